// Host construction of the device layout (see plan.h) and of query plans.
#include "plan.h"

#include <algorithm>
#include <cmath>

namespace peers {

namespace {
inline int32_t nwin_of(int32_t depth) { return (depth + kWin - 1) / kWin; }
}  // namespace

Status build_plan(const Symbolic& S, const Numeric& F, FactorPlan& P) {
  const int32_t N = S.N;
  P = FactorPlan();
  P.N = N;
  P.height = S.height;
  P.isd.resize(N);
  for (int32_t i = 0; i < N; ++i) P.isd[i] = 1.0 / std::sqrt(F.D[i]);
  P.bdepth.assign(S.depth.begin(), S.depth.end());
  // subtree size and height
  std::vector<int32_t> size(N, 1), hsub(N, 1);
  for (int32_t i = 0; i < N; ++i) {
    const int32_t p = S.parent[i];
    if (p >= 0) {
      size[p] += size[i];
      hsub[p] = std::max(hsub[p], hsub[i] + 1);
    }
  }
  P.small.assign(N, 0);
  for (int32_t i = 0; i < N; ++i) P.small[i] = size[i] <= kBottomMaxNodes && hsub[i] <= kBottomMaxHeight;
  // top indices, store offsets
  P.top_index.assign(N, -1);
  for (int32_t i = 0; i < N; ++i) {
    if (P.small[i]) continue;
    P.top_index[i] = (int32_t)P.top_node.size();
    P.top_node.push_back(i);
    P.top_off.push_back(P.store_elems);
    P.top_depth.push_back(S.depth[i]);
    P.top_isd.push_back(P.isd[i]);
    P.store_elems += (int64_t)nwin_of(S.depth[i]) * kWin;
  }
  P.ntop = (int32_t)P.top_node.size();

  // ---------------------------------------------------------------- top chunks
  const int32_t ns = (int32_t)S.snptr.size() - 1;
  std::vector<int32_t> chunk_of(N, -1);
  for (int32_t s = ns - 1; s >= 0; --s) {
    const int32_t f = S.snptr[s], l = S.snptr[s + 1] - 1;
    if (P.small[l]) continue;
    int32_t x = l;
    while (x > f && !P.small[x - 1]) --x;
    for (int32_t b = l; b >= x;) {
      const int32_t a = std::max(x, b - kChunk + 1);
      TopChunk c{};
      c.a = a;
      c.b = b;
      c.depth_b = S.depth[b];
      c.top_a = P.top_index[a];
      const int64_t e0 = S.colptr[b], e1 = S.colptr[b + 1];
      c.next = (int32_t)(e1 - e0);
      c.ext_begin = (int64_t)P.ext_top.size();
      for (int64_t p = e0; p < e1; ++p) {
        const int32_t k = S.rowidx[p];
        if (P.top_index[k] < 0) { set_error("plan: an ancestor of a top node is not top"); return E_INTERNAL; }
        P.ext_top.push_back(P.top_index[k]);
        P.ext_off.push_back(P.top_off[P.top_index[k]]);
        P.ext_depth.push_back(S.depth[k]);
      }
      const int32_t wc = b - a + 1;
      c.coef_begin = (int64_t)P.coef.size();
      P.coef.resize(P.coef.size() + (size_t)c.next * kChunk, 0.0);
      for (int32_t j = 0; j < wc; ++j) {
        const int64_t base = S.colptr[a + j] + (b - a - j);
        for (int32_t e = 0; e < c.next; ++e) P.coef[c.coef_begin + (int64_t)e * kChunk + j] = -F.Lx[base + e];
      }
      c.tri_begin = (int64_t)P.tri.size();
      P.tri.resize(P.tri.size() + (size_t)kChunk * kChunk, 0.0);
      for (int32_t j = 0; j < wc; ++j)
        for (int32_t jj = 0; jj < j; ++jj) {
          const int64_t p = S.colptr[a + jj] + (j - jj - 1);
          if (S.rowidx[p] != a + j) { set_error("plan: chunk is not a dense chain"); return E_INTERNAL; }
          P.tri[c.tri_begin + (int64_t)j * kChunk + jj] = -F.Lx[p];
        }
      // level: one more than the chunk holding b's parent
      const int32_t pb = S.parent[b];
      c.level = pb < 0 ? 0 : P.chunks[chunk_of[pb]].level + 1;
      const int32_t cid = (int32_t)P.chunks.size();
      for (int32_t v = a; v <= b; ++v) chunk_of[v] = cid;
      P.chunks.push_back(c);
      for (int32_t v = a; v <= b; ++v)
        for (int64_t p = S.colptr[v]; p < S.colptr[v + 1]; ++p) P.f_top += S.depth[S.rowidx[p]];
      b = a - 1;
    }
  }
  int32_t maxlev = -1;
  for (const auto& c : P.chunks) maxlev = std::max(maxlev, c.level);
  P.nlevels = maxlev + 1;
  {
    std::vector<int64_t> cnt(P.nlevels + 1, 0);
    for (const auto& c : P.chunks) cnt[c.level + 1] += nwin_of(S.depth[c.a]);
    for (int32_t l = 0; l < P.nlevels; ++l) cnt[l + 1] += cnt[l];
    P.level_ptr = cnt;
    P.task_chunk.assign(cnt[P.nlevels], 0);
    P.task_win.assign(cnt[P.nlevels], 0);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int32_t ci = 0; ci < (int32_t)P.chunks.size(); ++ci) {
      const auto& c = P.chunks[ci];
      const int32_t nw = nwin_of(S.depth[c.a]);
      for (int32_t t = 0; t < nw; ++t) {
        P.task_chunk[fill[c.level]] = ci;
        P.task_win[fill[c.level]++] = t;
      }
    }
  }

  // ---------------------------------------------------------------- bottom subtrees
  P.lslot.assign(N, -1);
  for (int32_t i = N - 1; i >= 0; --i) {
    if (!P.small[i]) continue;
    const int32_t p = S.parent[i];
    P.lslot[i] = (p < 0 || !P.small[p]) ? 0 : P.lslot[p] + 1;
    P.max_lslot = std::max(P.max_lslot, P.lslot[i]);
  }
  P.btask_ptr.assign(1, 0);
  int32_t cur = 0, curmaxd = 0;
  auto close_task = [&]() {
    if (cur == 0) return;
    P.btask_ptr.push_back((int32_t)P.bnodes.size());
    P.btask_nwin.push_back(nwin_of(curmaxd));
    cur = 0;
    curmaxd = 0;
  };
  for (int32_t r = 0; r < N; ++r) {
    if (!P.small[r]) continue;
    const int32_t p = S.parent[r];
    if (p >= 0 && P.small[p]) continue;  // not a bottom root
    const int32_t sz = r - S.first[r] + 1;
    if (cur > 0 && cur + sz > kBottomMaxNodes) close_task();
    for (int32_t v = r; v >= S.first[r]; --v) {
      P.bnodes.push_back(v);
      curmaxd = std::max(curmaxd, S.depth[v]);
    }
    cur += sz;
  }
  close_task();
  const int32_t nbt = (int32_t)P.btask_nwin.size();
  for (int32_t t = 0; t < nbt; ++t)
    for (int32_t w = 0; w < P.btask_nwin[t]; ++w) {
      P.bwork_task.push_back(t);
      P.bwork_win.push_back(w);
    }
  P.bent_ptr.assign(N + 1, 0);
  for (int32_t i = 0; i < N; ++i)
    P.bent_ptr[i + 1] = P.bent_ptr[i] + (P.small[i] ? S.colptr[i + 1] - S.colptr[i] : 0);
  P.bent_src.resize(P.bent_ptr[N]);
  P.bent_coef.resize(P.bent_ptr[N]);
  for (int32_t i = 0; i < N; ++i) {
    if (!P.small[i]) continue;
    int64_t q = P.bent_ptr[i];
    for (int64_t p = S.colptr[i]; p < S.colptr[i + 1]; ++p, ++q) {
      const int32_t k = S.rowidx[p];
      P.bent_src[q] = P.small[k] ? P.lslot[k] : -(P.top_index[k] + 1);
      P.bent_coef[q] = -F.Lx[p];
    }
  }
  for (int32_t t = 0; t < nbt; ++t) {
    int64_t nnz = 0;
    for (int32_t k = P.btask_ptr[t]; k < P.btask_ptr[t + 1]; ++k) {
      const int32_t v = P.bnodes[k];
      nnz += S.colptr[v + 1] - S.colptr[v];
    }
    P.f_bottom_computed += (double)nnz * kWin * P.btask_nwin[t];
  }
  return OK;
}

Status build_query_plan(const std::vector<int32_t>& first, const std::vector<int32_t>& depth,
                        const FactorPlan& P, int64_t q, const int32_t* a, const int32_t* b, QueryPlan& Q) {
  const int32_t N = P.N;
  Q = QueryPlan();
  Q.q = q;
  Q.bq_ptr.assign(N + 1, 0);
  std::vector<int32_t> lo_of(q, -2), hi_of(q, -1);
  for (int64_t k = 0; k < q; ++k) {
    const int32_t x = a[k], y = b[k];
    if (x == y) { Q.zero_out.push_back(k); continue; }
    int32_t lo, hi;
    if (x < 0) { lo = y; hi = -1; }
    else if (y < 0) { lo = x; hi = -1; }
    else { lo = std::min(x, y); hi = std::max(x, y); }
    if (hi >= 0 && first[hi] > lo) { Q.n_general++; continue; }
    lo_of[k] = lo;
    hi_of[k] = hi;
    if (P.small[lo]) Q.bq_ptr[lo + 1]++;
    else {
      Q.tq_lo.push_back(P.top_index[lo]);
      Q.tq_hi.push_back(hi < 0 ? -1 : P.top_index[hi]);
      Q.tq_out.push_back(k);
    }
  }
  for (int32_t i = 0; i < N; ++i) Q.bq_ptr[i + 1] += Q.bq_ptr[i];
  const int64_t nb = Q.bq_ptr[N];
  Q.bq_hicode.resize(nb);
  Q.bq_out.resize(nb);
  Q.bq_slot.resize(nb);
  Q.bq_nwin.resize(nb);
  std::vector<int32_t> fill(Q.bq_ptr.begin(), Q.bq_ptr.end() - 1);
  for (int64_t k = 0; k < q; ++k) {
    const int32_t lo = lo_of[k];
    if (lo < 0 || !P.small[lo]) continue;
    const int32_t hi = hi_of[k];
    const int32_t j = fill[lo]++;
    Q.bq_out[j] = k;
    Q.bq_hicode[j] = hi < 0 ? kGroundCode : (P.small[hi] ? P.lslot[hi] : -(P.top_index[hi] + 1));
  }
  int64_t slot = 0;
  for (int32_t i = 0; i < N; ++i)
    for (int32_t j = Q.bq_ptr[i]; j < Q.bq_ptr[i + 1]; ++j) {
      Q.bq_slot[j] = slot;
      Q.bq_nwin[j] = nwin_of(depth[i]);
      slot += Q.bq_nwin[j];
    }
  Q.nslots = slot;
  return OK;
}

}  // namespace peers
