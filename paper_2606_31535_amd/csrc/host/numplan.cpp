// Host plan of the device factorization (see numplan.h).
#include "numplan.h"

#include <algorithm>

namespace peers {

namespace {
inline int64_t find_row(const Symbolic& S, int32_t col, int32_t row) {
  const int32_t* b = S.rowidx.data() + S.colptr[col];
  const int32_t* e = S.rowidx.data() + S.colptr[col + 1];
  const int32_t* it = std::lower_bound(b, e, row);
  return (it != e && *it == row) ? (int64_t)(it - S.rowidx.data()) : -1;
}
}  // namespace

Status build_numeric_plan(const Ingested& ing, const Symbolic& S, const FactorPlan& P, NumericPlan& Q) {
  const int32_t N = S.N;
  Q = NumericPlan();
  Q.N = N;
  Q.nnz = S.colptr[N];
  Q.height = S.height;
  // A at the factor's positions
  Q.lx0.assign(Q.nnz, 0.0);
  Q.r0.assign(N, 0.0);
  for (int32_t j = 0; j < N; ++j) {
    const int32_t r = S.perm[j];
    Q.r0[j] = ing.gnd[r];
    for (int64_t p = ing.A.ptr[r]; p < ing.A.ptr[r + 1]; ++p) {
      const int32_t i = S.iperm[ing.A.idx[p]];
      if (i <= j) continue;
      const int64_t pos = find_row(S, j, i);
      if (pos < 0) { set_error("numeric plan: an entry of A outside the factor pattern"); return E_INTERNAL; }
      Q.lx0[pos] += ing.A.val[p];
    }
  }
  // 1. bottom tasks, columns ascending, and their pair targets
  const int32_t nbt = (int32_t)P.btask_nwin.size();
  Q.bt_ptr.assign(1, 0);
  Q.bpair_ptr.assign(1, 0);
  for (int32_t t = 0; t < nbt; ++t) {
    // the task's records are in descending node order
    for (int32_t k = P.btask_ptr[t + 1] - 1; k >= P.btask_ptr[t]; --k) {
      const int32_t v = P.bnode_node[k];
      Q.bcol.push_back(v);
      for (int64_t p = S.colptr[v]; p < S.colptr[v + 1]; ++p) {
        const int32_t j = S.rowidx[p];
        if (!P.small[j]) continue;
        for (int64_t q = p + 1; q < S.colptr[v + 1]; ++q) {
          const int64_t pos = find_row(S, j, S.rowidx[q]);
          if (pos < 0) { set_error("numeric plan: fill outside the factor pattern"); return E_INTERNAL; }
          Q.bpair.push_back(pos);
        }
      }
      Q.bpair_ptr.push_back((int64_t)Q.bpair.size());
    }
    Q.bt_ptr.push_back((int32_t)Q.bcol.size());
  }
  // 2. top columns' pulls from bottom columns (k ascending)
  {
    std::vector<int32_t> cnt(P.ntop + 1, 0);
    for (int32_t k = 0; k < N; ++k) {
      if (!P.small[k]) continue;
      for (int64_t p = S.colptr[k]; p < S.colptr[k + 1]; ++p)
        if (!P.small[S.rowidx[p]]) cnt[P.top_index[S.rowidx[p]] + 1]++;
    }
    for (int32_t t = 0; t < P.ntop; ++t) cnt[t + 1] += cnt[t];
    Q.tg_ptr = cnt;
    Q.tg_k.resize(cnt[P.ntop]);
    Q.tg_p.resize(cnt[P.ntop]);
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (int32_t k = 0; k < N; ++k) {
      if (!P.small[k]) continue;
      for (int64_t p = S.colptr[k]; p < S.colptr[k + 1]; ++p) {
        const int32_t j = S.rowidx[p];
        if (P.small[j]) continue;
        const int32_t slot = fill[P.top_index[j]]++;
        Q.tg_k[slot] = k;
        Q.tg_p[slot] = p;
      }
    }
  }
  // 3. chain levels, deepest first
  const int32_t nch = (int32_t)P.chains.size();
  std::vector<std::vector<int32_t>> lev(P.nchain_levels);
  for (int32_t c = 0; c < nch; ++c) lev[P.chains[c].level].push_back(c);
  Q.lev_ptr.assign(1, 0);
  Q.ur_ptr.assign(1, 0);
  Q.gemm_ptr.assign(1, 0);
  Q.sc_ptr.assign(1, 0);
  Q.sc_src_ptr.assign(1, 0);
  Q.g_off.assign(nch, 0);
  for (int32_t l = P.nchain_levels - 1; l >= 0; --l) {
    int64_t goff = 0;
    for (int32_t c : lev[l]) {
      const Chain& C = P.chains[c];
      Q.lev_chain.push_back(c);
      if (C.nU == 0) continue;
      for (int32_t e0 = 0; e0 < C.nU; e0 += 64) {
        Q.ur_chain.push_back(c);
        Q.ur_row0.push_back(e0);
      }
      GemmProb g{};
      g.a_buf = BUF_LUC; g.a_off = C.luc_off; g.lda = C.ldb; g.aoff_begin = -1; g.gather = 0;
      g.b_buf = BUF_BT; g.b_off = C.bt_off; g.ldb = C.ldb; g.trans = 1;  // (k, j) at k * ldb + j
      g.c_buf = BUF_G; g.c_off = goff; g.ldc = C.ldb;
      g.M = C.nU; g.N = C.nU; g.K = C.w; g.alpha = 1.0;
      const int32_t pid = (int32_t)Q.probs.size();
      Q.probs.push_back(g);
      for (int32_t r0 = 0; r0 < C.nU; r0 += kTileM)
        for (int32_t c0 = 0; c0 < C.nU; c0 += kTileN)
          if (r0 + kTileM - 1 > c0) Q.tasks.push_back(GemmTask{pid, r0, c0, 0, C.w});  // below the diagonal
      Q.g_off[c] = goff;
      goff += C.ldb * C.nU;
    }
    Q.g_elems = std::max(Q.g_elems, goff);
    Q.lev_ptr.push_back((int32_t)Q.lev_chain.size());
    Q.ur_ptr.push_back((int32_t)Q.ur_chain.size());
    Q.gemm_ptr.push_back((int64_t)Q.tasks.size());
  }
  Q.steps = P.nchain_levels;
  // scatter lists per step: U_C's nodes are known by their store offsets in
  // the gather table, mapped back to top indices here
  {
    std::vector<std::pair<int64_t, int32_t>> off2t(P.ntop);
    for (int32_t t = 0; t < P.ntop; ++t) off2t[t] = {P.top_off[t], t};
    std::sort(off2t.begin(), off2t.end());
    auto top_of_off = [&](int64_t off) -> int32_t {
      auto it = std::lower_bound(off2t.begin(), off2t.end(), std::make_pair(off, (int32_t)-1));
      return (it != off2t.end() && it->first == off) ? it->second : -1;
    };
    for (int32_t step = 0; step < Q.steps; ++step) {
      std::vector<std::pair<int32_t, std::pair<int32_t, int32_t>>> dst;  // (top index, (chain, pos))
      for (int32_t x = Q.lev_ptr[step]; x < Q.lev_ptr[step + 1]; ++x) {
        const int32_t c = Q.lev_chain[x];
        const Chain& C = P.chains[c];
        for (int32_t e = 0; e < C.nU; ++e) {
          const int32_t t = top_of_off(P.u_off[C.u_begin + e]);
          if (t < 0) { set_error("numeric plan: a U column is not a top column"); return E_INTERNAL; }
          dst.push_back({t, {c, e}});
        }
      }
      std::stable_sort(dst.begin(), dst.end(), [](const auto& x, const auto& y) {
        return x.first != y.first ? x.first < y.first : x.second.first < y.second.first;
      });
      for (size_t i = 0; i < dst.size(); ++i) {
        if (i == 0 || dst[i].first != dst[i - 1].first) {
          if (i) Q.sc_src_ptr.push_back((int32_t)Q.sc_chain.size());
          Q.sc_dest.push_back(dst[i].first);
        }
        Q.sc_chain.push_back(dst[i].second.first);
        Q.sc_pos.push_back(dst[i].second.second);
      }
      if (!dst.empty()) Q.sc_src_ptr.push_back((int32_t)Q.sc_chain.size());
      Q.sc_ptr.push_back((int32_t)Q.sc_dest.size());
    }
  }
  // 4. top columns' factor values come from L_CC (lcc) or L_{U,C} (luc)
  for (int32_t t = 0; t < P.ntop; ++t) {
    const int32_t j = P.top_node[t];
    const Chain& C = P.chains[P.top_chain[t]];
    const int32_t jj = j - C.a;
    int64_t e = 0;
    for (int64_t p = S.colptr[j]; p < S.colptr[j + 1]; ++p) {
      const int32_t i = S.rowidx[p];
      Q.top_pos.push_back(p);
      if (i <= C.b) {
        Q.top_src.push_back(C.lcc_off + (int64_t)jj * C.ldl + (i - C.a));
      } else {
        // position of i in U_C: U_C ascending; rows of column j above the
        // chain are a subset of it in the same order
        const int64_t off = P.top_off[P.top_index[i]];
        while (e < C.nU && P.u_off[C.u_begin + e] != off) ++e;
        if (e == C.nU) { set_error("numeric plan: a row above a chain is not in U_C"); return E_INTERNAL; }
        Q.top_src.push_back(kLxFromLuc | (C.luc_off + (int64_t)jj * C.ldb + e));
      }
    }
  }
  Q.bnode_node = P.bnode_node;
  Q.bottom_records = (int64_t)P.bnode_node.size();
  return OK;
}

}  // namespace peers
