// Host plan of the device factorization (see numplan.h).
#include "numplan.h"

#include <algorithm>
#include <atomic>

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
  const int threads = default_threads();
  // A at the factor's positions (columns in parallel: each writes its own)
  Q.lx0.assign(Q.nnz, 0.0);
  Q.r0.assign(N, 0.0);
  std::atomic<bool> outside{false};
  parallel_for((N + 4095) / 4096, threads, [&](int64_t blk) {
    const int32_t j1 = (int32_t)std::min<int64_t>(N, (blk + 1) * 4096);
    for (int32_t j = (int32_t)(blk * 4096); j < j1; ++j) {
      const int32_t r = S.perm[j];
      Q.r0[j] = ing.gnd[r];
      for (int64_t p = ing.A.ptr[r]; p < ing.A.ptr[r + 1]; ++p) {
        const int32_t i = S.iperm[ing.A.idx[p]];
        if (i <= j) continue;
        const int64_t pos = find_row(S, j, i);
        if (pos < 0) outside = true;
        else Q.lx0[pos] += ing.A.val[p];
      }
    }
  });
  if (outside) { set_error("numeric plan: an entry of A outside the factor pattern"); return E_INTERNAL; }
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
  // 3. pieces of the top chains and the tree they form
  std::vector<int32_t> piece_of(N, -1);
  for (int32_t c = 0; c < (int32_t)P.chains.size(); ++c) {
    const Chain& C = P.chains[c];
    for (int32_t a = C.a; a <= C.b; a += kFacPiece) {
      FacPiece f{};
      f.a = a;
      f.b = std::min(C.b, a + kFacPiece - 1);
      f.w = f.b - f.a + 1;
      f.dp = S.depth[f.b] - 1;
      f.col_base = C.store_base + (int64_t)(a - C.a) * C.ld;
      f.ld = C.ld;
      f.u_begin = (int64_t)Q.pu_depth.size();
      for (int64_t p = S.colptr[f.b]; p < S.colptr[f.b + 1]; ++p) {
        const int32_t u = S.rowidx[p];
        if (P.top_index[u] < 0) { set_error("numeric plan: a row above a top chain is not a top node"); return E_INTERNAL; }
        Q.pu_depth.push_back(S.depth[u]);
        Q.pu_top.push_back(P.top_index[u]);
      }
      f.nU = (int32_t)((int64_t)Q.pu_depth.size() - f.u_begin);
      f.ldu = (int64_t)((std::max(f.nU, 1) + 63) / 64) * 64;
      for (int32_t v = f.a; v <= f.b; ++v) piece_of[v] = (int32_t)Q.pieces.size();
      Q.pieces.push_back(f);
    }
  }
  const int32_t np = (int32_t)Q.pieces.size();
  // levels: parents first (a piece's parent holds parent(b), a larger index)
  int32_t nlev = 0;
  for (int32_t x = np - 1; x >= 0; --x) {
    FacPiece& f = Q.pieces[x];
    const int32_t pb = S.parent[f.b];
    f.level = pb < 0 ? 0 : Q.pieces[piece_of[pb]].level + 1;
    nlev = std::max(nlev, f.level + 1);
  }
  std::vector<std::vector<int32_t>> lev(nlev);
  for (int32_t x = 0; x < np; ++x) lev[Q.pieces[x].level].push_back(x);
  Q.lev_ptr.assign(1, 0);
  Q.ur_ptr.assign(1, 0);
  Q.gemm_ptr.assign(1, 0);
  Q.sc_ptr.assign(1, 0);
  Q.sc_src_ptr.assign(1, 0);
  for (int32_t l = nlev - 1; l >= 0; --l) {
    int64_t goff = 0, loff = 0;
    std::vector<std::pair<int32_t, std::pair<int32_t, int32_t>>> dst;  // (top index, (piece, pos))
    for (int32_t x : lev[l]) {
      FacPiece& f = Q.pieces[x];
      Q.lev_piece.push_back(x);
      if (f.nU == 0) continue;
      f.luc_off = loff;
      loff += f.ldu * f.w;
      f.g_off = goff;
      goff += f.ldu * f.nU;
      for (int32_t e0 = 0; e0 < f.nU; e0 += kFacRowTile) {
        Q.ur_piece.push_back(x);
        Q.ur_row0.push_back(e0);
      }
      GemmProb g{};
      g.a_buf = BUF_LUC; g.a_off = f.luc_off; g.lda = f.ldu; g.aoff_begin = -1; g.gather = 0;
      g.b_buf = BUF_BT; g.b_off = f.luc_off; g.ldb = f.ldu; g.trans = 1;  // (k, j) at k * ldb + j
      g.c_buf = BUF_G; g.c_off = f.g_off; g.ldc = f.ldu;
      g.M = f.nU; g.N = f.nU; g.K = f.w; g.alpha = 1.0;
      const int32_t pid = (int32_t)Q.probs.size();
      Q.probs.push_back(g);
      for (int32_t r0 = 0; r0 < f.nU; r0 += kTileM)
        for (int32_t c0 = 0; c0 < f.nU; c0 += kTileN)
          if (r0 + kTileM - 1 > c0) Q.tasks.push_back(GemmTask{pid, r0, c0, 0, f.w});  // below the diagonal
      for (int32_t e = 0; e < f.nU; ++e) dst.push_back({Q.pu_top[f.u_begin + e], {x, e}});
    }
    Q.luc_elems = std::max(Q.luc_elems, loff);
    Q.g_elems = std::max(Q.g_elems, goff);
    Q.lev_ptr.push_back((int32_t)Q.lev_piece.size());
    Q.ur_ptr.push_back((int32_t)Q.ur_piece.size());
    Q.gemm_ptr.push_back((int64_t)Q.tasks.size());
    std::stable_sort(dst.begin(), dst.end(), [](const auto& x, const auto& y) {
      return x.first != y.first ? x.first < y.first : x.second.first < y.second.first;
    });
    for (size_t i = 0; i < dst.size(); ++i) {
      if (i == 0 || dst[i].first != dst[i - 1].first) {
        if (i) Q.sc_src_ptr.push_back((int32_t)Q.sc_piece.size());
        Q.sc_dest.push_back(dst[i].first);
      }
      Q.sc_piece.push_back(dst[i].second.first);
      Q.sc_pos.push_back(dst[i].second.second);
    }
    if (!dst.empty()) Q.sc_src_ptr.push_back((int32_t)Q.sc_piece.size());
    Q.sc_ptr.push_back((int32_t)Q.sc_dest.size());
  }
  Q.steps = nlev;
  // 4. top columns' factor values go to L_CC (lcc) or L_{U,C} (luc): rows
  //    of the chain by their offset, rows above it by their position in U_C
  //    (the pattern of the chain's last column, ascending)
  Q.top_x_ptr.assign(P.ntop + 1, 0);
  for (int32_t t = 0; t < P.ntop; ++t) {
    const int32_t j = P.top_node[t];
    Q.top_x_ptr[t + 1] = Q.top_x_ptr[t] + (S.colptr[j + 1] - S.colptr[j]);
  }
  Q.top_src.assign(Q.top_x_ptr[P.ntop], 0);
  std::atomic<bool> bad{false};
  parallel_for((int64_t)P.chains.size(), threads, [&](int64_t ci) {
    const Chain& C = P.chains[ci];
    const int32_t* U = S.rowidx.data() + S.colptr[C.b];
    for (int32_t v = C.a; v <= C.b; ++v) {
      const int32_t jj = v - C.a;
      int64_t x = Q.top_x_ptr[P.top_index[v]];
      int32_t e = 0;
      for (int64_t p = S.colptr[v]; p < S.colptr[v + 1]; ++p, ++x) {
        const int32_t i = S.rowidx[p];
        if (i <= C.b) {
          Q.top_src[x] = C.lcc_off + (int64_t)jj * C.ldl + (i - C.a);
        } else {
          while (e < C.nU && U[e] != i) ++e;  // both ascending
          if (e == C.nU) { bad = true; return; }
          Q.top_src[x] = kLxFromLuc | (C.luc_off + (int64_t)jj * C.ldb + e);
        }
      }
    }
  });
  if (bad) { set_error("numeric plan: a row above a chain is not in U_C"); return E_INTERNAL; }
  Q.bnode_node = P.bnode_node;
  Q.bottom_records = (int64_t)P.bnode_node.size();
  return OK;
}

}  // namespace peers
