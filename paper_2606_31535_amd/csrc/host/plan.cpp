// Host construction of the device layout (see plan.h) and of query plans.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <functional>

namespace peers {

namespace {
inline int32_t nwin_of(int32_t depth) { return (depth + kWin - 1) / kWin; }
// windows of a top column as the sweep reads them: whole groups of kWinPerWave
inline int32_t nwin_grouped(int32_t depth) {
  return (nwin_of(depth) + kWinPerWave - 1) / kWinPerWave * kWinPerWave;
}
}  // namespace

Status build_plan(const Symbolic& S, const Numeric* Fp, FactorPlan& P) {
  const int32_t N = S.N;
  P = FactorPlan();
  P.N = N;
  P.height = S.height;
  const bool record = Fp == nullptr;
  auto lval = [&](int64_t q) { return Fp ? Fp->Lx[q] : 0.0; };
  P.isd.resize(N);
  for (int32_t i = 0; i < N; ++i) P.isd[i] = Fp ? 1.0 / std::sqrt(Fp->D[i]) : 1.0;
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
    P.top_off.push_back(-1);
    P.top_depth.push_back(S.depth[i]);
    P.top_isd.push_back(P.isd[i]);
  }
  P.ntop = (int32_t)P.top_node.size();

  // ---------------------------------------------------------------- top chains
  // maximal runs a..b of top nodes with parent(i) = i+1 (top indices of a run
  // are consecutive because top nodes are numbered in increasing node order)
  P.top_chain.assign(P.ntop, -1);
  std::vector<int32_t> chain_of(N, -1);
  for (int32_t t = 0; t < P.ntop;) {
    const int32_t a = P.top_node[t];
    int32_t b = a, t2 = t;
    while (t2 + 1 < P.ntop && P.top_node[t2 + 1] == b + 1 && S.parent[b] == b + 1) { ++b; ++t2; }
    Chain c{};
    c.a = a;
    c.b = b;
    c.w = b - a + 1;
    c.dp = S.parent[b] < 0 ? 0 : S.depth[S.parent[b]];
    for (int32_t v = a; v <= b; ++v) {
      chain_of[v] = (int32_t)P.chains.size();
      P.top_chain[P.top_index[v]] = (int32_t)P.chains.size();
    }
    P.chains.push_back(c);
    t = t2 + 1;
  }
  const int32_t nch = (int32_t)P.chains.size();
  // levels (parents first: chains with larger node indices come later)
  for (int32_t ci = nch - 1; ci >= 0; --ci) {
    Chain& c = P.chains[ci];
    const int32_t pb = S.parent[c.b];
    c.level = pb < 0 ? 0 : P.chains[chain_of[pb]].level + 1;
    P.nchain_levels = std::max(P.nchain_levels, c.level + 1);
  }
  P.chain_parent.assign(nch, -1);
  for (int32_t ci = 0; ci < nch; ++ci) {
    const int32_t pb = S.parent[P.chains[ci].b];
    P.chain_parent[ci] = pb < 0 ? -1 : chain_of[pb];
  }
  // U_C, store layout, dense blocks
  std::vector<int32_t> mark(N, -1), upos(N, -1);
  int64_t lcc_elems = 0, luc_elems = 0;
  P.store_elems = kStoreZeroBlock;  // leading zero block
  for (int32_t ci = 0; ci < nch; ++ci) {
    Chain& c = P.chains[ci];
    std::vector<int32_t> U;
    for (int32_t v = c.a; v <= c.b; ++v)
      for (int64_t p = S.colptr[v]; p < S.colptr[v + 1]; ++p) {
        const int32_t r = S.rowidx[p];
        if (r > c.b && mark[r] != ci) { mark[r] = ci; U.push_back(r); }
      }
    // the rows above the chain that any of its columns reaches are exactly
    // the pattern of its last column (parent(v) = v + 1 inside the chain, and
    // struct(v) minus parent(v) lies in struct(parent(v)))
    if ((int64_t)U.size() != S.colptr[c.b + 1] - S.colptr[c.b]) { set_error("plan: inconsistent U"); return E_INTERNAL; }
    U.assign(S.rowidx.begin() + S.colptr[c.b], S.rowidx.begin() + S.colptr[c.b + 1]);
    c.nU = (int32_t)U.size();
    c.u_begin = (int64_t)P.u_off.size();
    for (int32_t e = 0; e < c.nU; ++e) {
      if (P.top_index[U[e]] < 0) { set_error("plan: an ancestor of a top node is not top"); return E_INTERNAL; }
      P.u_depth.push_back(S.depth[U[e]]);
      P.u_off.push_back(-1);  // filled once every chain has its store base
    }
    c.ld = (int64_t)nwin_grouped(c.dp + c.w) * kWin;
    c.store_base = P.store_elems;
    P.store_elems += c.ld * c.w;
    for (int32_t j = 0; j < c.w; ++j) P.top_off[P.top_index[c.a + j]] = c.store_base + (int64_t)j * c.ld;
    c.ldl = (int64_t)nwin_of(c.w) * kWin;
    c.lcc_off = lcc_elems;
    c.x_off = lcc_elems;
    lcc_elems += c.ldl * c.w;
    c.ldb = (int64_t)nwin_of(std::max(c.nU, 1)) * kWin;
    c.bt_off = luc_elems;
    c.luc_off = luc_elems;
    luc_elems += c.nU > 0 ? c.ldb * c.w : 0;
  }
  // gather table: store offset of every U_C column (needs all store bases)
  for (int32_t ci = 0; ci < nch; ++ci) {
    const Chain& c = P.chains[ci];
    const int32_t* U = S.rowidx.data() + S.colptr[c.b];
    for (int32_t e = 0; e < c.nU; ++e) P.u_off[c.u_begin + e] = P.top_off[P.top_index[U[e]]];
  }
  // dense L_CC (unit diagonal stored) and L_{U,C}, column-major
  P.lcc.assign(lcc_elems, 0.0);
  P.luc.assign(luc_elems, 0.0);
  {
    for (int32_t ci = 0; ci < nch; ++ci) {
      const Chain& c = P.chains[ci];
      const int32_t* U = S.rowidx.data() + S.colptr[c.b];
      for (int32_t e = 0; e < c.nU; ++e) upos[U[e]] = e;
      for (int32_t j = 0; j < c.w; ++j) {
        const int32_t v = c.a + j;
        P.lcc[c.lcc_off + (int64_t)j * c.ldl + j] = 1.0;
        for (int64_t p = S.colptr[v]; p < S.colptr[v + 1]; ++p) {
          const int32_t r = S.rowidx[p];
          if (r <= c.b) P.lcc[c.lcc_off + (int64_t)j * c.ldl + (r - c.a)] = lval(p);
          else P.luc[c.luc_off + (int64_t)j * c.ldb + upos[r]] = lval(p);
        }
        for (int64_t p = S.colptr[v]; p < S.colptr[v + 1]; ++p) P.f_top += S.depth[S.rowidx[p]];
      }
    }
  }
  P.x_elems = lcc_elems;
  P.bt_elems = luc_elems;

  // ---------------------------------------------------------------- GEMM task lists
  auto add_tiles = [&](int32_t prob, int32_t M, int32_t Nn, auto krange) {
    for (int32_t r0 = 0; r0 < M; r0 += kTileM)
      for (int32_t c0 = 0; c0 < Nn; c0 += kTileN) {
        int32_t k0, k1;
        krange(r0, c0, k0, k1);
        P.tasks.push_back(GemmTask{prob, r0, c0, k0, k1});
      }
  };
  // upload: B_C = -L_{U,C} L_CC^{-1} (B operand lower triangular: k >= column)
  P.bpre_begin = (int64_t)P.tasks.size();
  for (int32_t ci = 0; ci < nch; ++ci) {
    const Chain& c = P.chains[ci];
    if (c.nU == 0) continue;
    GemmProb g{};
    g.a_buf = BUF_LUC; g.a_off = c.luc_off; g.lda = c.ldb; g.aoff_begin = -1; g.gather = 0;
    g.b_buf = BUF_X; g.b_off = c.x_off; g.ldb = c.ldl;
    g.c_buf = BUF_BT; g.c_off = c.bt_off; g.ldc = c.w; g.trans = 2;  // B_C row-major
    g.M = c.nU; g.N = c.w; g.K = c.w; g.alpha = -1.0;
    const int32_t pid = (int32_t)P.probs.size();
    P.probs.push_back(g);
    P.prob_chain.push_back(ci);
    add_tiles(pid, g.M, g.N, [&](int32_t, int32_t c0, int32_t& k0, int32_t& k1) { k0 = c0; k1 = g.K; });
    P.f_bpre += (double)c.nU * c.w * c.w / 2.0;
  }
  P.bpre_end = (int64_t)P.tasks.size();
  // recursive blocked inverse of every L_CC: merge nodes by height
  struct Merge { int32_t chain, lo, mid, hi; };
  std::vector<std::vector<Merge>> by_height(1);
  std::function<int(int32_t, int32_t, int32_t)> rec = [&](int32_t ci, int32_t lo, int32_t hi) -> int {
    if (hi - lo <= kBase) {
      P.base_blocks.push_back(BaseBlock{ci, lo, hi - lo});
      return 0;
    }
    const int32_t nb = (hi - lo + kBase - 1) / kBase;
    const int32_t mid = lo + (nb / 2) * kBase;
    const int h = 1 + std::max(rec(ci, lo, mid), rec(ci, mid, hi));
    if ((int)by_height.size() <= h) by_height.resize(h + 1);
    by_height[h].push_back(Merge{ci, lo, mid, hi});
    return h;
  };
  for (int32_t ci = 0; ci < nch; ++ci) rec(ci, 0, P.chains[ci].w);
  P.inv_heights = (int32_t)by_height.size() - 1;
  P.inv_T_ptr.assign(1, (int64_t)P.tasks.size());
  P.inv_X_ptr.assign(1, (int64_t)P.tasks.size());
  P.t_elems = 1;
  for (int32_t h = 1; h <= P.inv_heights; ++h) {
    int64_t toff = 0;
    std::vector<int64_t> tof;
    for (const Merge& mg : by_height[h]) {
      const Chain& c = P.chains[mg.chain];
      const int32_t n1 = mg.mid - mg.lo, n2 = mg.hi - mg.mid;
      const int64_t ldt = (int64_t)nwin_of(n2) * kWin;
      tof.push_back(toff);
      GemmProb g{};
      g.a_buf = BUF_LCC; g.a_off = c.lcc_off + (int64_t)mg.lo * c.ldl + mg.mid; g.lda = c.ldl; g.aoff_begin = -1;
      g.b_buf = BUF_X; g.b_off = c.x_off + (int64_t)mg.lo * c.ldl + mg.lo; g.ldb = c.ldl;
      g.c_buf = BUF_T; g.c_off = toff; g.ldc = ldt;
      g.M = n2; g.N = n1; g.K = n1; g.alpha = 1.0;
      const int32_t pid = (int32_t)P.probs.size();
      P.probs.push_back(g);
      P.prob_chain.push_back(mg.chain);
      add_tiles(pid, n2, n1, [&](int32_t, int32_t c0, int32_t& k0, int32_t& k1) { k0 = c0; k1 = n1; });
      P.f_top_inv += (double)n2 * n1 * n1 / 2.0;
      toff += ldt * n1;
    }
    P.t_elems = std::max(P.t_elems, toff);
    P.inv_T_ptr.push_back((int64_t)P.tasks.size());
    for (size_t q = 0; q < by_height[h].size(); ++q) {
      const Merge& mg = by_height[h][q];
      const Chain& c = P.chains[mg.chain];
      const int32_t n1 = mg.mid - mg.lo, n2 = mg.hi - mg.mid;
      const int64_t ldt = (int64_t)nwin_of(n2) * kWin;
      GemmProb g{};
      g.a_buf = BUF_X; g.a_off = c.x_off + (int64_t)mg.mid * c.ldl + mg.mid; g.lda = c.ldl; g.aoff_begin = -1;
      g.b_buf = BUF_T; g.b_off = tof[q]; g.ldb = ldt;
      g.c_buf = BUF_X; g.c_off = c.x_off + (int64_t)mg.lo * c.ldl + mg.mid; g.ldc = c.ldl;
      g.M = n2; g.N = n1; g.K = n2; g.alpha = -1.0;
      const int32_t pid = (int32_t)P.probs.size();
      P.probs.push_back(g);
      P.prob_chain.push_back(mg.chain);
      add_tiles(pid, n2, n1, [&](int32_t r0, int32_t, int32_t& k0, int32_t& k1) {
        k0 = 0;
        k1 = std::min(n2, r0 + kTileM);
      });
      P.f_top_inv += (double)n2 * n2 * n1 / 2.0;
    }
    P.inv_X_ptr.push_back((int64_t)P.tasks.size());
  }
  for (const BaseBlock& bb : P.base_blocks) P.f_top_inv += (double)bb.size * bb.size * bb.size / 6.0;
  // per sweep, level by level: Z[0:dp, C] = Z[0:dp, U_C] B_C (rows r need U with depth > r)
  P.t2_ptr.assign(1, (int64_t)P.tasks.size());
  P.t2n_ptr.assign(1, 0);
  {
    std::vector<std::vector<int32_t>> lev(P.nchain_levels);
    for (int32_t ci = 0; ci < nch; ++ci) lev[P.chains[ci].level].push_back(ci);
    for (int32_t l = 1; l < P.nchain_levels; ++l) {
      for (int32_t ci : lev[l]) {
        const Chain& c = P.chains[ci];
        GemmProb g{};
        g.a_buf = BUF_STORE; g.a_off = 0; g.lda = 0; g.aoff_begin = c.u_begin; g.gather = 1;
        g.b_buf = BUF_BT; g.b_off = c.bt_off; g.ldb = c.w; g.trans = 1;  // B_C row-major
        g.c_buf = BUF_STORE; g.c_off = c.store_base; g.ldc = c.ld;
        g.M = c.dp; g.N = c.w; g.K = c.nU; g.alpha = 1.0;
        const int32_t pid = (int32_t)P.probs.size();
        P.probs.push_back(g);
        P.prob_chain.push_back(ci);
        const int32_t* ud = P.u_depth.data() + c.u_begin;
        auto krange = [&](int32_t r0, int32_t, int32_t& k0, int32_t& k1) {
          k0 = 0;
          k1 = (int32_t)(std::lower_bound(ud, ud + c.nU, r0, std::greater<int32_t>()) - ud);  // depth > r0
        };
        if (g.N <= kNarrowN) {
          // narrow chains: one wavefront per 64 x 16 tile over the whole reduction
          for (int32_t r0 = 0; r0 < g.M; r0 += kTileM) {
            int32_t k0, k1;
            krange(r0, 0, k0, k1);
            P.ntasks.push_back(GemmTask{pid, r0, 0, k0, k1});
          }
        } else {
          add_tiles(pid, g.M, g.N, krange);
        }
        for (int32_t e = 0; e < c.nU; ++e) P.f_top_gemm += (double)ud[e] * c.w;
      }
      P.t2_ptr.push_back((int64_t)P.tasks.size());
      P.t2n_ptr.push_back((int64_t)P.ntasks.size());
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
  auto topref = [&](int32_t k) -> int64_t {
    const int32_t t = P.top_index[k];
    return store_ref(P.top_off[t], nwin_grouped(P.top_depth[t]));
  };
  // the bottom sweep addresses the store with 32-bit byte offsets when it can
  P.store_wide = P.store_elems * 8 >= (int64_t)UINT32_MAX;
  P.btask_ptr.assign(1, 0);
  P.btask_attach_ptr.assign(1, 0);
  int32_t cur = 0, curmaxd = 0;
  auto close_task = [&]() {
    if (cur == 0) return;
    P.btask_ptr.push_back((int32_t)P.bnode.size());
    P.btask_nwin.push_back(nwin_of(curmaxd));
    auto b = P.btask_attach.begin() + P.btask_attach_ptr.back();
    std::sort(b, P.btask_attach.end());
    P.btask_attach.erase(std::unique(b, P.btask_attach.end()), P.btask_attach.end());
    P.btask_attach_ptr.push_back((int32_t)P.btask_attach.size());
    cur = 0;
    curmaxd = 0;
  };
  for (int32_t r = 0; r < N; ++r) {
    if (!P.small[r]) continue;
    const int32_t p = S.parent[r];
    if (p >= 0 && P.small[p]) continue;  // not a bottom root
    const int32_t sz = r - S.first[r] + 1;
    if (cur > 0 && cur + sz > kBottomMaxNodes) close_task();
    if (p >= 0) P.btask_attach.push_back(chain_of[p]);  // the chain this subtree hangs from
    {
      // U_S = struct(r): every row of the subtree's columns outside it
      const int32_t K = (int32_t)(S.colptr[r + 1] - S.colptr[r]);
      P.sub_p0.push_back((int32_t)P.bnode.size());
      P.sub_p1.push_back((int32_t)P.bnode.size() + sz);
      P.sub_K.push_back(K);
      P.sub_ubeg.push_back((int32_t)P.sub_uoff.size());
      for (int64_t q = S.colptr[r]; q < S.colptr[r + 1]; ++q) {
        const int32_t u = S.rowidx[q];
        if (P.top_index[u] < 0) { set_error("plan: a row outside a bottom subtree is not a top node"); return E_INTERNAL; }
        P.sub_uoff.push_back(P.top_off[P.top_index[u]]);
        P.sub_udep.push_back(S.depth[u]);
        P.sub_unode.push_back(u);
      }
      P.sub_bbase.push_back(P.b_elems);
      if (K <= kDenseMaxK) P.b_elems += (int64_t)K * sz;
      P.bpos_sub.insert(P.bpos_sub.end(), sz, (int32_t)P.sub_p0.size() - 1);
    }
    for (int32_t v = r; v >= S.first[r]; --v) {
      BNode bn{};
      bn.isd = P.isd[v];
      bn.depth = S.depth[v];
      bn.slots = slot_code(P.lslot[v]) << kOwnSlotShift;
      int32_t tinl[2] = {-1, -1};
      std::vector<BEnt> more_lds, more_top;
      int32_t nl = 0, nt = 0;
      const int64_t bidx = (int64_t)P.bnode.size();
      std::vector<std::pair<int64_t, int64_t>> lds_q, top_q;  // (CSC position, index in its overflow list)
      for (int64_t q = S.colptr[v]; q < S.colptr[v + 1]; ++q) {
        const int32_t k = S.rowidx[q];
        const double c = -lval(q);
        if (P.small[k]) {
          if (nl < 3) {
            bn.lc[nl] = c;
            bn.slots |= slot_code(P.lslot[k]) << (kSlotBits * nl);
            if (record) {
              P.coef_p.push_back(q);
              P.coef_off.push_back(bidx * (int64_t)sizeof(BNode) + (int64_t)offsetof(BNode, lc) + 8 * nl);
            }
          } else {
            if (record) lds_q.push_back({q, (int64_t)more_lds.size()});
            more_lds.push_back(BEnt{slot_code(P.lslot[k]), c});
          }
          ++nl;
        } else {
          if (nt < 2) {
            bn.tref[nt] = topref(k);
            bn.tc[nt] = c;
            tinl[nt] = k;
            if (record) {
              P.coef_p.push_back(q);
              P.coef_off.push_back(bidx * (int64_t)sizeof(BNode) + (int64_t)offsetof(BNode, tc) + 8 * nt);
            }
          } else {
            if (record) top_q.push_back({q, (int64_t)more_top.size()});
            more_top.push_back(BEnt{topref(k), c});
          }
          ++nt;
        }
      }
      if (record) {
        const int64_t b0 = (int64_t)P.bent.size();
        for (auto& e : lds_q) {
          P.coef_p.push_back(e.first);
          P.coef_off.push_back(kCoefInBent | ((b0 + e.second) * (int64_t)sizeof(BEnt) + (int64_t)offsetof(BEnt, coef)));
        }
        for (auto& e : top_q) {
          P.coef_p.push_back(e.first);
          P.coef_off.push_back(kCoefInBent | ((b0 + (int64_t)more_lds.size() + e.second) * (int64_t)sizeof(BEnt) +
                                              (int64_t)offsetof(BEnt, coef)));
        }
      }
      bn.slots |= std::min(nl, 3) << kInlineCountShift;
      if (more_top.size() > 32767 || P.bent.size() + more_lds.size() + more_top.size() > (size_t)INT32_MAX) {
        set_error("plan: bottom column too long for the node record");
        return E_INTERNAL;
      }
      bn.ent = (int32_t)P.bent.size();
      bn.n_more = (int32_t)more_lds.size() | ((int32_t)more_top.size() << 16);
      P.bent.insert(P.bent.end(), more_lds.begin(), more_lds.end());
      P.bent.insert(P.bent.end(), more_top.begin(), more_top.end());
      P.bnode_tinl.push_back(tinl[0]);
      P.bnode_tinl.push_back(tinl[1]);
      P.bnode.push_back(bn);
      P.bnode_node.push_back(v);
      curmaxd = std::max(curmaxd, S.depth[v]);
    }
    cur += sz;
  }
  close_task();
  // the sweep reads the records of the next three positions ahead of time
  P.bnode.push_back(BNode{});
  P.bnode.push_back(BNode{});
  P.bnode.push_back(BNode{});
  P.bent.push_back(BEnt{0, 0.0});
  const int32_t nbt = (int32_t)P.btask_nwin.size();
  P.bpos_task.assign(P.bnode_node.size(), 0);
  P.node_pos.assign(N, -1);
  for (int32_t k = 0; k < (int32_t)P.bnode_node.size(); ++k) P.node_pos[P.bnode_node[k]] = k;
  for (int32_t t = 0; t < nbt; ++t)
    for (int32_t k = P.btask_ptr[t]; k < P.btask_ptr[t + 1]; ++k) P.bpos_task[k] = t;
  P.max_btask_nwin = 0;
  {
    double fb = 0;
    for (int32_t t = 0; t < nbt; ++t) {
      P.max_btask_nwin = std::max(P.max_btask_nwin, P.btask_nwin[t]);
      int64_t nnz = 0;
      for (int32_t k = P.btask_ptr[t]; k < P.btask_ptr[t + 1]; ++k) {
        const int32_t v = P.bnode_node[k];
        nnz += S.colptr[v + 1] - S.colptr[v];
      }
      fb += (double)nnz * kWin * P.btask_nwin[t];
    }
    P.f_bottom_computed = fb;
  }
  return OK;
}

void AncestorTable::build(const std::vector<int32_t>& parent_in, const std::vector<int32_t>& depth_in,
                          const FactorPlan& plan) {
  P = &plan;
  parent = parent_in;
  depth = depth_in;
  const int32_t N = (int32_t)parent.size();
  broot.assign(N, -1);
  for (int32_t i = N - 1; i >= 0; --i) {  // parents come after their children
    if (!P->small[i]) continue;
    const int32_t p = parent[i];
    broot[i] = (p >= 0 && P->small[p]) ? broot[p] : i;
  }
}

int32_t AncestorTable::lca(int32_t a, int32_t b) const {
  if (a == b) return a;
  if (P->small[a] && P->small[b] && broot[a] == broot[b]) {
    while (a != b) {
      if (depth[a] >= depth[b]) a = parent[a];
      else b = parent[b];
    }
    return a;
  }
  // the top nodes the two root paths enter the top tree at
  if (P->small[a]) a = parent[broot[a]];
  if (P->small[b]) b = parent[broot[b]];
  if (a < 0 || b < 0) return -1;  // a bottom subtree that is a whole tree of its own
  int32_t ca = P->top_chain[P->top_index[a]], cb = P->top_chain[P->top_index[b]];
  while (ca != cb) {
    if (P->chains[ca].level >= P->chains[cb].level) {
      a = parent[P->chains[ca].b];
      if (a < 0) return -1;
      ca = P->top_chain[P->top_index[a]];
    } else {
      b = parent[P->chains[cb].b];
      if (b < 0) return -1;
      cb = P->top_chain[P->top_index[b]];
    }
  }
  return std::max(a, b);
}

// The dense form's part of a query plan (see kDenseMaxK): which tasks use it,
// their first sweep window, the w of every query, and the dense work items.
static void plan_dense(const FactorPlan& P, const std::vector<int32_t>& depth, int64_t nb,
                       const std::vector<int32_t>& jlo, const std::vector<int32_t>& jhi, QueryPlan& Q,
                       std::vector<int32_t>& tw0) {
  // the dense sums address the store with 32-bit element offsets
  if (P.store_elems > INT32_MAX) return;
  const std::vector<int32_t>& pos = P.node_pos;
  Q.bq_bu.assign(nb + 1, 0);
  Q.bq_bv.assign(nb + 1, kDenseNoV);
  Q.bq_g0.assign(nb + 1, 0);
  std::vector<char> ok(nb, 0);
  for (int64_t j = 0; j < nb; ++j) {
    // (a staging entry has hi -1 like a ground pair: its w is B_S e_lo)
    const int32_t lo = jlo[j], hi = jhi[j];
    if (lo < 0) continue;
    const int32_t sub = P.bpos_sub[pos[lo]];
    const int32_t K = P.sub_K[sub];
    if (K > kDenseMaxK) continue;
    int64_t bv = kDenseNoV;
    if (hi >= 0 && P.small[hi]) {
      // an ancestor in the same subtree
      if (P.bpos_sub[pos[hi]] != sub) continue;
      bv = P.sub_bbase[sub] + (int64_t)(pos[hi] - P.sub_p0[sub]) * K;
    } else if (hi >= 0) {
      // a top node: one of the columns of U_S, or the form does not apply
      const int32_t* U = P.sub_unode.data() + P.sub_ubeg[sub];
      const int32_t* it = std::lower_bound(U, U + K, hi);
      if (it == U + K || *it != hi) continue;
      bv = -1 - (int64_t)(it - U);
    }
    Q.bq_bu[j] = P.sub_bbase[sub] + (int64_t)(pos[lo] - P.sub_p0[sub]) * K;
    Q.bq_bv[j] = bv;
    ok[j] = 1;
  }
  const int32_t nbt = (int32_t)P.btask_nwin.size();
  std::vector<DItem> items;
  std::vector<int32_t> cls;
  for (int32_t t = 0; t < nbt; ++t) {
    const int32_t j0 = Q.bq_ptr[P.btask_ptr[t]], j1 = Q.bq_ptr[P.btask_ptr[t + 1]];
    if (j0 == j1) continue;
    // rows above the task's shallowest subtree, in whole window groups
    int32_t rmin = INT32_MAX;
    for (int32_t p = P.btask_ptr[t]; p < P.btask_ptr[t + 1]; p = P.sub_p1[P.bpos_sub[p]])
      rmin = std::min(rmin, depth[P.bnode_node[p]] - 1);  // a subtree's first record is its root
    const int32_t w0 = kWinPerWave * (rmin / (kWin * kWinPerWave));
    if (w0 == 0) continue;
    bool all = true;
    for (int32_t j = j0; j < j1; ++j) {
      if (!ok[j]) { all = false; continue; }
      Q.bq_g0[j] = w0 / kWinPerWave;
      if (Q.bq[j].kind == kQStage) Q.bq[j].out = w0;  // the dense form writes the windows below
    }
    if (all) tw0[t] = w0;
    for (int32_t p = P.btask_ptr[t]; p < P.btask_ptr[t + 1];) {
      const int32_t sub = P.bpos_sub[p];
      const int32_t s0 = Q.bq_ptr[P.sub_p0[sub]], s1 = Q.bq_ptr[P.sub_p1[sub]];
      const int cl = dense_class(P.sub_K[sub]);
      // staged columns: one column tile per item
      const int32_t m0 = (int32_t)Q.dq_list.size();
      for (int32_t j = s0; j < s1; ++j)
        if (ok[j] && Q.bq[j].kind == kQStage) Q.dq_list.push_back(j);
      const int32_t m1 = (int32_t)Q.dq_list.size();
      for (int32_t c = m0; c < m1; c += kDenseTile) {
        items.push_back(DItem{sub, c, std::min(kDenseTile, m1 - c), kWin * w0});
        cls.push_back(kDenseGroups + cl);
      }
      const int32_t l0 = (int32_t)Q.dq_list.size();
      for (int32_t j = s0; j < s1; ++j)
        if (ok[j] && Q.bq[j].kind != kQStage) Q.dq_list.push_back(j);
      const int32_t l1 = (int32_t)Q.dq_list.size();
      // the subtree's column tiles in items of 1, 2, 4 or 8 tiles, largest first
      for (int32_t c = l0; c < l1;) {
        const int32_t tiles = (l1 - c + kDenseTile - 1) / kDenseTile;
        int lg = 0;
        while (lg + 1 < kDenseTileKinds && (1 << (lg + 1)) <= std::min(tiles, dense_tiles(cl))) ++lg;
        const int32_t nq = std::min((int32_t)kDenseTile << lg, l1 - c);
        items.push_back(DItem{sub, c, nq, kWin * w0});
        cls.push_back(cl * kDenseTileKinds + lg);
        c += nq;
      }
      p = P.sub_p1[sub];
    }
  }
  // by class, then largest first (rows times column tiles; a subtree's items
  // stay adjacent)
  std::vector<int64_t> ord(items.size());
  for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int64_t)i;
  auto cost = [&](int64_t x) { return (int64_t)items[x].rows * ((items[x].nq + kDenseTile - 1) / kDenseTile); };
  std::stable_sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) {
    if (cls[x] != cls[y]) return cls[x] < cls[y];
    return cost(x) > cost(y);
  });
  Q.dclass_ptr.assign(kDenseAllGroups + 1, 0);
  for (int64_t x : ord) {
    Q.ditems.push_back(items[x]);
    Q.dclass_ptr[cls[x] + 1]++;
  }
  for (int c = 0; c < kDenseAllGroups; ++c) Q.dclass_ptr[c + 1] += Q.dclass_ptr[c];
  Q.dense = !Q.ditems.empty();
}

Status build_query_plan(const std::vector<int32_t>& first, const std::vector<int32_t>& depth,
                        const FactorPlan& P, int64_t q, const int32_t* a, const int32_t* b, QueryPlan& Q,
                        const AncestorTable* anc, const std::vector<int32_t>* export_nodes, bool dense) {
  const int32_t N = P.N;
  Q = QueryPlan();
  Q.q = q;
  const std::vector<int32_t>& pos = P.node_pos;  // bottom position of every bottom node
  const int32_t nbn = (int32_t)P.bnode_node.size();
  Q.bq_ptr.assign(nbn + 1, 0);
  std::vector<int32_t> lo_of(q, -2), hi_of(q, -1);
  std::vector<char> general(q, 0);
  std::vector<int32_t> gp_top;  // top endpoints of non-ancestor pairs
  std::vector<int64_t> stage_of;  // per node: staging offset of its column, -1 if not staged
  auto column = [&](int32_t x, int64_t& off, int32_t& staged) {
    if (!P.small[x]) {
      off = P.top_off[P.top_index[x]];
      staged = 0;
      return;
    }
    if (stage_of[x] < 0) {
      stage_of[x] = Q.stage_elems;
      // whole groups of kWinPerWave windows: the sweep writes its window
      // group unconditionally (zeros past the column's depth)
      Q.stage_elems += (int64_t)nwin_grouped(depth[x]) * kWin;
      Q.bq_ptr[pos[x] + 1]++;  // one staging entry at the node
    }
    off = stage_of[x];
    staged = 1;
  };
  for (int64_t k = 0; k < q; ++k) {
    const int32_t x = a[k], y = b[k];
    if (x == y) { Q.zero_out.push_back(k); continue; }
    int32_t lo, hi;
    if (x < 0) { lo = y; hi = -1; }
    else if (y < 0) { lo = x; hi = -1; }
    else { lo = std::min(x, y); hi = std::max(x, y); }
    if (hi >= 0 && first[hi] > lo) {
      Q.n_general++;
      if (!anc) continue;
      if (stage_of.empty()) stage_of.assign(N, -1);
      GPair g{};
      column(lo, g.a_off, g.a_stage);
      column(hi, g.b_off, g.b_stage);
      g.da = depth[lo];
      g.db = depth[hi];
      const int32_t c = anc->lca(lo, hi);
      g.dl = c < 0 ? 0 : depth[c];
      g.out = k;
      Q.gp.push_back(g);
      if (!P.small[lo]) gp_top.push_back(lo);
      if (!P.small[hi]) gp_top.push_back(hi);
      general[k] = 1;
      continue;
    }
    lo_of[k] = lo;
    hi_of[k] = hi;
    if (P.small[lo]) Q.bq_ptr[pos[lo] + 1]++;
    else {
      Q.tq_lo.push_back(P.top_index[lo]);
      Q.tq_hi.push_back(hi < 0 ? -1 : P.top_index[hi]);
      Q.tq_out.push_back(k);
    }
  }
  if (export_nodes) {
    if (stage_of.empty()) stage_of.assign(N, -1);
    for (int32_t x : *export_nodes) {
      int64_t off;
      int32_t staged;
      column(x, off, staged);
      Q.export_off.push_back(off);
      Q.export_staged.push_back((char)staged);
      if (!staged) gp_top.push_back(x);
    }
  }
  if (!Q.tq_lo.empty()) {
    // top queries by lower endpoint, so that the queries of one column run
    // side by side and share its reads in the caches
    std::vector<int64_t> ord(Q.tq_lo.size());
    for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int64_t)i;
    std::stable_sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) { return Q.tq_lo[x] < Q.tq_lo[y]; });
    std::vector<int32_t> lo2(ord.size()), hi2(ord.size());
    std::vector<int64_t> out2(ord.size());
    for (size_t i = 0; i < ord.size(); ++i) {
      lo2[i] = Q.tq_lo[ord[i]];
      hi2[i] = Q.tq_hi[ord[i]];
      out2[i] = Q.tq_out[ord[i]];
    }
    Q.tq_lo.swap(lo2);
    Q.tq_hi.swap(hi2);
    Q.tq_out.swap(out2);
  }
  {
    // the sweep forms record byte offsets in 32 bits (one padding record)
    int64_t total = 0;
    for (int32_t i = 0; i < nbn; ++i) total += Q.bq_ptr[i + 1];
    if ((total + 1) * (int64_t)sizeof(BQuery) > (int64_t)UINT32_MAX) {
      set_error("query plan: too many queries with a bottom lower endpoint for one plan (split the request)");
      return E_INVALID_ARG;
    }
  }
  for (int32_t i = 0; i < nbn; ++i) Q.bq_ptr[i + 1] += Q.bq_ptr[i];
  const int64_t nb = Q.bq_ptr[nbn];
  Q.bq.resize(nb);
  std::vector<int32_t> fill(Q.bq_ptr.begin(), Q.bq_ptr.end() - 1);
  std::vector<int32_t> jlo(dense ? nb : 0, -1), jhi(dense ? nb : 0, -1);  // endpoints per entry (-1: staging)
  // staging entries first within their node's bucket
  if (!stage_of.empty())
    for (int32_t x = 0; x < N; ++x) {
      if (stage_of[x] < 0) continue;
      if (dense) jlo[fill[pos[x]]] = x;  // (jhi stays -1: the staged node's own column)
      BQuery& bq = Q.bq[fill[pos[x]]++];
      bq.kind = kQStage;
      bq.hiref = stage_of[x];
      bq.out = -1;
      bq.nwin = nwin_of(depth[x]);
      Q.max_nwin = std::max(Q.max_nwin, bq.nwin);
    }
  for (int64_t k = 0; k < q; ++k) {
    const int32_t lo = lo_of[k];
    if (lo < 0 || !P.small[lo]) continue;
    const int32_t hi = hi_of[k];
    if (dense) {
      jlo[fill[pos[lo]]] = lo;
      jhi[fill[pos[lo]]] = hi;
    }
    BQuery& bq = Q.bq[fill[pos[lo]]++];
    bq.out = k;
    bq.nwin = nwin_of(depth[lo]);
    const int32_t ps = pos[lo];
    bq.hiref = 0;
    if (hi < 0) bq.kind = kQGround;
    else if (P.small[hi]) {
      bq.kind = kQSlot;
      bq.hiref = slot_code(P.lslot[hi]);
    } else if (P.bnode_tinl[2 * ps] == hi) bq.kind = kQInl0;
    else if (P.bnode_tinl[2 * ps + 1] == hi) bq.kind = kQInl1;
    else {
      const int32_t t = P.top_index[hi];
      bq.kind = kQStore;
      bq.hiref = store_ref(P.top_off[t], nwin_grouped(P.top_depth[t]));
    }
    Q.max_nwin = std::max(Q.max_nwin, bq.nwin);
  }
  // one padding entry each: the sweep reads bucket bounds two positions and
  // first entries one position ahead of time
  Q.bq.push_back(BQuery{0, kQGround, 0, -1});
  Q.bq_ptr.push_back(Q.bq_ptr.back());
  // a sweep wavefront writes one slot per query of its task for its group of
  // kWinPerWave windows (groups past a query's column are never read)
  const int32_t groups = (std::max(Q.max_nwin, P.max_btask_nwin) + kWinPerWave - 1) / kWinPerWave;
  Q.nslots = (int64_t)groups * nb;
  // top chains the plan reads: those of the swept subtrees' attachment
  // points (subtrees with at least one bucket entry), of its top endpoints,
  // and every ancestor chain of those
  const int32_t nbt = (int32_t)P.btask_nwin.size();
  const int32_t nch = (int32_t)P.chains.size();
  auto swept = [&](int32_t t) { return Q.bq_ptr[P.btask_ptr[t + 1]] != Q.bq_ptr[P.btask_ptr[t]]; };
  Q.chain_need.assign(nch, 0);
  for (int32_t t = 0; t < nbt; ++t)
    if (swept(t))
      for (int32_t k = P.btask_attach_ptr[t]; k < P.btask_attach_ptr[t + 1]; ++k) Q.chain_need[P.btask_attach[k]] = 1;
  for (int32_t lo : Q.tq_lo) Q.chain_need[P.top_chain[lo]] = 1;
  for (int32_t x : gp_top) Q.chain_need[P.top_chain[P.top_index[x]]] = 1;
  for (int32_t c = 0; c < nch; ++c)
    if (Q.chain_need[c] && P.chain_parent[c] >= 0) Q.chain_need[P.chain_parent[c]] = 1;
  int32_t need = 0;
  for (int32_t c = 0; c < nch; ++c) need += Q.chain_need[c];
  Q.prune_top = need < nch;
  // first window of each task's sweep: 0, or past the rows that the dense
  // form covers for every subtree of the task
  std::vector<int32_t> tw0(nbt, 0);
  if (dense && nb > 0 && !P.sub_p0.empty()) plan_dense(P, depth, nb, jlo, jhi, Q, tw0);
  // work list: the swept tasks, every window from the first
  for (int32_t t = 0; t < nbt; ++t) {
    if (!swept(t)) continue;
    for (int32_t w = tw0[t]; w < P.btask_nwin[t]; w += kBottomWaves * kWinPerWave) {
      Q.work_task.push_back(t);
      Q.work_win.push_back(w);
    }
  }
  return OK;
}

}  // namespace peers
