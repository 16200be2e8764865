// CPU emulation of the device sweep's address arithmetic, with bounds checks.
//
// Test infrastructure: it runs the library's host preparation (ingest,
// ordering, symbolic, numeric, device-layout plan and query plans) on a
// graph read from a file, then replays what every kernel of one sweep
// addresses -- in the exact integer widths the kernels use (the bottom
// sweep's 32-bit record, query and store byte offsets included) -- and
// checks each access against the size of the buffer it falls in, plus the
// layout invariants those offsets rely on. It never touches a GPU. Built with
// AddressSanitizer and UndefinedBehaviorSanitizer by the test that runs it,
// so the host preparation is checked at the same time.
//
// Usage: sweep_addressing GRAPH_FILE NUM_RANDOM_PAIRS SEED
// GRAPH_FILE: int64 n, int64 m, int32 ground, int32 has_coords, then eu[m],
// ev[m] (int32), w[m] (float64), coords[n*3] (float64) if has_coords.
#include <algorithm>
#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <unordered_map>
#include <vector>

#include "../../paper_2606_31535_amd/csrc/host/graph_handle.h"
#include "../../paper_2606_31535_amd/csrc/host/plan.h"

using namespace peers;

namespace {

int64_t g_checks = 0;

#define REQUIRE(cond, ...)                                               \
  do {                                                                   \
    ++g_checks;                                                          \
    if (!(cond)) {                                                       \
      std::fprintf(stderr, "VIOLATION %s:%d: %s: ", __FILE__, __LINE__, #cond); \
      std::fprintf(stderr, __VA_ARGS__);                                 \
      std::fprintf(stderr, "\n");                                        \
      std::exit(1);                                                      \
    }                                                                    \
  } while (0)

constexpr int NW = kWinPerWave;
constexpr uint32_t kBQ = sizeof(BQuery);

struct Sizes {
  int64_t store_elems;   // elements the store allocation holds
  int64_t stage_elems;
  int64_t nslots;        // partial slots, then the dense sums
};

// The bottom sweep's read of a top-store column (32-bit byte offsets): the
// windows t0 .. t0+NW-1 of the column named by `ref`, lanes 0..63.
void check_store_ref(const FactorPlan& P, const Sizes& Z, int64_t ref, int32_t t0, bool wide, const char* what) {
  const int32_t wb = (int32_t)ref, nw = (int32_t)(ref >> 32);
  REQUIRE(nw >= 0 && nw % NW == 0, "%s: window count %d", what, nw);
  REQUIRE(wb >= 0 && (int64_t)wb + t0 <= INT32_MAX, "%s: first window %d + t0 %d", what, wb, t0);
  const int32_t wi = t0 < nw ? wb + t0 : 0;
  // the last byte the wave reads
  const uint64_t last = (uint64_t)(wi + NW - 1) * (kWin * 8) + 63 * 8 + 7;
  if (!wide) {
    // (uint32)wi * 512 + lane * 8 must not wrap in 32 bits
    REQUIRE((uint64_t)wi * (kWin * 8) + 63 * 8 <= UINT32_MAX, "%s: 32-bit store offset wraps (wi %d)", what, wi);
  }
  REQUIRE(last < (uint64_t)Z.store_elems * 8, "%s: store byte %" PRIu64 " of %" PRId64, what, last,
          Z.store_elems * 8);
  (void)P;
}

struct Marks {
  std::vector<uint8_t> part_written;
  std::vector<uint8_t> dense_written;
};

// B_S of every subtree (upload): the records each wave walks, the columns of
// B it writes, and the LDS path stack it indexes.
void check_bxfer(const FactorPlan& P) {
  const int32_t nsub = (int32_t)P.sub_p0.size();
  REQUIRE((int32_t)P.sub_p1.size() == nsub && (int32_t)P.sub_K.size() == nsub && (int32_t)P.sub_bbase.size() == nsub,
          "subtree tables");
  for (int32_t s = 0; s < nsub; ++s) {
    const int32_t K = P.sub_K[s], p0 = P.sub_p0[s], p1 = P.sub_p1[s];
    REQUIRE(p0 < p1 && p1 <= (int32_t)P.bnode_node.size(), "subtree records [%d, %d)", p0, p1);
    REQUIRE(P.sub_ubeg[s] >= 0 && (int64_t)P.sub_ubeg[s] + K <= (int64_t)P.sub_uoff.size(), "U_S range");
    if (K == 0 || K > kDenseMaxK) continue;
    REQUIRE(P.sub_bbase[s] >= 0 && P.sub_bbase[s] + (int64_t)K * (p1 - p0) <= P.b_elems, "B_S of subtree %d", s);
    for (int32_t k = 1; k < K; ++k)
      REQUIRE(P.sub_udep[P.sub_ubeg[s] + k] < P.sub_udep[P.sub_ubeg[s] + k - 1], "U_S depths descending");
    for (int32_t p = p0; p < p1; ++p) {
      REQUIRE(P.bpos_sub[p] == s, "position %d's subtree", p);
      const BNode& b = P.bnode[p];
      const int32_t nl = b.n_more & 0xffff, nt = (int32_t)((uint32_t)b.n_more >> 16);
      REQUIRE(b.ent >= 0 && (int64_t)b.ent + nl + nt <= (int64_t)P.bent.size(), "overflow entries");
    }
  }
}

// Dense items: every read of B (forming w), U_S and the store, and every
// dense sum written.
void check_dense(const FactorPlan& P, const QueryPlan& Q, const Sizes& Z, const std::vector<int32_t>& depth,
                 Marks& M) {
  const int64_t nbq = Q.nbq();
  M.dense_written.assign((size_t)std::max<int64_t>(nbq, 1), 0);
  if (!Q.dense) {
    REQUIRE(Q.ditems.empty(), "items without the dense flag");
    return;
  }
  REQUIRE((int)Q.dclass_ptr.size() == kDenseAllGroups + 1 && Q.dclass_ptr[0] == 0 &&
              Q.dclass_ptr[kDenseAllGroups] == (int64_t)Q.ditems.size(), "group ranges");
  REQUIRE((int64_t)Q.bq_bu.size() == nbq + 1 && (int64_t)Q.bq_bv.size() == nbq + 1 && (int64_t)Q.bq_g0.size() == nbq + 1,
          "per-query dense tables");
  REQUIRE(kStoreZeroBlock >= kDenseTile, "zero block covers a row tile");
  REQUIRE(Z.store_elems <= INT32_MAX, "dense sums address the store with 32-bit element offsets");
  for (int x = 0; x < kDenseAllGroups; ++x) {
    const bool stage = x >= kDenseGroups;
    const int c = stage ? x - kDenseGroups : x / kDenseTileKinds, tiles = stage ? 1 : 1 << (x % kDenseTileKinds);
    REQUIRE(Q.dclass_ptr[x + 1] == Q.dclass_ptr[x] || tiles <= dense_tiles(c), "group %d", x);
    for (int64_t it = Q.dclass_ptr[x]; it < Q.dclass_ptr[x + 1]; ++it) {
      const DItem& d = Q.ditems[it];
      REQUIRE(d.sub >= 0 && d.sub < (int32_t)P.sub_p0.size(), "item subtree");
      const int32_t K = P.sub_K[d.sub], ub = P.sub_ubeg[d.sub];
      REQUIRE(K > 0 && K <= kDenseMaxK && dense_class(K) == c, "item class %d for |U_S| %d", c, K);
      REQUIRE(d.nq >= 1 && d.nq <= kDenseTile * tiles, "item queries %d", d.nq);
      const int32_t js0 = Q.bq_ptr[P.sub_p0[d.sub]], js1 = Q.bq_ptr[P.sub_p1[d.sub]];
      REQUIRE(d.q0 >= 0 && (int64_t)d.q0 + d.nq <= (int64_t)Q.dq_list.size(), "item query list");
      for (int32_t q = 0; q < d.nq; ++q)
        REQUIRE(Q.dq_list[d.q0 + q] >= js0 && Q.dq_list[d.q0 + q] < js1, "item query outside the subtree");
      const int32_t root = P.bnode_node[P.sub_p0[d.sub]];
      REQUIRE(d.rows > 0 && d.rows % (kWin * NW) == 0 && d.rows <= depth[root] - 1, "item rows %d (root depth %d)",
              d.rows, depth[root]);
      // U_S columns: rows read are below min(rows, depth) of each column
      for (int32_t k = 0; k < K; ++k) {
        const int64_t off = P.sub_uoff[ub + k];
        const int32_t rmax = std::min(d.rows, P.sub_udep[ub + k]);
        REQUIRE(off >= kStoreZeroBlock && off + rmax <= Z.store_elems, "U_S column read");
      }
      for (int32_t q = 0; q < d.nq; ++q) {
        const int64_t j = Q.dq_list[d.q0 + q];
        REQUIRE(Q.bq_g0[j] * kWin * NW == d.rows, "first sweep window of query %" PRId64, j);
        const int64_t bb = P.sub_bbase[d.sub], be = bb + (int64_t)K * (P.sub_p1[d.sub] - P.sub_p0[d.sub]);
        REQUIRE(Q.bq_bu[j] >= bb && Q.bq_bu[j] + K <= be, "B column of u");
        const int64_t bv = Q.bq_bv[j];
        if (bv >= 0) REQUIRE(bv >= bb && bv + K <= be, "B column of v");
        else if (bv != kDenseNoV) REQUIRE(-1 - bv < K, "U_S column of v");
        REQUIRE((Q.bq[j].kind == kQStage) == stage, "staging entries in exactly the staging groups");
        if (stage) {
          // the item writes rows [0, rows) of the staged column; the sweep the rest
          REQUIRE(Q.bq[j].out * kWin == d.rows && Q.bq[j].hiref >= 0 && Q.bq[j].hiref + d.rows <= Z.stage_elems,
                  "staged rows of entry %" PRId64, j);
          REQUIRE(Q.bq_bv[j] == kDenseNoV, "staging w is B_S e_x");
        }
        const int64_t slot = Q.nslots + j;
        REQUIRE(stage || slot < Z.nslots, "dense sum slot %" PRId64 " of %" PRId64, slot, Z.nslots);
        REQUIRE(!M.dense_written[j], "query %" PRId64 " in two dense items", j);
        M.dense_written[j] = 1;
      }
    }
  }
}

void check_bottom(const FactorPlan& P, const QueryPlan& Q, const Sizes& Z, bool wide, Marks& M, int64_t& node_waves) {
  const int64_t nbq = Q.nbq();
  const int32_t nbn = (int32_t)P.bnode_node.size();
  REQUIRE((int64_t)P.bnode.size() == nbn + 3, "record padding %zu vs %d", P.bnode.size(), nbn);
  REQUIRE((int64_t)Q.bq_ptr.size() == nbn + 2, "bucket bounds %zu vs %d", Q.bq_ptr.size(), nbn);
  REQUIRE((int64_t)Q.bq.size() == nbq + 1, "query padding");
  REQUIRE((nbq + 1) * (int64_t)kBQ <= (int64_t)UINT32_MAX, "query records beyond 32-bit offsets");
  M.part_written.assign((size_t)std::max<int64_t>(Q.nslots, 1), 0);
  for (size_t w = 0; w < Q.work_task.size(); ++w) {
    const int32_t task = Q.work_task[w];
    REQUIRE(task >= 0 && task + 1 < (int32_t)P.btask_ptr.size(), "task %d", task);
    for (int wave = 0; wave < kBottomWaves; ++wave) {
      const int32_t t0 = Q.work_win[w] + wave * NW;
      REQUIRE(t0 % NW == 0, "t0 %d", t0);
      const int32_t p0 = P.btask_ptr[task], p1 = P.btask_ptr[task + 1];
      if (t0 >= P.btask_nwin[task]) continue;
      REQUIRE(p1 - p0 <= kBottomMaxNodes && p1 > p0, "task size %d", p1 - p0);
      const int32_t grp = t0 / NW;
      const int32_t t0d = t0 * kWin;
      int32_t jb = Q.bq_ptr[p0];
      const int32_t jend = Q.bq_ptr[p1];
      // prologue reads: records p0, p0+1, p0+2; bounds p0, p0+1; first entry
      REQUIRE(p0 + 2 < (int32_t)P.bnode.size(), "prologue record");
      check_store_ref(P, Z, P.bnode[p0].tref[0], t0, wide, "inline 0");
      check_store_ref(P, Z, P.bnode[p0].tref[1], t0, wide, "inline 1");
      check_store_ref(P, Z, P.bnode[p0 + 1].tref[0], t0, wide, "next inline 0");
      check_store_ref(P, Z, P.bnode[p0 + 1].tref[1], t0, wide, "next inline 1");
      REQUIRE((uint64_t)Q.bq_ptr[p0] * kBQ <= UINT32_MAX, "first query offset");
      for (int32_t p = p0; p < p1; ++p) {
        ++node_waves;
        const uint32_t ro = (uint32_t)(p - p0) * (uint32_t)sizeof(BNode);
        REQUIRE((uint64_t)(p - p0 + 3) * sizeof(BNode) <= UINT32_MAX && p + 3 < (int32_t)P.bnode.size(),
                "record read ahead at %d", p);
        (void)ro;
        REQUIRE(p + 2 < (int32_t)Q.bq_ptr.size(), "bucket bound read ahead at %d", p);
        const BNode& cur = P.bnode[p];
        // top-store values two nodes ahead
        check_store_ref(P, Z, P.bnode[p + 2].tref[0], t0, wide, "read-ahead inline 0");
        check_store_ref(P, Z, P.bnode[p + 2].tref[1], t0, wide, "read-ahead inline 1");
        // slot codes
        for (int e = 0; e < 3; ++e) {
          const int32_t code = (cur.slots >> (kSlotBits * e)) & kSlotMask;
          REQUIRE(code % 2 == 0 && code / 2 < kBottomMaxHeight, "slot code %d", code);
        }
        const int32_t own = (cur.slots >> kOwnSlotShift) & kSlotMask;
        REQUIRE(own % 2 == 0 && own / 2 < kBottomMaxHeight, "own slot code %d", own);
        const int32_t nl = cur.n_more & 0xffff, nt = (int32_t)((uint32_t)cur.n_more >> 16);
        REQUIRE(cur.ent >= 0 && (int64_t)cur.ent + nl + nt < (int64_t)P.bent.size(), "overflow entries");
        for (int32_t e = 0; e < nl; ++e) {
          const int32_t code = (int32_t)P.bent[cur.ent + e].ref & kSlotMask;
          REQUIRE(code % 2 == 0 && code / 2 < kBottomMaxHeight, "overflow slot code %d", code);
        }
        for (int32_t e = 0; e < nt; ++e) check_store_ref(P, Z, P.bent[cur.ent + nl + e].ref, t0, wide, "overflow store");
        // query entries of this node; the next bucket end is read two ahead
        const int32_t q0 = Q.bq_ptr[p], q1 = Q.bq_ptr[p + 1];
        REQUIRE(q0 <= q1 && q1 <= nbq, "bucket [%d, %d) of %" PRId64, q0, q1, nbq);
        REQUIRE((uint64_t)q1 * kBQ + kBQ <= (uint64_t)Q.bq.size() * kBQ, "entry read ahead");
        if (q1 > q0 && cur.depth - 1 - t0d >= 0) {
          for (int32_t j = q0; j < q1; ++j) {
            REQUIRE((uint64_t)(j + 1) * kBQ <= UINT32_MAX && j + 1 < (int64_t)Q.bq.size(), "next entry");
            const BQuery& b = Q.bq[j];
            if (b.kind == kQSlot) {
              const int32_t code = (int32_t)b.hiref & kSlotMask;
              REQUIRE(code % 2 == 0 && code / 2 < kBottomMaxHeight, "query slot %d", code);
            } else if (b.kind == kQStore) {
              check_store_ref(P, Z, b.hiref, t0, wide, "query store column");
            } else if (b.kind == kQStage) {
              const int64_t lo = b.hiref + (int64_t)t0 * kWin, hi = b.hiref + (int64_t)(t0 + NW - 1) * kWin + 63;
              REQUIRE(lo >= 0 && hi < Z.stage_elems, "staging write [%" PRId64 ", %" PRId64 "] of %" PRId64, lo, hi,
                      Z.stage_elems);
            } else {
              REQUIRE(b.kind == kQInl0 || b.kind == kQInl1 || b.kind == kQGround, "kind %d", b.kind);
            }
          }
        }
      }
      // the wave's partial slots: grp * nbq + [jb, jend)
      for (int32_t j = jb; j < jend; ++j) {
        const int64_t slot = (int64_t)grp * nbq + j;
        REQUIRE(slot >= 0 && slot < Q.nslots, "partial slot %" PRId64 " of %" PRId64, slot, Q.nslots);
        M.part_written[slot] = 1;
      }
    }
  }
}

void check_finish(const FactorPlan& P, const QueryPlan& Q, const Sizes& Z, const Marks& M) {
  const int64_t nbq = Q.nbq();
  // ordered window reduction: every slot it reads was written by the sweep
  for (int64_t j = 0; j < nbq; ++j) {
    const BQuery& b = Q.bq[j];
    if (b.kind == kQStage) continue;
    REQUIRE(b.out >= 0 && b.out < Q.q, "output index %" PRId64, b.out);
    const int32_t ng = (b.nwin + NW - 1) / NW;
    const int32_t g0 = Q.dense ? Q.bq_g0[j] : 0;
    REQUIRE(g0 >= 0 && g0 < ng, "first window group %d of %d", g0, ng);
    if (g0 > 0) REQUIRE(M.dense_written[j], "reduction reads an unwritten dense sum %" PRId64, j);
    for (int32_t g = g0; g < ng; ++g) {
      const int64_t slot = (int64_t)g * nbq + j;
      REQUIRE(slot < Q.nslots && M.part_written[slot], "reduction reads unwritten slot %" PRId64, slot);
    }
  }
  // top-node pairs
  for (size_t k = 0; k < Q.tq_lo.size(); ++k) {
    const int32_t lo = Q.tq_lo[k], hi = Q.tq_hi[k];
    REQUIRE(lo >= 0 && lo < P.ntop && hi >= -1 && hi < P.ntop, "top pair");
    const int32_t nwl = (P.top_depth[lo] + kWin - 1) / kWin;
    REQUIRE(P.top_off[lo] + (int64_t)nwl * kWin <= Z.store_elems, "top pair lower column");
    if (hi >= 0) {
      const int32_t nwh = (P.top_depth[hi] + kWin - 1) / kWin;
      REQUIRE(P.top_off[hi] + (int64_t)nwh * kWin <= Z.store_elems, "top pair upper column");
    }
    REQUIRE(Q.tq_out[k] >= 0 && Q.tq_out[k] < Q.q, "top pair output");
  }
  for (const GPair& g : Q.gp) {
    REQUIRE(g.a_off + g.da <= (g.a_stage ? Z.stage_elems : Z.store_elems), "non-ancestor column a");
    REQUIRE(g.b_off + g.db <= (g.b_stage ? Z.stage_elems : Z.store_elems), "non-ancestor column b");
    REQUIRE(g.dl <= g.da && g.dl <= g.db, "lowest common ancestor depth");
    REQUIRE(g.out >= 0 && g.out < Q.q, "non-ancestor output");
  }
  for (int64_t o : Q.zero_out) REQUIRE(o >= 0 && o < Q.q, "zero output");
}

// Values of the dense form on a small graph: for every query with a dense
// sum, the rows above its subtree from B_S (formed from the records as the
// upload kernel does) and w, plus its rows from the subtree on, against the
// plain sum over all rows of its columns of Z (eq 11 on the factor, eq 12).
void check_dense_values(const GraphHandle& G, const FactorPlan& P, const QueryPlan& Q, const int32_t* a,
                        const int32_t* b, double& worst) {
  if (!Q.dense) return;
  const Symbolic& S = G.sym;
  const int32_t N = S.N;
  std::vector<std::vector<double>> z(N);
  for (int32_t i = N - 1; i >= 0; --i) {
    z[i].assign(S.depth[i], 0.0);
    z[i][S.depth[i] - 1] = 1.0 / std::sqrt(G.num.D[i]);
    for (int64_t p = S.colptr[i]; p < S.colptr[i + 1]; ++p) {
      const int32_t k = S.rowidx[p];
      for (int32_t d = 0; d < S.depth[k]; ++d) z[i][d] -= G.num.Lx[p] * z[k][d];
    }
  }
  std::vector<double> store((size_t)std::max<int64_t>(P.store_elems, kWin), 0.0);
  for (int32_t t = 0; t < P.ntop; ++t)
    for (int32_t d = 0; d < P.top_depth[t]; ++d) store[P.top_off[t] + d] = z[P.top_node[t]][d];
  // B_S per subtree
  std::vector<double> B((size_t)std::max<int64_t>(P.b_elems, 1), 0.0);
  for (size_t sb = 0; sb < P.sub_p0.size(); ++sb) {
    const int32_t K = P.sub_K[sb];
    if (K == 0 || K > kDenseMaxK) continue;
    std::vector<double> st((size_t)kBottomMaxHeight * K, 0.0), acc(K);
    for (int32_t p = P.sub_p0[sb]; p < P.sub_p1[sb]; ++p) {
      const BNode& bn = P.bnode[p];
      const int32_t ninl = (bn.slots >> kInlineCountShift) & 3;
      const int32_t nl = bn.n_more & 0xffff, nt = (int32_t)((uint32_t)bn.n_more >> 16);
      std::fill(acc.begin(), acc.end(), 0.0);
      auto path = [&](int32_t code, double c) {
        for (int32_t k = 0; k < K; ++k) acc[k] += c * st[(size_t)((code & kSlotMask) >> 1) * K + k];
      };
      auto top = [&](int64_t ref, double c) {
        for (int32_t k = 0; k < K; ++k)
          if ((int64_t)(uint32_t)ref * kWin == P.sub_uoff[P.sub_ubeg[sb] + k]) acc[k] += c;
      };
      for (int32_t e = 0; e < ninl; ++e) path(bn.slots >> (kSlotBits * e), bn.lc[e]);
      for (int32_t e = 0; e < nl; ++e) path((int32_t)P.bent[bn.ent + e].ref, P.bent[bn.ent + e].coef);
      top(bn.tref[0], bn.tc[0]);
      top(bn.tref[1], bn.tc[1]);
      for (int32_t e = 0; e < nt; ++e) top(P.bent[bn.ent + nl + e].ref, P.bent[bn.ent + nl + e].coef);
      const int32_t own = ((bn.slots >> kOwnSlotShift) & kSlotMask) >> 1;
      for (int32_t k = 0; k < K; ++k) {
        st[(size_t)own * K + k] = acc[k];
        B[P.sub_bbase[sb] + (int64_t)(p - P.sub_p0[sb]) * K + k] = acc[k];
      }
    }
  }
  for (const DItem& d : Q.ditems) {
    const int32_t K = P.sub_K[d.sub], ub = P.sub_ubeg[d.sub];
    for (int32_t c = 0; c < d.nq; ++c) {
      const int64_t j = Q.dq_list[d.q0 + c];
      std::vector<double> w(K);
      for (int32_t k = 0; k < K; ++k) {
        const int64_t bv = Q.bq_bv[j];
        w[k] = B[Q.bq_bu[j] + k] - (bv >= 0 ? B[bv + k] : (bv != kDenseNoV && k == -1 - bv) ? 1.0 : 0.0);
      }
      double dense = 0.0;
      for (int32_t row = 0; row < d.rows; ++row) {
        double y = 0.0;
        for (int32_t k = 0; k < K; ++k)
          if (row < P.sub_udep[ub + k]) y += w[k] * store[P.sub_uoff[ub + k] + row];
        dense += y * y;
      }
      if (Q.bq[j].kind == kQStage) {
        // a staged column: rows [0, rows) against the node's column of Z
        int32_t node = -1;
        for (int32_t p = P.sub_p0[d.sub]; p < P.sub_p1[d.sub] && node < 0; ++p)
          if (Q.bq_ptr[p] <= j && j < Q.bq_ptr[p + 1]) node = P.bnode_node[p];
        REQUIRE(node >= 0, "staged node of entry %" PRId64, j);
        double zmax = 0.0, dmax = 0.0;
        for (int32_t row = 0; row < d.rows; ++row) {
          double yv = 0.0;
          for (int32_t k2 = 0; k2 < K; ++k2)
            if (row < P.sub_udep[ub + k2]) yv += w[k2] * store[P.sub_uoff[ub + k2] + row];
          zmax = std::max(zmax, std::fabs(z[node][row]));
          dmax = std::max(dmax, std::fabs(yv - z[node][row]));
        }
        const double err = zmax > 0 ? dmax / zmax : dmax;
        worst = std::max(worst, err);
        REQUIRE(err < 1e-12, "staged column of entry %" PRId64 ": difference %.3g of %.3g", j, dmax, zmax);
        continue;
      }
      const int64_t k = Q.bq[j].out;
      const int32_t x = a[k], y = b[k];
      const int32_t lo = x < 0 ? y : (y < 0 ? x : std::min(x, y));
      const int32_t hi = (x < 0 || y < 0) ? -1 : std::max(x, y);
      double rest = 0.0, full = 0.0;
      for (int32_t r = 0; r < S.depth[lo]; ++r) {
        const double zh = (hi >= 0 && r < S.depth[hi]) ? z[hi][r] : 0.0;
        const double df = z[lo][r] - zh;
        full += df * df;
        if (r >= d.rows) rest += df * df;
      }
      const double err = std::fabs(dense + rest - full) / full;
      worst = std::max(worst, err);
      REQUIRE(err < 1e-11, "query %" PRId64 ": dense %.17g + sweep rows %.17g vs %.17g", j, dense, rest, full);
    }
  }
}

// Chain rows and the chain-level GEMM tiles of the top phase.
void check_top(const FactorPlan& P, const Sizes& Z) {
  std::unordered_map<int64_t, int64_t> col_ld;  // store column offset -> rows its region holds
  for (int32_t t = 0; t < P.ntop; ++t) {
    const Chain& c = P.chains[P.top_chain[t]];
    REQUIRE(P.top_off[t] % kWin == 0, "store columns start on a window");
    REQUIRE(P.top_off[t] == c.store_base + (int64_t)(P.top_node[t] - c.a) * c.ld, "column offset");
    REQUIRE(P.top_off[t] + c.ld <= Z.store_elems, "chain column");
    REQUIRE((int64_t)((P.top_depth[t] + NW * kWin - 1) / (NW * kWin)) * NW * kWin <= c.ld, "column padding");
    col_ld[P.top_off[t]] = c.ld;
  }
  for (size_t l = 0; l + 1 < P.t2_ptr.size(); ++l) {
    auto tiles = [&](const GemmTask& tk, int32_t width) {
      const GemmProb& pb = P.probs[tk.prob];
      const Chain& c = P.chains[P.prob_chain[tk.prob]];
      REQUIRE(pb.gather && pb.c_buf == BUF_STORE && pb.ldc == c.ld && pb.M == c.dp, "level problem");
      const int32_t rmax = std::min(tk.row0 + kTileM, pb.M) - 1;
      for (int32_t e = tk.k0; e < tk.k1; ++e) {
        const int64_t col = P.u_off[pb.aoff_begin + e];
        auto it = col_ld.find(col);
        REQUIRE(it != col_ld.end(), "gathered offset is not a store column");
        // the tile reads rows up to rmax of every gathered column: they stay
        // inside that column's region (zeros past its depth)
        REQUIRE(rmax < it->second, "gathered column region %" PRId64 " rows, tile reads row %d", it->second, rmax);
        REQUIRE(P.u_depth[pb.aoff_begin + e] > tk.row0, "reduction index below the tile's rows");
      }
      const int32_t cmax = std::min(tk.col0 + width, pb.N) - 1;
      REQUIRE(pb.c_off + (int64_t)cmax * pb.ldc + rmax < Z.store_elems, "tile store");
      REQUIRE(rmax < pb.ldc, "tile rows inside the output column");
    };
    for (int64_t t = P.t2_ptr[l]; t < P.t2_ptr[l + 1]; ++t) tiles(P.tasks[t], kTileN);
    for (int64_t t = P.t2n_ptr[l]; t < P.t2n_ptr[l + 1]; ++t) tiles(P.ntasks[t], kNarrowN);
  }
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 4) {
    std::fprintf(stderr, "usage: %s GRAPH_FILE NUM_RANDOM_PAIRS SEED\n", argv[0]);
    return 2;
  }
  FILE* fp = std::fopen(argv[1], "rb");
  if (!fp) { std::perror("open"); return 2; }
  int64_t n = 0, m = 0;
  int32_t ground = 0, has_coords = 0;
  bool ok = std::fread(&n, 8, 1, fp) == 1 && std::fread(&m, 8, 1, fp) == 1 && std::fread(&ground, 4, 1, fp) == 1 &&
            std::fread(&has_coords, 4, 1, fp) == 1;
  std::vector<int32_t> eu(m), ev(m);
  std::vector<double> w(m), coords(has_coords ? n * 3 : 0);
  ok = ok && std::fread(eu.data(), 4, m, fp) == (size_t)m && std::fread(ev.data(), 4, m, fp) == (size_t)m &&
       std::fread(w.data(), 8, m, fp) == (size_t)m;
  if (has_coords) ok = ok && std::fread(coords.data(), 8, n * 3, fp) == (size_t)(n * 3);
  std::fclose(fp);
  if (!ok) { std::fprintf(stderr, "short graph file\n"); return 2; }
  const int64_t npairs = std::atoll(argv[2]);
  const uint64_t seed = std::strtoull(argv[3], nullptr, 10);

  peers_graph_opts o{};
  o.coords = has_coords ? coords.data() : nullptr;
  GraphHandle G;
  Status st = build_graph(n, m, eu.data(), ev.data(), w.data(), ground, o, G);
  if (st != OK) { std::fprintf(stderr, "build_graph: %d %s\n", st, last_error()); return 3; }
  FactorPlan P;
  st = build_plan(G.sym, &G.num, P);
  if (st != OK) { std::fprintf(stderr, "build_plan: %d %s\n", st, last_error()); return 3; }
  AncestorTable anc;
  anc.build(G.sym.parent, G.sym.depth, P);
  auto pidx = [&](int32_t x) -> int32_t {
    if (x == ground) return -1;
    return G.sym.iperm[x < ground ? x : x - 1];
  };
  Sizes Z{};
  Z.store_elems = std::max<int64_t>(P.store_elems, kWin);
  const bool wide = P.store_wide;
  int64_t node_waves = 0;
  Marks M;
  check_bxfer(P);
  const bool small = n <= 20000;
  double worst = 0.0;
  auto run_plan = [&](const QueryPlan& Q, const int32_t* qa, const int32_t* qb) {
    Z.stage_elems = std::max<int64_t>(Q.stage_elems, 1);
    Z.nslots = Q.nslots + (Q.dense ? Q.nbq() : 0);
    check_dense(P, Q, Z, G.sym.depth, M);
    check_bottom(P, Q, Z, wide, M, node_waves);
    check_finish(P, Q, Z, M);
    if (small) check_dense_values(G, P, Q, qa, qb, worst);
  };
  // 1. all edges, as the resident plan of an uploaded factor
  {
    std::vector<int32_t> a(m), b(m);
    for (int64_t e = 0; e < m; ++e) {
      a[e] = pidx(eu[e]);
      b[e] = pidx(ev[e]);
      if (eu[e] == ev[e]) a[e] = b[e];
    }
    for (int dense = 0; dense < 2; ++dense) {
      QueryPlan Q;
      st = build_query_plan(G.sym.first, G.sym.depth, P, m, a.data(), b.data(), Q, nullptr, nullptr, dense != 0);
      if (st != OK) { std::fprintf(stderr, "edge plan: %d %s\n", st, last_error()); return 3; }
      REQUIRE(Q.n_general == 0, "an edge whose endpoints are not ancestor-related");
      run_plan(Q, a.data(), b.data());
      if (dense) std::printf("edges: %zu dense items, %" PRId64 " sweep work items\n", Q.ditems.size(),
                             (int64_t)Q.work_task.size());
    }
  }
  // 2. random pairs (non-ancestor pairs stage bottom columns), ground pairs,
  //    self pairs and duplicated edges
  {
    std::mt19937_64 rng(seed);
    std::vector<int32_t> a, b;
    for (int64_t k = 0; k < npairs; ++k) {
      int32_t x = (int32_t)(rng() % (uint64_t)n), y = (int32_t)(rng() % (uint64_t)n);
      const uint64_t r = rng() % 10;
      if (r == 0) y = ground;
      if (r == 1) y = x;
      if (r == 2 && m > 0) {
        const int64_t e = (int64_t)(rng() % (uint64_t)m);
        x = eu[e];
        y = ev[e];
      }
      a.push_back(x == y ? pidx(y) : pidx(x));
      b.push_back(pidx(y));
    }
    for (int dense = 0; dense < 2; ++dense) {
      QueryPlan Q;
      st = build_query_plan(G.sym.first, G.sym.depth, P, (int64_t)a.size(), a.data(), b.data(), Q, &anc, nullptr,
                            dense != 0);
      if (st != OK) { std::fprintf(stderr, "pair plan: %d %s\n", st, last_error()); return 3; }
      run_plan(Q, a.data(), b.data());
      std::printf("pairs: %" PRId64 " non-ancestor, %" PRId64 " staged elements, %zu dense items\n", Q.n_general,
                  Q.stage_elems, Q.ditems.size());
    }
    // a few edges: a plan that reads only some top chains
    {
      std::vector<int32_t> fa, fb;
      for (int64_t e = 0; e < std::min<int64_t>(m, 64); ++e) {
        fa.push_back(pidx(eu[e * (m / std::min<int64_t>(m, 64))]));
        fb.push_back(pidx(ev[e * (m / std::min<int64_t>(m, 64))]));
        if (fa.back() == fb.back()) fa.back() = fb.back();
      }
      QueryPlan Q;
      st = build_query_plan(G.sym.first, G.sym.depth, P, (int64_t)fa.size(), fa.data(), fb.data(), Q, &anc, nullptr, true);
      if (st != OK) { std::fprintf(stderr, "few-pair plan: %d %s\n", st, last_error()); return 3; }
      run_plan(Q, fa.data(), fb.data());
      std::printf("few pairs: %s top, %zu dense items\n", Q.prune_top ? "pruned" : "whole", Q.ditems.size());
    }
    // every node with the ground
    std::vector<int32_t> ga(n), gb(n, -1);
    for (int64_t x = 0; x < n; ++x) ga[x] = pidx((int32_t)x);
    QueryPlan Q;
    st = build_query_plan(G.sym.first, G.sym.depth, P, n, ga.data(), gb.data(), Q, &anc, nullptr, true);
    if (st != OK) { std::fprintf(stderr, "ground plan: %d %s\n", st, last_error()); return 3; }
    run_plan(Q, ga.data(), gb.data());
  }
  if (small) std::printf("dense values: worst relative difference %.3g\n", worst);
  check_top(P, Z);
  std::printf("ok: n %" PRId64 " m %" PRId64 " height %d store %.3f GB (%s offsets) node-waves %" PRId64
              " checks %" PRId64 "\n",
              n, m, G.sym.height, Z.store_elems * 8e-9, wide ? "64-bit" : "32-bit", node_waves, g_checks);
  return 0;
}
