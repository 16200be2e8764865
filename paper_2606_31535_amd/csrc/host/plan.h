// Device layout of one factor for the implicit sweep, built on the host.
//
// Notation: Z = D^{-1/2} L^{-1} is the paper's inverse Cholesky factor
// (eq 3, eq 11). Column i of Z is supported on the root path anc*(i)
// (Lemma 1), so it is stored depth-indexed: z_i[d] = Z_{a_d(i), i} for the
// ancestor a_d(i) at depth d+1, d = 0..depth(i)-1, with z_i[depth(i)-1] =
// D_i^{-1/2}. Eq 11 with w~_ki = -L_ki (unit-lower L) reads
//     z_i[d] = sum over k in struct(L_:,i) of (-L_ki) z_k[d],   d < depth(i)-1,
// and eq 12 becomes R_uv = sum_d (z_u[d] - z_v[d])^2 (z_g = 0 for the ground).
// Lanes of a wavefront are 64 consecutive depths ("a window").
//
// The tree is split in two:
//  * bottom subtrees: maximal subtrees with at most kBottomMaxNodes nodes and
//    height at most kBottomMaxHeight. A workgroup sweeps one of them for one
//    window in descending index order (a topological order, Theorem 1),
//    keeping the column values of the current root path in an LDS stack
//    indexed by local depth; nothing else of Z is kept.
//  * the top tree (the separators of the nested dissection and everything
//    above the bottom subtrees): its columns are produced by dense
//    supernode chunks, level by level, into the "top store", which bottom
//    subtrees read as the path values above their root.
#pragma once

#include <cstdint>
#include <vector>

#include "host.h"

namespace peers {

constexpr int kWin = 64;              // depths per window = wavefront lanes
constexpr int kChunk = 32;            // top chunk width (columns per task)
constexpr int kBottomMaxHeight = 64;  // LDS path stack slots per window
constexpr int kBottomMaxNodes = 2048;
constexpr int32_t kGroundCode = INT32_MIN;

struct TopChunk {
  int32_t a, b;          // node range [a, b], a chain inside one supernode
  int32_t depth_b;       // depth of b (depth(a + j) = depth_b + b - a - j)
  int32_t next;          // ext = struct(b): number of ancestors referenced
  int64_t ext_begin;     // into ext_top / ext_depth
  int64_t coef_begin;    // into coef: next rows of kChunk doubles
  int64_t tri_begin;     // into tri: kChunk x kChunk
  int32_t level;         // chunk depth in the chunk tree (root chunk = 0)
  int32_t top_a;         // top index of node a (top indices of a..b are consecutive)
};

struct FactorPlan {
  int32_t N = 0;
  int32_t height = 0;
  // top tree
  int32_t ntop = 0;
  std::vector<int32_t> top_index;   // per node: top index or -1
  std::vector<int32_t> top_node;    // per top index: node
  std::vector<int64_t> top_off;     // per top index: element offset in the store (multiple of kWin)
  std::vector<int32_t> top_depth;   // per top index
  std::vector<double> top_isd;      // per top index: D^{-1/2}
  int64_t store_elems = 0;
  std::vector<TopChunk> chunks;
  std::vector<int32_t> ext_top;     // top index of each ext entry
  std::vector<int64_t> ext_off;     // its store offset (top_off of ext_top)
  std::vector<int32_t> ext_depth;
  std::vector<double> coef;         // -L_{ext[e], a+j} at [coef_begin + e*kChunk + j]
  std::vector<double> tri;          // -L_{a+j, a+jj} at [tri_begin + j*kChunk + jj], jj < j
  std::vector<int64_t> level_ptr;   // top tasks grouped by level
  std::vector<int32_t> task_chunk;  // (chunk, window) tasks, sorted by level
  std::vector<int32_t> task_win;
  int32_t nlevels = 0;
  // bottom subtrees
  std::vector<char> small;          // per node
  std::vector<int32_t> lslot;       // per bottom node: local depth (LDS slot)
  std::vector<int32_t> btask_ptr;   // per bottom task: range in bnodes
  std::vector<int32_t> bnodes;      // processing order (descending within each subtree)
  std::vector<int32_t> btask_nwin;  // windows per task
  std::vector<int32_t> bwork_task;  // (task, window) work items
  std::vector<int32_t> bwork_win;
  std::vector<int64_t> bent_ptr;    // per node (N+1): entries of bottom nodes only
  std::vector<int32_t> bent_src;    // >= 0: LDS slot; < 0: -(top index + 1)
  std::vector<double> bent_coef;    // -L_ki
  std::vector<int32_t> bdepth;      // per node depth
  std::vector<double> isd;          // per node D^{-1/2}
  int32_t max_lslot = 0;
  // work statistics
  double f_top = 0, f_bottom_computed = 0;
};

Status build_plan(const Symbolic& S, const Numeric& F, FactorPlan& P);

// Query plan for a list of pairs in reduced-permuted indices.
struct QueryPlan {
  int64_t q = 0;
  // bottom queries bucketed by lower endpoint
  std::vector<int32_t> bq_ptr;     // N+1
  std::vector<int32_t> bq_hicode;  // LDS slot, -(top+1), or kGroundCode
  std::vector<int64_t> bq_slot;    // first partial slot
  std::vector<int64_t> bq_out;     // output index
  std::vector<int32_t> bq_nwin;    // windows (partials) of the query
  int64_t nslots = 0;
  // top queries
  std::vector<int32_t> tq_lo, tq_hi;  // top indices (hi -1 = ground)
  std::vector<int64_t> tq_out;
  // pairs with R = 0
  std::vector<int64_t> zero_out;
  int64_t n_general = 0;  // pairs whose endpoints are not ancestor-related
};

// a, b: permuted node indices (-1 = ground), per query; out = query number.
// first/depth: subtree ranges and depths of the postordered elimination tree.
Status build_query_plan(const std::vector<int32_t>& first, const std::vector<int32_t>& depth,
                        const FactorPlan& P, int64_t q, const int32_t* a, const int32_t* b, QueryPlan& Q);

}  // namespace peers
