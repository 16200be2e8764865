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
//    height at most kBottomMaxHeight. A wavefront sweeps one of them for a
//    group of windows in descending index order (a topological order,
//    Theorem 1), keeping the column values of the current root path in a
//    register stack indexed by local depth; nothing else of Z is kept.
//  * the top tree (the separators of the nested dissection and everything
//    above the bottom subtrees). It is cut into chains: maximal runs of top
//    nodes a..b with parent(i) = i+1. For a chain C with diagonal block L_CC
//    and outside ancestors U_C (every row of L_{:,C} outside C), the rows of
//    Z above C follow from eq 11 as one product
//        Z[rows above C, C] = Z[rows above C, U_C] * B_C,
//        B_C = -L_{U_C, C} L_CC^{-1}      (formed once per factor, on the GPU),
//    and the rows inside C are Z[C, C] = D_C^{-1/2} L_CC^{-1} (L_CC^{-1} by a
//    recursive blocked triangular inverse at upload; the scaled rows written
//    every sweep). Every term is >= 0
//    (-L_ki >= 0 and L^{-1} >= 0 for a grounded Laplacian), so these blocked
//    forms add nonnegative terms only. Chains depend only on their ancestor
//    chains, so the top tree is a handful of levels of dense FP64 GEMMs. The
//    columns land in the "top store" (each top column over its whole depth),
//    which bottom subtrees read as the path values above their root.
#pragma once

#include <cstdint>
#include <vector>

#include "host.h"

namespace peers {

constexpr int kWin = 64;              // depths per window = wavefront lanes
constexpr int kTileM = 64;            // GEMM output tile rows
constexpr int kTileN = 32;            // GEMM output tile columns
constexpr int kNarrowN = 16;          // chain widths handled by the one-wavefront narrow GEMM tiles
constexpr int kBase = 64;             // base block of the triangular inverse
// path-stack slots (registers) per window: the stack is indexed with a
// wave-uniform slot, which stays in registers only up to 16 doubles (the
// widest register tuple, 32 dwords); a taller stack would spill to scratch
constexpr int kBottomMaxHeight = 16;
// Path-stack slots are stored as slot codes, twice the slot index (the
// register offset of the slot's double), so that the sweep gets a register
// offset from a record with one bit-field extraction.
// BNode::slots packing: code of inline entry e at bits kSlotBits*e, own code
// at kOwnSlotShift, number of inline path-stack entries at kInlineCountShift
constexpr int kSlotBits = 5;
constexpr int kSlotMask = (1 << kSlotBits) - 1;
constexpr int kOwnSlotShift = 3 * kSlotBits;
constexpr int kInlineCountShift = 20;
static_assert(2 * (kBottomMaxHeight - 1) <= kSlotMask && kOwnSlotShift + kSlotBits <= kInlineCountShift,
              "slot codes fit their bit fields");
inline int32_t slot_code(int32_t slot) { return 2 * slot; }
constexpr int kBottomMaxNodes = 512;
constexpr int kBottomWaves = 4;       // wavefronts per bottom workgroup
constexpr int kWinPerWave = 2;        // windows per bottom wavefront (lane l: depths t*64 + l)
constexpr int32_t kGroundCode = INT32_MIN;
// Dense form of the rows above a bottom subtree S with root r. Every column
// of S restricted to the rows above S is a combination of the columns of
// U_S = struct(r) (top nodes, all ancestors of r), by eq 11 applied inside S:
//     Z[above S, S] = Z[above S, U_S] B_S,   B_S = -L_{U_S,S} L_SS^{-1},
// with B_S >= 0 and every column summing to at most 1. A query (u, v) with u
// in S then gets its rows above S as
//     sum_d (Z[d, U_S] w)^2,   w = B_S e_u - (B_S e_v | e_v | 0)
// for v in S, v in U_S, or the ground: per subtree a product of the top-store
// columns of U_S (rows x |U_S|) with the queries' w (|U_S| x queries) on the
// FP64 matrix cores, squared and summed per query. The sweep then runs only
// the rows from the subtree's own depth on. Subtrees with |U_S| above
// kDenseMaxK keep the full sweep.
constexpr int kDenseMaxK = 64;
constexpr int kDenseTile = 16;        // queries per MFMA column tile
constexpr int kDenseClasses = 5;      // |U_S| padded to 4, 8, 16, 32 or 64
constexpr int dense_class(int32_t K) { return K <= 4 ? 0 : K <= 8 ? 1 : K <= 16 ? 2 : K <= 32 ? 3 : 4; }
constexpr int dense_steps(int cls) { return 1 << cls; }  // k-groups of 4 per class
// column tiles per dense work item: 1, 2, 4 or 8 (at most dense_tiles of
// the class; each loaded row block of U_S serves all of them), and row
// tiles per step, per class. Items are grouped by (class, tiles): group
// class * kDenseTileKinds + log2(tiles).
constexpr int dense_tiles(int cls) { return cls <= 1 ? 8 : cls <= 3 ? 4 : 2; }
constexpr int dense_rt(int cls) { return cls <= 1 ? 4 : cls == 2 ? 2 : 1; }
constexpr int kDenseTileKinds = 4;
constexpr int kDenseGroups = kDenseClasses * kDenseTileKinds;
// then one group per class of staging items: the rows above S of a staged
// column (a non-ancestor pair's bottom endpoint), Z[rows, U_S] B_S e_x,
// written to the staging buffer (one column tile per item)
constexpr int kDenseAllGroups = kDenseGroups + kDenseClasses;
// w of a query whose higher endpoint is the ground
constexpr int64_t kDenseNoV = INT64_MIN;

// Device buffers a GEMM operand can live in.
enum GemmBuf : int32_t { BUF_STORE = 0, BUF_LCC = 1, BUF_X = 2, BUF_T = 3, BUF_BT = 4, BUF_LUC = 5, BUF_G = 6, BUF_COUNT = 7 };

// C[M x N] = alpha * A[M x K] * B[K x N]; column-major unless `trans` says
// otherwise for B or C. Column k of A starts at
// buffer[a_buf] + (gather ? gather_table[aoff_begin + k] : a_off + k * lda).
struct GemmProb {
  int64_t a_off, lda, aoff_begin;
  int64_t b_off, ldb;
  int64_t c_off, ldc;
  int32_t M, N, K;
  int32_t a_buf, b_buf, c_buf;
  int32_t gather;
  int32_t trans;  // bit 0: B stored row-major (element (k, j) at b_off + k * ldb + j); bit 1: C row-major
  double alpha;
};

// One 64 x 32 output tile of a problem, over reduction indices [k0, k1).
struct GemmTask {
  int32_t prob, row0, col0, k0, k1;
};

struct Chain {
  int32_t a, b, w, dp;     // nodes a..b; dp = depth of parent(b) (rows above the chain)
  int32_t level, nU;       // chain-tree depth; |U_C|
  int64_t u_begin;         // into u_off / u_depth (U_C ascending = depth descending)
  int64_t store_base, ld;  // column a+j of the store at store_base + j*ld; ld = (dp + w) rounded up to whole window groups
  int64_t lcc_off, ldl;    // dense L_CC, column-major
  int64_t x_off;           // L_CC^{-1} workspace, same shape as L_CC
  int64_t bt_off, ldb;     // B_C, |U| x w row-major (row u at bt_off + u * w); ldb = roundup64(nU) sizes L_{U,C}
  int64_t luc_off;         // dense L_{U,C}, column-major (upload only), ld = ldb
};

struct BaseBlock {
  int32_t chain, lo, size;
};

// A bottom node in its task's processing order: one 80-byte record read by
// the scalar unit. The first three path-stack entries and the first two
// top-store entries of column i are inline; further ones are in bent (the
// path-stack ones first). Absent inline entries have coefficient 0 (slot 0,
// store reference 0).
struct BNode {
  double isd;                      // D_i^{-1/2}
  double lc[3];                    // -L_ki of the inline path-stack entries
  int64_t tref[2];                 // inline store entries: store_ref of column k (0 when absent)
  double tc[2];                    // their -L_ki
  int32_t slots;                   // path-stack slot codes and inline count (kSlotBits packing)
  int32_t depth;
  int32_t ent;                     // first overflow entry in bent
  int32_t n_more;                  // overflow path-stack entries (bits 0..15), then store entries (16..31)
};
static_assert(sizeof(BNode) == 80, "BNode is read as one 80-byte scalar record");

// An overflow entry -L_ki of a bottom column: ref = path-stack slot, or the
// store_ref of column k for a top-store entry.
struct BEnt {
  int64_t ref;
  double coef;
};
// A reference to a top-store column: low 32 bits = index of its first window
// (element offset / 64), high 32 bits = its number of windows, rounded up to
// a multiple of kWinPerWave (the column is zero-padded that far).
inline int64_t store_ref(int64_t elem_off, int32_t nwin) { return ((int64_t)nwin << 32) | (int64_t)(elem_off / 64); }

struct FactorPlan {
  int32_t N = 0;
  int32_t height = 0;
  // top tree
  int32_t ntop = 0;
  std::vector<int32_t> top_index;   // per node: top index or -1
  std::vector<int32_t> top_node;    // per top index: node
  std::vector<int64_t> top_off;     // per top index: element offset of its column in the store
  std::vector<int32_t> top_depth;   // per top index
  std::vector<double> top_isd;      // per top index: D^{-1/2}
  std::vector<int32_t> top_chain;   // per top index: chain
  int64_t store_elems = 0;
  bool store_wide = false;          // store bytes beyond 32-bit offsets
  std::vector<Chain> chains;
  int32_t nchain_levels = 0;
  std::vector<int64_t> u_off;       // gather table: store offset of each U_C column
  std::vector<int32_t> u_depth;
  std::vector<double> lcc;          // dense chain blocks L_CC (unit diagonal stored)
  std::vector<double> luc;          // dense L_{U,C} (upload only)
  int64_t x_elems = 0, t_elems = 0, bt_elems = 0;
  std::vector<BaseBlock> base_blocks;
  std::vector<GemmProb> probs;
  std::vector<GemmTask> tasks;
  std::vector<int64_t> inv_T_ptr;   // per recursion height h >= 1: tasks of T = L21 X11
  std::vector<int64_t> inv_X_ptr;   // per height: tasks of X21 = -X22 T
  std::vector<int64_t> t2_ptr;      // per chain level: tasks of Z[rows, C] = Z[rows, U] B_C
  std::vector<GemmTask> ntasks;     // narrow chains (w <= kNarrowN): one 64 x 16 tile per task
  std::vector<int64_t> t2n_ptr;     // per chain level: its narrow tasks
  int64_t bpre_begin = 0, bpre_end = 0;  // upload: B_C = -L_{U,C} L_CC^{-1}
  int32_t inv_heights = 0;
  // bottom subtrees
  std::vector<char> small;          // per node
  std::vector<int32_t> lslot;       // per bottom node: local depth (LDS slot)
  std::vector<int32_t> btask_ptr;   // per bottom task: range in bnode
  std::vector<BNode> bnode;         // processing order (descending within each subtree)
  std::vector<int32_t> bnode_node;  // node of each processing position (kept on the host)
  std::vector<int32_t> bnode_tinl;  // per position: the two inline top entries' nodes (-1 if absent)
  std::vector<BEnt> bent;
  std::vector<int32_t> btask_nwin;  // windows per task
  std::vector<int32_t> bpos_task;   // per processing position: its task
  std::vector<int32_t> node_pos;    // per node: its bottom processing position (-1 for top nodes)
  std::vector<int32_t> btask_attach_ptr, btask_attach;  // per task: chains its subtrees hang from
  std::vector<int32_t> prob_chain;  // per GEMM problem: its chain
  std::vector<int32_t> chain_parent;  // per chain: chain of parent(b), -1 at a root
  int32_t max_btask_nwin = 0;
  std::vector<double> isd;          // per node D^{-1/2}
  int32_t max_lslot = 0;
  // bottom subtrees (in processing order): record range, U_S = struct(root)
  // (ascending, so depth descending) with its store offsets and depths, and
  // the column-major B_S (column of the node at position p at
  // sub_bbase + (p - sub_p0) * sub_K; only for sub_K <= kDenseMaxK)
  std::vector<int32_t> sub_p0, sub_p1, sub_K, sub_ubeg, sub_udep, sub_unode;
  std::vector<int64_t> sub_uoff, sub_bbase;
  std::vector<int32_t> bpos_sub;    // per processing position: its subtree
  int64_t b_elems = 0;
  // work statistics (FMAs)
  double f_top = 0, f_top_gemm = 0, f_top_inv = 0, f_bpre = 0, f_bottom_computed = 0;
  // where the coefficient -L_ki of each bottom-column entry (CSC position)
  // went: a byte offset into the bnode array, or (with kCoefInBent set) into
  // the bent array; recorded only when the factor is computed on the device
  std::vector<int64_t> coef_p, coef_off;
};
constexpr int64_t kCoefInBent = int64_t(1) << 62;

// F may be null: the layout is then built with zero coefficients and unit
// pivots, and coef_p / coef_off record where the values belong.
Status build_plan(const Symbolic& S, const Numeric* F, FactorPlan& P);

// A query whose lower endpoint is a bottom node, or a staging entry.
struct BQuery {
  int64_t hiref;   // kQSlot: path-stack slot; kQStore: store_ref; kQStage: staging offset
  int32_t kind;    // how the higher endpoint's column is found (kQ*)
  int32_t nwin;    // windows of the lower endpoint's column
  int64_t out;     // output index; kQStage: the first window the sweep writes
};
// BQuery::kind: the higher endpoint's column in the lower endpoint's sweep
//   kQSlot   on the path stack (the higher endpoint is in the same subtree)
//   kQInl0/1 the lower endpoint's inline top-store entry 0 / 1
//   kQGround the ground (z = 0)
//   kQStore  another top-store column: hiref = its store_ref
//   kQStage  not a pair: the sweep writes the node's column to the staging
//            buffer at element offset hiref (non-ancestor pairs)
enum BQueryKind : int32_t { kQSlot = 0, kQInl0 = 1, kQInl1 = 2, kQGround = 3, kQStore = 4, kQStage = 5 };
// The first kWinPerWave windows of the top store are zero; loads of windows
// past a column's depth are pointed there.
constexpr int64_t kStoreZeroBlock = (int64_t)kWin * kWinPerWave;

// One dense work item: up to kDenseTile * (its tiles) bottom queries of one
// subtree (dq_list[q0 .. q0 + nq)), rows [0, rows) of their sums.
struct DItem {
  int32_t sub;     // subtree
  int32_t q0;      // first of the item's entries in dq_list
  int32_t nq;      // queries
  int32_t rows;    // a multiple of kWin * kWinPerWave
};

// A pair whose endpoints are not ancestor-related: both columns are read
// whole after the sweep (top store, or the staging buffer for bottom nodes)
// and split at their lowest common ancestor.
struct GPair {
  int64_t a_off, b_off;   // element offsets of the two columns
  int32_t da, db;         // their depths
  int32_t dl;             // depth of the lowest common ancestor (0: none)
  int32_t a_stage, b_stage;  // 1: the column is in the staging buffer, 0: in the top store
  int32_t pad_;
  int64_t out;
};

// Lowest common ancestors in the elimination tree, using the split into
// bottom subtrees and top chains: inside one bottom subtree by climbing
// parents (at most its height), otherwise from the top nodes the two subtrees
// hang from, chain to chain up the chain tree (each chain is a path of
// consecutive indices, so within a chain the ancestor is the larger index).
struct AncestorTable {
  const FactorPlan* P = nullptr;
  std::vector<int32_t> parent, depth;
  std::vector<int32_t> broot;   // per bottom node: root of its bottom subtree (-1 for top nodes)
  void build(const std::vector<int32_t>& parent_in, const std::vector<int32_t>& depth_in, const FactorPlan& plan);
  int32_t lca(int32_t a, int32_t b) const;  // -1 if a and b are in different trees
};

// Query plan for a list of pairs in reduced-permuted indices.
struct QueryPlan {
  int64_t q = 0;
  // bottom queries bucketed by lower endpoint, in the order of the bottom
  // nodes' processing positions (FactorPlan::bnode)
  std::vector<int32_t> bq_ptr;     // #bottom positions + 1, plus one padding entry
  std::vector<BQuery> bq;          // bucket order, plus one padding entry; partial of window group g at part[g * nbq() + j]
  int64_t nbq() const { return bq.empty() ? 0 : (int64_t)bq.size() - 1; }
  int32_t max_nwin = 0;
  int64_t nslots = 0;
  // top queries
  std::vector<int32_t> tq_lo, tq_hi;  // top indices (hi -1 = ground)
  std::vector<int64_t> tq_out;
  // pairs with R = 0
  std::vector<int64_t> zero_out;
  // pairs whose endpoints are not ancestor-related
  std::vector<GPair> gp;
  int64_t stage_elems = 0;
  int64_t n_general = 0;
  // bottom work items (task, first window): only the subtrees that hold a
  // lower endpoint or a staged column are swept
  std::vector<int32_t> work_task, work_win;
  // top chains the plan reads (closed under ancestors); prune_top when that
  // is not every chain, and only those chains' top steps need to run
  std::vector<char> chain_need;
  bool prune_top = false;
  // dense rows above bottom subtrees. Which rows of a query the dense form
  // covers depends only on the factor and on the query itself (not on the
  // other queries of the plan), so a query gets the same bits in any plan.
  // Work items grouped by class and tiles (items [dclass_ptr[x],
  // dclass_ptr[x+1]) of group x), then the staging items of each class
  // (group kDenseGroups + class), their bottom queries in dq_list; per bottom
  // query the B_S column offsets of its endpoints (bq_bv: >= 0 a column of B,
  // -1 - e for the e-th column of U_S, kDenseNoV for the ground) and the
  // first window group its sweep sums (bq_g0 > 0: the dense sum covers the
  // rows above it). A task's sweep starts past the dense rows when every one
  // of its queries has a dense sum.
  std::vector<DItem> ditems;
  std::vector<int32_t> dq_list;
  std::vector<int64_t> dclass_ptr;
  std::vector<int64_t> bq_bu, bq_bv;
  std::vector<int32_t> bq_g0;
  bool dense = false;
  // columns requested for export (in request order): element offset in the
  // top store (export_staged 0) or in the staging buffer (1)
  std::vector<int64_t> export_off;
  std::vector<char> export_staged;
};

// a, b: permuted node indices (-1 = ground), per query; out = query number.
// first/depth: subtree ranges and depths of the postordered elimination tree.
// anc: ancestor table for non-ancestor pairs; without it such pairs are only
// counted (n_general) and left out of the plan.
// export_nodes (optional, permuted indices): columns the sweep must leave in
// device memory for export (bottom columns are staged, top columns are in
// the store); their locations land in export_off / export_staged.
// dense: sum the rows above bottom subtrees in the dense form for the queries
// that allow it.
Status build_query_plan(const std::vector<int32_t>& first, const std::vector<int32_t>& depth,
                        const FactorPlan& P, int64_t q, const int32_t* a, const int32_t* b, QueryPlan& Q,
                        const AncestorTable* anc = nullptr, const std::vector<int32_t>* export_nodes = nullptr,
                        bool dense = false);

}  // namespace peers
