// Host plan of the device factorization P L_r P^T = L D L^T (Algorithm 8,
// step 1, on the GPU).
//
// The factorization follows the split of the elimination tree used by the
// sweep (plan.h): bottom subtrees first, then the top chains level by level
// from the deepest chain level to the roots. Every pivot is formed without
// cancellation: each Schur complement of a grounded Laplacian is again a
// grounded Laplacian, so its pivot is its conductance to the ground r_j plus
// the magnitudes of its off-diagonal entries, and eliminating node k adds
// (-L_ik) r_k to r_i; off-diagonal entries only receive terms of their own
// sign (the host factorization does the same; numeric.cpp).
//
//  1. Bottom subtrees: one wavefront per bottom task takes its columns in
//     ascending order (children first) in the factor's compressed columns:
//     pivot, scaling, and the updates of the pairs (p < q) of the column whose
//     row index at p is a bottom node (the target position of row(q) in
//     column row(p) is precomputed here). Updates into top columns are left
//     to step 2.
//  2. Top columns are dense fronts indexed by depth (the layout of the
//     sweep's top store, which serves as workspace): column j holds the
//     Schur complement entry of its ancestor at depth d+1 in element d. Each
//     top column pulls the contributions of the bottom columns that reach it,
//     in a fixed order.
//  3. The top chains are cut into pieces of at most kFacPiece consecutive
//     columns; a piece P = a..b has the outside rows U_P = struct(b) (the
//     pattern of its last column holds every row above the piece that any of
//     its columns reaches). Per level of the tree of pieces, deepest first:
//     each piece's diagonal block is factored in one workgroup (its pivots
//     need only the block and the running sums of the rows above it, carried
//     like r); the rows of U_P are solved one row per thread (L_{U,P}); the
//     products L_{U,P} D_P L_{U,P}^T are dense GEMMs on the matrix cores; and
//     each destination column subtracts its share of them, and adds its r, in
//     a fixed order of source pieces.
//  4. The factor values of the top columns are read back from the fronts,
//     and the sweep layout (L_CC and L_{U,C} blocks, bottom records,
//     D^{-1/2}) is filled from the factor.
#pragma once

#include <cstdint>
#include <vector>

#include "host.h"
#include "plan.h"

namespace peers {

constexpr int32_t kFacPiece = 64;     // columns per piece of a top chain
constexpr int32_t kFacRowTile = 256;  // rows of U_P per U-row workgroup

// A piece a..b of a top chain (parent(i) = i+1 inside it).
struct FacPiece {
  int32_t a, b, w, dp;    // dp = depth of parent(b): rows above the piece
  int32_t nU, level;      // |U_P|, depth in the tree of pieces
  int64_t col_base, ld;   // front of column a+t at col_base + t*ld (the top store)
  int64_t u_begin;        // into pu_depth / pu_top
  int64_t luc_off, ldu;   // L_{U,P} in its step's scratch, column-major, ld = ldu = roundup64(nU)
  int64_t g_off;          // its product in the step's product buffer (column-major, ld = ldu)
};

struct NumericPlan {
  int32_t N = 0;
  int64_t nnz = 0;
  int32_t height = 0;
  std::vector<double> lx0;      // A's strict-lower entries at the factor's positions (0 at fill)
  std::vector<double> r0;       // conductance of each node to the ground
  // 1. bottom subtrees
  std::vector<int32_t> bt_ptr;  // per bottom task: its columns in bcol
  std::vector<int32_t> bcol;    // ascending within each task
  std::vector<int64_t> bpair_ptr;  // per bcol entry: its update targets in bpair
  std::vector<int64_t> bpair;      // factor positions, in (p, q) order over p with a bottom row
  // 2. pulls of top columns: for top index t, the bottom columns k reaching it
  //    and the position of L_{node(t), k} in column k
  std::vector<int32_t> tg_ptr;
  std::vector<int32_t> tg_k;
  std::vector<int64_t> tg_p;
  // 3. pieces of the top chains, by level of the piece tree, deepest first
  std::vector<FacPiece> pieces;
  std::vector<int32_t> pu_depth;  // per piece, U_P ascending (depth descending): depths
  std::vector<int32_t> pu_top;    // ... and top indices
  std::vector<int32_t> lev_ptr;   // per step: pieces in lev_piece
  std::vector<int32_t> lev_piece;
  std::vector<int32_t> ur_ptr;    // per step: U-row tiles (kFacRowTile rows) in ur_piece / ur_row0
  std::vector<int32_t> ur_piece, ur_row0;
  std::vector<GemmProb> probs;    // L_{U,P} D_P L_{U,P}^T of every piece (tiles below the diagonal)
  std::vector<GemmTask> tasks;
  std::vector<int64_t> gemm_ptr;  // per step: its tiles in tasks
  int64_t luc_elems = 0;          // largest step's L_{U,P} scratch (and its D-scaled copy)
  int64_t g_elems = 0;            // largest step's product buffer
  std::vector<int32_t> sc_ptr;    // per step: destination top indices in sc_dest
  std::vector<int32_t> sc_dest;
  std::vector<int32_t> sc_src_ptr;  // per destination: its (piece, position in U_P) sources
  std::vector<int32_t> sc_piece, sc_pos;
  int32_t steps = 0;
  // 4. outputs into the sweep layout
  std::vector<int64_t> top_x_ptr;   // per top index: its factor positions' entries in top_src
  std::vector<int64_t> top_src;     // per top-column factor position: lcc index, or luc index | kLxFromLuc
  std::vector<int32_t> bnode_node;  // per bottom record: its node (for D^{-1/2})
  int64_t bottom_records = 0;
};
constexpr int64_t kLxFromLuc = int64_t(1) << 62;

// Plans the factorization of the graph handle's matrix (A's off-diagonal
// entries and ground conductances, permuted by S) over the sweep layout P.
Status build_numeric_plan(const Ingested& ing, const Symbolic& S, const FactorPlan& P, NumericPlan& Q);

}  // namespace peers
