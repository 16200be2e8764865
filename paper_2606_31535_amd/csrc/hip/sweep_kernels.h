// Device kernels of the implicit-inverse sweep (gfx950, wave64, FP64).
//
// Layout and notation are those of host/plan.h: lanes of a wavefront are 64
// consecutive depths d of a window, and the value a lane holds for node i is
// z_i[d] = Z_{a_d(i), i}, the entry of the inverse Cholesky factor in the row
// of i's ancestor at depth d+1 (eq 11: Z_jj = D_j^{-1/2}, Z_ji = sum over
// H-edges (k, i) of w~_ki Z_jk with w~_ki = -L_ki for unit-lower L).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../host/plan.h"

namespace peers {

// Generic FP64 GEMM over task lists (see GemmProb / GemmTask in host/plan.h).
struct GemmArgs {
  double* buf[BUF_COUNT];
  const GemmProb* probs;
  const GemmTask* tasks;
  const GemmTask* ntasks;  // narrow-chain tasks (one wavefront each)
  const int64_t* gather;
};

struct SweepArgs {
  // top tree
  const Chain* chains;
  const BaseBlock* base_blocks;
  int32_t nbase;
  const int32_t* top_chain;
  const int32_t* top_node;
  const double* lcc;
  double* X;
  const int64_t* top_off;
  const int32_t* top_depth;
  const double* top_isd;
  double* store;
  // bottom subtrees
  const int32_t* btask_ptr;
  const int32_t* btask_nwin;
  const BNode* bnode;
  const BEnt* bent;
  const double* isd;
  int32_t store_wide;  // 1: store byte offsets need 64 bits
  // dense form of the rows above bottom subtrees (host/plan.h, kDenseMaxK)
  int32_t nsub;
  const int32_t* sub_p0;
  const int32_t* sub_p1;
  const int32_t* sub_K;
  const int32_t* sub_ubeg;
  const int32_t* sub_udep;
  const int64_t* sub_uoff;
  const int64_t* sub_bbase;
  double* B;  // B_S of every subtree, formed at upload
};

struct QueryArgs {
  // bottom work items of this plan: (task, first window)
  const int32_t* work_task;
  const int32_t* work_win;
  int64_t nwork;
  const int32_t* bq_ptr;
  const BQuery* bq;
  int64_t nbq;
  const int32_t* tq_lo;
  const int32_t* tq_hi;
  const int64_t* tq_out;
  int64_t ntq;
  const int64_t* zero_out;
  int64_t nzero;
  const GPair* gp;
  int64_t ngp;
  double* stage;  // staged bottom columns of non-ancestor pairs
  double* part;
  double* R;
  // dense work items (null when the plan has none): their queries in
  // dq_list, the dense sum of bottom query j at part[dpart_off + j]
  const DItem* ditems;
  int64_t nditems;
  const int32_t* dq_list;
  const int64_t* bq_bu;
  const int64_t* bq_bv;
  const int32_t* bq_g0;
  int64_t dpart_off;
};

// Everything one factor's sweep reads, for grouped launches over many factors.
struct FactorArgs {
  GemmArgs g;
  SweepArgs a;
  QueryArgs q;
};

// One workgroup item of a grouped launch: a factor's argument block and the
// item's index in that factor's own launch of the same step (GEMM task, base
// block, top column, bottom work item, or finish block).
struct GroupItem {
  int32_t fa;
  int32_t pad_;
  int64_t local;
};

enum GroupKind : int {
  GK_GEMM = 0, GK_INV_BASE = 1, GK_CHAIN_ROWS = 2, GK_BOTTOM = 3,
  GK_REDUCE = 4, GK_TOP_QUERY = 5, GK_ZERO = 6, GK_GENERAL = 7, GK_GEMM_NARROW = 8,
  // the bottom step of a group holding a factor with 64-bit store offsets
  // (GK_BOTTOM runs only the 32-bit form, which keeps its register count low)
  GK_BOTTOM_WIDE = 9,
  // dense rows above bottom subtrees: the items of each group (GK_DENSE + group)
  GK_DENSE = 10
};

// Items per finish block of each kind (threads, or wavefronts per item; the
// top-node pairs take two per wavefront).
constexpr int kReduceBlock = 256, kTopQueryBlock = 8, kZeroBlock = 256, kGeneralBlock = 4;

hipError_t launch_grouped(int kind, const FactorArgs* fa, const GroupItem* items, int64_t nitems, int64_t grid,
                          hipStream_t s);
hipError_t launch_gemm(const GemmArgs& g, int64_t task0, int64_t ntasks, hipStream_t s);
// wide tiles [task0, task0 + ntasks) and narrow tiles [ntask0, ntask0 + nntasks) of one chain level
hipError_t launch_gemm_level(const GemmArgs& g, int64_t task0, int64_t ntasks, int64_t ntask0, int64_t nntasks,
                             hipStream_t s);
hipError_t launch_inv_base(const SweepArgs& a, hipStream_t s);
hipError_t launch_chain_rows(const SweepArgs& a, int32_t ntop, hipStream_t s);
hipError_t launch_bottom(const SweepArgs& a, const QueryArgs& q, hipStream_t s);
// B_S of every subtree with |U_S| <= kDenseMaxK (upload, after the records hold the factor)
hipError_t launch_bxfer(const SweepArgs& a, hipStream_t s);
// the dense sums of the items of group x, or of every group for x < 0
// (dclass_ptr: the plan's item ranges per group, host memory)
hipError_t launch_dense(const SweepArgs& a, const QueryArgs& q, const int64_t* dclass_ptr, int x, hipStream_t s);
hipError_t launch_finish(const SweepArgs& a, const QueryArgs& q, hipStream_t s);

}  // namespace peers
