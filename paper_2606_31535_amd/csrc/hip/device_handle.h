// Device and factor handles shared by the plain, batched and served paths.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <memory>
#include <mutex>
#include <vector>

#include "../host/plan.h"
#include "sweep_kernels.h"

namespace peers {

struct BatchCache;   // captured batch launches (batch.hip)
struct FactorHandle;

struct DeviceHandle {
  int32_t ordinal = 0;
  int32_t cus = 0;
  uint64_t total = 0;
  uint64_t budget = 0;
  uint64_t used = 0;
  std::mutex mu;
  Status reserve(uint64_t bytes);
  void release(uint64_t bytes);
  BatchCache* batches = nullptr;  // guarded by batch_mu
  std::mutex batch_mu;
  // side streams of the bottom step (dense groups beside the sweep) with
  // their fork and join events, made when the device is opened; side_mu is
  // held while one sweep enqueues its fork, side launches and join
  static constexpr int kSideStreams = 3;
  hipStream_t side[kSideStreams] = {nullptr, nullptr, nullptr};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kSideStreams] = {nullptr, nullptr, nullptr};
  std::mutex side_mu;
};

void batch_cache_free(DeviceHandle& D);
void batch_cache_forget(DeviceHandle& D, const FactorHandle* F);

struct DeviceQueryPlan {
  void* base = nullptr;
  uint64_t bytes = 0;
  QueryArgs args{};
  int64_t nslots = 0;
  int64_t stage_elems = 0;
  int64_t q = 0;
  std::vector<int32_t> work_task, work_win;  // host copies (batch schedules)
  std::vector<char> chain_need;              // top chains the plan reads
  bool prune_top = false;
  // dense rows above bottom subtrees: item ranges per group and each
  // group's matrix-core work (MFMA count estimate) (host)
  bool dense = false;
  std::vector<int64_t> dclass_ptr;
  std::vector<double> dgroup_cost;
  // grouped-launch image of a pruned plan on its own factor (owned)
  void* layout_mem = nullptr;
  uint64_t layout_bytes = 0;
  std::shared_ptr<void> layout_host;
};

struct FactorHandle {
  DeviceHandle* dev = nullptr;
  int64_t n = 0, m = 0;
  int32_t ground = 0;
  int32_t N = 0;
  std::vector<int32_t> iperm;  // reduced id -> permuted index
  std::vector<int32_t> first, depth;
  AncestorTable anc;  // lowest common ancestors for non-ancestor pairs
  std::unique_ptr<FactorPlan> plan;
  bool dense_ok = true;  // plans may use the dense sums (not with peers_graph_opts::sweep_only)
  SweepArgs sweep{};
  GemmArgs gemm{};
  void* base = nullptr;
  void* store = nullptr;
  void* xbuf = nullptr;   // L_CC^{-1} workspace
  void* tbuf = nullptr;   // recursion temporaries
  void* btbuf = nullptr;  // transfer blocks B_C (resident)
  void* bbuf = nullptr;   // bottom subtrees' B_S (resident)
  double t_transform = 0, t_layout = 0, t_edge_plan = 0, t_transfer = 0, t_numeric_device = 0;
  void* part = nullptr;
  void* res = nullptr;
  void* stage = nullptr;  // staged bottom columns of non-ancestor pairs
  uint64_t resident_bytes = 0, store_bytes = 0, part_bytes = 0, res_bytes = 0, stage_bytes = 0, reserved = 0;
  DeviceQueryPlan edges;  // all-edge queries, resident
  DeviceQueryPlan to_ground;  // every node with the ground, resident after its first use
  bool to_ground_ready = false;
  std::mutex mu;          // one sweep at a time on the factor's own workspace (part/res/stage)
  // requests of any server that are queued or on the device for this factor;
  // release waits for them
  std::atomic<int64_t> server_refs{0};
  // per-phase timing of the last profiled sweep
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  bool timed = false;
  int32_t top_launches = 0, bottom_launches = 0;
  double top_flops = 0, bottom_flops = 0, top_bytes = 0, bottom_bytes = 0, finish_flops = 0;
};

Status hip_fail(hipError_t e, const char* what);
struct GraphHandle;
struct NumericPlan;
struct Numeric;
// The numeric factorization on the device (factor.hip): fills the sweep
// layout's coefficients, D^{-1/2}, L_CC (lcc_dev) and L_{U,C} (luc_dev), and
// copies L and D into host_out.
Status device_factor(FactorHandle& F, const GraphHandle& G, const NumericPlan& Q, double* lcc_dev, double* luc_dev,
                     hipStream_t s, Numeric* host_out, double* device_ms);
Status upload_query_plan(FactorHandle& F, const QueryPlan& Q, DeviceQueryPlan& D, hipStream_t s);
// Device bytes of a plan, and its upload into caller memory (not owned by D).
uint64_t query_plan_bytes(const QueryPlan& Q);
Status upload_query_plan_to(const QueryPlan& Q, DeviceQueryPlan& D, void* mem, hipStream_t s);
void free_query_plan(FactorHandle& F, DeviceQueryPlan& D);
Status ensure_workspace(FactorHandle& F, int64_t nslots, int64_t nres, int64_t nstage);
// Matrix-core work of a plan's dense groups (host estimates for scheduling).
void dense_costs(const QueryPlan& Q, std::vector<double>& group);
// Workspace of one sweep given by the caller instead of the factor's own
// (partial slots, staging, and the launch layout of a pruned sweep).
struct SweepWork {
  double* part = nullptr;  // partial slots, then the dense sums (the plan's nslots)
  double* stage = nullptr;
  void* layout = nullptr;
  uint64_t layout_cap = 0;  // bytes available at `layout`
};
Status run_sweep(FactorHandle& F, DeviceQueryPlan& D, double* R_dev, hipStream_t s, bool profile,
                 const SweepWork* work = nullptr);
// dense: the plan may sum rows above bottom subtrees in the dense form (for
// plans that run through run_sweep or a batch on the factor's own workspace)
Status build_query_plan_handle(const FactorHandle& F, int64_t q, const int32_t* a, const int32_t* b,
                               QueryPlan& Q, bool dense = false);
// Validates q pairs of original ids, builds their plan and uploads it.
Status plan_for_pairs(FactorHandle& F, int64_t q, const int32_t* u, const int32_t* v, DeviceQueryPlan& D,
                      hipStream_t s, bool dense = false);

// Reduced-permuted index of an original node id (-1 for the ground).
inline int32_t perm_index(const FactorHandle& F, int32_t x) {
  if (x == F.ground) return -1;
  return F.iperm[x < F.ground ? x : x - 1];
}

}  // namespace peers
