// Device half of the C ABI: device handles, factor upload into HBM, and the
// plain all-edge / pair queries (Algorithm 8 steps 2-3 on one GPU).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>

#include "../../../include/peers.h"
#include "../host/graph_handle.h"
#include "../host/numplan.h"
#include "batch.h"
#include "device_handle.h"
#include "sweep_kernels.h"

namespace peers {

Status hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return E_HIP;
}

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) return hip_fail(_e, #expr);   \
  } while (0)

namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Packs host vectors into one device allocation.
struct Packer {
  struct Item { const void* src; size_t bytes; size_t off; void** dst; };
  std::vector<Item> items;
  size_t total = 0;
  template <class T>
  void add(const std::vector<T>& v, const T** dst) {
    const size_t b = v.size() * sizeof(T);
    items.push_back({v.data(), b, total, (void**)dst});
    total = align_up(total + std::max<size_t>(b, 1), 256);
  }
  template <class T>
  void add(const std::vector<T>& v, T** dst) { add(v, (const T**)dst); }
  Status commit(void* base, hipStream_t s) {
    for (auto& it : items) {
      *it.dst = (char*)base + it.off;
      if (it.bytes) HIP_TRY(hipMemcpyAsync((char*)base + it.off, it.src, it.bytes, hipMemcpyHostToDevice, s));
    }
    return OK;
  }
};

}  // namespace

Status DeviceHandle::reserve(uint64_t bytes) {
  std::lock_guard<std::mutex> g(mu);
  if (used + bytes > budget) {
    set_error("HBM budget: " + std::to_string(used) + " used + " + std::to_string(bytes) + " requested > " +
              std::to_string(budget));
    return E_OVER_BUDGET;
  }
  used += bytes;
  return OK;
}

void DeviceHandle::release(uint64_t bytes) {
  std::lock_guard<std::mutex> g(mu);
  used = bytes > used ? 0 : used - bytes;
}

// Extra cost counted per dense launch when the groups are spread over the
// side streams: 2e7 units of dense_costs take 40-80 us at the rates of the
// large groups on the 1M-node mesh, about the time a launch of a few items
// (a few long row walks) lasts.
constexpr double kDenseLaunchFloor = 2e7;

// Matrix-core work of each dense group (rows x column tiles x k-groups).
void dense_costs(const QueryPlan& Q, std::vector<double>& group) {
  group.assign(Q.dense ? kDenseAllGroups : 0, 0.0);
  for (int x = 0; Q.dense && x < kDenseAllGroups; ++x) {
    const int cls = x < kDenseGroups ? x / kDenseTileKinds : x - kDenseGroups;
    const int tiles = x < kDenseGroups ? 1 << (x % kDenseTileKinds) : 1;
    for (int64_t i = Q.dclass_ptr[x]; i < Q.dclass_ptr[x + 1]; ++i) group[x] += (double)Q.ditems[i].rows * tiles * dense_steps(cls);
  }
}

static void pack_query_plan(const QueryPlan& Q, DeviceQueryPlan& D, Packer& pk) {
  pk.add(Q.work_task, &D.args.work_task);
  pk.add(Q.work_win, &D.args.work_win);
  pk.add(Q.gp, &D.args.gp);
  pk.add(Q.bq_ptr, &D.args.bq_ptr);
  pk.add(Q.bq, &D.args.bq);
  pk.add(Q.tq_lo, &D.args.tq_lo);
  pk.add(Q.tq_hi, &D.args.tq_hi);
  pk.add(Q.tq_out, &D.args.tq_out);
  pk.add(Q.zero_out, &D.args.zero_out);
  D.args.ditems = nullptr;
  D.args.dq_list = nullptr;
  D.args.bq_bu = D.args.bq_bv = nullptr;
  D.args.bq_g0 = nullptr;
  D.args.nditems = 0;
  D.args.dpart_off = Q.nslots;
  if (Q.dense) {
    pk.add(Q.ditems, &D.args.ditems);
    pk.add(Q.dq_list, &D.args.dq_list);
    pk.add(Q.bq_bu, &D.args.bq_bu);
    pk.add(Q.bq_bv, &D.args.bq_bv);
    pk.add(Q.bq_g0, &D.args.bq_g0);
    D.args.nditems = (int64_t)Q.ditems.size();
  }
  D.dense = Q.dense;
  D.dclass_ptr = Q.dclass_ptr;
  dense_costs(Q, D.dgroup_cost);
  D.args.nbq = Q.nbq();
  D.args.ntq = (int64_t)Q.tq_out.size();
  D.args.nzero = (int64_t)Q.zero_out.size();
  D.args.nwork = (int64_t)Q.work_task.size();
  D.args.ngp = (int64_t)Q.gp.size();
  D.nslots = Q.nslots + (Q.dense ? Q.nbq() : 0);  // the dense sums follow the window-group slots
  D.stage_elems = Q.stage_elems;
  D.work_task = Q.work_task;
  D.work_win = Q.work_win;
  D.chain_need = Q.chain_need;
  D.prune_top = Q.prune_top;
  D.q = Q.q;
}

uint64_t query_plan_bytes(const QueryPlan& Q) {
  Packer pk;
  DeviceQueryPlan D;
  pack_query_plan(Q, D, pk);
  return pk.total;
}

Status upload_query_plan_to(const QueryPlan& Q, DeviceQueryPlan& D, void* mem, hipStream_t s) {
  Packer pk;
  pack_query_plan(Q, D, pk);
  D.base = nullptr;  // not owned
  D.bytes = 0;
  return pk.commit(mem, s);
}

Status upload_query_plan(FactorHandle& F, const QueryPlan& Q, DeviceQueryPlan& D, hipStream_t s) {
  Packer pk;
  pack_query_plan(Q, D, pk);
  D.bytes = pk.total;
  Status st = F.dev->reserve(D.bytes);
  if (st != OK) return st;
  hipError_t e = hipMalloc(&D.base, std::max<size_t>(D.bytes, 256));
  if (e != hipSuccess) { F.dev->release(D.bytes); D.bytes = 0; return hip_fail(e, "hipMalloc(query plan)"); }
  return pk.commit(D.base, s);
}

void free_query_plan(FactorHandle& F, DeviceQueryPlan& D) {
  if (D.layout_mem) { (void)hipFree(D.layout_mem); F.dev->release(D.layout_bytes); }
  D.layout_mem = nullptr;
  D.layout_bytes = 0;
  D.layout_host.reset();
  if (D.base) { (void)hipFree(D.base); F.dev->release(D.bytes); }
  D.base = nullptr;
  D.bytes = 0;
}

// Grows one workspace buffer of the factor to at least `need` bytes.
static Status grow(FactorHandle& F, void*& buf, uint64_t& have, uint64_t need, const char* what) {
  if (need <= have) return OK;
  // captured batches hold this factor's workspace addresses
  batch_cache_forget(*F.dev, &F);
  if (buf) {
    (void)hipFree(buf);
    F.dev->release(have);
    buf = nullptr;
    have = 0;
  }
  Status st = F.dev->reserve(need);
  if (st != OK) return st;
  hipError_t e = hipMalloc(&buf, need);
  if (e != hipSuccess) {
    F.dev->release(need);
    return hip_fail(e, what);
  }
  have = need;
  return OK;
}

Status ensure_workspace(FactorHandle& F, int64_t nslots, int64_t nres, int64_t nstage) {
  Status st = grow(F, F.part, F.part_bytes, (uint64_t)std::max<int64_t>(nslots, 1) * 8, "hipMalloc(partials)");
  if (st == OK) st = grow(F, F.res, F.res_bytes, (uint64_t)std::max<int64_t>(nres, 1) * 8, "hipMalloc(results)");
  if (st == OK) st = grow(F, F.stage, F.stage_bytes, (uint64_t)std::max<int64_t>(nstage, 1) * 8, "hipMalloc(staging)");
  return st;
}

// L_CC^{-1} of every top chain into F.X: 64 x 64 diagonal inverses, then per
// recursion height T = L21 X11 and X21 = -X22 T. Returns the launch count.
static Status run_chain_inverse(FactorHandle& F, hipStream_t s, int32_t& launches) {
  const FactorPlan& P = *F.plan;
  HIP_TRY(launch_inv_base(F.sweep, s));
  launches += P.base_blocks.empty() ? 0 : 1;
  for (int32_t h = 1; h <= P.inv_heights; ++h) {
    HIP_TRY(launch_gemm(F.gemm, P.inv_X_ptr[h - 1], P.inv_T_ptr[h] - P.inv_X_ptr[h - 1], s));
    HIP_TRY(launch_gemm(F.gemm, P.inv_T_ptr[h], P.inv_X_ptr[h] - P.inv_T_ptr[h], s));
    launches += 2;
  }
  return OK;
}

Status run_sweep(FactorHandle& F, DeviceQueryPlan& D, double* R_dev, hipStream_t s, bool profile,
                 const SweepWork* work) {
  if (D.prune_top) return run_sweep_pruned(F, D, R_dev, s, profile, work);
  QueryArgs q = D.args;
  q.part = work && work->part ? work->part : (double*)F.part;
  q.stage = work && work->stage ? work->stage : (double*)F.stage;
  q.R = R_dev;
  const FactorPlan& P = *F.plan;
  if (profile && !F.ev[0])
    for (auto& e : F.ev) HIP_TRY(hipEventCreate(&e));
  F.timed = profile;
  if (profile) HIP_TRY(hipEventRecord(F.ev[0], s));
  // L_CC^{-1} of every chain is part of the prepared factor (formed at
  // upload with B_C); the sweep starts from the chain-internal rows
  int32_t launches = 0;
  HIP_TRY(launch_chain_rows(F.sweep, P.ntop, s));
  launches += P.ntop > 0 ? 1 : 0;
  for (size_t l = 0; l + 1 < P.t2_ptr.size(); ++l) {
    HIP_TRY(launch_gemm_level(F.gemm, P.t2_ptr[l], P.t2_ptr[l + 1] - P.t2_ptr[l], P.t2n_ptr[l],
                              P.t2n_ptr[l + 1] - P.t2n_ptr[l], s));
    launches += 1;
  }
  F.top_launches = launches;
  if (profile) HIP_TRY(hipEventRecord(F.ev[1], s));
  int32_t bl = 0;
  if (D.dense) {
    for (int c = 0; c < kDenseAllGroups; ++c) bl += D.dclass_ptr[c + 1] > D.dclass_ptr[c] ? 1 : 0;
    if (work) {
      // caller workspace (a caller that may capture the stream): one stream
      HIP_TRY(launch_dense(F.sweep, q, D.dclass_ptr.data(), -1, s));
    } else {
      // the dense groups on the device's side streams beside the sweep on s
      // (they write disjoint sums; the finish step on s waits for all of
      // them). Largest first to the least loaded stream, counting each launch
      // at its cost plus kDenseLaunchFloor: a group with fewer items than the
      // device holds workgroups takes about as long as its longest item, so
      // the small groups are spread over the streams. Each stream then runs
      // its groups smallest first, so those latency-bound launches of the
      // three streams overlap at the start instead of queueing at the end.
      DeviceHandle& V = *F.dev;
      std::lock_guard<std::mutex> g(V.side_mu);
      constexpr int NS = DeviceHandle::kSideStreams;
      HIP_TRY(hipEventRecord(V.fork_ev, s));
      std::vector<int> ord;
      for (int x = 0; x < kDenseAllGroups; ++x)
        if (D.dclass_ptr[x + 1] > D.dclass_ptr[x]) ord.push_back(x);
      std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return D.dgroup_cost[x] > D.dgroup_cost[y]; });
      double load[NS] = {0, 0, 0};
      std::vector<int> on(ord.size());
      for (size_t i = 0; i < ord.size(); ++i) {
        int k = 0;
        for (int j = 1; j < NS; ++j)
          if (load[j] < load[k]) k = j;
        load[k] += D.dgroup_cost[ord[i]] + kDenseLaunchFloor;
        on[i] = k;
      }
      for (int k = 0; k < NS; ++k) HIP_TRY(hipStreamWaitEvent(V.side[k], V.fork_ev, 0));
      for (size_t i = ord.size(); i-- > 0;) HIP_TRY(launch_dense(F.sweep, q, D.dclass_ptr.data(), ord[i], V.side[on[i]]));
      for (int k = 0; k < NS; ++k) HIP_TRY(hipEventRecord(V.join_ev[k], V.side[k]));
      HIP_TRY(launch_bottom(F.sweep, q, s));
      for (int k = 0; k < NS; ++k) HIP_TRY(hipStreamWaitEvent(s, V.join_ev[k], 0));
      F.bottom_launches = bl + (q.nwork > 0 ? 1 : 0);
      if (profile) HIP_TRY(hipEventRecord(F.ev[2], s));
      HIP_TRY(launch_finish(F.sweep, q, s));
      if (profile) HIP_TRY(hipEventRecord(F.ev[3], s));
      return OK;
    }
  }
  HIP_TRY(launch_bottom(F.sweep, q, s));
  F.bottom_launches = bl + (q.nwork > 0 ? 1 : 0);
  if (profile) HIP_TRY(hipEventRecord(F.ev[2], s));
  HIP_TRY(launch_finish(F.sweep, q, s));
  if (profile) HIP_TRY(hipEventRecord(F.ev[3], s));
  return OK;
}

Status build_query_plan_handle(const FactorHandle& F, int64_t q, const int32_t* a, const int32_t* b,
                               QueryPlan& Q, bool dense) {
  return build_query_plan(F.first, F.depth, *F.plan, q, a, b, Q, &F.anc, nullptr, dense && F.dense_ok);
}

Status plan_for_pairs(FactorHandle& F, int64_t q, const int32_t* u, const int32_t* v, DeviceQueryPlan& DQ,
                      hipStream_t s, bool dense) {
  std::vector<int32_t> a(q), b(q);
  for (int64_t k = 0; k < q; ++k) {
    if (u[k] < 0 || u[k] >= F.n || v[k] < 0 || v[k] >= F.n) {
      set_error("query " + std::to_string(k) + " has a node id outside [0, n)");
      return E_NODE_RANGE;
    }
    a[k] = perm_index(F, u[k]);
    b[k] = perm_index(F, v[k]);
    if (u[k] == v[k]) a[k] = b[k];
  }
  QueryPlan Q;
  Status st = build_query_plan_handle(F, q, a.data(), b.data(), Q, dense);
  if (st != OK) return st;
  return upload_query_plan(F, Q, DQ, s);
}

}  // namespace peers

using namespace peers;

extern "C" {

peers_status peers_device_open(int32_t ordinal, uint64_t hbm_budget_bytes, peers_device* out) {
  if (!out) { set_error("out is null"); return PEERS_E_INVALID_ARG; }
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return (peers_status)hip_fail(e, "hipGetDeviceCount");
  if (ordinal < 0 || ordinal >= count) { set_error("device ordinal out of range"); return PEERS_E_INVALID_ARG; }
  e = hipSetDevice(ordinal);
  if (e != hipSuccess) return (peers_status)hip_fail(e, "hipSetDevice");
  size_t freeb = 0, total = 0;
  e = hipMemGetInfo(&freeb, &total);
  if (e != hipSuccess) return (peers_status)hip_fail(e, "hipMemGetInfo");
  auto* D = new DeviceHandle();
  D->ordinal = ordinal;
  if (hipDeviceGetAttribute(&D->cus, hipDeviceAttributeMultiprocessorCount, ordinal) != hipSuccess || D->cus <= 0)
    D->cus = 256;
  D->total = total;
  D->budget = hbm_budget_bytes ? std::min<uint64_t>(hbm_budget_bytes, total) : (uint64_t)(0.9 * (double)total);
  e = hipEventCreateWithFlags(&D->fork_ev, hipEventDisableTiming);
  for (int k = 0; k < DeviceHandle::kSideStreams && e == hipSuccess; ++k) {
    e = hipStreamCreateWithFlags(&D->side[k], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&D->join_ev[k], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    peers_device_close(reinterpret_cast<peers_device>(D));
    return (peers_status)hip_fail(e, "side streams");
  }
  *out = reinterpret_cast<peers_device>(D);
  return PEERS_OK;
}

void peers_device_close(peers_device d) {
  if (!d) return;
  auto* D = reinterpret_cast<DeviceHandle*>(d);
  batch_cache_free(*D);
  (void)hipSetDevice(D->ordinal);
  for (int k = 0; k < DeviceHandle::kSideStreams; ++k) {
    if (D->side[k]) (void)hipStreamDestroy(D->side[k]);
    if (D->join_ev[k]) (void)hipEventDestroy(D->join_ev[k]);
  }
  if (D->fork_ev) (void)hipEventDestroy(D->fork_ev);
  delete D;
}

peers_status peers_device_usage(peers_device d, uint64_t* used, uint64_t* budget) {
  if (!d) { set_error("null device"); return PEERS_E_INVALID_ARG; }
  auto* D = reinterpret_cast<DeviceHandle*>(d);
  std::lock_guard<std::mutex> g(D->mu);
  if (used) *used = D->used;
  if (budget) *budget = D->budget;
  return PEERS_OK;
}

peers_status peers_device_set_budget(peers_device d, uint64_t hbm_budget_bytes) {
  if (!d) { set_error("null device"); return PEERS_E_INVALID_ARG; }
  auto* D = reinterpret_cast<DeviceHandle*>(d);
  std::lock_guard<std::mutex> g(D->mu);
  const uint64_t b = hbm_budget_bytes ? std::min<uint64_t>(hbm_budget_bytes, D->total) : (uint64_t)(0.9 * (double)D->total);
  if (D->used > b) {
    set_error("the library holds " + std::to_string(D->used) + " bytes, more than the new budget " + std::to_string(b));
    return PEERS_E_OVER_BUDGET;
  }
  D->budget = b;
  return PEERS_OK;
}

peers_status peers_factor_upload(peers_device d, peers_graph g, void* hip_stream, peers_factor* out) {
  if (!d || !g || !out) { set_error("null argument"); return PEERS_E_INVALID_ARG; }
  *out = nullptr;
  auto* D = reinterpret_cast<DeviceHandle*>(d);
  const GraphHandle& G = *reinterpret_cast<GraphHandle*>(g);
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t he = hipSetDevice(D->ordinal);
  if (he != hipSuccess) return (peers_status)hip_fail(he, "hipSetDevice");
  // the upload reads the graph's factor, and forms it first for a graph
  // created with numeric_on_device: uploads of such a graph run one at a time
  std::unique_lock<std::mutex> num_lock(G.num_mu, std::defer_lock);
  if (G.numeric_on_device) num_lock.lock();
  std::unique_ptr<FactorHandle> F(new FactorHandle());
  F->dev = D;
  F->n = G.ing.n;
  F->m = G.ing.m;
  F->ground = G.ing.ground;
  F->N = G.sym.N;
  F->iperm = G.sym.iperm;
  F->first = G.sym.first;
  F->depth = G.sym.depth;
  F->dense_ok = !G.sweep_only;
  F->plan.reset(new FactorPlan());
  double tp = now_s();
  // a graph created with numeric_on_device has no factor values yet: the
  // layout is built with placeholders and the device factorization fills them
  const bool dev_numeric = !G.numeric_ready;
  Status st = build_plan(G.sym, dev_numeric ? nullptr : &G.num, *F->plan);
  if (st != OK) return (peers_status)st;
  std::unique_ptr<NumericPlan> NP;
  if (dev_numeric) {
    NP.reset(new NumericPlan());
    st = build_numeric_plan(G.ing, G.sym, *F->plan, *NP);
    if (st != OK) return (peers_status)st;
  }
  F->t_layout = now_s() - tp;
  const FactorPlan& P = *F->plan;
  F->anc.build(G.sym.parent, G.sym.depth, P);
  // resident all-edge query plan
  double acc_bottom = 0, acc_top = 0;
  tp = now_s();
  {
    std::vector<int32_t> a(F->m), b(F->m);
    for (int64_t e = 0; e < F->m; ++e) {
      a[e] = perm_index(*F, G.eu[e]);
      b[e] = perm_index(*F, G.ev[e]);
      if (G.eu[e] == G.ev[e]) a[e] = b[e];  // self-loop: R = 0
    }
    QueryPlan Q;
    st = build_query_plan(F->first, F->depth, P, F->m, a.data(), b.data(), Q, nullptr, nullptr, F->dense_ok);
    if (st != OK) return (peers_status)st;
    if (Q.n_general) { set_error("internal: an edge whose endpoints are not etree-related"); return PEERS_E_INTERNAL; }
    F->t_edge_plan = now_s() - tp;
    // eq 12 terms: depth of the lower endpoint, per pair with R > 0
    for (int64_t e = 0; e < F->m; ++e) {
      if (a[e] == b[e]) continue;
      const int32_t lo = a[e] < 0 ? b[e] : (b[e] < 0 ? a[e] : std::min(a[e], b[e]));
      (P.small[lo] ? acc_bottom : acc_top) += (double)G.sym.depth[lo];
    }
    tp = now_s();
    st = upload_query_plan(*F, Q, F->edges, s);
    if (st != OK) return (peers_status)st;
  }
  Packer pk;
  SweepArgs& A = F->sweep;
  GemmArgs& GA = F->gemm;
  const double* lcc_dev = nullptr;
  pk.add(P.chains, &A.chains);
  pk.add(P.base_blocks, &A.base_blocks);
  pk.add(P.top_chain, &A.top_chain);
  pk.add(P.top_node, &A.top_node);
  pk.add(P.lcc, &lcc_dev);
  pk.add(P.u_off, &GA.gather);
  pk.add(P.probs, &GA.probs);
  pk.add(P.tasks, &GA.tasks);
  pk.add(P.ntasks, &GA.ntasks);
  pk.add(P.top_off, &A.top_off);
  pk.add(P.top_depth, &A.top_depth);
  pk.add(P.top_isd, &A.top_isd);
  pk.add(P.btask_ptr, &A.btask_ptr);
  pk.add(P.btask_nwin, &A.btask_nwin);
  pk.add(P.bnode, &A.bnode);
  pk.add(P.bent, &A.bent);
  pk.add(P.isd, &A.isd);
  pk.add(P.sub_p0, &A.sub_p0);
  pk.add(P.sub_p1, &A.sub_p1);
  pk.add(P.sub_K, &A.sub_K);
  pk.add(P.sub_ubeg, &A.sub_ubeg);
  pk.add(P.sub_udep, &A.sub_udep);
  pk.add(P.sub_uoff, &A.sub_uoff);
  pk.add(P.sub_bbase, &A.sub_bbase);
  A.nsub = (int32_t)P.sub_p0.size();
  A.nbase = (int32_t)P.base_blocks.size();
  A.store_wide = (P.store_wide || G.store64) ? 1 : 0;
  F->resident_bytes = pk.total + (uint64_t)std::max<int64_t>(P.bt_elems, 1) * 8 + (uint64_t)std::max<int64_t>(P.b_elems, 1) * 8;
  F->store_bytes = (uint64_t)(std::max<int64_t>(P.store_elems, kWin) + std::max<int64_t>(P.x_elems, 1) +
                              std::max<int64_t>(P.t_elems, 1)) * 8;
  const uint64_t luc_bytes = (uint64_t)std::max<int64_t>(P.bt_elems, 1) * 8;
  st = D->reserve(F->resident_bytes + F->store_bytes + luc_bytes);
  if (st != OK) { free_query_plan(*F, F->edges); return (peers_status)st; }
  F->reserved = F->resident_bytes + F->store_bytes;
  he = hipMalloc(&F->base, pk.total);
  if (he != hipSuccess) { D->release(luc_bytes); return (peers_status)hip_fail(he, "hipMalloc(factor)"); }
  he = hipMalloc(&F->store, (size_t)std::max<int64_t>(P.store_elems, kWin) * 8);
  if (he == hipSuccess) he = hipMalloc(&F->xbuf, (size_t)std::max<int64_t>(P.x_elems, 1) * 8);
  if (he == hipSuccess) he = hipMalloc(&F->tbuf, (size_t)std::max<int64_t>(P.t_elems, 1) * 8);
  if (he == hipSuccess) he = hipMalloc(&F->btbuf, (size_t)std::max<int64_t>(P.bt_elems, 1) * 8);
  if (he == hipSuccess) he = hipMalloc(&F->bbuf, (size_t)std::max<int64_t>(P.b_elems, 1) * 8);
  void* lucbuf = nullptr;
  if (he == hipSuccess) he = hipMalloc(&lucbuf, luc_bytes);
  if (he != hipSuccess) { D->release(luc_bytes); return (peers_status)hip_fail(he, "hipMalloc(top workspace)"); }
  A.store = (double*)F->store;
  A.X = (double*)F->xbuf;
  A.B = (double*)F->bbuf;
  st = pk.commit(F->base, s);
  if (st != OK) { (void)hipFree(lucbuf); D->release(luc_bytes); return (peers_status)st; }
  A.lcc = lcc_dev;
  GA.buf[BUF_STORE] = (double*)F->store;
  GA.buf[BUF_LCC] = const_cast<double*>(lcc_dev);
  GA.buf[BUF_X] = (double*)F->xbuf;
  GA.buf[BUF_T] = (double*)F->tbuf;
  GA.buf[BUF_BT] = (double*)F->btbuf;
  GA.buf[BUF_LUC] = (double*)lucbuf;
  // zero the triangular-inverse workspace once (its upper blocks are never written)
  // and the transfer blocks' padding; then B_C = -L_{U,C} L_CC^{-1} on the GPU
  he = hipMemsetAsync(F->xbuf, 0, (size_t)std::max<int64_t>(P.x_elems, 1) * 8, s);
  // the store's leading zero block (windows past a column's depth read it)
  if (he == hipSuccess) he = hipMemsetAsync(F->store, 0, (size_t)kStoreZeroBlock * 8, s);
  if (he == hipSuccess) he = hipMemsetAsync(F->btbuf, 0, (size_t)std::max<int64_t>(P.bt_elems, 1) * 8, s);
  if (he == hipSuccess && !P.luc.empty())
    he = hipMemcpyAsync(lucbuf, P.luc.data(), P.luc.size() * 8, hipMemcpyHostToDevice, s);
  if (he != hipSuccess) { (void)hipFree(lucbuf); D->release(luc_bytes); return (peers_status)hip_fail(he, "upload"); }
  he = hipStreamSynchronize(s);
  if (he != hipSuccess) { (void)hipFree(lucbuf); D->release(luc_bytes); return (peers_status)hip_fail(he, "upload"); }
  F->t_transfer = now_s() - tp;
  if (dev_numeric) {
    // the factor on the device; its values are copied back into the graph
    // handle (exports, later uploads, the host scheme)
    GraphHandle& Gm = const_cast<GraphHandle&>(G);
    double ms = 0;
    st = device_factor(*F, G, *NP, const_cast<double*>(lcc_dev), (double*)lucbuf, s, &Gm.num, &ms);
    if (st != OK) { (void)hipFree(lucbuf); D->release(luc_bytes); return (peers_status)st; }
    Gm.numeric_ready = true;
    Gm.stats.t_numeric = ms * 1e-3;
    F->t_numeric_device = ms * 1e-3;
    NP.reset();
    std::vector<int64_t>().swap(F->plan->coef_p);
    std::vector<int64_t>().swap(F->plan->coef_off);
  }
  {
    const double t0 = now_s();
    int32_t nl = 0;
    // B_S of the bottom subtrees from the records' final coefficients
    he = launch_bxfer(F->sweep, s);
    st = he == hipSuccess ? OK : hip_fail(he, "bottom transfer blocks");
    if (st == OK) st = run_chain_inverse(*F, s, nl);
    if (st == OK) {
      he = launch_gemm(F->gemm, P.bpre_begin, P.bpre_end - P.bpre_begin, s);
      if (he != hipSuccess) st = hip_fail(he, "transfer blocks");
    }
    if (st == OK) {
      he = hipStreamSynchronize(s);
      if (he != hipSuccess) st = hip_fail(he, "hipStreamSynchronize(transfer blocks)");
    }
    F->t_transform = now_s() - t0;
  }
  (void)hipFree(lucbuf);
  D->release(luc_bytes);
  GA.buf[BUF_LUC] = nullptr;
  // the recursion temporaries are needed only while L_CC^{-1} is formed
  if (st == OK && F->tbuf) {
    (void)hipFree(F->tbuf);
    F->tbuf = nullptr;
    GA.buf[BUF_T] = nullptr;
    const uint64_t tb = (uint64_t)std::max<int64_t>(P.t_elems, 1) * 8;
    F->store_bytes -= tb;
    F->reserved -= tb;
    D->release(tb);
  }
  if (st != OK) return (peers_status)st;
  st = ensure_workspace(*F, F->edges.nslots, F->m, F->edges.stage_elems);
  if (st != OK) return (peers_status)st;
  he = hipStreamSynchronize(s);
  if (he != hipSuccess) return (peers_status)hip_fail(he, "hipStreamSynchronize(upload)");
  {
    // algorithmic work per phase: 2 flops per FMA of the exact count
    // F = sum over L_ki != 0 of depth(k) restricted to the phase's columns,
    // and 12 bytes (value + row index) per factor entry plus the top store
    double fb = 0, nb = 0, nt = 0;
    for (int32_t i = 0; i < G.sym.N; ++i) {
      double fi = 0;
      for (int64_t p = G.sym.colptr[i]; p < G.sym.colptr[i + 1]; ++p) fi += G.sym.depth[G.sym.rowidx[p]];
      if (P.small[i]) { fb += fi; nb += (double)(G.sym.colptr[i + 1] - G.sym.colptr[i]); }
      else nt += (double)(G.sym.colptr[i + 1] - G.sym.colptr[i]);
    }
    F->top_flops = 2.0 * P.f_top;  // exact count; the blocked forms do f_top_gemm + f_top_inv
    F->bottom_flops = 2.0 * fb + 3.0 * acc_bottom;
    F->finish_flops = 3.0 * acc_top;
    F->top_bytes = 12.0 * nt + 8.0 * (double)P.store_elems;
    F->bottom_bytes = 12.0 * nb + 16.0 * (double)F->m;
  }
  // host-side copies of the plan are only needed for query planning now
  FactorPlan& Pm = *F->plan;
  std::vector<double>().swap(Pm.lcc);
  std::vector<double>().swap(Pm.luc);
  std::vector<BEnt>().swap(Pm.bent);
  std::vector<BNode>().swap(Pm.bnode);
  *out = reinterpret_cast<peers_factor>(F.release());
  return PEERS_OK;
}

void peers_factor_release(peers_factor f) {
  if (!f) return;
  auto* F = reinterpret_cast<FactorHandle*>(f);
  // server requests on this factor (queued or running) finish first
  while (F->server_refs.load() > 0) std::this_thread::sleep_for(std::chrono::microseconds(100));
  { std::lock_guard<std::mutex> g(F->mu); }  // a plain or batched call on it has returned
  (void)hipSetDevice(F->dev->ordinal);
  (void)hipDeviceSynchronize();
  batch_cache_forget(*F->dev, F);
  free_query_plan(*F, F->edges);
  free_query_plan(*F, F->to_ground);
  if (F->base) (void)hipFree(F->base);
  if (F->store) (void)hipFree(F->store);
  if (F->xbuf) (void)hipFree(F->xbuf);
  if (F->tbuf) (void)hipFree(F->tbuf);
  if (F->btbuf) (void)hipFree(F->btbuf);
  if (F->bbuf) (void)hipFree(F->bbuf);
  for (auto& e : F->ev)
    if (e) (void)hipEventDestroy(e);

  if (F->part) (void)hipFree(F->part);
  if (F->res) (void)hipFree(F->res);
  if (F->stage) (void)hipFree(F->stage);
  F->dev->release(F->reserved + F->part_bytes + F->res_bytes + F->stage_bytes);
  delete F;
}

peers_status peers_factor_footprint(peers_factor f, uint64_t* resident_bytes, uint64_t* workspace_bytes) {
  if (!f) { set_error("null factor"); return PEERS_E_INVALID_ARG; }
  auto* F = reinterpret_cast<FactorHandle*>(f);
  if (resident_bytes) *resident_bytes = F->resident_bytes + F->edges.bytes;
  if (workspace_bytes) *workspace_bytes = F->store_bytes + F->part_bytes + F->res_bytes + F->stage_bytes;
  return PEERS_OK;
}

peers_status peers_factor_timings(peers_factor f, peers_sweep_timings* out) {
  if (!f || !out) { set_error("null argument"); return PEERS_E_INVALID_ARG; }
  auto* F = reinterpret_cast<FactorHandle*>(f);
  std::lock_guard<std::mutex> g(F->mu);
  *out = peers_sweep_timings{};
  out->top_launches = F->top_launches;
  out->bottom_launches = F->bottom_launches;
  out->top_flops = F->top_flops;
  out->bottom_flops = F->bottom_flops;
  out->top_bytes = F->top_bytes;
  out->bottom_bytes = F->bottom_bytes;
  out->finish_flops = F->finish_flops;
  out->t_layout_s = F->t_layout;
  out->t_edge_plan_s = F->t_edge_plan;
  out->t_transfer_s = F->t_transfer;
  out->t_transform_s = F->t_transform;
  if (!F->timed) return PEERS_OK;
  hipError_t e = hipEventSynchronize(F->ev[3]);
  if (e != hipSuccess) return (peers_status)hip_fail(e, "hipEventSynchronize");
  float ms[3] = {0, 0, 0};
  for (int k = 0; k < 3; ++k) {
    e = hipEventElapsedTime(&ms[k], F->ev[k], F->ev[k + 1]);
    if (e != hipSuccess) return (peers_status)hip_fail(e, "hipEventElapsedTime");
  }
  out->top_ms = ms[0];
  out->bottom_ms = ms[1];
  out->finish_ms = ms[2];
  out->total_ms = (double)ms[0] + ms[1] + ms[2];
  return PEERS_OK;
}

peers_status peers_factor_export_columns(peers_factor f, int64_t k, const int32_t* nodes, int64_t ld,
                                         double* Z_out, void* hip_stream) {
  if (!f || k < 0 || (k > 0 && (!nodes || !Z_out))) { set_error("null argument"); return PEERS_E_INVALID_ARG; }
  auto* F = reinterpret_cast<FactorHandle*>(f);
  hipStream_t s = (hipStream_t)hip_stream;
  std::lock_guard<std::mutex> g(F->mu);
  if (ld < F->plan->height) { set_error("ld is below the elimination tree height"); return PEERS_E_INVALID_ARG; }
  hipError_t he = hipSetDevice(F->dev->ordinal);
  if (he != hipSuccess) return (peers_status)hip_fail(he, "hipSetDevice");
  if (k == 0) return PEERS_OK;
  std::vector<int32_t> xs(k);
  for (int64_t i = 0; i < k; ++i) {
    if (nodes[i] < 0 || nodes[i] >= F->n) { set_error("node " + std::to_string(i) + " outside [0, n)"); return PEERS_E_NODE_RANGE; }
    if (nodes[i] == F->ground) { set_error("the ground node has no column"); return PEERS_E_INVALID_ARG; }
    xs[i] = perm_index(*F, nodes[i]);
  }
  QueryPlan Q;
  Status st = build_query_plan(F->first, F->depth, *F->plan, 0, nullptr, nullptr, Q, &F->anc, &xs);
  if (st != OK) return (peers_status)st;
  DeviceQueryPlan DQ;
  st = upload_query_plan(*F, Q, DQ, s);
  if (st == OK) st = ensure_workspace(*F, DQ.nslots, 1, DQ.stage_elems);
  if (st == OK) st = run_sweep(*F, DQ, (double*)F->res, s, false);
  for (int64_t i = 0; i < k && st == OK; ++i) {
    const int32_t dp = F->depth[xs[i]];
    const double* src = (Q.export_staged[i] ? (const double*)F->stage : (const double*)F->store) + Q.export_off[i];
    he = hipMemcpyAsync(Z_out + i * ld, src, (size_t)dp * 8, hipMemcpyDeviceToHost, s);
    if (he != hipSuccess) st = hip_fail(he, "hipMemcpyAsync(columns)");
  }
  he = hipStreamSynchronize(s);
  free_query_plan(*F, DQ);
  if (st != OK) return (peers_status)st;
  if (he != hipSuccess) return (peers_status)hip_fail(he, "hipStreamSynchronize");
  for (int64_t i = 0; i < k; ++i) {
    const int32_t dp = F->depth[xs[i]];
    std::fill(Z_out + i * ld + dp, Z_out + (i + 1) * ld, 0.0);
  }
  return PEERS_OK;
}

peers_status peers_query_all_edges(peers_factor f, double* R_out, uint32_t flags, void* hip_stream) {
  if (!f || (!R_out && reinterpret_cast<FactorHandle*>(f)->m > 0)) { set_error("null argument"); return PEERS_E_INVALID_ARG; }
  auto* F = reinterpret_cast<FactorHandle*>(f);
  hipStream_t s = (hipStream_t)hip_stream;
  std::lock_guard<std::mutex> g(F->mu);
  hipError_t he = hipSetDevice(F->dev->ordinal);
  if (he != hipSuccess) return (peers_status)hip_fail(he, "hipSetDevice");
  if (F->m == 0) return PEERS_OK;
  const bool dev_out = flags & PEERS_OUT_DEVICE;
  double* Rd = dev_out ? R_out : (double*)F->res;
  Status st = run_sweep(*F, F->edges, Rd, s, flags & PEERS_PROFILE);
  if (st != OK) return (peers_status)st;
  if (!dev_out) {
    he = hipMemcpyAsync(R_out, Rd, sizeof(double) * F->m, hipMemcpyDeviceToHost, s);
    if (he != hipSuccess) return (peers_status)hip_fail(he, "hipMemcpyAsync(results)");
  }
  if (!dev_out || (flags & PEERS_SYNC)) {
    he = hipStreamSynchronize(s);
    if (he != hipSuccess) return (peers_status)hip_fail(he, "hipStreamSynchronize");
  }
  return PEERS_OK;
}

peers_status peers_query_all_to_ground(peers_factor f, double* R_out, uint32_t flags, void* hip_stream) {
  if (!f || !R_out) { set_error("null argument"); return PEERS_E_INVALID_ARG; }
  auto* F = reinterpret_cast<FactorHandle*>(f);
  hipStream_t s = (hipStream_t)hip_stream;
  std::lock_guard<std::mutex> g(F->mu);
  hipError_t he = hipSetDevice(F->dev->ordinal);
  if (he != hipSuccess) return (peers_status)hip_fail(he, "hipSetDevice");
  if (!F->to_ground_ready) {
    // pairs (x, g) for every original id x, in id order; (g, g) gives 0
    std::vector<int32_t> a(F->n), b(F->n, -1);
    for (int64_t x = 0; x < F->n; ++x) a[x] = perm_index(*F, (int32_t)x);
    QueryPlan Q;
    Status st = build_query_plan_handle(*F, F->n, a.data(), b.data(), Q, true);
    if (st == OK) st = upload_query_plan(*F, Q, F->to_ground, s);
    if (st == OK) st = ensure_workspace(*F, F->to_ground.nslots, F->n, F->to_ground.stage_elems);
    if (st != OK) {
      free_query_plan(*F, F->to_ground);
      return (peers_status)st;
    }
    F->to_ground_ready = true;
  }
  const bool dev_out = flags & PEERS_OUT_DEVICE;
  double* Rd = dev_out ? R_out : (double*)F->res;
  Status st = run_sweep(*F, F->to_ground, Rd, s, flags & PEERS_PROFILE);
  if (st != OK) return (peers_status)st;
  if (!dev_out) {
    he = hipMemcpyAsync(R_out, Rd, sizeof(double) * F->n, hipMemcpyDeviceToHost, s);
    if (he != hipSuccess) return (peers_status)hip_fail(he, "hipMemcpyAsync(results)");
  }
  if (!dev_out || (flags & PEERS_SYNC)) {
    he = hipStreamSynchronize(s);
    if (he != hipSuccess) return (peers_status)hip_fail(he, "hipStreamSynchronize");
  }
  return PEERS_OK;
}

peers_status peers_query(peers_factor f, int64_t q, const int32_t* qu, const int32_t* qv, double* R_out,
                         uint32_t flags, void* hip_stream) {
  if (!f || q < 0 || (q > 0 && (!qu || !qv || !R_out))) { set_error("null argument"); return PEERS_E_INVALID_ARG; }
  auto* F = reinterpret_cast<FactorHandle*>(f);
  hipStream_t s = (hipStream_t)hip_stream;
  std::lock_guard<std::mutex> g(F->mu);
  hipError_t he = hipSetDevice(F->dev->ordinal);
  if (he != hipSuccess) return (peers_status)hip_fail(he, "hipSetDevice");
  if (q == 0) return PEERS_OK;
  std::vector<int32_t> hu, hv;
  const int32_t* u = qu;
  const int32_t* v = qv;
  if (flags & PEERS_IN_DEVICE) {
    hu.resize(q);
    hv.resize(q);
    he = hipMemcpyAsync(hu.data(), qu, sizeof(int32_t) * q, hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipMemcpyAsync(hv.data(), qv, sizeof(int32_t) * q, hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) return (peers_status)hip_fail(he, "copy query pairs");
    u = hu.data();
    v = hv.data();
  }
  DeviceQueryPlan DQ;
  Status st = plan_for_pairs(*F, q, u, v, DQ, s, true);
  if (st != OK) return (peers_status)st;
  st = ensure_workspace(*F, DQ.nslots, q, DQ.stage_elems);
  if (st == OK) {
    const bool dev_out = flags & PEERS_OUT_DEVICE;
    double* Rd = dev_out ? R_out : (double*)F->res;
    st = run_sweep(*F, DQ, Rd, s, flags & PEERS_PROFILE);
    if (st == OK && !dev_out) {
      he = hipMemcpyAsync(R_out, Rd, sizeof(double) * q, hipMemcpyDeviceToHost, s);
      if (he != hipSuccess) st = hip_fail(he, "hipMemcpyAsync(results)");
    }
  }
  he = hipStreamSynchronize(s);
  free_query_plan(*F, DQ);
  if (st != OK) return (peers_status)st;
  if (he != hipSuccess) return (peers_status)hip_fail(he, "hipStreamSynchronize");
  return PEERS_OK;
}

}  // extern "C"
