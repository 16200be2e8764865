// Batched form: the sweeps of many resident factors run as one sequence of
// grouped launches (one launch per step of the sweep, covering that step of
// every factor), captured once as a HIP graph and replayed. Each factor's
// arithmetic is exactly that of its own sweep, so every result is
// bit-identical to the same query run alone.
//
// The bottom step's schedule (the order in which subtree work items are
// handed to workgroups, and whether workgroups are one per item or a
// persistent grid looping over items) is picked by timing the candidates on
// the first call of a batch and kept with the captured graph. The choice is
// also remembered under a signature of the batch's structure (per factor:
// sizes, elimination-tree height, top-tree shape and the GEMM tiles of every
// chain level, bottom work items and query entries), so a later batch of
// other factors with the same structure skips the timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <list>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <unordered_map>

#include "../../../include/peers.h"
#include "batch.h"
#include "device_handle.h"
#include "sweep_kernels.h"

namespace peers {

const char* const kBatchScheduleNames[kBatchSchedules] = {"natural order, one workgroup per item",
                                                         "largest first, one workgroup per item",
                                                         "largest first, persistent 8 workgroups per CU",
                                                         "largest first, persistent 4 workgroups per CU"};

void BatchLayout::use_schedule(int c) {
  if (bottom_stage < 0) return;
  stages[bottom_stage].off = bottom_off[c];
  stages[bottom_stage].grid = bottom_grid[c];
}

void batch_layout(const DeviceHandle& D, const std::vector<BatchEntry>& E, BatchLayout& L) {
  L = BatchLayout();
  const int32_t nb = (int32_t)E.size();
  L.fargs.resize(nb);
  for (int32_t i = 0; i < nb; ++i) {
    const FactorHandle& F = *E[i].F;
    L.fargs[i].g = F.gemm;
    L.fargs[i].a = F.sweep;
    L.fargs[i].q = E[i].plan->args;
    L.fargs[i].q.part = E[i].part ? E[i].part : (double*)F.part;
    L.fargs[i].q.stage = E[i].stage ? E[i].stage : (double*)F.stage;
    L.fargs[i].q.R = E[i].R_dev;
  }
  std::vector<GroupItem>& items = L.items;
  auto stage = [&](int kind, auto&& per_factor) {
    BatchStage st{kind, (int64_t)items.size(), 0, 0};
    for (int32_t i = 0; i < nb; ++i) per_factor(i);
    st.n = (int64_t)items.size() - st.off;
    st.grid = st.n;
    if (st.n > 0) L.stages.push_back(st);
  };
  auto range = [&](int32_t i, int64_t a, int64_t b) {
    for (int64_t t = a; t < b; ++t) items.push_back(GroupItem{i, 0, t});
  };
  // top-step items of chains the entry's plan does not read are left out
  auto need = [&](int32_t i, int32_t chain) {
    const DeviceQueryPlan& Q = *E[i].plan;
    return !Q.prune_top || Q.chain_need[chain];
  };
  auto gemm_range = [&](int32_t i, int64_t a, int64_t b) {
    const FactorPlan& P = *E[i].F->plan;
    for (int64_t t = a; t < b; ++t)
      if (need(i, P.prob_chain[P.tasks[t].prob])) items.push_back(GroupItem{i, 0, t});
  };
  int32_t lmax = 0;
  for (int32_t i = 0; i < nb; ++i) lmax = std::max(lmax, (int32_t)E[i].F->plan->t2_ptr.size() - 1);
  // top tree (L_CC^{-1} is part of each prepared factor): chain-internal
  // rows, then the chain levels
  stage(GK_CHAIN_ROWS, [&](int32_t i) {
    const FactorPlan& P = *E[i].F->plan;
    for (int64_t k = 0; k < P.ntop; ++k)
      if (need(i, P.top_chain[k])) items.push_back(GroupItem{i, 0, k});
  });
  for (int32_t l = 0; l < lmax; ++l) {
    stage(GK_GEMM, [&](int32_t i) {
      const FactorPlan& P = *E[i].F->plan;
      if (l + 1 < (int32_t)P.t2_ptr.size()) gemm_range(i, P.t2_ptr[l], P.t2_ptr[l + 1]);
    });
    stage(GK_GEMM_NARROW, [&](int32_t i) {
      const FactorPlan& P = *E[i].F->plan;
      if (l + 1 < (int32_t)P.t2n_ptr.size())
        for (int64_t t = P.t2n_ptr[l]; t < P.t2n_ptr[l + 1]; ++t)
          if (need(i, P.prob_chain[P.ntasks[t].prob])) items.push_back(GroupItem{i, 0, t});
    });
  }
  // dense rows above bottom subtrees: the items of each group
  for (int c = 0; c < kDenseAllGroups; ++c)
    stage(GK_DENSE + c, [&](int32_t i) {
      const DeviceQueryPlan& Q = *E[i].plan;
      if (Q.dense) range(i, Q.dclass_ptr[c], Q.dclass_ptr[c + 1]);
    });
  // bottom subtrees: one item list per candidate schedule
  {
    std::vector<GroupItem> nat;
    std::vector<double> cost;
    for (int32_t i = 0; i < nb; ++i) {
      const FactorPlan& P = *E[i].F->plan;
      const DeviceQueryPlan& Q = *E[i].plan;
      for (size_t w = 0; w < Q.work_task.size(); ++w) {
        const int32_t t = Q.work_task[w];
        const double nodes = P.btask_ptr[t + 1] - P.btask_ptr[t];
        const double wins = std::min(kBottomWaves * kWinPerWave, P.btask_nwin[t] - Q.work_win[w]);
        nat.push_back(GroupItem{i, 0, (int64_t)w});
        cost.push_back(nodes * wins);
      }
    }
    std::vector<int64_t> ord(nat.size());
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) { return cost[x] > cost[y]; });
    L.bottom_n = (int64_t)nat.size();
    for (int c = 0; c < kBatchSchedules; ++c) {
      L.bottom_off[c] = (int64_t)items.size();
      if (c == 0) items.insert(items.end(), nat.begin(), nat.end());
      else
        for (int64_t k : ord) items.push_back(nat[k]);
      L.bottom_grid[c] = c == 2 ? 8 * (int64_t)D.cus : c == 3 ? 4 * (int64_t)D.cus : L.bottom_n;
    }
    if (L.bottom_n > 0) {
      bool wide = false;
      for (int32_t i = 0; i < nb; ++i) wide = wide || L.fargs[i].a.store_wide != 0;
      L.bottom_stage = (int)L.stages.size();
      L.stages.push_back(BatchStage{wide ? GK_BOTTOM_WIDE : GK_BOTTOM, L.bottom_off[0], L.bottom_n, L.bottom_n});
    }
  }
  // finish: ordered window sums, top-node pairs, zero pairs, non-ancestor pairs
  auto blocks = [](int64_t n, int64_t per) { return (n + per - 1) / per; };
  stage(GK_REDUCE, [&](int32_t i) { range(i, 0, blocks(E[i].plan->args.nbq, kReduceBlock)); });
  stage(GK_TOP_QUERY, [&](int32_t i) { range(i, 0, blocks(E[i].plan->args.ntq, kTopQueryBlock)); });
  stage(GK_ZERO, [&](int32_t i) { range(i, 0, blocks(E[i].plan->args.nzero, kZeroBlock)); });
  stage(GK_GENERAL, [&](int32_t i) { range(i, 0, blocks(E[i].plan->args.ngp, kGeneralBlock)); });
  const uint64_t fa_bytes = (uint64_t)nb * sizeof(FactorArgs);
  L.items_offset = (fa_bytes + 255) / 256 * 256;
  L.bytes = L.items_offset + std::max<uint64_t>(items.size(), 1) * sizeof(GroupItem);
}

Status batch_upload(const BatchLayout& L, void* mem, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(mem, L.fargs.data(), L.fargs.size() * sizeof(FactorArgs), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !L.items.empty())
    e = hipMemcpyAsync((char*)mem + L.items_offset, L.items.data(), L.items.size() * sizeof(GroupItem),
                       hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "batch upload");
  return OK;
}

Status batch_launch_stage(const BatchLayout& L, const BatchStage& st, void* mem, hipStream_t s) {
  const auto* fa = (const FactorArgs*)mem;
  const auto* items = (const GroupItem*)((char*)mem + L.items_offset);
  hipError_t e = launch_grouped(st.kind, fa, items + st.off, st.n, st.grid, s);
  if (e != hipSuccess) return hip_fail(e, "grouped launch");
  return OK;
}

Status batch_launch(const BatchLayout& L, void* mem, hipStream_t s) {
  for (const BatchStage& st : L.stages) {
    Status r = batch_launch_stage(L, st, mem, s);
    if (r != OK) return r;
  }
  return OK;
}

Status run_sweep_pruned(FactorHandle& F, DeviceQueryPlan& D, double* R_dev, hipStream_t s, bool profile,
                        const SweepWork* work) {
  std::vector<BatchEntry> be{
      BatchEntry{&F, &D, R_dev, work ? work->part : nullptr, work ? work->stage : nullptr}};
  auto L = std::make_shared<BatchLayout>();
  batch_layout(*F.dev, be, *L);
  void* mem = D.layout_mem;
  if (work && work->layout) {
    // caller memory (nothing is allocated)
    if (L->bytes > work->layout_cap) {
      set_error("the launch layout needs " + std::to_string(L->bytes) + " bytes, " +
                std::to_string(work->layout_cap) + " are left in the caller's workspace");
      return E_OVER_BUDGET;
    }
    mem = work->layout;
  } else if (L->bytes > D.layout_bytes) {
    if (D.layout_mem) {
      (void)hipFree(D.layout_mem);
      F.dev->release(D.layout_bytes);
      D.layout_mem = nullptr;
      D.layout_bytes = 0;
    }
    Status st = F.dev->reserve(L->bytes);
    if (st != OK) return st;
    hipError_t e = hipMalloc(&D.layout_mem, L->bytes);
    if (e != hipSuccess) {
      F.dev->release(L->bytes);
      return hip_fail(e, "hipMalloc(pruned sweep)");
    }
    D.layout_bytes = L->bytes;
    mem = D.layout_mem;
  }
  Status st = batch_upload(*L, mem, s);
  if (st != OK) return st;
  D.layout_host = L;  // host image stays alive while the copies may be pending
  if (profile && !F.ev[0])
    for (auto& e : F.ev) {
      hipError_t he = hipEventCreate(&e);
      if (he != hipSuccess) return hip_fail(he, "hipEventCreate");
    }
  F.timed = profile;
  int32_t top = 0, bottom = 0;
  const int nst = (int)L->stages.size();
  // phase boundaries (events 1 and 2): the first bottom-or-finish step and the first finish step
  int b1 = nst, b2 = nst;
  for (int k = nst - 1; k >= 0; --k) {
    const int kd = L->stages[k].kind;
    const bool finish = kd == GK_REDUCE || kd == GK_TOP_QUERY || kd == GK_ZERO || kd == GK_GENERAL;
    if (kd == GK_BOTTOM || kd == GK_BOTTOM_WIDE || kd >= GK_DENSE || finish) b1 = k;
    if (finish) b2 = k;
  }
  if (profile) (void)hipEventRecord(F.ev[0], s);
  for (int k = 0; k <= nst; ++k) {
    if (profile && k == b1) (void)hipEventRecord(F.ev[1], s);
    if (profile && k == b2) (void)hipEventRecord(F.ev[2], s);
    if (k == nst) break;
    st = batch_launch_stage(*L, L->stages[k], mem, s);
    if (st != OK) return st;
    const int kd = L->stages[k].kind;
    if (kd == GK_BOTTOM || kd == GK_BOTTOM_WIDE || kd >= GK_DENSE) ++bottom;
    else if (k < b1) ++top;
  }
  if (profile) (void)hipEventRecord(F.ev[3], s);
  F.top_launches = top;
  F.bottom_launches = bottom;
  return OK;
}

namespace {

struct Entry {
  FactorHandle* F = nullptr;
  DeviceQueryPlan* plan = nullptr;  // the factor's all-edge plan or `own`
  DeviceQueryPlan own;
  double* R_dev = nullptr;
  double* R_host = nullptr;
  int64_t q = 0;
};

}  // namespace

// A built batch: layout in device memory and the captured graph.
struct BatchExec {
  std::vector<const FactorHandle*> factors;
  std::vector<const void*> key;
  DeviceHandle* dev = nullptr;
  BatchLayout L;
  void* mem = nullptr;
  uint64_t bytes = 0;
  int schedule = -1;
  double cand_ms[kBatchSchedules] = {0, 0, 0, 0};
  bool schedule_cached = false;  // taken from the signature memo, not timed
  uint64_t signature = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~BatchExec() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (mem) {
      (void)hipFree(mem);
      dev->release(bytes);
    }
  }
};

struct ScheduleMemo {
  int schedule = 0;
  double cand_ms[kBatchSchedules] = {0, 0, 0, 0};
};

struct BatchCache {
  std::list<std::unique_ptr<BatchExec>> execs;  // most recent first
  std::unordered_map<uint64_t, ScheduleMemo> schedules;  // by batch signature
  peers_batch_info last{};
};

void batch_cache_free(DeviceHandle& D) {
  std::lock_guard<std::mutex> g(D.batch_mu);
  delete D.batches;
  D.batches = nullptr;
}

void batch_cache_forget(DeviceHandle& D, const FactorHandle* F) {
  std::lock_guard<std::mutex> g(D.batch_mu);
  if (!D.batches) return;
  auto& Lst = D.batches->execs;
  for (auto it = Lst.begin(); it != Lst.end();) {
    if (std::find((*it)->factors.begin(), (*it)->factors.end(), F) != (*it)->factors.end()) it = Lst.erase(it);
    else ++it;
  }
}

namespace {

constexpr size_t kMaxCached = 4;

Status build_exec(DeviceHandle& D, std::vector<Entry>& E, BatchExec& X, hipStream_t s) {
  std::vector<BatchEntry> be;
  for (auto& e : E) {
    be.push_back(BatchEntry{e.F, e.plan, e.R_dev});
    X.factors.push_back(e.F);
  }
  batch_layout(D, be, X.L);
  Status st = D.reserve(X.L.bytes);
  if (st != OK) return st;
  X.dev = &D;
  X.bytes = X.L.bytes;
  hipError_t e = hipMalloc(&X.mem, X.bytes);
  if (e != hipSuccess) {
    D.release(X.bytes);
    X.bytes = 0;
    X.mem = nullptr;
    return hip_fail(e, "hipMalloc(batch)");
  }
  st = batch_upload(X.L, X.mem, s);
  if (st == OK) {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize(batch upload)");
  }
  return st;
}

// Structure signature of a batch (splitmix64 over the fields, in order).
uint64_t batch_signature(const std::vector<Entry>& E, bool all_edges) {
  uint64_t h = 0x6a09e667f3bcc909ull;
  auto mix = [&](uint64_t x) {
    uint64_t z = (h ^ x) + 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    h = z ^ (z >> 31);
  };
  mix(E.size());
  mix(all_edges ? 1 : 0);
  for (const Entry& e : E) {
    const FactorPlan& P = *e.F->plan;
    const DeviceQueryPlan& Q = *e.plan;
    mix((uint64_t)e.F->n);
    mix((uint64_t)e.F->m);
    mix((uint64_t)P.height);
    mix((uint64_t)P.ntop);
    mix(P.chains.size());
    mix(P.btask_nwin.size());
    mix(P.bnode_node.size());
    mix(P.t2_ptr.size());
    for (size_t l = 0; l + 1 < P.t2_ptr.size(); ++l) mix((uint64_t)(P.t2_ptr[l + 1] - P.t2_ptr[l]));
    for (size_t l = 0; l + 1 < P.t2n_ptr.size(); ++l) mix((uint64_t)(P.t2n_ptr[l + 1] - P.t2n_ptr[l]));
    // pair batches: the query-dependent counts to within a factor of two
    auto bucket = [&](uint64_t x) { return all_edges ? x : (uint64_t)(64 - __builtin_clzll(x | 1)); };
    mix(bucket(Q.work_task.size()));
    mix(bucket((uint64_t)Q.args.nbq));
    mix(bucket((uint64_t)e.q));
  }
  return h;
}

// Times each bottom schedule (after one pass of the top steps, which the
// bottom step only reads) and keeps the fastest.
Status autotune(BatchExec& X, hipStream_t s) {
  BatchLayout& L = X.L;
  if (L.bottom_stage < 0) {
    X.schedule = 0;
    return OK;
  }
  for (int k = 0; k < L.bottom_stage; ++k) {
    Status r = batch_launch_stage(L, L.stages[k], X.mem, s);
    if (r != OK) return r;
  }
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t ce = hipEventCreate(&ev[0]);
  if (ce == hipSuccess) ce = hipEventCreate(&ev[1]);
  if (ce != hipSuccess) {
    if (ev[0]) (void)hipEventDestroy(ev[0]);
    return hip_fail(ce, "hipEventCreate");
  }
  Status r = OK;
  double best = 1e300;
  for (int c = 0; c < kBatchSchedules && r == OK; ++c) {
    const BatchStage st{L.stages[L.bottom_stage].kind, L.bottom_off[c], L.bottom_n, L.bottom_grid[c]};
    double tmin = 1e300;
    for (int rep = 0; rep < 2 && r == OK; ++rep) {
      hipError_t e = hipEventRecord(ev[0], s);
      if (e == hipSuccess) r = batch_launch_stage(L, st, X.mem, s);
      if (r == OK && e == hipSuccess) e = hipEventRecord(ev[1], s);
      if (r == OK && e == hipSuccess) e = hipEventSynchronize(ev[1]);
      float ms = 0;
      if (r == OK && e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
      if (e != hipSuccess) r = hip_fail(e, "autotune timing");
      tmin = std::min(tmin, (double)ms);
    }
    X.cand_ms[c] = tmin;
    if (tmin < best) {
      best = tmin;
      X.schedule = c;
    }
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (r != OK) return r;
  L.use_schedule(X.schedule);
  return OK;
}

Status capture(BatchExec& X) {
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "hipStreamCreate(capture)");
  Status r = OK;
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) r = hip_fail(e, "hipStreamBeginCapture");
  if (r == OK) {
    r = batch_launch(X.L, X.mem, cs);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    if (r == OK && e != hipSuccess) r = hip_fail(e, "hipStreamEndCapture");
    X.graph = g;
  }
  if (r == OK) {
    e = hipGraphInstantiate(&X.exec, X.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) r = hip_fail(e, "hipGraphInstantiate");
  }
  (void)hipStreamDestroy(cs);
  return r;
}

}  // namespace

}  // namespace peers

using namespace peers;

extern "C" {

peers_status peers_batch_query(peers_device d, int32_t nb, const peers_factor* f, const int64_t* q,
                               const int32_t* const* qu, const int32_t* const* qv, double* const* R_out,
                               uint32_t flags, void* hip_stream) {
  if (!d || nb < 0 || (nb > 0 && (!f || !R_out))) { set_error("null argument"); return PEERS_E_INVALID_ARG; }
  if (nb == 0) return PEERS_OK;
  auto* D = reinterpret_cast<DeviceHandle*>(d);
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t he = hipSetDevice(D->ordinal);
  if (he != hipSuccess) return (peers_status)hip_fail(he, "hipSetDevice");
  std::vector<Entry> E(nb);
  std::vector<FactorHandle*> order;
  bool all_edges = true;
  for (int32_t i = 0; i < nb; ++i) {
    auto* F = reinterpret_cast<FactorHandle*>(f[i]);
    if (!F || F->dev != D) { set_error("factor " + std::to_string(i) + " is null or on another device"); return PEERS_E_INVALID_ARG; }
    const bool edges = !qu || !qv || !qu[i] || !qv[i];
    if (!edges && (!q || q[i] < 0)) { set_error("negative pair count"); return PEERS_E_INVALID_ARG; }
    E[i].F = F;
    E[i].q = edges ? F->m : q[i];
    if (E[i].q > 0 && !R_out[i]) { set_error("null output " + std::to_string(i)); return PEERS_E_INVALID_ARG; }
    all_edges = all_edges && edges;
    order.push_back(F);
  }
  std::sort(order.begin(), order.end());
  if (std::adjacent_find(order.begin(), order.end()) != order.end()) {
    set_error("a factor appears twice in one batch");
    return PEERS_E_INVALID_ARG;
  }
  // one sweep at a time per factor: lock every factor, in address order
  std::vector<std::unique_lock<std::mutex>> locks;
  for (FactorHandle* F : order) locks.emplace_back(F->mu);

  const bool dev_out = flags & PEERS_OUT_DEVICE;
  Status st = OK;
  for (int32_t i = 0; i < nb && st == OK; ++i) {
    Entry& e = E[i];
    const bool edges = !qu || !qv || !qu[i] || !qv[i];
    if (edges) {
      e.plan = &e.F->edges;
    } else {
      std::vector<int32_t> hu, hv;
      const int32_t* u = qu[i];
      const int32_t* v = qv[i];
      if ((flags & PEERS_IN_DEVICE) && e.q > 0) {
        hu.resize(e.q);
        hv.resize(e.q);
        he = hipMemcpy(hu.data(), qu[i], sizeof(int32_t) * e.q, hipMemcpyDeviceToHost);
        if (he == hipSuccess) he = hipMemcpy(hv.data(), qv[i], sizeof(int32_t) * e.q, hipMemcpyDeviceToHost);
        if (he != hipSuccess) { st = hip_fail(he, "copy query pairs"); break; }
        u = hu.data();
        v = hv.data();
      }
      st = plan_for_pairs(*e.F, e.q, u, v, e.own, s, true);
      if (st != OK) break;
      e.plan = &e.own;
    }
    st = ensure_workspace(*e.F, e.plan->nslots, e.q, e.plan->stage_elems);
    e.R_dev = dev_out ? R_out[i] : (double*)e.F->res;
    e.R_host = dev_out ? nullptr : R_out[i];
  }
  if (st == OK) {
    he = hipStreamSynchronize(s);  // plan uploads complete before the graph reads them
    if (he != hipSuccess) st = hip_fail(he, "hipStreamSynchronize(plans)");
  }

  std::lock_guard<std::mutex> bg(D->batch_mu);
  if (!D->batches) D->batches = new BatchCache();
  BatchCache& C = *D->batches;
  BatchExec* X = nullptr;
  std::unique_ptr<BatchExec> owned;
  std::vector<const void*> key;
  for (auto& e : E) {
    key.push_back(e.F);
    key.push_back(e.R_dev);
  }
  bool reused = false;
  if (st == OK && all_edges) {
    for (auto it = C.execs.begin(); it != C.execs.end(); ++it)
      if ((*it)->key == key) {
        C.execs.splice(C.execs.begin(), C.execs, it);
        X = C.execs.front().get();
        reused = true;
        break;
      }
  }
  if (st == OK && !X) {
    owned.reset(new BatchExec());
    owned->key = key;
    owned->signature = batch_signature(E, all_edges);
    st = build_exec(*D, E, *owned, s);
    if (st == OK) {
      auto it = C.schedules.find(owned->signature);
      if (it != C.schedules.end() && owned->L.bottom_stage >= 0) {
        owned->schedule = it->second.schedule;
        std::copy(it->second.cand_ms, it->second.cand_ms + kBatchSchedules, owned->cand_ms);
        owned->schedule_cached = true;
        owned->L.use_schedule(owned->schedule);
      } else {
        st = autotune(*owned, s);
        if (st == OK && owned->L.bottom_stage >= 0) {
          ScheduleMemo& m = C.schedules[owned->signature];
          m.schedule = owned->schedule;
          std::copy(owned->cand_ms, owned->cand_ms + kBatchSchedules, m.cand_ms);
        }
      }
    }
    if (st == OK) st = capture(*owned);
    if (st == OK) X = owned.get();
  }
  hipEvent_t ev[2] = {nullptr, nullptr};
  float total_ms = 0;
  if (st == OK) {
    (void)hipEventCreate(&ev[0]);
    (void)hipEventCreate(&ev[1]);
    (void)hipEventRecord(ev[0], s);
    he = hipGraphLaunch(X->exec, s);
    if (he != hipSuccess) st = hip_fail(he, "hipGraphLaunch");
    (void)hipEventRecord(ev[1], s);
  }
  for (int32_t i = 0; i < nb && st == OK; ++i)
    if (E[i].R_host && E[i].q > 0) {
      he = hipMemcpyAsync(E[i].R_host, E[i].R_dev, sizeof(double) * E[i].q, hipMemcpyDeviceToHost, s);
      if (he != hipSuccess) st = hip_fail(he, "hipMemcpyAsync(results)");
    }
  const bool must_sync = !dev_out || (flags & PEERS_SYNC) || !all_edges;
  if (must_sync) {
    he = hipStreamSynchronize(s);
    if (st == OK && he != hipSuccess) st = hip_fail(he, "hipStreamSynchronize");
  }
  if (st == OK) {
    peers_batch_info& I = C.last;
    I = peers_batch_info{};
    I.factors = nb;
    I.stages = (int32_t)X->L.stages.size();
    I.bottom_items = X->L.bottom_n;
    I.schedule = X->schedule;
    I.candidates = kBatchSchedules;
    for (int c = 0; c < kBatchSchedules; ++c) I.candidate_ms[c] = X->cand_ms[c];
    std::snprintf(I.schedule_name, sizeof(I.schedule_name), "%s", kBatchScheduleNames[std::max(0, X->schedule)]);
    I.graph_reused = reused ? 1 : 0;
    I.schedule_cached = X->schedule_cached ? 1 : 0;
    I.signature = X->signature;
    if (must_sync && hipEventElapsedTime(&total_ms, ev[0], ev[1]) == hipSuccess) I.last_ms = total_ms;
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  if (owned && st == OK && all_edges) {
    C.execs.push_front(std::move(owned));
    while (C.execs.size() > kMaxCached) C.execs.pop_back();
  }
  if (st != OK) (void)hipStreamSynchronize(s);
  owned.reset();  // per-call graphs (their plans die with this call)
  for (auto& e : E) free_query_plan(*e.F, e.own);
  return (peers_status)st;
}

peers_status peers_batch_last_info(peers_device d, peers_batch_info* out) {
  if (!d || !out) { set_error("null argument"); return PEERS_E_INVALID_ARG; }
  auto* D = reinterpret_cast<DeviceHandle*>(d);
  std::lock_guard<std::mutex> g(D->batch_mu);
  *out = D->batches ? D->batches->last : peers_batch_info{};
  return PEERS_OK;
}

}  // extern "C"
