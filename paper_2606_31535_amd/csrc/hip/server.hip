// Served form: a request loop over resident factors with continuous batching.
//
// Callers submit pair requests against resident factors from any thread. One
// worker keeps up to `streams` device batches in flight, each on its own HIP
// stream: a batch takes the pending requests (oldest first, up to a pair cap),
// merges those of the same factor into one pruned query plan, and runs the
// plans of all its factors as one grouped launch sequence (the batched form's
// steps). Requests that arrive while batches are on the device go into the
// next batch that a free stream forms, so work from different requests
// overlaps on the device.
//
// One factor may be in several batches at once. Each batch has its own
// partial slots, staging and result buffers (in its stream's arena); the only
// factor memory two batches share is the top store, and every sweep writes
// the same values there (each top column is formed from the factor alone, in
// a fixed order), so overlapping sweeps of one factor read exactly the values
// a lone sweep reads. Every result is therefore the same bits as the request
// run alone: the plan computes each pair independently of the other pairs.
//
// Admission by memory: factors are admitted at upload (their footprint
// against the device's HBM budget). A batch's arena (plans, launch layout,
// workspaces) is reserved against the same budget when the batch is formed.
// If it does not fit while other batches are on the device, its requests go
// back to the head of the queue and wait until a batch completes and frees
// memory; idle streams give their arenas back. A batch that does not fit on
// an otherwise idle device is cut to its first request, and only a single
// request that cannot fit an idle device fails with PEERS_E_OVER_BUDGET.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <unordered_map>

#include "../../../include/peers.h"
#include "batch.h"
#include "device_handle.h"

namespace peers {

namespace {

using Clock = std::chrono::steady_clock;

// an idle stream keeps its arena this long before giving it back to the budget
constexpr auto kArenaIdleRelease = std::chrono::milliseconds(20);

struct Request {
  uint64_t ticket = 0;
  FactorHandle* F = nullptr;
  std::vector<int32_t> a, b;  // reduced-permuted endpoints (-1 = ground)
  double* R_out = nullptr;
  int64_t q = 0;
  Clock::time_point t_submit;
  peers_status status = PEERS_OK;
  bool done = false;
  bool cancelled = false;  // results are not copied out
  bool on_device = false;  // taken into a batch
};
using ReqPtr = std::shared_ptr<Request>;

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  void* arena = nullptr;  // plans, batch layout and workspaces of the batch in flight
  uint64_t arena_bytes = 0;
  double* pinned = nullptr;  // results, device -> host
  int64_t pinned_elems = 0;
  bool busy = false;
  Clock::time_point idle_since = Clock::now();
  std::vector<ReqPtr> reqs;
  std::vector<int64_t> req_off;  // each request's first result in `pinned`
  std::vector<QueryPlan> hplans;
  std::vector<DeviceQueryPlan> dplans;
  BatchLayout L;
};

enum class Launch { Started, WaitForMemory, TooBig, Failed };

}  // namespace

struct Server {
  DeviceHandle* D = nullptr;
  peers_server_opts o{};
  std::mutex mu;
  std::condition_variable cv_req, cv_done;
  std::deque<ReqPtr> pending;
  std::unordered_map<uint64_t, ReqPtr> reqs;
  uint64_t next_ticket = 1;
  bool stopping = false;
  bool mem_blocked = false;  // the head batch waits for a batch to complete
  std::vector<Slot> slots;
  std::thread worker;
  // statistics
  uint64_t submitted = 0, completed = 0, rejected = 0, batches = 0, pairs_done = 0, memory_waits = 0;
  std::vector<double> lat_us;
  double busy_s = 0;
  Clock::time_point busy_since;
  int busy_slots = 0;
};

namespace {

uint64_t align256(uint64_t x) { return (x + 255) / 256 * 256; }

void free_arena(Server& S, Slot& sl) {
  if (!sl.arena) return;
  (void)hipFree(sl.arena);
  S.D->release(sl.arena_bytes);
  sl.arena = nullptr;
  sl.arena_bytes = 0;
}

// Makes the slot's arena at least `need` bytes (budgeted). On a budget
// refusal, idle slots give their arenas back and the reservation is tried
// again; the result says whether it is worth waiting for busy slots.
Launch reserve_arena(Server& S, Slot& sl, uint64_t need, Status& err) {
  if (need <= sl.arena_bytes) return Launch::Started;
  free_arena(S, sl);
  need = std::max<uint64_t>(need, 1 << 20);
  Status st = S.D->reserve(need);
  if (st == E_OVER_BUDGET) {
    for (Slot& o : S.slots)
      if (&o != &sl && !o.busy) free_arena(S, o);
    st = S.D->reserve(need);
  }
  if (st == E_OVER_BUDGET) {
    for (Slot& o : S.slots)
      if (&o != &sl && o.busy) return Launch::WaitForMemory;
    err = st;
    return Launch::TooBig;
  }
  if (st != OK) {
    err = st;
    return Launch::Failed;
  }
  hipError_t e = hipMalloc(&sl.arena, need);
  if (e != hipSuccess) {
    S.D->release(need);
    err = hip_fail(e, "hipMalloc(server arena)");
    return Launch::Failed;
  }
  sl.arena_bytes = need;
  return Launch::Started;
}

Status grow_pinned(Slot& sl, int64_t need) {
  if (need <= sl.pinned_elems) return OK;
  need = std::max<int64_t>(need, sl.pinned_elems + sl.pinned_elems / 2);
  if (sl.pinned) (void)hipHostFree(sl.pinned);
  sl.pinned = nullptr;
  sl.pinned_elems = 0;
  hipError_t e = hipHostMalloc((void**)&sl.pinned, (size_t)need * 8, hipHostMallocDefault);
  if (e != hipSuccess) return hip_fail(e, "hipHostMalloc(results)");
  sl.pinned_elems = need;
  return OK;
}

// (server lock held)
void finish_request(Server& S, Request* r, peers_status st) {
  if (r->done) return;
  r->status = r->cancelled && st == PEERS_OK ? PEERS_E_CANCELLED : st;
  r->done = true;
  r->F->server_refs.fetch_sub(1);
  const double us = std::chrono::duration<double, std::micro>(Clock::now() - r->t_submit).count();
  if (r->status == PEERS_OK) {
    S.completed++;
    S.pairs_done += (uint64_t)r->q;
    S.lat_us.push_back(us);
  } else {
    S.rejected++;
  }
}

// Builds and launches one batch on a free slot (worker thread, server lock
// not held). Requests whose factor could not be planned fail individually
// (reported through `failed`); a batch that does not fit the budget is not
// launched and its requests stay with the caller.
Launch launch(Server& S, Slot& sl, const std::vector<ReqPtr>& take,
              std::vector<std::pair<ReqPtr, peers_status>>& failed, Status& err) {
  sl.reqs.clear();
  sl.req_off.clear();
  sl.hplans.clear();
  sl.dplans.clear();
  // group by factor, keeping submission order inside each factor
  std::map<FactorHandle*, std::vector<ReqPtr>> groups;
  std::vector<FactorHandle*> forder;
  for (const ReqPtr& r : take) {
    if (!groups.count(r->F)) forder.push_back(r->F);
    groups[r->F].push_back(r);
  }
  // host plans of the factors, in parallel (independent per factor)
  const size_t nf = forder.size();
  std::vector<QueryPlan> plans(nf);
  std::vector<Status> pst(nf, OK);
  auto plan_one = [&](size_t i) {
    FactorHandle* F = forder[i];
    const std::vector<ReqPtr>& G = groups.at(F);
    int64_t q = 0;
    for (const ReqPtr& r : G) q += r->q;
    std::vector<int32_t> a, b;
    a.reserve(q);
    b.reserve(q);
    for (const ReqPtr& r : G) {
      a.insert(a.end(), r->a.begin(), r->a.end());
      b.insert(b.end(), r->b.begin(), r->b.end());
    }
    pst[i] = build_query_plan_handle(*F, q, a.data(), b.data(), plans[i], true);
  };
  {
    std::vector<std::thread> th;
    for (size_t i = 1; i < nf; ++i) th.emplace_back(plan_one, i);
    if (nf) plan_one(0);
    for (auto& t : th) t.join();
  }
  std::vector<FactorHandle*> planned;
  std::vector<ReqPtr> reqs;
  std::vector<int64_t> req_off;
  int64_t total = 0;
  for (size_t i = 0; i < nf; ++i) {
    FactorHandle* F = forder[i];
    if (pst[i] != OK) {
      for (const ReqPtr& r : groups[F]) failed.push_back({r, (peers_status)pst[i]});
      continue;
    }
    sl.hplans.push_back(std::move(plans[i]));
    planned.push_back(F);
    for (const ReqPtr& r : groups[F]) {
      reqs.push_back(r);
      req_off.push_back(total);
      total += r->q;
    }
  }
  if (planned.empty()) return Launch::Started;  // nothing left to run
  // arena: plans, then the batch layout, then per-plan workspaces
  // (partial slots, results, staging)
  const size_t np = planned.size();
  std::vector<uint64_t> poff(np), woff(np);
  uint64_t bytes = 0;
  for (size_t i = 0; i < np; ++i) {
    poff[i] = bytes;
    bytes += align256(query_plan_bytes(sl.hplans[i]));
  }
  sl.dplans.resize(np);
  std::vector<BatchEntry> be;
  for (size_t i = 0; i < np; ++i) {
    // host-side plan fields (counts, work lists) are what the layout reads
    DeviceQueryPlan& d = sl.dplans[i];
    d.work_task = sl.hplans[i].work_task;
    d.work_win = sl.hplans[i].work_win;
    d.chain_need = sl.hplans[i].chain_need;
    d.prune_top = sl.hplans[i].prune_top;
    d.args.nbq = sl.hplans[i].nbq();
    d.args.ntq = (int64_t)sl.hplans[i].tq_out.size();
    d.args.nzero = (int64_t)sl.hplans[i].zero_out.size();
    d.args.ngp = (int64_t)sl.hplans[i].gp.size();
    d.args.nditems = (int64_t)sl.hplans[i].ditems.size();
    d.dense = sl.hplans[i].dense;
    d.dclass_ptr = sl.hplans[i].dclass_ptr;
    be.push_back(BatchEntry{planned[i], &sl.dplans[i], nullptr, nullptr, nullptr});
  }
  BatchLayout probe;
  batch_layout(*S.D, be, probe);
  const uint64_t layout_off = bytes;
  bytes += align256(probe.bytes);
  // partial slots (with the dense sums after them), results, staging
  auto part_bytes = [](const QueryPlan& Q) {
    return align256((uint64_t)std::max<int64_t>(Q.nslots + (Q.dense ? Q.nbq() : 0), 1) * 8);
  };
  for (size_t i = 0; i < np; ++i) {
    const QueryPlan& Q = sl.hplans[i];
    woff[i] = bytes;
    bytes += part_bytes(Q) + align256((uint64_t)std::max<int64_t>(Q.q, 1) * 8) +
             align256((uint64_t)std::max<int64_t>(Q.stage_elems, 1) * 8);
  }
  Launch how = reserve_arena(S, sl, bytes, err);
  if (how != Launch::Started) return how;
  Status st = grow_pinned(sl, std::max<int64_t>(total, 1));
  char* ar = (char*)sl.arena;
  for (size_t i = 0; i < np && st == OK; ++i) {
    const QueryPlan& Q = sl.hplans[i];
    st = upload_query_plan_to(Q, sl.dplans[i], ar + poff[i], sl.stream);
    be[i].part = (double*)(ar + woff[i]);
    be[i].R_dev = (double*)(ar + woff[i] + part_bytes(Q));
    be[i].stage = (double*)((char*)be[i].R_dev + align256((uint64_t)std::max<int64_t>(Q.q, 1) * 8));
  }
  if (st == OK) {
    batch_layout(*S.D, be, sl.L);
    st = batch_upload(sl.L, ar + layout_off, sl.stream);
  }
  if (st == OK) st = batch_launch(sl.L, ar + layout_off, sl.stream);
  // results of each factor, in request order, into the pinned buffer
  int64_t off = 0;
  for (size_t i = 0; i < np && st == OK; ++i) {
    const int64_t q = sl.hplans[i].q;
    if (q > 0) {
      hipError_t e = hipMemcpyAsync(sl.pinned + off, be[i].R_dev, (size_t)q * 8, hipMemcpyDeviceToHost, sl.stream);
      if (e != hipSuccess) st = hip_fail(e, "hipMemcpyAsync(server results)");
    }
    off += q;
  }
  if (st == OK) {
    hipError_t e = hipEventRecord(sl.ev, sl.stream);
    if (e != hipSuccess) st = hip_fail(e, "hipEventRecord(server)");
  }
  if (st != OK) {
    (void)hipStreamSynchronize(sl.stream);
    for (const ReqPtr& r : reqs) failed.push_back({r, (peers_status)st});
    return Launch::Started;
  }
  sl.reqs = std::move(reqs);
  sl.req_off = std::move(req_off);
  return Launch::Started;
}

// Hands a finished batch's results to its requests (server lock held).
void complete(Server& S, Slot& sl, hipError_t e) {
  for (size_t i = 0; i < sl.reqs.size(); ++i) {
    Request* r = sl.reqs[i].get();
    if (e == hipSuccess && r->q > 0 && !r->cancelled)
      std::memcpy(r->R_out, sl.pinned + sl.req_off[i], (size_t)r->q * 8);
    finish_request(S, r, e == hipSuccess ? PEERS_OK : PEERS_E_HIP);
  }
  sl.reqs.clear();
  sl.busy = false;
  sl.idle_since = Clock::now();
  S.mem_blocked = false;
  if (--S.busy_slots == 0) S.busy_s += std::chrono::duration<double>(Clock::now() - S.busy_since).count();
  S.cv_done.notify_all();
}

void run(Server& S) {
  (void)hipSetDevice(S.D->ordinal);
  const int64_t cap = S.o.max_batch_pairs > 0 ? S.o.max_batch_pairs : (1 << 20);
  const auto max_wait = std::chrono::microseconds(S.o.max_wait_us > 0 ? S.o.max_wait_us : 200);
  std::unique_lock<std::mutex> lk(S.mu);
  for (;;) {
    bool progressed = false;
    for (Slot& sl : S.slots) {
      if (!sl.busy) continue;
      const hipError_t e = hipEventQuery(sl.ev);
      if (e == hipErrorNotReady) continue;
      complete(S, sl, e);
      progressed = true;
    }
    Slot* free_slot = nullptr;
    for (Slot& sl : S.slots)
      if (!sl.busy) {
        free_slot = &sl;
        break;
      }
    if (free_slot && !S.pending.empty() && !S.mem_blocked) {
      // while another batch keeps the device busy, let a small batch wait a
      // little for batch-mates
      int64_t pend = 0;
      for (const ReqPtr& r : S.pending) pend += r->q;
      const bool young = Clock::now() - S.pending.front()->t_submit < max_wait;
      if (!(S.busy_slots > 0 && pend < cap && young)) {
        std::vector<ReqPtr> take;
        int64_t pairs = 0;
        while (!S.pending.empty()) {
          const ReqPtr& r = S.pending.front();
          if (pairs > 0 && pairs + r->q > cap) break;
          pairs += r->q;
          r->on_device = true;
          take.push_back(r);
          S.pending.pop_front();
        }
        // form and launch without the lock; a batch too large for an idle
        // device is retried with its first request alone
        for (;;) {
          lk.unlock();
          std::vector<std::pair<ReqPtr, peers_status>> failed;
          Status err = OK;
          const Launch how = launch(S, *free_slot, take, failed, err);
          lk.lock();
          for (auto& fr : failed) finish_request(S, fr.first.get(), fr.second);
          if (!failed.empty()) S.cv_done.notify_all();
          // requests that failed to plan are finished: never queue them again
          take.erase(std::remove_if(take.begin(), take.end(), [](const ReqPtr& r) { return r->done; }), take.end());
          if (take.empty() && how != Launch::Started) break;
          if (how == Launch::Started) {
            if (!free_slot->reqs.empty()) {
              free_slot->busy = true;
              if (S.busy_slots++ == 0) S.busy_since = Clock::now();
              S.batches++;
            }
            break;
          }
          if (how == Launch::WaitForMemory || (how == Launch::TooBig && take.size() > 1)) {
            // back to the head of the queue, in order: all of them when
            // memory frees up later, all but the first when the batch is
            // too large even for an idle device
            const size_t keep = how == Launch::WaitForMemory ? 0 : 1;
            for (size_t i = take.size(); i > keep; --i) {
              take[i - 1]->on_device = false;
              S.pending.push_front(take[i - 1]);
            }
            take.resize(keep);
            if (how == Launch::WaitForMemory) {
              S.mem_blocked = true;
              S.memory_waits++;
              break;
            }
            continue;
          }
          // a lone request that does not fit, or a failure
          for (const ReqPtr& r : take) finish_request(S, r.get(), (peers_status)(err != OK ? err : E_OVER_BUDGET));
          S.cv_done.notify_all();
          break;
        }
        progressed = true;
      }
    }
    // idle streams give their arenas back to the budget
    if (S.pending.empty()) {
      const auto now = Clock::now();
      for (Slot& sl : S.slots)
        if (!sl.busy && sl.arena && now - sl.idle_since > kArenaIdleRelease) free_arena(S, sl);
    }
    if (S.stopping && S.pending.empty() && S.busy_slots == 0) break;
    if (!progressed) {
      bool arenas = false;
      for (Slot& sl : S.slots) arenas = arenas || (!sl.busy && sl.arena);
      if (S.busy_slots > 0 || (!S.pending.empty() && !S.mem_blocked) || arenas)
        S.cv_req.wait_for(lk, std::chrono::microseconds(50));
      else if (S.busy_slots == 0 && S.mem_blocked)
        S.mem_blocked = false;  // nothing on the device: try again
      else
        S.cv_req.wait(lk, [&] { return S.stopping || !S.pending.empty(); });
    }
  }
}

double percentile(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double x = p * (double)(v.size() - 1);
  const size_t i = (size_t)x;
  const double f = x - (double)i;
  return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

}  // namespace

}  // namespace peers

using namespace peers;

extern "C" {

peers_status peers_server_start(peers_device d, const peers_server_opts* opts, peers_server* out) {
  if (!d || !out) { set_error("null argument"); return PEERS_E_INVALID_ARG; }
  *out = nullptr;
  auto* D = reinterpret_cast<DeviceHandle*>(d);
  hipError_t e = hipSetDevice(D->ordinal);
  if (e != hipSuccess) return (peers_status)hip_fail(e, "hipSetDevice");
  std::unique_ptr<Server> S(new Server());
  S->D = D;
  if (opts) S->o = *opts;
  const int ns = std::max(1, std::min(8, S->o.streams > 0 ? S->o.streams : 2));
  S->slots.resize(ns);
  for (Slot& sl : S->slots) {
    e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
    if (e != hipSuccess) {
      for (Slot& t : S->slots) {
        if (t.ev) (void)hipEventDestroy(t.ev);
        if (t.stream) (void)hipStreamDestroy(t.stream);
      }
      return (peers_status)hip_fail(e, "server streams");
    }
  }
  Server* raw = S.get();
  raw->worker = std::thread([raw] { run(*raw); });
  *out = reinterpret_cast<peers_server>(S.release());
  return PEERS_OK;
}

peers_status peers_server_submit(peers_server s, peers_factor f, int64_t q, const int32_t* qu, const int32_t* qv,
                                 double* R_out, uint64_t* ticket) {
  if (!s || !f || q < 0 || (q > 0 && (!qu || !qv || !R_out)) || !ticket) {
    set_error("null argument");
    return PEERS_E_INVALID_ARG;
  }
  auto* S = reinterpret_cast<Server*>(s);
  auto* F = reinterpret_cast<FactorHandle*>(f);
  if (F->dev != S->D) { set_error("factor is on another device"); return PEERS_E_INVALID_ARG; }
  auto r = std::make_shared<Request>();
  r->F = F;
  r->q = q;
  r->R_out = R_out;
  r->a.resize(q);
  r->b.resize(q);
  for (int64_t k = 0; k < q; ++k) {
    if (qu[k] < 0 || qu[k] >= F->n || qv[k] < 0 || qv[k] >= F->n) {
      set_error("query " + std::to_string(k) + " has a node id outside [0, n)");
      return PEERS_E_NODE_RANGE;
    }
    r->a[k] = perm_index(*F, qu[k]);
    r->b[k] = perm_index(*F, qv[k]);
    if (qu[k] == qv[k]) r->a[k] = r->b[k];
  }
  const int64_t capq = S->o.queue_capacity > 0 ? S->o.queue_capacity : 4096;
  std::lock_guard<std::mutex> g(S->mu);
  if (S->stopping) { set_error("server is stopping"); return PEERS_E_CANCELLED; }
  if ((int64_t)S->pending.size() >= capq) {
    S->rejected++;
    set_error("request queue full");
    return PEERS_E_BUSY;
  }
  r->ticket = S->next_ticket++;
  r->t_submit = Clock::now();
  *ticket = r->ticket;
  S->submitted++;
  F->server_refs.fetch_add(1);
  S->reqs[r->ticket] = r;
  if (q == 0) {
    finish_request(*S, r.get(), PEERS_OK);
    S->cv_done.notify_all();
    return PEERS_OK;
  }
  S->pending.push_back(r);
  S->cv_req.notify_one();
  return PEERS_OK;
}

peers_status peers_server_wait(peers_server s, uint64_t ticket, int64_t timeout_us, peers_status* result) {
  if (!s) { set_error("null server"); return PEERS_E_INVALID_ARG; }
  auto* S = reinterpret_cast<Server*>(s);
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) { set_error("unknown ticket"); return PEERS_E_INVALID_ARG; }
  ReqPtr r = it->second;  // keeps the request alive for this waiter
  auto ready = [&] { return r->done; };
  if (timeout_us < 0) S->cv_done.wait(lk, ready);
  else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
    set_error("request not finished within the timeout");
    return PEERS_E_TIMEOUT;
  }
  if (result) *result = r->status;
  S->reqs.erase(ticket);  // (another waiter on the same ticket may have erased it)
  return PEERS_OK;
}

peers_status peers_server_cancel(peers_server s, uint64_t ticket) {
  if (!s) { set_error("null server"); return PEERS_E_INVALID_ARG; }
  auto* S = reinterpret_cast<Server*>(s);
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) { set_error("unknown ticket"); return PEERS_E_INVALID_ARG; }
  ReqPtr r = it->second;
  if (r->done) return PEERS_OK;
  r->cancelled = true;
  if (!r->on_device) {
    auto p = std::find(S->pending.begin(), S->pending.end(), r);
    if (p != S->pending.end()) S->pending.erase(p);
    finish_request(*S, r.get(), PEERS_E_CANCELLED);
    S->cv_done.notify_all();
  }
  // a request on the device finishes as CANCELLED when its batch completes,
  // without its results being copied out
  return PEERS_OK;
}

peers_status peers_server_stats_get(peers_server s, peers_server_stats* out) {
  if (!s || !out) { set_error("null argument"); return PEERS_E_INVALID_ARG; }
  auto* S = reinterpret_cast<Server*>(s);
  std::lock_guard<std::mutex> g(S->mu);
  *out = peers_server_stats{};
  out->submitted = S->submitted;
  out->completed = S->completed;
  out->rejected = S->rejected;
  out->batches = S->batches;
  out->p50_us = percentile(S->lat_us, 0.50);
  out->p99_us = percentile(S->lat_us, 0.99);
  out->max_us = S->lat_us.empty() ? 0.0 : *std::max_element(S->lat_us.begin(), S->lat_us.end());
  double busy = S->busy_s;
  if (S->busy_slots > 0) busy += std::chrono::duration<double>(Clock::now() - S->busy_since).count();
  out->resistances_per_s = busy > 0 ? (double)S->pairs_done / busy : 0.0;
  out->memory_waits = S->memory_waits;
  for (const Slot& sl : S->slots) out->arena_bytes += sl.arena_bytes;
  out->pending = S->pending.size();
  return PEERS_OK;
}

peers_status peers_server_stop(peers_server s) {
  if (!s) return PEERS_OK;
  auto* S = reinterpret_cast<Server*>(s);
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stopping = true;
  }
  S->cv_req.notify_all();
  if (S->worker.joinable()) S->worker.join();
  (void)hipSetDevice(S->D->ordinal);
  for (Slot& sl : S->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    free_arena(*S, sl);
    if (sl.pinned) (void)hipHostFree(sl.pinned);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  delete S;
  return PEERS_OK;
}

}  // extern "C"
