// Served form: a request loop over resident factors with continuous batching.
//
// Callers submit pair requests against resident factors from any thread. One
// worker keeps up to `streams` device batches in flight, each on its own HIP
// stream: a batch takes the pending requests (oldest first, up to a pair cap),
// merges those of the same factor into one pruned query plan, and runs the
// plans of all its factors as one grouped launch sequence (the batched form's
// steps). Requests that arrive while batches are on the device wait for the
// next free slot, so work from different requests overlaps on the device.
// Each factor is in at most one batch at a time (it has one top store and
// one workspace). Every result is the same bits as the request run alone:
// the plan computes each pair independently of the other pairs in it.
//
// Admission: factors are admitted when uploaded (their footprint against the
// device's HBM budget); a batch's plans, partial slots and staging must also
// fit the budget, else its requests fail with PEERS_E_OVER_BUDGET.
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

struct Request {
  uint64_t ticket = 0;
  FactorHandle* F = nullptr;
  std::vector<int32_t> a, b;  // reduced-permuted endpoints (-1 = ground)
  double* R_out = nullptr;
  int64_t q = 0;
  Clock::time_point t_submit;
  peers_status status = PEERS_OK;
  bool done = false;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  void* arena = nullptr;  // plans and batch layout of the batch in flight
  uint64_t arena_bytes = 0;
  double* pinned = nullptr;  // results, device -> host
  int64_t pinned_elems = 0;
  bool busy = false;
  std::vector<Request*> reqs;
  std::vector<int64_t> req_off;  // each request's first result in `pinned`
  std::vector<FactorHandle*> factors;
  std::vector<std::unique_lock<std::mutex>> locks;
  std::vector<QueryPlan> hplans;
  std::vector<DeviceQueryPlan> dplans;
  BatchLayout L;
};

}  // namespace

struct Server {
  DeviceHandle* D = nullptr;
  peers_server_opts o{};
  std::mutex mu;
  std::condition_variable cv_req, cv_done;
  std::deque<Request*> pending;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  uint64_t next_ticket = 1;
  bool stopping = false;
  std::vector<Slot> slots;
  std::set<const FactorHandle*> in_flight;
  std::thread worker;
  // statistics
  uint64_t submitted = 0, completed = 0, rejected = 0, batches = 0, pairs_done = 0;
  std::vector<double> lat_us;
  double busy_s = 0;
  Clock::time_point busy_since;
  int busy_slots = 0;
};

namespace {

// Grows a device buffer (budgeted); growth only, so steady serving allocates nothing.
Status grow_device(DeviceHandle& D, void*& buf, uint64_t& have, uint64_t need, const char* what) {
  if (need <= have) return OK;
  need = std::max<uint64_t>(need, have + have / 2);
  if (buf) {
    (void)hipFree(buf);
    D.release(have);
    buf = nullptr;
    have = 0;
  }
  Status st = D.reserve(need);
  if (st != OK) return st;
  hipError_t e = hipMalloc(&buf, need);
  if (e != hipSuccess) {
    D.release(need);
    return hip_fail(e, what);
  }
  have = need;
  return OK;
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

void finish_request(Server& S, Request* r, peers_status st) {
  r->status = st;
  r->done = true;
  const double us = std::chrono::duration<double, std::micro>(Clock::now() - r->t_submit).count();
  if (st == PEERS_OK) {
    S.completed++;
    S.pairs_done += (uint64_t)r->q;
    S.lat_us.push_back(us);
  } else {
    S.rejected++;
  }
}

// Builds and launches one batch on a free slot (worker thread, server lock
// not held). Requests whose factor could not be planned fail individually.
void launch(Server& S, Slot& sl, std::vector<Request*> take) {
  sl.reqs.clear();
  sl.req_off.clear();
  sl.factors.clear();
  sl.hplans.clear();
  sl.dplans.clear();
  // group by factor, keeping submission order inside each factor
  std::map<FactorHandle*, std::vector<Request*>> groups;
  std::vector<FactorHandle*> forder;
  for (Request* r : take) {
    if (!groups.count(r->F)) forder.push_back(r->F);
    groups[r->F].push_back(r);
  }
  std::vector<std::pair<Request*, peers_status>> failed;
  std::vector<FactorHandle*> planned;
  int64_t total = 0;
  // host plans of the factors, in parallel (independent per factor)
  const size_t nf = forder.size();
  std::vector<QueryPlan> plans(nf);
  std::vector<Status> pst(nf, OK);
  auto plan_one = [&](size_t i) {
    FactorHandle* F = forder[i];
    const std::vector<Request*>& G = groups[F];
    int64_t q = 0;
    for (Request* r : G) q += r->q;
    std::vector<int32_t> a, b;
    a.reserve(q);
    b.reserve(q);
    for (Request* r : G) {
      a.insert(a.end(), r->a.begin(), r->a.end());
      b.insert(b.end(), r->b.begin(), r->b.end());
    }
    pst[i] = build_query_plan_handle(*F, q, a.data(), b.data(), plans[i]);
  };
  {
    std::vector<std::thread> th;
    for (size_t i = 1; i < nf; ++i) th.emplace_back(plan_one, i);
    if (nf) plan_one(0);
    for (auto& t : th) t.join();
  }
  for (size_t i = 0; i < nf; ++i) {
    FactorHandle* F = forder[i];
    std::vector<Request*>& G = groups[F];
    Status st = pst[i];
    if (st == OK) st = ensure_workspace(*F, plans[i].nslots, plans[i].q, plans[i].stage_elems);
    if (st != OK) {
      for (Request* r : G) failed.push_back({r, (peers_status)st});
      continue;
    }
    sl.hplans.push_back(std::move(plans[i]));
    planned.push_back(F);
    for (Request* r : G) {
      sl.reqs.push_back(r);
      sl.req_off.push_back(total);
      total += r->q;
    }
  }
  // device image: plans, then the batch layout
  std::vector<uint64_t> poff;
  uint64_t bytes = 0;
  for (const QueryPlan& Q : sl.hplans) {
    poff.push_back(bytes);
    bytes += (query_plan_bytes(Q) + 255) / 256 * 256;
  }
  sl.dplans.resize(sl.hplans.size());
  Status st = OK;
  if (!planned.empty()) {
    // the layout needs the plans' device addresses: size it with a first pass
    std::vector<BatchEntry> be;
    for (size_t i = 0; i < planned.size(); ++i) be.push_back(BatchEntry{planned[i], &sl.dplans[i], nullptr});
    for (size_t i = 0; i < planned.size(); ++i) {
      // host-side plan fields (counts, work lists) are what the layout reads
      DeviceQueryPlan& d = sl.dplans[i];
      d.work_task = sl.hplans[i].work_task;
      d.work_win = sl.hplans[i].work_win;
      d.args.nbq = sl.hplans[i].nbq();
      d.args.ntq = (int64_t)sl.hplans[i].tq_out.size();
      d.args.nzero = (int64_t)sl.hplans[i].zero_out.size();
      d.args.ngp = (int64_t)sl.hplans[i].gp.size();
    }
    BatchLayout probe;
    batch_layout(*S.D, be, probe);
    const uint64_t need = bytes + probe.bytes;
    st = grow_device(*S.D, sl.arena, sl.arena_bytes, need, "hipMalloc(server arena)");
    if (st == OK) st = grow_pinned(sl, std::max<int64_t>(total, 1));
    for (size_t i = 0; i < planned.size() && st == OK; ++i)
      st = upload_query_plan_to(sl.hplans[i], sl.dplans[i], (char*)sl.arena + poff[i], sl.stream);
    if (st == OK) {
      for (size_t i = 0; i < planned.size(); ++i) be[i].R_dev = (double*)planned[i]->res;
      batch_layout(*S.D, be, sl.L);
      st = batch_upload(sl.L, (char*)sl.arena + bytes, sl.stream);
    }
    if (st == OK) st = batch_launch(sl.L, (char*)sl.arena + bytes, sl.stream);
    // results of each factor, in request order, into the pinned buffer
    int64_t off = 0;
    for (size_t i = 0; i < planned.size() && st == OK; ++i) {
      const int64_t q = sl.hplans[i].q;
      if (q > 0) {
        hipError_t e = hipMemcpyAsync(sl.pinned + off, planned[i]->res, (size_t)q * 8, hipMemcpyDeviceToHost,
                                      sl.stream);
        if (e != hipSuccess) st = hip_fail(e, "hipMemcpyAsync(server results)");
      }
      off += q;
    }
    if (st == OK) {
      hipError_t e = hipEventRecord(sl.ev, sl.stream);
      if (e != hipSuccess) st = hip_fail(e, "hipEventRecord(server)");
    }
  }
  std::lock_guard<std::mutex> g(S.mu);
  for (auto& fr : failed) finish_request(S, fr.first, fr.second);
  if (st != OK) {
    (void)hipStreamSynchronize(sl.stream);
    for (Request* r : sl.reqs) finish_request(S, r, (peers_status)st);
    sl.reqs.clear();
  }
  if (sl.reqs.empty()) {
    // nothing in flight on this slot: release its factors now
    for (FactorHandle* F : forder) S.in_flight.erase(F);
    sl.locks.clear();
    S.cv_done.notify_all();
    return;
  }
  sl.factors = forder;
  sl.busy = true;
  if (S.busy_slots++ == 0) S.busy_since = Clock::now();
  S.batches++;
  if (!failed.empty()) S.cv_done.notify_all();
}

// Hands a finished batch's results to its requests (server lock held).
void complete(Server& S, Slot& sl, hipError_t e) {
  for (size_t i = 0; i < sl.reqs.size(); ++i) {
    Request* r = sl.reqs[i];
    if (e == hipSuccess && r->q > 0) std::memcpy(r->R_out, sl.pinned + sl.req_off[i], (size_t)r->q * 8);
    finish_request(S, r, e == hipSuccess ? PEERS_OK : PEERS_E_HIP);
  }
  sl.reqs.clear();
  for (FactorHandle* F : sl.factors) S.in_flight.erase(F);
  sl.factors.clear();
  sl.locks.clear();
  sl.busy = false;
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
    if (free_slot && !S.pending.empty()) {
      // while another batch keeps the device busy, let a small batch wait a
      // little for batch-mates
      int64_t pend = 0;
      for (Request* r : S.pending) pend += r->q;
      const bool young = Clock::now() - S.pending.front()->t_submit < max_wait;
      if (!(S.busy_slots > 0 && pend < cap && young)) {
        std::vector<Request*> take;
        std::deque<Request*> keep;
        std::set<FactorHandle*> claimed;
        std::vector<std::unique_lock<std::mutex>> locks;
        int64_t pairs = 0;
        while (!S.pending.empty()) {
          Request* r = S.pending.front();
          S.pending.pop_front();
          bool ok = pairs == 0 || pairs + r->q <= cap;
          if (ok && !claimed.count(r->F)) {
            if (S.in_flight.count(r->F)) ok = false;
            else {
              std::unique_lock<std::mutex> fl(r->F->mu, std::try_to_lock);
              if (fl.owns_lock()) {
                locks.push_back(std::move(fl));
                claimed.insert(r->F);
              } else {
                ok = false;
              }
            }
          }
          if (ok) {
            take.push_back(r);
            pairs += r->q;
          } else {
            keep.push_back(r);
          }
        }
        S.pending.swap(keep);
        if (!take.empty()) {
          for (FactorHandle* F : claimed) S.in_flight.insert(F);
          free_slot->locks = std::move(locks);
          lk.unlock();
          launch(S, *free_slot, std::move(take));
          lk.lock();
          progressed = true;
        }
      }
    }
    if (S.stopping && S.pending.empty() && S.busy_slots == 0) break;
    if (!progressed) {
      if (S.busy_slots > 0 || !S.pending.empty()) S.cv_req.wait_for(lk, std::chrono::microseconds(50));
      else S.cv_req.wait(lk, [&] { return S.stopping || !S.pending.empty(); });
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
  std::unique_ptr<Request> r(new Request());
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
  if (q == 0) {
    finish_request(*S, r.get(), PEERS_OK);
    S->reqs[r->ticket] = std::move(r);
    S->cv_done.notify_all();
    return PEERS_OK;
  }
  S->pending.push_back(r.get());
  S->reqs[r->ticket] = std::move(r);
  S->cv_req.notify_one();
  return PEERS_OK;
}

peers_status peers_server_wait(peers_server s, uint64_t ticket, int64_t timeout_us, peers_status* result) {
  if (!s) { set_error("null server"); return PEERS_E_INVALID_ARG; }
  auto* S = reinterpret_cast<Server*>(s);
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) { set_error("unknown ticket"); return PEERS_E_INVALID_ARG; }
  Request* r = it->second.get();
  auto ready = [&] { return r->done; };
  if (timeout_us < 0) S->cv_done.wait(lk, ready);
  else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
    set_error("request not finished within the timeout");
    return PEERS_E_TIMEOUT;
  }
  if (result) *result = r->status;
  S->reqs.erase(it);
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
    if (sl.arena) {
      (void)hipFree(sl.arena);
      S->D->release(sl.arena_bytes);
    }
    if (sl.pinned) (void)hipHostFree(sl.pinned);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  delete S;
  return PEERS_OK;
}

}  // extern "C"
