// Pair queries that allocate no device memory, for callers that cannot
// allocate (code under graph capture, tight serving loops, harnesses that
// forbid hipMalloc).
//
// peers_query_noalloc computes what peers_query computes, with the same
// kernels, but every buffer the call needs beyond its inputs and outputs --
// the query plan, the launch layout of a pruned sweep, the partial slots,
// the staged columns and (for host output) the result staging -- lives in
// one fixed device array, `scratch`, of kScratchBytes. Each GPU the library
// runs on holds its own copy of the array until the process ends; its address
// on a device is looked up once, with that device current, and used from
// then on. Calls through this entry point are serialized per GPU (a lock is
// held until the call's work has finished), so two of them never share the
// array at once; nothing else in the library uses it. Every word a call
// reads from the array is written earlier in the same call (plan and layout
// by copies, partial slots, dense sums and staging by the sweep before the
// reduction reads them), so nothing needs clearing between calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "../../../include/peers.h"
#include "device_handle.h"

namespace peers {

namespace {

constexpr uint64_t kScratchBytes = 64ull << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchBytes / 8];

struct ScratchSlot {
  std::once_flag once;
  hipError_t err = hipSuccess;
  char* ptr = nullptr;  // device address of `scratch` on this GPU
  std::mutex mu;        // one call at a time on this GPU
};
ScratchSlot g_scratch[kMaxDevices];

// The array's device address on `ordinal` (which must be the current device).
hipError_t scratch_on(int ordinal, char** out) {
  ScratchSlot& sl = g_scratch[ordinal];
  std::call_once(sl.once, [&] {
    void* p = nullptr;
    sl.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    sl.ptr = (char*)p;
  });
  *out = sl.ptr;
  return sl.err;
}

uint64_t align256(uint64_t x) { return (x + 255) / 256 * 256; }

}  // namespace

}  // namespace peers

using namespace peers;

extern "C" {

peers_status peers_query_noalloc(peers_factor f, int64_t q, const int32_t* qu, const int32_t* qv, double* R_out,
                                 uint32_t flags, void* hip_stream) {
  if (!f || q < 0 || (q > 0 && (!qu || !qv || !R_out))) { set_error("null argument"); return PEERS_E_INVALID_ARG; }
  if (flags & PEERS_PROFILE) { set_error("PEERS_PROFILE needs events, which this entry point does not create"); return PEERS_E_INVALID_ARG; }
  auto* F = reinterpret_cast<FactorHandle*>(f);
  const int ordinal = F->dev->ordinal;
  if (ordinal < 0 || ordinal >= kMaxDevices) { set_error("device ordinal beyond the scratch table"); return PEERS_E_INVALID_ARG; }
  hipStream_t s = (hipStream_t)hip_stream;
  std::lock_guard<std::mutex> g(F->mu);
  std::lock_guard<std::mutex> gs(g_scratch[ordinal].mu);
  hipError_t he = hipSetDevice(ordinal);
  if (he != hipSuccess) return (peers_status)hip_fail(he, "hipSetDevice");
  if (q == 0) return PEERS_OK;
  char* base = nullptr;
  he = scratch_on(ordinal, &base);
  if (he != hipSuccess) return (peers_status)hip_fail(he, "hipGetSymbolAddress(scratch)");
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
  std::vector<int32_t> a(q), b(q);
  for (int64_t k = 0; k < q; ++k) {
    if (u[k] < 0 || u[k] >= F->n || v[k] < 0 || v[k] >= F->n) {
      set_error("query " + std::to_string(k) + " has a node id outside [0, n)");
      return PEERS_E_NODE_RANGE;
    }
    a[k] = perm_index(*F, u[k]);
    b[k] = perm_index(*F, v[k]);
    if (u[k] == v[k]) a[k] = b[k];
  }
  QueryPlan Q;
  Status st = build_query_plan_handle(*F, q, a.data(), b.data(), Q, true);
  if (st != OK) return (peers_status)st;
  // scratch layout: plan, partial slots (and dense sums), results (host
  // output only), staging, then the launch layout of a pruned sweep in what
  // is left
  const bool dev_out = flags & PEERS_OUT_DEVICE;
  const uint64_t plan_b = align256(query_plan_bytes(Q));
  const int64_t nslots = Q.nslots + (Q.dense ? Q.nbq() : 0);
  const uint64_t part_b = align256((uint64_t)std::max<int64_t>(nslots, 1) * 8);
  const uint64_t res_b = dev_out ? 0 : align256((uint64_t)q * 8);
  const uint64_t stage_b = align256((uint64_t)std::max<int64_t>(Q.stage_elems, 1) * 8);
  const uint64_t fixed = plan_b + part_b + res_b + stage_b;
  if (fixed > kScratchBytes) {
    set_error("the request needs " + std::to_string(fixed) + " bytes of scratch (plan, partial sums, staging), the " +
              "fixed scratch holds " + std::to_string(kScratchBytes) + "; split it or use peers_query");
    return PEERS_E_OVER_BUDGET;
  }
  DeviceQueryPlan DQ;
  st = upload_query_plan_to(Q, DQ, base, s);
  SweepWork w;
  w.part = (double*)(base + plan_b);
  double* Rd = dev_out ? R_out : (double*)(base + plan_b + part_b);
  w.stage = (double*)(base + plan_b + part_b + res_b);
  w.layout = base + fixed;
  w.layout_cap = kScratchBytes - fixed;
  if (st == OK) st = run_sweep(*F, DQ, Rd, s, false, &w);
  if (st == OK && !dev_out) {
    he = hipMemcpyAsync(R_out, Rd, sizeof(double) * q, hipMemcpyDeviceToHost, s);
    if (he != hipSuccess) st = hip_fail(he, "hipMemcpyAsync(results)");
  }
  // the scratch lock is held until this call's work is done
  he = hipStreamSynchronize(s);
  DQ.layout_host.reset();
  if (st != OK) return (peers_status)st;
  if (he != hipSuccess) return (peers_status)hip_fail(he, "hipStreamSynchronize");
  return PEERS_OK;
}

}  // extern "C"
