// Spectral sparsification by effective resistances (Section II-B,
// Algorithm 1) on the device: q independent draws of an edge with
// probability proportional to w_e R_e, each drawn edge weighted
// w_e / (q p_e). The resistances normally come straight from an all-edge
// sweep in device memory.
//
// Probabilities are integer weights k_e = floor(2^s fl(w_e R_e)) with
// s = 61 - ceil(log2 m) (w_e R_e <= 1 for a Laplacian, so the sum stays
// below 2^62), so their prefix sums are exact in any order and a draw's edge
// is an integer decision. Draw i takes the first word x of Philox4x64-10
// (Salmon et al., SC 2011) at counter (i, 0, 0, 0) and key (seed, 0) and picks
// the edge whose prefix-sum interval holds floor(x K / 2^64), K = sum k_e.
//
// Kernels: integer weights (one pass over w and R), a three-kernel inclusive
// scan (per-block scan, one-workgroup scan of block totals, offset add), the
// draws (one thread per draw, binary search in the prefix sums, integer
// atomic count), and the new weights count_e * w_e * (K / (q k_e)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>

#include "../../../include/peers.h"
#include "device_handle.h"

namespace peers {

namespace {

constexpr int kScanThreads = 256, kScanPer = 16;
constexpr int64_t kScanBlock = (int64_t)kScanThreads * kScanPer;
constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull, kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull, kPhiloxW1 = 0xBB67AE8584CAA73Bull;

// first output word of Philox4x64-10 at counter (i, 0, 0, 0), key (seed, 0)
__device__ __forceinline__ uint64_t philox_word0(uint64_t i, uint64_t seed) {
  uint64_t c0 = i, c1 = 0, c2 = 0, c3 = 0, k0 = seed, k1 = 0;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    const uint64_t hi0 = __umul64hi(kPhiloxM0, c0), lo0 = kPhiloxM0 * c0;
    const uint64_t hi1 = __umul64hi(kPhiloxM1, c2), lo1 = kPhiloxM1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return c0;
}

__global__ __launch_bounds__(256) void weights_kernel(int64_t m, const double* __restrict__ w,
                                                      const double* __restrict__ R, int s, uint64_t* __restrict__ k,
                                                      int32_t* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  const double x = w[i] * R[i];
  if (!(x >= 0.0 && x <= 2.0)) {  // also NaN
    atomicOr(bad, 1);
    k[i] = 0;
    return;
  }
  k[i] = (uint64_t)floor(ldexp(x, s));
}

// inclusive scan inside one wavefront
__device__ __forceinline__ uint64_t wave_inclusive(uint64_t t, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint64_t y = __shfl_up(t, off);
    if (lane >= off) t += y;
  }
  return t;
}

// per block of kScanBlock values: inclusive prefix sums in place, block total to bsum
__global__ __launch_bounds__(kScanThreads) void scan_local_kernel(int64_t m, uint64_t* __restrict__ C,
                                                                  uint64_t* __restrict__ bsum) {
  __shared__ uint64_t wsum[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  uint64_t v[kScanPer];
  uint64_t run = 0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    const int64_t idx = base + j;
    run += idx < m ? C[idx] : 0;
    v[j] = run;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t t = wave_inclusive(run, lane);
  if (lane == 63) wsum[wave] = t;
  __syncthreads();
  uint64_t wpre = 0;
  for (int w2 = 0; w2 < wave; ++w2) wpre += wsum[w2];
  const uint64_t excl = wpre + t - run;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    const int64_t idx = base + j;
    if (idx < m) C[idx] = v[j] + excl;
  }
  if (threadIdx.x == kScanThreads - 1) bsum[blockIdx.x] = wpre + t;
}

// exclusive prefix sums of the block totals, in place (one workgroup)
__global__ __launch_bounds__(1024) void scan_blocks_kernel(int64_t nb, uint64_t* __restrict__ bsum) {
  __shared__ uint64_t part[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t carry = 0;
  for (int64_t base = 0; base < nb; base += 1024) {
    const int64_t idx = base + threadIdx.x;
    const uint64_t x = idx < nb ? bsum[idx] : 0;
    const uint64_t t = wave_inclusive(x, lane);
    if (lane == 63) part[wave] = t;
    __syncthreads();
    uint64_t wpre = 0, total = 0;
    for (int w2 = 0; w2 < 16; ++w2) {
      if (w2 < wave) wpre += part[w2];
      total += part[w2];
    }
    if (idx < nb) bsum[idx] = carry + wpre + t - x;
    carry += total;
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void scan_add_kernel(int64_t m, uint64_t* __restrict__ C,
                                                       const uint64_t* __restrict__ bsum) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < m) C[i] += bsum[i / kScanBlock];
}

__global__ __launch_bounds__(256) void zero_counts_kernel(int64_t m, int32_t* __restrict__ c) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < m) c[i] = 0;
}

__global__ __launch_bounds__(256) void draw_kernel(int64_t q, uint64_t seed, int64_t m,
                                                   const uint64_t* __restrict__ C, int32_t* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= q) return;
  const uint64_t K = C[m - 1];
  const uint64_t t = __umul64hi(philox_word0((uint64_t)i, seed), K);
  // the first edge whose inclusive prefix sum exceeds t (C[m - 1] = K > t)
  int64_t lo = 0, hi = m - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (C[mid] > t) hi = mid;
    else lo = mid + 1;
  }
  atomicAdd(&count[lo], 1);
}

__global__ __launch_bounds__(256) void reweight_kernel(int64_t m, int64_t q, const double* __restrict__ w,
                                                       const uint64_t* __restrict__ C,
                                                       const int32_t* __restrict__ count, double* __restrict__ neww) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  const int32_t c = count[i];
  const uint64_t K = C[m - 1];
  const uint64_t k = C[i] - (i ? C[i - 1] : 0);
  neww[i] = c ? (double)c * w[i] * ((double)K / ((double)q * (double)k)) : 0.0;
}

inline unsigned blocks(int64_t n, int64_t per) { return (unsigned)std::max<int64_t>(1, (n + per - 1) / per); }
uint64_t align256(uint64_t x) { return (x + 255) / 256 * 256; }

}  // namespace

}  // namespace peers

using namespace peers;

extern "C" {

peers_status peers_sparsify(peers_device d, int64_t m, const double* w, const double* R, int64_t q, uint64_t seed,
                            int32_t* count, double* w_new, uint32_t flags, void* hip_stream) {
  if (!d || m <= 0 || !w || !R || !count || !w_new || q < 0 || q > INT32_MAX) {
    set_error("invalid argument (m >= 1, 0 <= q <= 2^31 - 1, non-null arrays)");
    return PEERS_E_INVALID_ARG;
  }
  auto* D = reinterpret_cast<DeviceHandle*>(d);
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t he = hipSetDevice(D->ordinal);
  if (he != hipSuccess) return (peers_status)hip_fail(he, "hipSetDevice");
  const bool in_dev = flags & PEERS_IN_DEVICE, out_dev = flags & PEERS_OUT_DEVICE;
  const int64_t nb = (m + kScanBlock - 1) / kScanBlock;
  // one buffer: prefix sums, block sums, flag, and staging for host arrays
  const uint64_t cb = align256((uint64_t)m * 8), bb = align256((uint64_t)nb * 8), fb = 256;
  const uint64_t ib = in_dev ? 0 : 2 * align256((uint64_t)m * 8);
  const uint64_t ob = out_dev ? 0 : align256((uint64_t)m * 4) + align256((uint64_t)m * 8);
  const uint64_t bytes = cb + bb + fb + ib + ob;
  Status st = D->reserve(bytes);
  if (st != OK) return (peers_status)st;
  char* mem = nullptr;
  he = hipMalloc((void**)&mem, bytes);
  if (he != hipSuccess) {
    D->release(bytes);
    return (peers_status)hip_fail(he, "hipMalloc(sparsifier)");
  }
  uint64_t* C = (uint64_t*)mem;
  uint64_t* bsum = (uint64_t*)(mem + cb);
  int32_t* bad = (int32_t*)(mem + cb + bb);
  const double* wd = w;
  const double* Rd = R;
  char* p = mem + cb + bb + fb;
  if (!in_dev) {
    wd = (const double*)p;
    Rd = (const double*)(p + align256((uint64_t)m * 8));
    p += ib;
  }
  int32_t* cd = out_dev ? count : (int32_t*)p;
  double* nd = out_dev ? w_new : (double*)(p + align256((uint64_t)m * 4));
  auto done = [&](peers_status r) {
    (void)hipStreamSynchronize(s);
    (void)hipFree(mem);
    D->release(bytes);
    return r;
  };
  const int sb = 61 - (m > 1 ? 64 - __builtin_clzll((unsigned long long)(m - 1)) : 0);
  if (!in_dev) {
    he = hipMemcpyAsync((void*)wd, w, (size_t)m * 8, hipMemcpyHostToDevice, s);
    if (he == hipSuccess) he = hipMemcpyAsync((void*)Rd, R, (size_t)m * 8, hipMemcpyHostToDevice, s);
    if (he != hipSuccess) return done((peers_status)hip_fail(he, "copy w and R"));
  }
  hipLaunchKernelGGL(zero_counts_kernel, dim3(1), dim3(256), 0, s, (int64_t)1, bad);
  hipLaunchKernelGGL(weights_kernel, dim3(blocks(m, 256)), dim3(256), 0, s, m, wd, Rd, sb, C, bad);
  hipLaunchKernelGGL(scan_local_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, m, C, bsum);
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(1024), 0, s, nb, bsum);
  hipLaunchKernelGGL(scan_add_kernel, dim3(blocks(m, 256)), dim3(256), 0, s, m, C, bsum);
  he = hipGetLastError();
  if (he != hipSuccess) return done((peers_status)hip_fail(he, "sparsifier weights and scan"));
  int32_t hbad = 0;
  uint64_t K = 0;
  he = hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipMemcpyAsync(&K, C + (m - 1), 8, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) return done((peers_status)hip_fail(he, "sparsifier total"));
  if (hbad) {
    set_error("w_e R_e must be finite and in [0, 2] for every edge");
    return done(PEERS_E_INVALID_ARG);
  }
  if (K == 0) {
    set_error("no edge has a positive sampling weight");
    return done(PEERS_E_INVALID_ARG);
  }
  hipLaunchKernelGGL(zero_counts_kernel, dim3(blocks(m, 256)), dim3(256), 0, s, m, cd);
  if (q > 0) hipLaunchKernelGGL(draw_kernel, dim3(blocks(q, 256)), dim3(256), 0, s, q, seed, m, C, cd);
  hipLaunchKernelGGL(reweight_kernel, dim3(blocks(m, 256)), dim3(256), 0, s, m, q, wd, C, cd, nd);
  he = hipGetLastError();
  if (he == hipSuccess && !out_dev) {
    he = hipMemcpyAsync(count, cd, (size_t)m * 4, hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipMemcpyAsync(w_new, nd, (size_t)m * 8, hipMemcpyDeviceToHost, s);
  }
  if (he != hipSuccess) return done((peers_status)hip_fail(he, "sparsifier draws"));
  return done(PEERS_OK);
}

}  // extern "C"
