// HIP kernels of the implicit sweep (Section III-C eq 11, Section III-G eq 12).
//
//  * top_chunk_kernel: one workgroup per (top chunk, window). A chunk is up to
//    kChunk consecutive columns of one supernode. Its columns share the
//    ancestors ext = struct(L_:,b), so the window values are a dense product
//    of the ext columns' window (read from the top store) with the chunk's
//    coefficient panel, done with FP64 MFMA tiles (v_mfma_f64_16x16x4f64:
//    both operands stay in VGPRs, so neither LDS nor scalar registers carry
//    the reuse), followed by the chunk's own unit-lower triangle on VALU
//    with scalar-broadcast coefficients. The four waves split the ancestors
//    and combine in LDS in a fixed order. Launched level by level down the
//    chunk tree.
//  * bottom_kernel: one wavefront per (bottom subtree task, window). Nodes are
//    visited in descending index, a topological order of every row's
//    traversal; the values of the current root path live in an LDS stack
//    indexed by local depth; values above the subtree come from the top
//    store. Each query whose lower endpoint is the current node adds
//    sum_d (z_u[d] - z_v[d])^2 over the window (eq 12) into its own slot.
//  * finish kernels: ordered sum of each bottom query's window slots, the
//    queries whose lower endpoint is a top node (both columns are in the top
//    store), and the pairs whose resistance is exactly zero.
#include "sweep_kernels.h"

namespace peers {

namespace {

__device__ __forceinline__ double wave_sum(double s) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Wave-uniform load through the scalar unit (constant address space).
template <class T>
__device__ __forceinline__ T load_uniform(const T* p) {
  return *(const __attribute__((address_space(4))) T*)p;
}

__global__ __launch_bounds__(256) void top_chunk_kernel(SweepArgs A, int64_t task0) {
  // partial 64 x kChunk tiles of waves 1..3 in the MFMA register layout, then
  // wave 0's row-major copy of the sum (reusing the same buffer)
  __shared__ double red[3][kChunk / 16 * 4][4][kWin];
  const int64_t task = task0 + blockIdx.x;
  const int32_t c = A.task_chunk[task];
  const int32_t t = A.task_win[task];
  const TopChunk ch = A.chunks[c];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int32_t d0 = t * kWin;
  // ext depths strictly decrease along ext (all are ancestors of b), so the
  // ancestors reaching this window form a prefix of ext
  int32_t lo = 0, hi = ch.next;
  const int32_t* ed = A.ext_depth + ch.ext_begin;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (ed[mid] > d0) lo = mid + 1; else hi = mid;
  }
  const int32_t ne = lo;
  const int32_t per = ((ne + 15) >> 4) << 2;  // multiple of 4 ancestors per wave
  const int32_t e0 = min(ne, wave * per), e1 = min(ne, e0 + per);
  // G (64 rows x kChunk cols) = Z[window, ext] * Cf[ext, chunk] with
  // v_mfma_f64_16x16x4f64: A operand lane l = (row l%16, k l/16),
  // B operand lane l = (k l/16, col l%16), C lane l reg r = (row 4r + l/16, col l%16).
  constexpr int RB = kWin / 16, CB = kChunk / 16;
  f64x4 C[RB][CB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) C[rb][cb] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int kk = lane >> 4, ii = lane & 15;
  const double* __restrict__ cf = A.coef + ch.coef_begin;
  const int64_t* __restrict__ eo = A.ext_off + ch.ext_begin;
  // operands of the 4 ancestors starting at e; lanes past e1 read a valid
  // address and contribute zero
  auto load_step = [&](int32_t e, double (&a)[RB], double (&b)[CB]) {
    const int32_t ek = e + kk;
    const bool ok = ek < e1;
    const int32_t ec = ok ? ek : e1 - 1;
    const double* zc = A.store + eo[ec] + d0 + ii;
    const double* bc = cf + (int64_t)ec * kChunk + ii;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) a[rb] = zc[16 * rb];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) b[cb] = bc[16 * cb];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) a[rb] = ok ? a[rb] : 0.0;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) b[cb] = ok ? b[cb] : 0.0;
  };
  if (e0 < e1) {
    double a[RB], b[CB];
    load_step(e0, a, b);
    for (int32_t e = e0; e < e1; e += 4) {
      double an[RB], bn[CB];
      const bool more = e + 4 < e1;
      if (more) load_step(e + 4, an, bn);
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) C[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb], b[cb], C[rb][cb], 0, 0, 0);
      if (more) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) a[rb] = an[rb];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) b[cb] = bn[cb];
      }
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[wave - 1][rb * CB + cb][r][lane] = C[rb][cb][r];
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
          for (int r = 0; r < 4; ++r) C[rb][cb][r] += red[w][rb * CB + cb][r][lane];
  }
  __syncthreads();
  // wave 0 re-lays the sum out row-major (row = window depth, padded stride);
  // every wave has finished reading the partial slabs at this point
  double* rowm = &red[0][0][0][0];
  constexpr int LD = kChunk + 1;
  static_assert(kWin * LD <= 3 * (kChunk / 16 * 4) * 4 * kWin, "row-major tile must fit the reduction buffer");
  if (wave == 0) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) rowm[(16 * rb + 4 * r + kk) * LD + 16 * cb + ii] = C[rb][cb][r];
  }
  __syncthreads();
  if (wave != 0) return;
  double acc[kChunk];
#pragma unroll
  for (int j = 0; j < kChunk; ++j) acc[j] = rowm[lane * LD + j];
  // the chunk's own unit-lower triangle, highest column first (eq 11)
  const double* __restrict__ tr = A.tri + ch.tri_begin;
  const int32_t wc = ch.b - ch.a + 1;
  const int32_t d = d0 + lane;
#pragma unroll
  for (int j = kChunk - 1; j >= 0; --j) {
    if (j < wc) {
      const int32_t dep = ch.depth_b + (wc - 1 - j);  // depth of node a + j
      if (d == dep - 1) acc[j] = A.top_isd[ch.top_a + j];
#pragma unroll
      for (int jj = 0; jj < j; ++jj) acc[jj] = fma(load_uniform(tr + j * kChunk + jj), acc[j], acc[jj]);
      if (d0 < dep) A.store[A.top_off[ch.top_a + j] + d0 + lane] = acc[j];
    }
  }
}

__global__ __launch_bounds__(64) void bottom_kernel(SweepArgs A, QueryArgs Q) {
  __shared__ double ps[kBottomMaxHeight][kWin];
  const int64_t w = blockIdx.x;
  const int32_t task = A.bwork_task[w];
  const int32_t t = A.bwork_win[w];
  const int lane = threadIdx.x;
  const int32_t d0 = t * kWin;
  const int32_t d = d0 + lane;
  const int32_t p0 = A.btask_ptr[task], p1 = A.btask_ptr[task + 1];
  for (int32_t p = p0; p < p1; ++p) {
    const int32_t i = A.bnodes[p];
    double acc = 0.0;
    const int64_t e1 = A.bent_ptr[i + 1];
    for (int64_t e = A.bent_ptr[i]; e < e1; ++e) {
      const int32_t src = A.bent_src[e];
      const double cf = A.bent_coef[e];
      double v;
      if (src >= 0) {
        v = ps[src][lane];
      } else {
        const int32_t k = -(src + 1);
        v = (d0 < A.top_depth[k]) ? A.store[A.top_off[k] + d0 + lane] : 0.0;
      }
      acc = fma(cf, v, acc);
    }
    if (d == A.depth[i] - 1) acc = A.isd[i];
    ps[A.lslot[i]][lane] = acc;
    const int32_t q1 = Q.bq_ptr[i + 1];
    for (int32_t q = Q.bq_ptr[i]; q < q1; ++q) {
      if (t >= Q.bq_nwin[q]) continue;
      const int32_t hc = Q.bq_hicode[q];
      double zh = 0.0;
      if (hc >= 0) {
        zh = ps[hc][lane];
      } else if (hc != kGroundCode) {
        const int32_t k = -(hc + 1);
        zh = (d0 < A.top_depth[k]) ? A.store[A.top_off[k] + d0 + lane] : 0.0;
      }
      const double df = acc - zh;
      const double s = wave_sum(df * df);
      if (lane == 0) Q.part[Q.bq_slot[q] + t] = s;
    }
  }
}

__global__ __launch_bounds__(256) void reduce_bottom_kernel(QueryArgs Q) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Q.nbq) return;
  const int64_t s0 = Q.bq_slot[j];
  const int32_t nw = Q.bq_nwin[j];
  double s = 0.0;
  for (int32_t t = 0; t < nw; ++t) s += Q.part[s0 + t];
  Q.R[Q.bq_out[j]] = s;
}

__global__ __launch_bounds__(256) void top_query_kernel(SweepArgs A, QueryArgs Q) {
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (q >= Q.ntq) return;
  const int32_t lo = Q.tq_lo[q], hi = Q.tq_hi[q];
  const int32_t dl = A.top_depth[lo];
  const int32_t dh = hi >= 0 ? A.top_depth[hi] : 0;
  const double* zl = A.store + A.top_off[lo];
  const double* zh = hi >= 0 ? A.store + A.top_off[hi] : nullptr;
  double s = 0.0;
  for (int32_t d = lane; d < dl; d += kWin) {
    const double v = zl[d] - (d < dh ? zh[d] : 0.0);
    s = fma(v, v, s);
  }
  s = wave_sum(s);
  if (lane == 0) Q.R[Q.tq_out[q]] = s;
}

__global__ __launch_bounds__(256) void zero_kernel(QueryArgs Q) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < Q.nzero) Q.R[Q.zero_out[j]] = 0.0;
}

}  // namespace

hipError_t launch_top_level(const SweepArgs& a, int64_t task0, int64_t ntasks, hipStream_t s) {
  if (ntasks <= 0) return hipSuccess;
  hipLaunchKernelGGL(top_chunk_kernel, dim3((unsigned)ntasks), dim3(256), 0, s, a, task0);
  return hipGetLastError();
}

hipError_t launch_bottom(const SweepArgs& a, const QueryArgs& q, int64_t nwork, hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
  hipLaunchKernelGGL(bottom_kernel, dim3((unsigned)nwork), dim3(64), 0, s, a, q);
  return hipGetLastError();
}

hipError_t launch_finish(const SweepArgs& a, const QueryArgs& q, hipStream_t s) {
  if (q.nbq > 0)
    hipLaunchKernelGGL(reduce_bottom_kernel, dim3((unsigned)((q.nbq + 255) / 256)), dim3(256), 0, s, q);
  if (q.ntq > 0)
    hipLaunchKernelGGL(top_query_kernel, dim3((unsigned)((q.ntq + 3) / 4)), dim3(256), 0, s, a, q);
  if (q.nzero > 0)
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((q.nzero + 255) / 256)), dim3(256), 0, s, q);
  return hipGetLastError();
}

}  // namespace peers
