// HIP kernels of the implicit sweep (Section III-C eq 11, Section III-G eq 12).
//
//  * top tree (chains of separator nodes, see host/plan.h): FP64 MFMA GEMMs
//    (v_mfma_f64_16x16x4f64, operands straight from global memory into
//    registers) driven by task lists. At upload, gemm_kernel forms L_CC^{-1}
//    of every chain by recursive 2x2 blocking on top of inv_base_kernel's
//    64 x 64 diagonal inverses, and the transfer blocks B_C. Every sweep,
//    chain_rows_kernel writes the chain rows D^{-1/2} L_CC^{-1} of every top
//    column; then gemm_level_kernel, one launch per chain level, forms
//    Z[rows above C, C] = Z[rows above C, U_C] B_C with the ancestor columns
//    gathered from the top store (64 x 32 tiles for wide chains, one-wave
//    64 x 16 tiles for narrow ones).
//  * dense rows above bottom subtrees (host/plan.h, kDenseMaxK): at upload,
//    bxfer_kernel forms B_S of every bottom subtree; every sweep,
//    dense_kernel sums the rows above each subtree for its queries as
//    ||Z[rows, U_S] w||^2 on the matrix cores, and the bottom sweep starts
//    past those rows where every query of a task has such a sum.
//  * bottom_kernel: one wavefront per (bottom subtree task, group of two
//    windows). Nodes are visited in descending index, a topological order of
//    every row's traversal; the values of the current root path live in a
//    register stack per window indexed by local depth; values above the
//    subtree come from the top store, requested two nodes ahead. Per-node
//    records come through the scalar unit. Each query whose lower endpoint is
//    the current node sums (z_u[d] - z_v[d])^2 over the windows (eq 12); the
//    per-lane sums go through a per-wave LDS block and are summed over the
//    lanes 16 queries at a time into window-group slots.
//  * finish kernels: ordered sum of each bottom query's window-group slots,
//    the queries whose lower endpoint is a top node (both columns are in the
//    top store), non-ancestor pairs, and the pairs whose resistance is exactly
//    zero.
#include "sweep_kernels.h"
#include "wave_ops.h"

namespace peers {

namespace {

// Wave-uniform load through the scalar unit (constant address space).
template <class T>
__device__ __forceinline__ T load_uniform(const T* p) {
  return *(const __attribute__((address_space(4))) T*)p;
}

// A wave-uniform record of whole 8-byte words through the scalar unit.
template <class T>
__device__ __forceinline__ T load_struct(const T* p) {
  static_assert(sizeof(T) % 8 == 0, "records are whole 8-byte words");
  uint64_t w[sizeof(T) / 8];
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 8); ++i) w[i] = load_uniform((const uint64_t*)p + i);
  T r;
  __builtin_memcpy(&r, w, sizeof(T));
  return r;
}

__device__ __forceinline__ BNode load_uniform(const BNode* p) {
  BNode r;
  r.isd = load_uniform(&p->isd);
#pragma unroll
  for (int e = 0; e < 3; ++e) r.lc[e] = load_uniform(&p->lc[e]);
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    r.tref[e] = load_uniform(&p->tref[e]);
    r.tc[e] = load_uniform(&p->tc[e]);
  }
  r.slots = load_uniform(&p->slots);
  r.depth = load_uniform(&p->depth);
  r.ent = load_uniform(&p->ent);
  r.n_more = load_uniform(&p->n_more);
  return r;
}

__device__ __forceinline__ BEnt load_uniform(const BEnt* p) {
  BEnt r;
  r.ref = load_uniform(&p->ref);
  r.coef = load_uniform(&p->coef);
  return r;
}

__device__ __forceinline__ BQuery load_uniform(const BQuery* p) {
  BQuery r;
  r.hiref = load_uniform(&p->hiref);
  r.out = load_uniform(&p->out);
  r.nwin = load_uniform(&p->nwin);
  return r;
}

// s_waitcnt vmcnt(0) (expcnt and lgkmcnt left at their maxima). Placed right
// after a load taken on a rare branch, so that the branch's merge point does
// not have to drain the loads that are prefetched for the next node.
__device__ __forceinline__ void wait_vector_loads() { __builtin_amdgcn_s_waitcnt(0x0F70); }

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Reduction loop of gemm_kernel for indices [e0, e1) in steps of 4 (one
// v_mfma_f64_16x16x4f64 k-group). Every load is unconditional: indices past
// e1 are clamped to a valid column and their B value is zeroed at use, so
// each load is waited for only right before its MFMAs. Gathered column
// offsets come through the scalar unit one step ahead. Operands are kept
// DEPTH - 1 steps ahead: the 64 x 32 tiles use two buffers, which keeps them
// within 128 registers (four waves per SIMD, with 32 KB of LDS per
// workgroup), measured faster than three buffers at three waves; the
// one-wave narrow tiles use three.
template <bool GATHER, bool BT, int NB = 2, int DEPTH = 2>
__device__ __forceinline__ void gemm_accumulate(f64x4 (&C)[4][NB], const double* __restrict__ A,
                                                const double* __restrict__ B, const int64_t* __restrict__ gt,
                                                const GemmProb& pb, const int32_t (&rows)[4], const int32_t (&cols)[NB],
                                                int kk, int32_t e0, int32_t e1) {
  // four separate scalars (an array here would be indexed per lane and
  // placed in scratch memory)
  struct Cols { int64_t g0, g1, g2, g3; };
  auto gathers = [&](int32_t e) -> Cols {
    Cols c{0, 0, 0, 0};
    if (GATHER) {
      c.g0 = load_uniform(gt + min(e, e1 - 1));
      c.g1 = load_uniform(gt + min(e + 1, e1 - 1));
      c.g2 = load_uniform(gt + min(e + 2, e1 - 1));
      c.g3 = load_uniform(gt + min(e + 3, e1 - 1));
    }
    return c;
  };
  auto load = [&](int32_t e, const Cols& gc, double (&a)[4], double (&b)[NB]) {
    const int32_t ec = min(e + kk, e1 - 1);
    int64_t acol;
    if (GATHER) {
      const int64_t lo = (kk & 1) ? gc.g1 : gc.g0;
      const int64_t hi = (kk & 1) ? gc.g3 : gc.g2;
      acol = (kk & 2) ? hi : lo;
    } else {
      acol = pb.a_off + (int64_t)ec * pb.lda;
    }
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) a[rb] = A[acol + rows[rb]];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) b[cb] = BT ? B[(int64_t)ec * pb.ldb + cols[cb]] : B[(int64_t)cols[cb] * pb.ldb + ec];
  };
  auto mma = [&](int32_t e, const double (&a)[4], const double (&b)[NB]) {
    const bool ok = e + kk < e1;
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const double bv = ok ? b[cb] : 0.0;
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) C[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb], bv, C[rb][cb], 0, 0, 0);
    }
  };
  // DEPTH operand buffers: step i's operands are requested DEPTH - 1 steps
  // before its MFMAs (steps wholly past e1 are skipped)
  double a[DEPTH][4], b[DEPTH][NB];
#pragma unroll
  for (int i = 0; i < DEPTH - 1; ++i) load(e0 + 4 * i, gathers(e0 + 4 * i), a[i], b[i]);
  Cols gn = gathers(e0 + 4 * (DEPTH - 1));
  for (int32_t e = e0; e < e1; e += 4 * DEPTH) {
#pragma unroll
    for (int i = 0; i < DEPTH; ++i) {
      const int nb = (i + DEPTH - 1) % DEPTH;
      load(e + 4 * (i + DEPTH - 1), gn, a[nb], b[nb]);
      gn = gathers(e + 4 * (i + DEPTH));
      if (i == 0 || e + 4 * i < e1) mma(e + 4 * i, a[i], b[i]);
    }
  }
}

// C[M x N] = alpha * A[M x K] * B[K x N] for one 64 x 32 output tile over the
// reduction range [k0, k1) of its task (a problem's last tile with at most 16
// columns left runs as 64 x 16). v_mfma_f64_16x16x4f64 operands:
// A lane l = (row l%16, k l/16), B lane l = (k l/16, col l%16), C lane l reg
// r = (row 4r + l/16, col l%16). The four waves take consecutive quarters of
// the reduction range (multiples of 4) and are summed in LDS in a fixed
// order, (C0 + C2) + (C1 + C3), so the result does not depend on scheduling.
typedef double GemmRed[2][8][4][kWin];

// Gp points at the argument block in kernel-argument or global memory; its
// buffer table is read with uniform loads at the problem's (uniform) index.
__device__ __forceinline__ void gemm_body(const GemmArgs* Gp, int64_t task, GemmRed& red) {
  const GemmTask* tasks = load_uniform(&Gp->tasks);
  const GemmProb* probs = load_uniform(&Gp->probs);
  const GemmTask tk = tasks[task];
  const GemmProb pb = probs[tk.prob];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int kk = lane >> 4, ii = lane & 15;
  const double* __restrict__ A = load_uniform(&Gp->buf[pb.a_buf]);
  const double* __restrict__ B = load_uniform(&Gp->buf[pb.b_buf]) + pb.b_off;
  const int32_t nk = tk.k1 - tk.k0;
  const int32_t per = ((nk + 15) >> 4) << 2;
  const int32_t e0 = tk.k0 + min(nk, wave * per);
  const int32_t e1 = tk.k0 + min(nk, wave * per + per);
  int32_t rows[4], cols[2];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) rows[rb] = min(tk.row0 + 16 * rb + ii, pb.M - 1);
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) cols[cb] = min(tk.col0 + 16 * cb + ii, pb.N - 1);
  const int64_t* __restrict__ gt = load_uniform(&Gp->gather) + (pb.gather ? pb.aoff_begin : 0);
  // operands of the 4 reduction indices starting at e. Every load is
  // unconditional: indices past e1 are clamped to a valid column and their B
  // value is zeroed at use, so the loop body has no branches and each load is
  // waited for only right before its MFMAs.
  f64x4 C[4][2];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) C[rb][cb] = f64x4{0.0, 0.0, 0.0, 0.0};
  if (e0 < e1) {
    if (tk.col0 + 16 >= pb.N) {
      // at most 16 columns left in the tile: the 64 x 16 form (the same
      // products and order for those columns, half the matrix instructions)
      f64x4 C1[4][1];
      const int32_t cols1[1] = {cols[0]};
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) C1[rb][0] = f64x4{0.0, 0.0, 0.0, 0.0};
      if (pb.gather) {
        if (pb.trans & 1) gemm_accumulate<true, true, 1>(C1, A, B, gt, pb, rows, cols1, kk, e0, e1);
        else gemm_accumulate<true, false, 1>(C1, A, B, gt, pb, rows, cols1, kk, e0, e1);
      } else {
        if (pb.trans & 1) gemm_accumulate<false, true, 1>(C1, A, B, gt, pb, rows, cols1, kk, e0, e1);
        else gemm_accumulate<false, false, 1>(C1, A, B, gt, pb, rows, cols1, kk, e0, e1);
      }
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) C[rb][0] = C1[rb][0];
    } else if (pb.gather) {
      if (pb.trans & 1) gemm_accumulate<true, true>(C, A, B, gt, pb, rows, cols, kk, e0, e1);
      else gemm_accumulate<true, false>(C, A, B, gt, pb, rows, cols, kk, e0, e1);
    } else {
      if (pb.trans & 1) gemm_accumulate<false, true>(C, A, B, gt, pb, rows, cols, kk, e0, e1);
      else gemm_accumulate<false, false>(C, A, B, gt, pb, rows, cols, kk, e0, e1);
    }
  }
  // (C0 + C2) + (C1 + C3), in two rounds through a two-wave buffer
  if (wave >= 2) {
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[wave - 2][rb * 2 + cb][r][lane] = C[rb][cb][r];
  }
  __syncthreads();
  if (wave < 2) {
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) C[rb][cb][r] += red[wave][rb * 2 + cb][r][lane];
  }
  __syncthreads();
  if (wave == 1) {
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[0][rb * 2 + cb][r][lane] = C[rb][cb][r];
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) C[rb][cb][r] += red[0][rb * 2 + cb][r][lane];
  }
  __syncthreads();
  constexpr int LD = kTileN + 1;
  double* tile = &red[0][0][0][0];
  if (wave == 0) {
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) tile[(16 * rb + 4 * r + kk) * LD + 16 * cb + ii] = C[rb][cb][r];
  }
  __syncthreads();
  double* __restrict__ Cm = load_uniform(&Gp->buf[pb.c_buf]) + pb.c_off;
  if (pb.trans & 2) {
    for (int idx = threadIdx.x; idx < kTileM * kTileN; idx += 256) {
      const int c = idx & (kTileN - 1), r = idx / kTileN;
      const int32_t gr = tk.row0 + r, gc = tk.col0 + c;
      if (gr < pb.M && gc < pb.N) Cm[(int64_t)gr * pb.ldc + gc] = pb.alpha * tile[r * LD + c];
    }
  } else {
    for (int idx = threadIdx.x; idx < kTileM * kTileN; idx += 256) {
      const int r = idx & (kTileM - 1), c = idx / kTileM;
      const int32_t gr = tk.row0 + r, gc = tk.col0 + c;
      if (gr < pb.M && gc < pb.N) Cm[(int64_t)gc * pb.ldc + gr] = pb.alpha * tile[r * LD + c];
    }
  }
}

// Workgroups go to the device's XCDs round-robin (block b to XCD b % kXcds),
// and each XCD has its own L2. The tile tasks of a problem are listed row
// tile by row tile, so neighbouring tasks share operand slabs: runs of kXcdRun
// consecutive tasks are given to one XCD (the grid is padded to whole rounds
// of runs; padding blocks exit at once).
constexpr int64_t kXcds = 8, kXcdRun = 32;
__device__ __forceinline__ int64_t xcd_task(int64_t b) {
  const int64_t x = b % kXcds, slot = b / kXcds;
  return (slot / kXcdRun) * (kXcds * kXcdRun) + x * kXcdRun + slot % kXcdRun;
}
__host__ __device__ inline int64_t xcd_grid(int64_t n) { return (n + kXcds * kXcdRun - 1) / (kXcds * kXcdRun) * (kXcds * kXcdRun); }

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void gemm_kernel(GemmArgs G, int64_t task0, int64_t ntasks) {
  __shared__ GemmRed red;
  const int64_t t = xcd_task(blockIdx.x);
  if (t >= ntasks) return;
  gemm_body(&G, task0 + t, red);
}

// Narrow chains (width at most 16): one 64 x 16 output tile over the task's
// whole reduction range, computed by one wavefront with no K split, no LDS
// and no barrier (four independent tasks per workgroup). Same operand layout
// and summation order within the wavefront as gemm_accumulate.
__device__ __forceinline__ void gemm_narrow_body(const GemmArgs* Gp, int64_t task) {
  const GemmTask* tasks = load_uniform(&Gp->ntasks);
  const GemmProb* probs = load_uniform(&Gp->probs);
  const GemmTask tk = tasks[task];
  const GemmProb pb = probs[tk.prob];
  const int lane = threadIdx.x & 63;
  const int kk = lane >> 4, ii = lane & 15;
  const double* __restrict__ A = load_uniform(&Gp->buf[pb.a_buf]);
  const double* __restrict__ B = load_uniform(&Gp->buf[pb.b_buf]) + pb.b_off;
  int32_t rows[4], cols[1];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) rows[rb] = min(tk.row0 + 16 * rb + ii, pb.M - 1);
  cols[0] = min(tk.col0 + ii, pb.N - 1);
  const int64_t* __restrict__ gt = load_uniform(&Gp->gather) + pb.aoff_begin;
  f64x4 C[4][1];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) C[rb][0] = f64x4{0.0, 0.0, 0.0, 0.0};
  if (tk.k0 < tk.k1) gemm_accumulate<true, true, 1, 3>(C, A, B, gt, pb, rows, cols, kk, tk.k0, tk.k1);
  double* __restrict__ Cm = load_uniform(&Gp->buf[pb.c_buf]) + pb.c_off;
  const int32_t gc = tk.col0 + ii;
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int32_t gr = tk.row0 + 16 * rb + 4 * r + kk;
      if (gr < pb.M && gc < pb.N) Cm[(int64_t)gc * pb.ldc + gr] = pb.alpha * C[rb][0][r];
    }
}

// One chain level: the 64 x 32 tiles of its wide chains (first, in XCD runs)
// and the 64 x 16 one-wave tiles of its narrow chains (after them) in one
// launch, so the narrow tiles fill the device as the wide ones drain.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void gemm_level_kernel(
    GemmArgs G, int64_t task0, int64_t ntasks, int64_t ntask0, int64_t nntasks) {
  __shared__ GemmRed red;
  const int64_t nwide = xcd_grid(ntasks);
  if ((int64_t)blockIdx.x < nwide) {
    const int64_t t = xcd_task(blockIdx.x);
    if (t < ntasks) gemm_body(&G, task0 + t, red);
  } else {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t i = ((int64_t)blockIdx.x - nwide) * 4 + wave;
    if (i < nntasks) gemm_narrow_body(&G, ntask0 + i);
  }
}

// Inverse of one diagonal block (at most 64 x 64) of a chain's unit-lower
// L_CC by forward substitution: lane j holds column j of the inverse.
typedef double BaseTile[kBase][kBase + 1];

__device__ __forceinline__ void inv_base_body(const SweepArgs& A, int64_t blk, BaseTile& Ls, BaseTile& Xs) {
  const BaseBlock bb = A.base_blocks[blk];
  const Chain c = A.chains[bb.chain];
  const int lane = threadIdx.x;
  const int n = bb.size, lo = bb.lo;
  const double* Lb = A.lcc + c.lcc_off + (int64_t)lo * c.ldl + lo;
  for (int j = 0; j < n; ++j) Ls[lane][j] = lane < n ? Lb[(int64_t)j * c.ldl + lane] : 0.0;
  __syncthreads();
  for (int i = 0; i < n; ++i) {
    double s = i == lane ? 1.0 : 0.0;
    for (int k = 0; k < i; ++k) s = fma(-Ls[i][k], Xs[k][lane], s);
    Xs[i][lane] = i >= lane ? s : 0.0;
  }
  __syncthreads();
  double* Xb = A.X + c.x_off + (int64_t)lo * c.ldl + lo;
  for (int j = 0; j < n; ++j)
    if (lane < n) Xb[(int64_t)j * c.ldl + lane] = Xs[lane][j];
}

__global__ __launch_bounds__(64) void inv_base_kernel(SweepArgs A) {
  __shared__ BaseTile Ls, Xs;
  inv_base_body(A, blockIdx.x, Ls, Xs);
}

// Rows of a top column that lie inside its own chain (Z[C, C] = D^{-1/2} L_CC^{-1})
// and the zero padding below the column's depth. One workgroup per top column.
// (threads tid, tid + nthr, ... of the caller write top node k's rows)
__device__ __forceinline__ void chain_rows_body(const SweepArgs& A, int64_t k, int tid, int nthr) {
  // the node's chain record and position through the scalar unit (k is
  // wave-uniform)
  const Chain c = load_struct(A.chains + load_uniform(A.top_chain + k));
  const int32_t j = load_uniform(A.top_node + k) - c.a;
  const int64_t nrow = c.ld - c.dp;
  double* col = A.store + c.store_base + (int64_t)j * c.ld + c.dp;
  const double* xc = A.X + c.x_off + (int64_t)j * c.ldl;
  for (int64_t r = tid; r < nrow; r += nthr) {
    double v = 0.0;
    if (r < c.w - j) v = A.isd[c.b - r] * xc[c.w - 1 - r];
    col[r] = v;
  }
}

__global__ __launch_bounds__(256) void chain_rows_kernel(SweepArgs A) { chain_rows_body(A, blockIdx.x, threadIdx.x, 256); }

// One wavefront sweeps kWinPerWave consecutive windows of one subtree task:
// lane l holds depth t*64 + l of window t for each of them. The per-node
// records, address arithmetic and query reductions are shared by the windows.
// Per-wave LDS blocks of the bottom sweep's query sums (32 KB per workgroup).
// Rows are not padded: the transposed reads of a flush conflict in the LDS
// banks, which measured slightly cheaper than padded rows.
constexpr int kQBlock = 16, kQRowPad = kWin;
typedef double BottomLds[kBottomWaves][kQBlock][kQRowPad];

template <bool WIDE>
__device__ __forceinline__ void bottom_body(const SweepArgs& A, const QueryArgs& Q, int64_t w, BottomLds& lds) {
  constexpr int NW = kWinPerWave;
  // the waves of a workgroup sweep the same subtree for consecutive windows
  // and share its records through the scalar cache
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int32_t task = load_uniform(Q.work_task + w);
  const int32_t t0 = load_uniform(Q.work_win + w) + wave * NW;
  const int32_t p0 = load_uniform(A.btask_ptr + task), p1 = load_uniform(A.btask_ptr + task + 1);
  if (t0 >= load_uniform(A.btask_nwin + task)) return;
  const int lane = threadIdx.x & 63;
  // Values of a top column at this lane's depths in windows t0 .. t0+NW-1.
  // Store columns are zero-padded to whole groups of NW windows and t0 is a
  // multiple of NW, so one bound check covers the group; groups past the
  // column read the store's leading zero block, so the loads are unconditional.
  // byte offsets in the store fit 32 bits unless WIDE
  const char* __restrict__ zsb = (const char*)A.store;
  const uint32_t lane_off = (uint32_t)lane * 8u;
  auto top_values = [&](int64_t ref, double (&x)[NW]) {
    const int32_t wb = (int32_t)ref, nw = (int32_t)(ref >> 32);
    const int32_t wi = t0 < nw ? wb + t0 : 0;
    const double* __restrict__ pz;
    if (WIDE) pz = (const double*)(zsb + (size_t)wi * (kWin * 8) + lane_off);
    else pz = (const double*)(zsb + (size_t)((uint32_t)wi * (uint32_t)(kWin * 8) + lane_off));
#pragma unroll
    for (int v = 0; v < NW; ++v) x[v] = pz[v * kWin];
  };
  // values of the current root path inside the subtree, by local depth
  // (register-resident; every slot index is wave-uniform)
  // one array per window: each stays small enough to live in registers
  // (arrays of windows past NW are never touched and compile away)
  static_assert(NW >= 1 && NW <= 4, "one to four windows per wavefront");
  double ps0[kBottomMaxHeight], ps1[kBottomMaxHeight], ps2[kBottomMaxHeight], ps3[kBottomMaxHeight];
#pragma unroll
  for (int k = 0; k < kBottomMaxHeight; ++k) ps0[k] = ps1[k] = ps2[k] = ps3[k] = 0.0;
  // slot index of a slot code (codes are even, which lets the register
  // offset be taken from the code as it is)
  auto slot_of = [](int32_t code) -> int32_t {
    __builtin_assume((code & 1) == 0);
    return code >> 1;
  };
  // the slot code in bits [at, at + kSlotBits) of x: one s_bfe_u32 (written
  // out, since the compiler would otherwise rewrite the extraction into a
  // shift and a mask)
  auto code_at = [](int32_t x, auto at) -> int32_t {
    int32_t r;
    asm("s_bfe_u32 %0, %1, %2" : "=s"(r) : "s"(x), "i"(decltype(at)::value | (kSlotBits << 16)));
    return r;
  };
  auto ps_get = [&](int v, int32_t k) -> double {
    return v == 0 ? ps0[k] : (v == 1 ? ps1[k] : (v == 2 ? ps2[k] : ps3[k]));
  };
  auto ps_set = [&](int v, int32_t k, double x) {
    if (v == 0) ps0[k] = x;
    else if (v == 1) ps1[k] = x;
    else if (v == 2) ps2[k] = x;
    else ps3[k] = x;
  };
  // query records by byte offset (the record table is below 4 GB, which the
  // planner checks, so offsets are carried in 32 bits)
  const char* __restrict__ bqb = (const char*)Q.bq;
  constexpr uint32_t kBQ = sizeof(BQuery);
  auto bq_at = [&](uint32_t off) -> const BQuery* { return (const BQuery*)(bqb + off); };
  const int32_t t0d = t0 * kWin;  // first depth of the wave's windows
  const int32_t grp = t0 / NW;
  const int32_t jend = load_uniform(Q.bq_ptr + p1);
  int32_t jb = load_uniform(Q.bq_ptr + p0);
  // Per-lane values of the task's entries are summed over the lanes in
  // blocks of kQBlock entries through LDS: entry jb + c's 64 values go to row
  // c of the wave's block; at the end of a block lane l adds up
  // the 16 values of row l/4 starting at 16 (l % 4), in a fixed tree, and
  // two butterflies inside each group of four lanes complete the row sums,
  // which are stored into the window-major partial slots.
  double (&qrow)[kQBlock][kQRowPad] = lds[wave];
  auto flush = [&](int32_t count) {
    const int e = lane >> 2, part = lane & 3;
    const double* __restrict__ src = &qrow[e][16 * part];
    double t4[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) t4[i] = (src[4 * i] + src[4 * i + 1]) + (src[4 * i + 2] + src[4 * i + 3]);
    double t = (t4[0] + t4[1]) + (t4[2] + t4[3]);
    t += dpp<0xB1>(t);
    t += dpp<0x4E>(t);
    if (part == 0 && e < count) Q.part[(int64_t)grp * Q.nbq + jb + e] = t;
  };

  // Software pipeline over the subtree's nodes: while node p is computed,
  // the store values of nodes p+1 and p+2, the record of node p+1 and the
  // store references of node p+3 are in flight.
  // records and bucket bounds of the task's nodes, addressed by 32-bit byte
  // offsets from the task's first node (a task has at most kBottomMaxNodes)
  const char* __restrict__ recb = (const char*)(A.bnode + p0);
  const char* __restrict__ bqpb = (const char*)(Q.bq_ptr + p0);
  uint32_t ro = 0, bo = 0;  // offsets of the current node's record and bounds
  auto rec_at = [&](int k) -> const BNode* { return (const BNode*)(recb + ro) + k; };
  auto bqp_at = [&](int k) -> const int32_t* { return (const int32_t*)(bqpb + bo) + k; };
  const BNode* rec = rec_at(0);
  const int32_t* bqp = bqp_at(0);
  BNode cur = load_uniform(rec);
  int64_t r0 = load_uniform(&rec[2].tref[0]), r1 = load_uniform(&rec[2].tref[1]);
  int32_t qa = load_uniform(bqp), qb = load_uniform(bqp + 1);
  uint32_t qao = (uint32_t)qa * kBQ;
  int64_t qh = load_uniform(&bq_at(qao)->hiref);
  int32_t qk = load_uniform(&bq_at(qao)->kind);
  double va[2][NW], vb[2][NW], vc[2][NW];
  top_values(cur.tref[0], va[0]);
  top_values(cur.tref[1], va[1]);
  top_values(load_uniform(&rec[1].tref[0]), vb[0]);
  top_values(load_uniform(&rec[1].tref[1]), vb[1]);
#pragma unroll
  for (int v = 0; v < NW; ++v) vc[0][v] = vc[1][v] = 0.0;
  auto step = [&](const double (&u)[2][NW], double (&nn)[2][NW]) {
    top_values(r0, nn[0]);
    top_values(r1, nn[1]);
    const BNode nfull = load_uniform(rec_at(1));
    const int64_t s0 = load_uniform(&rec_at(3)->tref[0]), s1 = load_uniform(&rec_at(3)->tref[1]);
    // bucket of this node is [q0, q1) (read two nodes ahead); request the end
    // of the bucket two nodes on and the next node's first entry (one padding
    // entry each at the end)
    const int32_t q0 = qa, q1 = qb;
    const uint32_t q0o = qao, q1o = (uint32_t)q1 * kBQ;
    const int32_t nqc = load_uniform(bqp_at(2));
    const int64_t nqh = load_uniform(&bq_at(q1o)->hiref);
    const int32_t nqk = load_uniform(&bq_at(q1o)->kind);
    // eq 11: entries on the path stack, then entries in the top store (the
    // windows' values of one slot are read together: one index setup each)
    const int32_t sl = cur.slots;
    double acc[NW], pa[NW], pb[NW];
#pragma unroll
    for (int v = 0; v < NW; ++v) pa[v] = ps_get(v, slot_of(sl & kSlotMask));
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int v = 0; v < NW; ++v) pb[v] = ps_get(v, slot_of(code_at(sl, std::integral_constant<int, kSlotBits>())));
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int v = 0; v < NW; ++v) acc[v] = fma(cur.lc[1], pb[v], cur.lc[0] * pa[v]);
    if (((sl >> kInlineCountShift) & 3) == 3) {  // a third inline entry (about one node in ten)
#pragma unroll
      for (int v = 0; v < NW; ++v) pa[v] = ps_get(v, slot_of(code_at(sl, std::integral_constant<int, 2 * kSlotBits>())));
#pragma unroll
      for (int v = 0; v < NW; ++v) acc[v] = fma(cur.lc[2], pa[v], acc[v]);
    }
    const int32_t n_lds_more = cur.n_more & 0xffff, n_top_more = cur.n_more >> 16;
    for (int32_t e = 0; e < n_lds_more; ++e) {
      const BEnt be = load_uniform(A.bent + cur.ent + e);
#pragma unroll
      for (int v = 0; v < NW; ++v) acc[v] = fma(be.coef, ps_get(v, slot_of((int32_t)be.ref & kSlotMask)), acc[v]);
    }
    double at[NW];
#pragma unroll
    for (int v = 0; v < NW; ++v) at[v] = fma(cur.tc[1], u[1][v], cur.tc[0] * u[0][v]);
    for (int32_t e = 0; e < n_top_more; ++e) {
      const BEnt be = load_uniform(A.bent + cur.ent + n_lds_more + e);
      double x[NW];
      top_values(be.ref, x);
      wait_vector_loads();
#pragma unroll
      for (int v = 0; v < NW; ++v) at[v] = fma(be.coef, x[v], at[v]);
    }
    const int32_t top_slot = slot_of(code_at(sl, std::integral_constant<int, kOwnSlotShift>()));
#pragma unroll
    for (int v = 0; v < NW; ++v) acc[v] += at[v];
    // the diagonal entry D^{-1/2} sits at depth - 1, in one window group of
    // the column only: the other waves skip the lane test
    const uint32_t dl = (uint32_t)(cur.depth - 1 - t0d);
    if (dl < (uint32_t)(NW * kWin)) {
      __builtin_amdgcn_sched_barrier(0);  // keeps this a branch (not selects)
#pragma unroll
      for (int v = 0; v < NW; ++v)
        if (v * kWin + lane == (int)dl) acc[v] = cur.isd;
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int v = 0; v < NW; ++v) ps_set(v, top_slot, acc[v]);
    __builtin_amdgcn_sched_barrier(0);
    // eq 12 over these windows for the queries whose lower endpoint is this node
    // (the wave's windows hold some of the node's depths iff t0d < depth;
    // both conditions as one sign test, which stays a single scalar branch)
    if (((q1 - q0 - 1) | (cur.depth - 1 - t0d)) >= 0) {
      // the node's first entry was read during the previous node; the rest
      // are read one ahead of use
      int64_t h = qh;
      int32_t kind = qk;
      uint32_t qo = q0o;
      int32_t jl = q0 - jb;  // row of entry j in the LDS block
      int32_t j = q0;
      do {
        // path-stack value first (nine entries in ten on the all-edge
        // workloads; any slot is in range for the other kinds)
        double zh[NW];
#pragma unroll
        for (int v = 0; v < NW; ++v) zh[v] = ps_get(v, slot_of((int32_t)h & kSlotMask));
        // next entry (the table ends with a padding entry), requested only
        // after this entry's fields are in use: scalar loads are waited for
        // all together, so the request must not precede that wait
        __builtin_amdgcn_sched_barrier(0);
        const int64_t h_next = load_uniform(&bq_at(qo + kBQ)->hiref);
        const int32_t kind_next = load_uniform(&bq_at(qo + kBQ)->kind);
        // (a bit test rather than a comparison keeps this one branch: the
        // compiler would otherwise fold it into a search tree over the kinds)
        static_assert(kQSlot == 0 && kQStage < 8, "query kinds");
        if ((kind & 7) != 0) {
          if (kind == kQInl0) {
#pragma unroll
            for (int v = 0; v < NW; ++v) zh[v] = u[0][v];
          } else if (kind == kQInl1) {
#pragma unroll
            for (int v = 0; v < NW; ++v) zh[v] = u[1][v];
          } else if (kind == kQStore) {
            top_values(h, zh);
            wait_vector_loads();
          } else {
            // ground (zero column), or a staging entry: this node's column is
            // one side of a non-ancestor pair (its sum below is never read);
            // staged columns span whole window groups, so every window of the
            // group is written (zeros past the node's depth)
            // (the windows below the entry's first one are the dense form's)
            if (kind == kQStage && t0 >= (int32_t)load_uniform(&bq_at(qo)->out)) {
#pragma unroll
              for (int v = 0; v < NW; ++v) Q.stage[h + (int64_t)(t0 + v) * kWin + lane] = acc[v];
            }
#pragma unroll
            for (int v = 0; v < NW; ++v) zh[v] = 0.0;
          }
        }
        // windows past the node's depth hold zeros on both sides
        double sacc = 0.0;
#pragma unroll
        for (int v = 0; v < NW; ++v) {
          const double df = acc[v] - zh[v];
          sacc = fma(df, df, sacc);
        }
        while (jl >= kQBlock) {
          flush(kQBlock);
          jb += kQBlock;
          jl -= kQBlock;
        }
        qrow[jl][lane] = sacc;
        h = h_next;
        kind = kind_next;
        qo += kBQ;
        ++jl;
      } while (++j < q1);
    }
    qh = nqh;
    qk = nqk;
    qa = q1;
    qao = q1o;
    qb = nqc;
    ro += (uint32_t)sizeof(BNode);
    bo += (uint32_t)sizeof(int32_t);
    cur = nfull;
    r0 = s0;
    r1 = s1;
  };
  // (every path back to the loop head has consumed all three buffers, so no
  // load is waited for there)
  for (int32_t p = p0;; p += 3) {
    step(va, vc);
    if (p + 1 >= p1) break;
    step(vb, va);
    if (p + 2 >= p1) break;
    step(vc, vb);
    if (p + 3 >= p1) break;
  }
  while (jend - jb > kQBlock) {
    flush(kQBlock);
    jb += kQBlock;
  }
  flush(jend - jb);
}

template <bool WIDE>
__global__ __launch_bounds__(64 * kBottomWaves) void bottom_kernel(SweepArgs A, QueryArgs Q) {
  __shared__ BottomLds lds;
  bottom_body<WIDE>(A, Q, blockIdx.x, lds);
}

__device__ __forceinline__ void reduce_body(const QueryArgs& Q, int64_t blk) {
  const int64_t j = blk * 256 + threadIdx.x;
  if (j >= Q.nbq) return;
  const BQuery bq = Q.bq[j];
  if (bq.kind == kQStage) return;
  // the dense sum of the rows above the subtree first (when the plan has
  // one for this query), then the sweep's window groups in order
  const int32_t g0 = Q.bq_g0 ? Q.bq_g0[j] : 0;
  double s = g0 > 0 ? Q.part[Q.dpart_off + j] : 0.0;
  const int32_t ng = (bq.nwin + kWinPerWave - 1) / kWinPerWave;
  for (int32_t g = g0; g < ng; ++g) s += Q.part[(int64_t)g * Q.nbq + j];
  Q.R[bq.out] = s;
}

__global__ __launch_bounds__(256) void reduce_bottom_kernel(QueryArgs Q) { reduce_body(Q, blockIdx.x); }

// B_S of one bottom subtree (one wavefront, lane e = column e of U_S): eq 11
// inside the subtree with the columns of U_S as unit vectors, nodes in
// processing order (every node after its ancestors), the columns of the
// current root path kept per local depth in LDS. Top-store entries of a
// record name their column by its store offset, which identifies its lane.
typedef double XferStack[kBottomMaxHeight][kWin];
__device__ __forceinline__ void bxfer_body(const SweepArgs& A, int32_t sub, XferStack& st) {
  const int lane = threadIdx.x & 63;
  const int32_t K = load_uniform(A.sub_K + sub);
  if (K == 0 || K > kDenseMaxK) return;
  const int64_t mine = lane < K ? A.sub_uoff[load_uniform(A.sub_ubeg + sub) + lane] : -1;
  const int32_t p0 = load_uniform(A.sub_p0 + sub), p1 = load_uniform(A.sub_p1 + sub);
  double* __restrict__ Bs = A.B + load_uniform(A.sub_bbase + sub);
  auto slot = [](int32_t code) { return (code & kSlotMask) >> 1; };
  for (int32_t p = p0; p < p1; ++p) {
    const BNode b = load_uniform(A.bnode + p);
    const int32_t sl = b.slots;
    const int32_t ninl = (sl >> kInlineCountShift) & 3;
    double acc = 0.0;
    if (ninl > 0) acc = fma(b.lc[0], st[slot(sl)][lane], acc);
    if (ninl > 1) acc = fma(b.lc[1], st[slot(sl >> kSlotBits)][lane], acc);
    if (ninl > 2) acc = fma(b.lc[2], st[slot(sl >> (2 * kSlotBits))][lane], acc);
    const int32_t nl = b.n_more & 0xffff, nt = (int32_t)((uint32_t)b.n_more >> 16);
    for (int32_t e = 0; e < nl; ++e) {
      const BEnt be = load_uniform(A.bent + b.ent + e);
      acc = fma(be.coef, st[slot((int32_t)be.ref)][lane], acc);
    }
    // a store reference's low word is its column's first window
    auto top = [&](int64_t ref, double c) {
      if ((int64_t)(uint32_t)ref * kWin == mine) acc += c;
    };
    top(b.tref[0], b.tc[0]);
    top(b.tref[1], b.tc[1]);
    for (int32_t e = 0; e < nt; ++e) {
      const BEnt be = load_uniform(A.bent + b.ent + nl + e);
      top(be.ref, be.coef);
    }
    st[slot(sl >> kOwnSlotShift)][lane] = acc;
    if (lane < K) Bs[(int64_t)(p - p0) * K + lane] = acc;
  }
}

__global__ __launch_bounds__(64 * kBottomWaves) void bxfer_kernel(SweepArgs A) {
  __shared__ XferStack st[kBottomWaves];
  const int wave = threadIdx.x >> 6;
  const int32_t sub = blockIdx.x * kBottomWaves + wave;
  if (sub < A.nsub) bxfer_body(A, sub, st[wave]);
}

// One dense item (one workgroup): rows [0, rows) of Z[rows, U_S] W for up
// to G column tiles of 16 queries, on v_mfma_f64_16x16x4f64 (A lane l: row
// l%16 of a 16-row tile, column 4s + l/16 of U_S; B lane l: element
// (4s + l/16, l%16) of a column tile of W; C lane l: four rows of query
// l%16). W is formed in LDS from B_S: column c of tile g is B_S e_u -
// B_S e_v (v in S), B_S e_u - e_k (v the k-th column of U_S) or B_S e_u
// (the ground), zero past the queries and past |U_S|. Each wave takes every
// fourth step of RT row tiles; a loaded row block serves all column tiles.
// Products are squared and added per lane; the four lanes of a query, then
// the four waves, are summed in a fixed order. Columns of U_S are ordered by
// depth, descending, so k-group s is needed only for rows above the depth
// of its first column; inside a group, rows at or past a column's depth read
// the store's leading zero block.
// Calls f(std::integral_constant<int, n>) for a run-time n in [1, KS).
template <int KS, class F>
__device__ __forceinline__ void dense_dispatch(int32_t n, F&& f) {
  if constexpr (KS > 1) {
    if (n == KS - 1) f(std::integral_constant<int, KS - 1>());
    else dense_dispatch<KS - 1>(n, f);
  }
}

template <int GRP>
struct DenseLds {
  double w[1 << (GRP % kDenseTileKinds)][dense_steps(GRP / kDenseTileKinds)][kWin];
  double red[kBottomWaves][1 << (GRP % kDenseTileKinds)][kDenseTile];
};

// GRP = class * kDenseTileKinds + log2(column tiles). STAGE: the item's
// columns are staged bottom columns (one tile): each product is written to
// the staging buffer at the rows it covers instead of squared.
template <int GRP, bool STAGE>
__device__ __forceinline__ void dense_body(const SweepArgs& A, const QueryArgs& Q, int64_t it, DenseLds<GRP>& L) {
  constexpr int CLS = GRP / kDenseTileKinds;
  constexpr int KS = dense_steps(CLS), G = 1 << (GRP % kDenseTileKinds), RT = dense_rt(CLS);
  static_assert(!STAGE || G == 1, "staging items hold one column tile");
  const int tid = threadIdx.x, lane = tid & 63, kq = lane >> 4, r = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const DItem d = load_struct(Q.ditems + it);
  const int32_t K = load_uniform(A.sub_K + d.sub), ub = load_uniform(A.sub_ubeg + d.sub);
  for (int e = tid; e < G * KS * kWin; e += 64 * kBottomWaves) {
    const int g = e / (KS * kWin), s = (e / kWin) % KS, l = e % kWin;
    const int32_t k = 4 * s + (l >> 4), qi = g * kDenseTile + (l & 15);
    double v = 0.0;
    if (qi < d.nq && k < K) {
      const int64_t j = Q.dq_list[d.q0 + qi];
      const int64_t bu = Q.bq_bu[j], bv = Q.bq_bv[j];
      v = A.B[bu + k];
      if (bv >= 0) v -= A.B[bv + k];
      else if (bv != kDenseNoV && k == (int32_t)(-1 - bv)) v -= 1.0;
    }
    L.w[g][s][l] = v;
  }
  __syncthreads();
  const double* __restrict__ z = A.store;
  int32_t uo[KS], ud[KS], sd[KS];  // (the planner keeps store offsets of dense plans below 2^31)
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int32_t k = 4 * s + kq;
    uo[s] = k < K ? (int32_t)A.sub_uoff[ub + k] : 0;
    ud[s] = k < K ? A.sub_udep[ub + k] : 0;
    sd[s] = 4 * s < K ? load_uniform(A.sub_udep + ub + 4 * s) : 0;
  }
  double sq[G];
#pragma unroll
  for (int g = 0; g < G; ++g) sq[g] = 0.0;
  // staging: this lane's column (its query's staging offset), -1 past the queries
  int64_t sbase = -1;
  if (STAGE && r < d.nq) sbase = Q.bq[Q.dq_list[d.q0 + r]].hiref;
  // row blocks of this wave, the next one's loads in flight during each
  constexpr int32_t kStep = kBottomWaves * 16 * RT;
  auto load = [&](int32_t d0, double (&a)[KS][RT]) {
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int i = 0; i < RT; ++i) {
        const int32_t row = d0 + 16 * i + r;
        // unconditional, also past the last block (a load on a branch would
        // make the join wait for it); rows past the item read zeros
        a[s][i] = z[sd[s] > d0 && row < ud[s] && row < d.rows ? uo[s] + row : r];
      }
  };
  // the k-groups needed for rows from d0 on (a prefix), as a constant per
  // case so that every product of a block is straight-line code
  auto nsteps = [&](int32_t d0) {
    int32_t n = 0;
#pragma unroll
    for (int s = 0; s < KS; ++s) n += sd[s] > d0 ? 1 : 0;
    return n;
  };
  auto block_n = [&](auto NS, int32_t d0, const double (&a)[KS][RT]) {
    constexpr int N = decltype(NS)::value;
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma unroll
      for (int i = 0; i < RT; ++i) {
        f64x4 c = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < N; ++s) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s][i], L.w[g][s][lane], c, 0, 0, 0);
        if constexpr (STAGE) {
          // C lane l, element e: row 4e + l/16 of the tile, column l%16
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int32_t row = d0 + 16 * i + 4 * e + kq;
            if (sbase >= 0 && row < d.rows) Q.stage[sbase + row] = c[e];
          }
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) sq[g] = fma(c[e], c[e], sq[g]);
        }
      }
      // one column tile's products at a time (their accumulators stay few)
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  auto block = [&](int32_t d0, const double (&a)[KS][RT]) {
    const int32_t n = nsteps(d0);
    if (KS == 1 || n == KS) block_n(std::integral_constant<int, KS>(), d0, a);
    else dense_dispatch<KS>(n, [&](auto NS) { block_n(NS, d0, a); });
  };
  double a0[KS][RT], a1[KS][RT];
  int32_t d0 = wave * 16 * RT;
  load(d0, a0);
  while (d0 < d.rows) {
    load(d0 + kStep, a1);
    block(d0, a0);
    d0 += kStep;
    if (d0 >= d.rows) break;
    load(d0 + kStep, a0);
    block(d0, a1);
    d0 += kStep;
  }
  if constexpr (STAGE) return;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    sq[g] += __shfl_xor(sq[g], 16);
    sq[g] += __shfl_xor(sq[g], 32);
    if (lane < kDenseTile) L.red[wave][g][lane] = sq[g];
  }
  __syncthreads();
  for (int t = tid; t < d.nq; t += 64 * kBottomWaves) {
    const int g = t / kDenseTile, c = t % kDenseTile;
    Q.part[Q.dpart_off + Q.dq_list[d.q0 + t]] = (L.red[0][g][c] + L.red[1][g][c]) + (L.red[2][g][c] + L.red[3][g][c]);
  }
}

template <int GRP, bool STAGE>
__global__ __launch_bounds__(64 * kBottomWaves) __attribute__((amdgpu_waves_per_eu(4))) void dense_kernel(
    SweepArgs A, QueryArgs Q, int64_t i0) {
  __shared__ DenseLds<GRP> L;
  dense_body<GRP, STAGE>(A, Q, i0 + blockIdx.x, L);
}

// Calls f(std::integral_constant<int, GRP>, std::bool_constant<STAGE>) for a
// run-time group x in [X, kDenseAllGroups) (staging group kDenseGroups + c
// runs the one-tile form of class c).
template <int X, class F>
void dense_group(int x, F&& f) {
  if constexpr (X < kDenseGroups) {
    // (groups with more tiles than their class takes hold no items)
    if constexpr ((1 << (X % kDenseTileKinds)) <= dense_tiles(X / kDenseTileKinds))
      if (x == X) return f(std::integral_constant<int, X>(), std::false_type());
    dense_group<X + 1>(x, f);
  } else if constexpr (X < kDenseAllGroups) {
    if (x == X) return f(std::integral_constant<int, (X - kDenseGroups) * kDenseTileKinds>(), std::true_type());
    dense_group<X + 1>(x, f);
  }
}

// Pairs whose endpoints are not ancestor-related (eq 12 over the union of the
// two root paths): rows above the lowest common ancestor are shared, so
//   R = sum_{d < dl} (z_a[d] - z_b[d])^2 + sum_{d >= dl} z_a[d]^2 + sum_{d >= dl} z_b[d]^2.
// One wavefront per pair, lanes over depths, fixed order.
__device__ __forceinline__ void general_pair_body(const SweepArgs& A, const QueryArgs& Q, int64_t blk) {
  const int64_t p = blk * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (p >= Q.ngp) return;
  const GPair g = Q.gp[p];
  const double* za = (g.a_stage ? Q.stage : A.store) + g.a_off;
  const double* zb = (g.b_stage ? Q.stage : A.store) + g.b_off;
  const int32_t dm = max(g.da, g.db);
  double s = 0.0;
  for (int32_t d = lane; d < dm; d += kWin) {
    const double va = d < g.da ? za[d] : 0.0;
    const double vb = d < g.db ? zb[d] : 0.0;
    if (d < g.dl) {
      const double t = va - vb;
      s = fma(t, t, s);
    } else {
      s = fma(va, va, s);
      s = fma(vb, vb, s);
    }
  }
  s = wave_sum(s);
  if (lane == 0) Q.R[g.out] = s;
}

__global__ __launch_bounds__(256) void general_pair_kernel(SweepArgs A, QueryArgs Q) {
  general_pair_body(A, Q, blockIdx.x);
}

// eq 12 for a pair whose lower endpoint lo is a top node and whose partner
// hi is an ancestor of it or the ground: R = sum_{d < depth(lo)} (z_lo[d] -
// z_hi[d])^2 with z_hi[d] = 0 past depth(hi), both columns read from the top
// store. Every sweep writes each top column over whole windows (zeros past
// the node's depth), so bounds are taken per window: a lane past a depth
// reads zeros and adds a zero term, which leaves its sum unchanged, and each
// pair's terms run in window order. Windows whose loads are issued together
// per step: 2 measured faster than 4 and 8 with two pairs per wavefront.
constexpr int kTopQueryUnroll = 2;
// pairs spanning this many windows or more take the one-pair-at-a-time path
constexpr int32_t kTopQueryDeep = 16;
__device__ __forceinline__ void top_query_body(const SweepArgs& A, const QueryArgs& Q, int64_t blk) {
  // two consecutive pairs per wavefront (pairs are sorted by lower endpoint,
  // so the two often share its column): indices and offsets are wave-uniform
  const int64_t q0 = (blk * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) * 2;
  const int lane = threadIdx.x & 63;
  if (q0 >= Q.ntq) return;
  const bool two = q0 + 1 < Q.ntq;
  const int64_t q1 = two ? q0 + 1 : q0;
  const int32_t lo0 = load_uniform(Q.tq_lo + q0), hi0 = load_uniform(Q.tq_hi + q0);
  const int32_t lo1 = load_uniform(Q.tq_lo + q1), hi1 = load_uniform(Q.tq_hi + q1);
  const int32_t dl0 = load_uniform(A.top_depth + lo0), dl1 = load_uniform(A.top_depth + lo1);
  const int32_t dh0 = hi0 >= 0 ? load_uniform(A.top_depth + hi0) : 0;
  const int32_t dh1 = hi1 >= 0 ? load_uniform(A.top_depth + hi1) : 0;
  const double* __restrict__ zl0 = A.store + load_uniform(A.top_off + lo0) + lane;
  const double* __restrict__ zl1 = A.store + load_uniform(A.top_off + lo1) + lane;
  const double* __restrict__ zh0 = A.store + (hi0 >= 0 ? load_uniform(A.top_off + hi0) : 0) + lane;
  const double* __restrict__ zh1 = A.store + (hi1 >= 0 ? load_uniform(A.top_off + hi1) : 0) + lane;
  const bool same = lo0 == lo1;
  const int32_t nwl0 = (dl0 + kWin - 1) / kWin, nwh0 = (dh0 + kWin - 1) / kWin;
  const int32_t nwl1 = (dl1 + kWin - 1) / kWin, nwh1 = (dh1 + kWin - 1) / kWin;
  const int32_t nw = max(nwl0, nwl1);
  double s0 = 0.0, s1 = 0.0;
  if (nw >= kTopQueryDeep) {
    // deep columns (few such pairs, long load chains): one pair after the
    // other, with 4 * kTopQueryUnroll windows of loads in flight in the same
    // registers
    constexpr int U = 4 * kTopQueryUnroll;
    auto one = [&](const double* __restrict__ zl, const double* __restrict__ zh, int32_t nwl, int32_t nwh) {
      double s = 0.0;
      for (int32_t w = 0; w < nwl; w += U) {
        double a[U], b[U];
#pragma unroll
        for (int i = 0; i < U; ++i) a[i] = w + i < nwl ? zl[(int64_t)(w + i) * kWin] : 0.0;
#pragma unroll
        for (int i = 0; i < U; ++i) b[i] = w + i < nwh ? zh[(int64_t)(w + i) * kWin] : 0.0;
#pragma unroll
        for (int i = 0; i < U; ++i) {
          const double v = a[i] - b[i];
          s = fma(v, v, s);
        }
      }
      return s;
    };
    s0 = one(zl0, zh0, nwl0, nwh0);
    if (two) s1 = one(zl1, zh1, nwl1, nwh1);
  } else {
    for (int32_t w = 0; w < nw; w += kTopQueryUnroll) {
      double a0[kTopQueryUnroll], b0[kTopQueryUnroll], a1[kTopQueryUnroll], b1[kTopQueryUnroll];
#pragma unroll
      for (int i = 0; i < kTopQueryUnroll; ++i) a0[i] = w + i < nwl0 ? zl0[(int64_t)(w + i) * kWin] : 0.0;
#pragma unroll
      for (int i = 0; i < kTopQueryUnroll; ++i) b0[i] = w + i < nwh0 ? zh0[(int64_t)(w + i) * kWin] : 0.0;
      if (same) {
#pragma unroll
        for (int i = 0; i < kTopQueryUnroll; ++i) a1[i] = a0[i];
      } else {
#pragma unroll
        for (int i = 0; i < kTopQueryUnroll; ++i) a1[i] = w + i < nwl1 ? zl1[(int64_t)(w + i) * kWin] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < kTopQueryUnroll; ++i) b1[i] = w + i < nwh1 ? zh1[(int64_t)(w + i) * kWin] : 0.0;
#pragma unroll
      for (int i = 0; i < kTopQueryUnroll; ++i) {
        const double v0 = a0[i] - b0[i], v1 = a1[i] - b1[i];
        s0 = fma(v0, v0, s0);
        s1 = fma(v1, v1, s1);
      }
    }
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  if (lane == 0) {
    Q.R[load_uniform(Q.tq_out + q0)] = s0;
    if (two) Q.R[load_uniform(Q.tq_out + q1)] = s1;
  }
}

// Blocks of pairs go to the XCDs in runs of consecutive blocks, as the GEMM
// tiles do: most partners are near the lower endpoint in the same chain, so
// a partner's column is usually the lower column of a pair a few blocks on,
// and the run keeps both reads in one L2 (measured 2% faster on the batched
// random geometric graphs than round-robin blocks).
__global__ __launch_bounds__(256) void top_query_kernel(SweepArgs A, QueryArgs Q) {
  top_query_body(A, Q, xcd_task(blockIdx.x));
}

__device__ __forceinline__ void zero_body(const QueryArgs& Q, int64_t blk) {
  const int64_t j = blk * 256 + threadIdx.x;
  if (j < Q.nzero) Q.R[Q.zero_out[j]] = 0.0;
}

__global__ __launch_bounds__(256) void zero_kernel(QueryArgs Q) { zero_body(Q, blockIdx.x); }

// ---------------------------------------------------------------- grouped launches
// One launch covers the same step of many factors: item i of the map names a
// factor's argument block and the item's index within that factor's own
// launch of the step. A grid smaller than the item count makes the workgroups
// loop over items with a fixed stride (persistent form). Every item computes
// exactly what it computes in the factor's own launch.

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void grouped_gemm_kernel(const FactorArgs* __restrict__ fa,
                                                           const GroupItem* __restrict__ items, int64_t nitems) {
  __shared__ GemmRed red;
  for (int64_t i = blockIdx.x; i < nitems; i += gridDim.x) {
    const int32_t f = load_uniform(&items[i].fa);
    const int64_t local = load_uniform(&items[i].local);
    gemm_body(&fa[f].g, local, red);
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void grouped_narrow_kernel(const FactorArgs* __restrict__ fa,
                                                             const GroupItem* __restrict__ items, int64_t nitems) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int64_t b = blockIdx.x; b * 4 < nitems; b += gridDim.x) {
    const int64_t i = b * 4 + wave;
    if (i < nitems) gemm_narrow_body(&fa[load_uniform(&items[i].fa)].g, load_uniform(&items[i].local));
  }
}

// chain rows of many factors: one wavefront per top node, four per workgroup
// (most top nodes of small graphs have a few windows of rows)
__global__ __launch_bounds__(256) void grouped_chain_rows_kernel(const FactorArgs* __restrict__ fa,
                                                                 const GroupItem* __restrict__ items, int64_t nitems) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int64_t b = blockIdx.x; b * 4 < nitems; b += gridDim.x) {
    const int64_t i = b * 4 + wave;
    if (i < nitems)
      chain_rows_body(load_struct(&fa[load_uniform(&items[i].fa)].a), load_uniform(&items[i].local), threadIdx.x & 63, 64);
  }
}

__global__ __launch_bounds__(64) void grouped_inv_base_kernel(const FactorArgs* __restrict__ fa,
                                                              const GroupItem* __restrict__ items, int64_t nitems) {
  __shared__ BaseTile Ls, Xs;
  for (int64_t i = blockIdx.x; i < nitems; i += gridDim.x) {
    const int32_t f = load_uniform(&items[i].fa);
    const int64_t local = load_uniform(&items[i].local);
    const SweepArgs A = load_struct(&fa[f].a);
    inv_base_body(A, local, Ls, Xs);
    __syncthreads();
  }
}

// One (factor, item) per workgroup of the bottom step (grids that cover the
// items); the persistent schedules use grouped_kernel's loop.
template <bool WIDE>
__global__ __launch_bounds__(64 * kBottomWaves) void grouped_bottom_once_kernel(const FactorArgs* __restrict__ fa,
                                                                               const GroupItem* __restrict__ items) {
  __shared__ BottomLds lds;
  const int32_t f = load_uniform(&items[blockIdx.x].fa);
  const int64_t local = load_uniform(&items[blockIdx.x].local);
  bottom_body<WIDE>(load_struct(&fa[f].a), load_struct(&fa[f].q), local, lds);
}

// top-node pairs of many factors, blocks mapped to XCDs as in top_query_kernel
__global__ __launch_bounds__(256) void grouped_top_query_kernel(const FactorArgs* __restrict__ fa,
                                                                const GroupItem* __restrict__ items, int64_t nitems) {
  const int64_t i = xcd_task(blockIdx.x);
  if (i >= nitems) return;
  const int32_t f = load_uniform(&items[i].fa);
  top_query_body(load_struct(&fa[f].a), load_struct(&fa[f].q), load_uniform(&items[i].local));
}

// dense items of many factors, one group per launch: one workgroup per item
template <int GRP, bool STAGE>
__global__ __launch_bounds__(64 * kBottomWaves) __attribute__((amdgpu_waves_per_eu(4))) void grouped_dense_kernel(
    const FactorArgs* __restrict__ fa, const GroupItem* __restrict__ items, int64_t nitems) {
  __shared__ DenseLds<GRP> L;
  for (int64_t i = blockIdx.x; i < nitems; i += gridDim.x) {
    const int32_t f = load_uniform(&items[i].fa);
    dense_body<GRP, STAGE>(load_struct(&fa[f].a), load_struct(&fa[f].q), load_uniform(&items[i].local), L);
    __syncthreads();
  }
}

template <int KIND>
__global__ __launch_bounds__(256) void grouped_kernel(const FactorArgs* __restrict__ fa,
                                                      const GroupItem* __restrict__ items, int64_t nitems) {
  for (int64_t i = blockIdx.x; i < nitems; i += gridDim.x) {
    const int32_t f = load_uniform(&items[i].fa);
    const int64_t local = load_uniform(&items[i].local);
    if constexpr (KIND == GK_BOTTOM || KIND == GK_BOTTOM_WIDE) {
      __shared__ BottomLds lds;
      bottom_body<KIND == GK_BOTTOM_WIDE>(load_struct(&fa[f].a), load_struct(&fa[f].q), local, lds);
    } else if constexpr (KIND == GK_REDUCE) {
      reduce_body(load_struct(&fa[f].q), local);
    } else if constexpr (KIND == GK_ZERO) {
      zero_body(load_struct(&fa[f].q), local);
    } else if constexpr (KIND == GK_GENERAL) {
      general_pair_body(load_struct(&fa[f].a), load_struct(&fa[f].q), local);
    }
  }
}

}  // namespace

hipError_t launch_grouped(int kind, const FactorArgs* fa, const GroupItem* items, int64_t nitems, int64_t grid,
                          hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  const dim3 g((unsigned)std::max<int64_t>(1, std::min(grid, nitems)));
  switch (kind) {
    case GK_GEMM: hipLaunchKernelGGL(grouped_gemm_kernel, g, dim3(256), 0, s, fa, items, nitems); break;
    case GK_GEMM_NARROW: {
      // four tasks per workgroup
      const dim3 gn((unsigned)std::max<int64_t>(1, (std::min(grid, nitems) + 3) / 4));
      hipLaunchKernelGGL(grouped_narrow_kernel, gn, dim3(256), 0, s, fa, items, nitems);
      break;
    }
    case GK_INV_BASE: hipLaunchKernelGGL(grouped_inv_base_kernel, g, dim3(64), 0, s, fa, items, nitems); break;
    case GK_CHAIN_ROWS: {
      // four top nodes per workgroup
      const dim3 gr((unsigned)std::max<int64_t>(1, (std::min(grid, nitems) + 3) / 4));
      hipLaunchKernelGGL(grouped_chain_rows_kernel, gr, dim3(256), 0, s, fa, items, nitems);
      break;
    }
    case GK_BOTTOM:
      if ((int64_t)g.x == nitems)
        hipLaunchKernelGGL(grouped_bottom_once_kernel<false>, g, dim3(64 * kBottomWaves), 0, s, fa, items);
      else
        hipLaunchKernelGGL(grouped_kernel<GK_BOTTOM>, g, dim3(64 * kBottomWaves), 0, s, fa, items, nitems);
      break;
    case GK_BOTTOM_WIDE:
      if ((int64_t)g.x == nitems)
        hipLaunchKernelGGL(grouped_bottom_once_kernel<true>, g, dim3(64 * kBottomWaves), 0, s, fa, items);
      else
        hipLaunchKernelGGL(grouped_kernel<GK_BOTTOM_WIDE>, g, dim3(64 * kBottomWaves), 0, s, fa, items, nitems);
      break;
    case GK_REDUCE: hipLaunchKernelGGL(grouped_kernel<GK_REDUCE>, g, dim3(256), 0, s, fa, items, nitems); break;
    case GK_TOP_QUERY:
      hipLaunchKernelGGL(grouped_top_query_kernel, dim3((unsigned)xcd_grid(nitems)), dim3(256), 0, s, fa, items, nitems);
      break;
    case GK_ZERO: hipLaunchKernelGGL(grouped_kernel<GK_ZERO>, g, dim3(256), 0, s, fa, items, nitems); break;
    case GK_GENERAL: hipLaunchKernelGGL(grouped_kernel<GK_GENERAL>, g, dim3(256), 0, s, fa, items, nitems); break;
    default:
      if (kind >= GK_DENSE && kind < GK_DENSE + kDenseAllGroups) {
        dense_group<0>(kind - GK_DENSE, [&](auto X, auto ST) {
          hipLaunchKernelGGL((grouped_dense_kernel<decltype(X)::value, decltype(ST)::value>), g,
                             dim3(64 * kBottomWaves), 0, s, fa, items, nitems);
        });
        break;
      }
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gemm_level(const GemmArgs& g, int64_t task0, int64_t ntasks, int64_t ntask0, int64_t nntasks,
                             hipStream_t s) {
  const int64_t grid = xcd_grid(ntasks) + (nntasks + 3) / 4;
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(gemm_level_kernel, dim3((unsigned)grid), dim3(256), 0, s, g, task0, ntasks, ntask0, nntasks);
  return hipGetLastError();
}


hipError_t launch_gemm(const GemmArgs& g, int64_t task0, int64_t ntasks, hipStream_t s) {
  if (ntasks <= 0) return hipSuccess;
  hipLaunchKernelGGL(gemm_kernel, dim3((unsigned)xcd_grid(ntasks)), dim3(256), 0, s, g, task0, ntasks);
  return hipGetLastError();
}

hipError_t launch_inv_base(const SweepArgs& a, hipStream_t s) {
  if (a.nbase <= 0) return hipSuccess;
  hipLaunchKernelGGL(inv_base_kernel, dim3((unsigned)a.nbase), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_chain_rows(const SweepArgs& a, int32_t ntop, hipStream_t s) {
  if (ntop <= 0) return hipSuccess;
  hipLaunchKernelGGL(chain_rows_kernel, dim3((unsigned)ntop), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_bottom(const SweepArgs& a, const QueryArgs& q, hipStream_t s) {
  if (q.nwork <= 0) return hipSuccess;
  if (a.store_wide)
    hipLaunchKernelGGL(bottom_kernel<true>, dim3((unsigned)q.nwork), dim3(64 * kBottomWaves), 0, s, a, q);
  else
    hipLaunchKernelGGL(bottom_kernel<false>, dim3((unsigned)q.nwork), dim3(64 * kBottomWaves), 0, s, a, q);
  return hipGetLastError();
}

hipError_t launch_bxfer(const SweepArgs& a, hipStream_t s) {
  if (a.nsub <= 0) return hipSuccess;
  hipLaunchKernelGGL(bxfer_kernel, dim3((unsigned)((a.nsub + kBottomWaves - 1) / kBottomWaves)), dim3(64 * kBottomWaves),
                     0, s, a);
  return hipGetLastError();
}

hipError_t launch_dense(const SweepArgs& a, const QueryArgs& q, const int64_t* dclass_ptr, int only, hipStream_t s) {
  for (int x = 0; x < kDenseAllGroups; ++x) {
    const int64_t i0 = dclass_ptr[x], n = dclass_ptr[x + 1] - dclass_ptr[x];
    if (n <= 0 || (only >= 0 && x != only)) continue;
    dense_group<0>(x, [&](auto X, auto ST) {
      hipLaunchKernelGGL((dense_kernel<decltype(X)::value, decltype(ST)::value>), dim3((unsigned)n),
                         dim3(64 * kBottomWaves), 0, s, a, q, i0);
    });
  }
  return hipGetLastError();
}

hipError_t launch_finish(const SweepArgs& a, const QueryArgs& q, hipStream_t s) {
  if (q.nbq > 0)
    hipLaunchKernelGGL(reduce_bottom_kernel, dim3((unsigned)((q.nbq + 255) / 256)), dim3(256), 0, s, q);
  if (q.ntq > 0)
    hipLaunchKernelGGL(top_query_kernel, dim3((unsigned)xcd_grid((q.ntq + kTopQueryBlock - 1) / kTopQueryBlock)),
                       dim3(256), 0, s, a, q);
  if (q.nzero > 0)
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((q.nzero + 255) / 256)), dim3(256), 0, s, q);
  if (q.ngp > 0)
    hipLaunchKernelGGL(general_pair_kernel, dim3((unsigned)((q.ngp + 3) / 4)), dim3(256), 0, s, a, q);
  return hipGetLastError();
}

}  // namespace peers
