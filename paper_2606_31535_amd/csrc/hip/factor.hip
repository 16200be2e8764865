// Numeric factorization P L_r P^T = L D L^T on the device (Algorithm 8,
// step 1), following the plan of host/numplan.h: bottom subtrees (one
// wavefront per task, right-looking in the factor's compressed columns), the
// pulls of bottom contributions into the top columns' dense depth-indexed
// fronts (the top store's layout, used as workspace), then per level of the
// tree of chain pieces (at most 64 columns each) the pieces' diagonal blocks
// in LDS, the rows of U_P, the products L_{U,P} D_P L_{U,P}^T on the matrix
// cores (the sweep's GEMM body) and the subtraction of those products from
// the ancestor columns. The factor's top values are left in the fronts and
// copied into the sweep layout at the end. Every pivot is the node's
// conductance to the ground plus the magnitudes of its off-diagonal Schur
// entries, and every update adds terms of the sign of what it updates, so no
// step cancels. Each reduction and each update runs in a fixed order: the
// factor is the same bits on every run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "../host/graph_handle.h"
#include "../host/numplan.h"
#include "device_handle.h"
#include "sweep_kernels.h"
#include "wave_ops.h"

namespace peers {

namespace {

struct FacArgs {
  const int64_t* colptr;
  const int32_t* rowidx;
  const int32_t* depth;
  const int32_t* top_index;  // per node, -1 for bottom nodes
  double* Lx;
  double* D;
  double* r;     // conductance to the ground, accumulated per node
  double* rfin;  // r of each node when it is eliminated
  double* e;     // per top index: r plus the magnitudes of the column's U-row entries
  // bottom
  const int32_t* bt_ptr;
  const int32_t* bcol;
  const int64_t* bpair_ptr;
  const int64_t* bpair;
  // pulls
  const int32_t* tg_ptr;
  const int32_t* tg_k;
  const int64_t* tg_p;
  // pieces of the top chains
  const int32_t* top_node;
  const int64_t* top_off;
  double* T;
  const FacPiece* pieces;
  const int32_t* pu_depth;
  const int32_t* pu_top;
  double* lu;   // L_{U,P} of the step's pieces
  double* lud;  // the same scaled by D_P
  double* G;
  const int32_t* lev_piece;
  const int32_t* ur_piece;
  const int32_t* ur_row0;
  const int32_t* sc_dest;
  const int32_t* sc_src_ptr;
  const int32_t* sc_piece;
  const int32_t* sc_pos;
  // outputs into the sweep layout
  double* lcc;
  double* luc;
  const int64_t* top_x_ptr;
  const int64_t* top_src;
  const int64_t* coef_p;
  const int64_t* coef_off;
  char* bnode_base;
  char* bent_base;
  const int32_t* bnode_node;
  double* isd;
  double* top_isd;
};

// Top columns' fronts: element depth(i) - 1 of top column j holds A_ij.
__global__ __launch_bounds__(64) void fac_front_init_kernel(FacArgs F, int32_t ntop) {
  const int32_t t = blockIdx.x;
  if (t >= ntop) return;
  const int32_t j = F.top_node[t];
  const int64_t base = F.top_off[t];
  for (int64_t p = F.colptr[j] + threadIdx.x; p < F.colptr[j + 1]; p += 64)
    F.T[base + F.depth[F.rowidx[p]] - 1] = F.Lx[p];
}

// One bottom task: its columns children first.
__global__ __launch_bounds__(64) void fac_bottom_kernel(FacArgs F) {
  const int32_t task = blockIdx.x;
  const int lane = threadIdx.x;
  for (int32_t x = F.bt_ptr[task]; x < F.bt_ptr[task + 1]; ++x) {
    const int32_t k = F.bcol[x];
    const int64_t p0 = F.colptr[k], p1 = F.colptr[k + 1];
    double s = 0.0;
    for (int64_t p = p0 + lane; p < p1; p += 64) s -= F.Lx[p];
    s = wave_sum(s);
    const double rk = F.r[k];
    const double d = rk + s;
    if (lane == 0) {
      F.D[k] = d;
      F.rfin[k] = rk;
    }
    for (int64_t p = p0 + lane; p < p1; p += 64) F.Lx[p] = F.Lx[p] / d;
    __syncthreads();
    // rows of the column that are bottom nodes: their ground conductance and
    // their columns' entries below them
    int64_t pb = F.bpair_ptr[x];
    for (int64_t p = p0; p < p1; ++p) {
      const int32_t j = F.rowidx[p];
      if (F.top_index[j] >= 0) continue;
      const double lp = F.Lx[p];
      if (lane == 0) F.r[j] = fma(-lp, rk, F.r[j]);
      const double sp = d * lp;
      for (int64_t q = p + 1 + lane; q < p1; q += 64) {
        const int64_t tgt = F.bpair[pb + (q - p - 1)];
        F.Lx[tgt] = fma(-F.Lx[q], sp, F.Lx[tgt]);
      }
      pb += p1 - p - 1;
    }
    __syncthreads();
  }
}

// Each top column subtracts the contributions of the bottom columns that
// reach it, in the plan's order.
__global__ __launch_bounds__(64) void fac_pull_kernel(FacArgs F, int32_t ntop) {
  const int32_t t = blockIdx.x;
  if (t >= ntop) return;
  const int lane = threadIdx.x;
  const int32_t j = F.top_node[t];
  const int64_t base = F.top_off[t];
  double racc = 0.0;
  for (int32_t x = F.tg_ptr[t]; x < F.tg_ptr[t + 1]; ++x) {
    const int32_t k = F.tg_k[x];
    const int64_t p = F.tg_p[x];
    const double lp = F.Lx[p];
    const double sp = F.D[k] * lp;
    racc = fma(-lp, F.rfin[k], racc);
    for (int64_t q = p + 1 + lane; q < F.colptr[k + 1]; q += 64) {
      double* dst = F.T + base + F.depth[F.rowidx[q]] - 1;
      *dst = fma(-F.Lx[q], sp, *dst);
    }
    __syncthreads();
  }
  if (lane == 0) F.r[j] += racc;
}

// e_t = r + the magnitudes of column t's entries in the rows of U_P, for
// every column of this level's pieces: one wavefront per column (four
// columns per workgroup, 16 workgroups per piece), the rows in four
// interleaved lane-strided sums added in a fixed order.
__global__ __launch_bounds__(256) void fac_esum_kernel(FacArgs F, int32_t lev0) {
  const FacPiece Pc = F.pieces[F.lev_piece[lev0 + blockIdx.x / 16]];
  const int lane = threadIdx.x & 63;
  const int32_t t = (int32_t)(blockIdx.x % 16) * 4 + (int32_t)(threadIdx.x >> 6);
  if (t >= Pc.w) return;
  const double* col = F.T + Pc.col_base + (int64_t)t * Pc.ld;
  const int32_t* pd = F.pu_depth + Pc.u_begin;
  double u0 = 0.0, u1 = 0.0, u2 = 0.0, u3 = 0.0;
  int32_t e = lane;
  for (; e + 192 < Pc.nU; e += 256) {
    u0 -= col[pd[e] - 1];
    u1 -= col[pd[e + 64] - 1];
    u2 -= col[pd[e + 128] - 1];
    u3 -= col[pd[e + 192] - 1];
  }
  for (; e < Pc.nU; e += 64) u0 -= col[pd[e] - 1];
  const double u = wave_sum((u0 + u1) + (u2 + u3));
  if (lane == 0) F.e[F.top_index[Pc.a] + t] = F.r[Pc.a + t] + u;
}

// Diagonal block of one piece a..b, one wavefront: lane i holds row i of
// the block (x[t] = S_{a+i,a+t}) in registers. Column t (node a+t) is the
// front at T + col_base + t*ld; row a+i (i > t) of it sits at depth index
// dp + w - 1 - i. e_t (from fac_esum_kernel) is r plus the magnitudes of
// column t's U-row entries, so column t's pivot is e_t plus the magnitudes of
// its entries below the diagonal (a wave sum). Eliminating column t adds
// (-L_{a+i,a+t}) e_t and (-L_{a+i,a+t}) r_t to e and r of the later rows
// (the U rows' own updates are formed afterwards, row by row) and subtracts
// L_{a+i,a+t} S_{a+t2,a+t} from the entries (i, t2), t < t2, with column t
// broadcast through LDS (entries at or above the diagonal are updated too;
// they are never read). The L values go back into the fronts.
__global__ __launch_bounds__(64) void fac_diag_kernel(FacArgs F, int32_t lev0) {
  __shared__ double colS[kFacPiece];
  const FacPiece Pc = F.pieces[F.lev_piece[lev0 + blockIdx.x]];
  const int lane = threadIdx.x;
  const int32_t w = Pc.w, dp = Pc.dp;
  double* col0 = F.T + Pc.col_base;
  double x[kFacPiece];
#pragma unroll
  for (int t = 0; t < kFacPiece; ++t) x[t] = (t < w && lane > t && lane < w) ? col0[(int64_t)t * Pc.ld + dp + w - 1 - lane] : 0.0;
  double er = 0.0, rr = 0.0;
  if (lane < w) {
    er = F.e[F.top_index[Pc.a] + lane];
    rr = F.r[Pc.a + lane];
  }
  const bool live = lane < w;
#pragma unroll
  for (int t = 0; t < kFacPiece; ++t) {
    if (t < w) {
      const double et = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(er), t),
                                         __builtin_amdgcn_readlane(__double2loint(er), t));
      const double rt = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(rr), t),
                                         __builtin_amdgcn_readlane(__double2loint(rr), t));
      const bool below = live && lane > t;
      const double dv = et + wave_sum(below ? -x[t] : 0.0);
      const double l = below ? x[t] / dv : 0.0;
      if (lane == 0) {
        F.D[Pc.a + t] = dv;
        F.rfin[Pc.a + t] = rt;
      }
      if (below) col0[(int64_t)t * Pc.ld + dp + w - 1 - lane] = l;
      er = fma(-l, et, er);
      rr = fma(-l, rt, rr);
      colS[lane] = x[t];
      __syncthreads();
#pragma unroll
      for (int t2 = t + 1; t2 < kFacPiece; ++t2) x[t2] = fma(-l, colS[t2], x[t2]);
      __syncthreads();
    }
  }
}

// Rows of U_P: one thread per U node (kFacRowTile rows per workgroup). The
// row's 64 entries S_{u,a+t} stay in registers and are finished in column
// order: L_{u,t} = S_{u,t} / D_t, then S_{u,t2} -= L_{u,t} D_t L_{a+t2,t} for
// the later columns (so each entry takes its terms in increasing t), with the
// piece's L block and pivots staged in LDS. Writes L_{U,P} back into the
// fronts and into the step's scratch (plain and D-scaled) for the product.
__global__ __launch_bounds__(kFacRowTile) void fac_urows_kernel(FacArgs F, int32_t ur0) {
  __shared__ double lpp[kFacPiece * kFacPiece];  // lpp[t * 64 + i] = L_{a+i, a+t}, i > t
  __shared__ double dsh[kFacPiece];
  const FacPiece Pc = F.pieces[F.ur_piece[ur0 + blockIdx.x]];
  double* col0 = F.T + Pc.col_base;
  const int32_t w = Pc.w;
  const int32_t dtop = Pc.dp + w - 1;  // depth index of row a
  for (int32_t x = threadIdx.x; x < w * kFacPiece; x += kFacRowTile) {
    const int32_t t = x >> 6, i = x & 63;
    if (i > t && i < w) lpp[x] = col0[(int64_t)t * Pc.ld + dtop - i];
  }
  if ((int32_t)threadIdx.x < w) dsh[threadIdx.x] = F.D[Pc.a + threadIdx.x];
  __syncthreads();
  const int32_t e = F.ur_row0[ur0 + blockIdx.x] + threadIdx.x;
  if (e >= Pc.nU) return;
  const int32_t du = F.pu_depth[Pc.u_begin + e] - 1;
  double* lu = F.lu + Pc.luc_off + e;
  double* ld = F.lud + Pc.luc_off + e;
  double x[kFacPiece];
#pragma unroll
  for (int t = 0; t < kFacPiece; ++t) x[t] = t < w ? col0[(int64_t)t * Pc.ld + du] : 0.0;
#pragma unroll
  for (int t = 0; t < kFacPiece; ++t) {
    if (t < w) {
      const double dv = dsh[t];
      const double l = x[t] / dv;
      const double sl = l * dv;
      lu[(int64_t)t * Pc.ldu] = l;
      ld[(int64_t)t * Pc.ldu] = sl;
      col0[(int64_t)t * Pc.ld + du] = l;
#pragma unroll
      for (int t2 = t + 1; t2 < kFacPiece; ++t2) x[t2] = fma(-sl, lpp[t * kFacPiece + t2], x[t2]);
    }
  }
}

// Each destination column subtracts the products of this level's pieces
// whose U_P holds it, in piece order, and takes their ground conductance.
__global__ __launch_bounds__(64) void fac_scatter_kernel(FacArgs F, int32_t d0) {
  const int32_t di = d0 + blockIdx.x;
  const int32_t t = F.sc_dest[di];
  const int lane = threadIdx.x;
  const int64_t base = F.top_off[t];
  double racc = 0.0;
  for (int32_t x = F.sc_src_ptr[di]; x < F.sc_src_ptr[di + 1]; ++x) {
    const FacPiece Pc = F.pieces[F.sc_piece[x]];
    const int32_t e = F.sc_pos[x];
    const double* g = F.G + Pc.g_off + (int64_t)e * Pc.ldu;
    for (int32_t i = e + 1 + lane; i < Pc.nU; i += 64) {
      double* dst = F.T + base + F.pu_depth[Pc.u_begin + i] - 1;
      *dst -= g[i];
    }
    double rsum = 0.0;
    for (int32_t k = lane; k < Pc.w; k += 64) rsum = fma(-F.lu[Pc.luc_off + (int64_t)k * Pc.ldu + e], F.rfin[Pc.a + k], rsum);
    racc += wave_sum(rsum);
    __syncthreads();
  }
  if (lane == 0) F.r[F.top_node[t]] += racc;
}

// The top columns' factor values from their fronts into the compressed
// columns and the sweep's L_CC / L_{U,C} blocks.
__global__ __launch_bounds__(64) void fac_top_lx_kernel(FacArgs F, int32_t ntop) {
  const int32_t t = blockIdx.x;
  if (t >= ntop) return;
  const int32_t j = F.top_node[t];
  const int64_t base = F.top_off[t], p0 = F.colptr[j], x0 = F.top_x_ptr[t];
  for (int64_t p = p0 + threadIdx.x; p < F.colptr[j + 1]; p += 64) {
    const double v = F.T[base + F.depth[F.rowidx[p]] - 1];
    F.Lx[p] = v;
    const int64_t src = F.top_src[x0 + (p - p0)];
    if (src & kLxFromLuc) F.luc[src & ~kLxFromLuc] = v;
    else F.lcc[src] = v;
  }
}

__global__ __launch_bounds__(256) void fac_coef_kernel(FacArgs F, int64_t n) {
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (x >= n) return;
  const int64_t off = F.coef_off[x];
  char* dst = (off & kCoefInBent) ? F.bent_base + (off & ~kCoefInBent) : F.bnode_base + off;
  *(double*)dst = -F.Lx[F.coef_p[x]];
}

__global__ __launch_bounds__(256) void fac_isd_kernel(FacArgs F, int32_t N, int32_t ntop, int64_t nrec) {
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (x < N) F.isd[x] = 1.0 / sqrt(F.D[x]);
  if (x < ntop) F.top_isd[x] = 1.0 / sqrt(F.D[F.top_node[x]]);
  if (x < nrec) *(double*)(F.bnode_base + x * (int64_t)sizeof(BNode)) = 1.0 / sqrt(F.D[F.bnode_node[x]]);
}

inline unsigned grid1(int64_t n, int64_t per) { return (unsigned)std::max<int64_t>(1, (n + per - 1) / per); }

// Device buffers of the factorization. With `dry` set nothing is allocated:
// the calls only add up the bytes (so the budget is reserved exactly first).
struct DevBufs {
  bool dry = false;
  std::vector<void*> ptrs;
  uint64_t bytes = 0;
  hipError_t err = hipSuccess;
  template <class T>
  T* put(const std::vector<T>& v, hipStream_t s) {
    void* p = nullptr;
    const size_t b = std::max<size_t>(v.size() * sizeof(T), 8);
    if (dry) {
      bytes += b;
      return nullptr;
    }
    if (err == hipSuccess) err = hipMalloc(&p, b);
    if (err != hipSuccess) return nullptr;
    ptrs.push_back(p);
    bytes += b;
    if (!v.empty()) err = hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
    return (T*)p;
  }
  template <class T>
  T* alloc(size_t n) {
    void* p = nullptr;
    const size_t b = std::max<size_t>(n * sizeof(T), 8);
    if (dry) {
      bytes += b;
      return nullptr;
    }
    if (err == hipSuccess) err = hipMalloc(&p, b);
    if (err != hipSuccess) return nullptr;
    ptrs.push_back(p);
    bytes += b;
    return (T*)p;
  }
  void free_all() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

}  // namespace

Status device_factor(FactorHandle& Fh, const GraphHandle& G, const NumericPlan& Q, double* lcc_dev, double* luc_dev,
                     hipStream_t s, Numeric* host_out, double* device_ms) {
  const FactorPlan& P = *Fh.plan;
  const Symbolic& S = G.sym;
  const int32_t N = S.N;
  // the factorization's buffers; a dry pass first adds up their bytes, which
  // are reserved against the device budget while the factorization runs
  auto setup = [&](DevBufs& B, FacArgs& A, GemmArgs& GA) {
    A.colptr = B.put(S.colptr, s);
    A.rowidx = B.put(S.rowidx, s);
    A.depth = B.put(S.depth, s);
    A.top_index = B.put(P.top_index, s);
    A.Lx = B.put(Q.lx0, s);
    A.D = B.alloc<double>(N);
    A.r = B.put(Q.r0, s);
    A.rfin = B.alloc<double>(N);
    A.e = B.alloc<double>((size_t)std::max<int32_t>(P.ntop, 1));
    A.bt_ptr = B.put(Q.bt_ptr, s);
    A.bcol = B.put(Q.bcol, s);
    A.bpair_ptr = B.put(Q.bpair_ptr, s);
    A.bpair = B.put(Q.bpair, s);
    A.tg_ptr = B.put(Q.tg_ptr, s);
    A.tg_k = B.put(Q.tg_k, s);
    A.tg_p = B.put(Q.tg_p, s);
    A.top_node = Fh.sweep.top_node;
    A.top_off = Fh.sweep.top_off;
    A.T = (double*)Fh.store;
    A.pieces = B.put(Q.pieces, s);
    A.pu_depth = B.put(Q.pu_depth, s);
    A.pu_top = B.put(Q.pu_top, s);
    A.lu = B.alloc<double>((size_t)std::max<int64_t>(Q.luc_elems, 1));
    A.lud = B.alloc<double>((size_t)std::max<int64_t>(Q.luc_elems, 1));
    A.G = B.alloc<double>((size_t)std::max<int64_t>(Q.g_elems, 1));
    A.lev_piece = B.put(Q.lev_piece, s);
    A.ur_piece = B.put(Q.ur_piece, s);
    A.ur_row0 = B.put(Q.ur_row0, s);
    A.sc_dest = B.put(Q.sc_dest, s);
    A.sc_src_ptr = B.put(Q.sc_src_ptr, s);
    A.sc_piece = B.put(Q.sc_piece, s);
    A.sc_pos = B.put(Q.sc_pos, s);
    A.lcc = lcc_dev;
    A.luc = luc_dev;
    A.top_x_ptr = B.put(Q.top_x_ptr, s);
    A.top_src = B.put(Q.top_src, s);
    A.coef_p = B.put(P.coef_p, s);
    A.coef_off = B.put(P.coef_off, s);
    A.bnode_base = (char*)Fh.sweep.bnode;
    A.bent_base = (char*)Fh.sweep.bent;
    A.bnode_node = B.put(Q.bnode_node, s);
    A.isd = const_cast<double*>(Fh.sweep.isd);
    A.top_isd = const_cast<double*>(Fh.sweep.top_isd);
    GA = Fh.gemm;
    GA.probs = B.put(Q.probs, s);
    GA.tasks = B.put(Q.tasks, s);
    GA.buf[BUF_LUC] = A.lu;
    GA.buf[BUF_BT] = A.lud;
    GA.buf[BUF_G] = A.G;
  };
  uint64_t est = 0;
  {
    DevBufs dry;
    dry.dry = true;
    FacArgs A0{};
    GemmArgs G0{};
    setup(dry, A0, G0);
    est = dry.bytes;
  }
  Status st = Fh.dev->reserve(est);
  if (st != OK) return st;
  DevBufs B;
  FacArgs A{};
  GemmArgs GA{};
  setup(B, A, GA);
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipError_t e = B.err;
  auto finish = [&](Status r) {
    (void)hipStreamSynchronize(s);
    for (auto& x : ev)
      if (x) (void)hipEventDestroy(x);
    B.free_all();
    Fh.dev->release(est);
    return r;
  };
  if (e != hipSuccess) return finish(hip_fail(e, "device factorization buffers"));
  e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  if (e == hipSuccess) e = hipMemsetAsync(Fh.store, 0, (size_t)std::max<int64_t>(P.store_elems, kWin) * 8, s);
  if (e == hipSuccess) e = hipEventRecord(ev[0], s);
  if (e != hipSuccess) return finish(hip_fail(e, "device factorization setup"));
  const int32_t ntop = P.ntop;
  const int32_t nbt = (int32_t)Q.bt_ptr.size() - 1;
  if (ntop > 0) hipLaunchKernelGGL(fac_front_init_kernel, dim3(ntop), dim3(64), 0, s, A, ntop);
  if (nbt > 0) hipLaunchKernelGGL(fac_bottom_kernel, dim3(nbt), dim3(64), 0, s, A);
  if (ntop > 0) hipLaunchKernelGGL(fac_pull_kernel, dim3(ntop), dim3(64), 0, s, A, ntop);
  for (int32_t step = 0; step < Q.steps; ++step) {
    const int32_t nc = Q.lev_ptr[step + 1] - Q.lev_ptr[step];
    if (nc > 0) {
      hipLaunchKernelGGL(fac_esum_kernel, dim3(nc * 16), dim3(256), 0, s, A, Q.lev_ptr[step]);
      hipLaunchKernelGGL(fac_diag_kernel, dim3(nc), dim3(64), 0, s, A, Q.lev_ptr[step]);
    }
    const int32_t nu = Q.ur_ptr[step + 1] - Q.ur_ptr[step];
    if (nu > 0) hipLaunchKernelGGL(fac_urows_kernel, dim3(nu), dim3(kFacRowTile), 0, s, A, Q.ur_ptr[step]);
    e = launch_gemm(GA, Q.gemm_ptr[step], Q.gemm_ptr[step + 1] - Q.gemm_ptr[step], s);
    if (e != hipSuccess) return finish(hip_fail(e, "device factorization products"));
    const int32_t nd = Q.sc_ptr[step + 1] - Q.sc_ptr[step];
    if (nd > 0) hipLaunchKernelGGL(fac_scatter_kernel, dim3(nd), dim3(64), 0, s, A, Q.sc_ptr[step]);
  }
  const int64_t ncoef = (int64_t)P.coef_p.size();
  if (ntop > 0) hipLaunchKernelGGL(fac_top_lx_kernel, dim3(ntop), dim3(64), 0, s, A, ntop);
  if (ncoef > 0) hipLaunchKernelGGL(fac_coef_kernel, dim3(grid1(ncoef, 256)), dim3(256), 0, s, A, ncoef);
  const int64_t nmax = std::max<int64_t>({(int64_t)N, (int64_t)ntop, Q.bottom_records});
  hipLaunchKernelGGL(fac_isd_kernel, dim3(grid1(nmax, 256)), dim3(256), 0, s, A, N, ntop, Q.bottom_records);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(ev[1], s);
  // the store's leading zero block again (windows past a column's depth read it)
  if (e == hipSuccess) e = hipMemsetAsync(Fh.store, 0, (size_t)kStoreZeroBlock * 8, s);
  if (e == hipSuccess && host_out) {
    host_out->Lx.resize(Q.nnz);
    host_out->D.resize(N);
    e = hipMemcpyAsync(host_out->Lx.data(), A.Lx, (size_t)Q.nnz * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(host_out->D.data(), A.D, (size_t)N * 8, hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return finish(hip_fail(e, "device factorization"));
  float ms = 0;
  if (hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess && device_ms) *device_ms = ms;
  if (host_out) {
    for (int32_t i = 0; i < N; ++i)
      if (!(host_out->D[i] > 0.0) || !std::isfinite(host_out->D[i])) {
        set_error("non-positive pivot at column " + std::to_string(i));
        return finish(E_NOT_SPD);
      }
  }
  return finish(OK);
}

}  // namespace peers
