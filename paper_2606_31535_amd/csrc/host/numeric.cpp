// Numeric L D L^T factorization of the permuted grounded Laplacian
// (Algorithm 8, step 1: the paper factors L_r before the parallel sweep).
//
// Supernodal multifrontal method over the fundamental supernodes: each
// supernode assembles a dense frontal matrix from the original entries and its
// children's update matrices (extend-add), eliminates its own columns with a
// blocked right-looking L D L^T, and passes the Schur complement to its parent.
// No pivoting: L_r is SPD, and a non-positive pivot is reported as E_NOT_SPD.
//
// Pivots without cancellation. Every Schur complement of a grounded
// Laplacian is again a grounded Laplacian: its off-diagonal entries are <= 0,
// and each row's sum r_i >= 0 is that node's (effective) conductance to the
// ground. Eliminating node k changes them by adding same-signed terms only:
// S_ij -= L_ik D_k L_jk (a positive amount taken from a value <= 0) and
// r_i += (-L_ik) r_k. The usual diagonal update a_ii - sum l^2 d subtracts
// nearly equal numbers once r_i is small against the off-diagonals (nodes far
// from the ground), and the rounding then grows with the condition number of
// L_r. Here the updated diagonal is never used; each pivot is assembled when its
// column is eliminated as D_j = r_j + sum over rows i below j of (-S_ij), a
// sum of nonnegative terms, with r carried through the fronts beside the
// update matrices (extend-add of one more vector). This is the reformulation
// Grassmann, Taksar and Heyman use for Markov chains; every entry of L and D
// is then computed from same-signed sums, to high relative accuracy.
//
// Parallelism: independent subtrees of the supernodal tree run on separate
// threads, each in postorder with its own update stack; the few large fronts
// near the root run one at a time with a thread-parallel trailing update.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>

#include "host.h"

namespace peers {

namespace {

struct Ctx {
  const Symbolic& S;
  const std::vector<int64_t>& aptr;  // permuted lower columns of A (strict lower)
  const std::vector<int32_t>& arow;
  const std::vector<double>& aval;
  const std::vector<double>& agnd;   // permuted conductance to the ground
  std::vector<int32_t> sn_of;
  std::vector<int32_t> snpar;
  std::vector<std::vector<int32_t>> children;
  std::vector<std::vector<double>> upd;   // update matrix per supernode (lower, col-major)
  std::vector<std::vector<double>> updr;  // ground-conductance contributions to its rows
  Numeric& F;
  std::mutex err_mu;
  Status err = OK;
  std::string err_msg;
};

// Trailing update C[i,k] -= sum_j L[i,j] * d_j * L[k,j] over columns k in [k0, k1),
// rows i >= k, for panel columns j in [j0, j1). F is col-major with leading dim ld.
void trailing_update(double* Fm, int64_t ld, int64_t nrow, int64_t j0, int64_t j1, int64_t k0, int64_t k1,
                     const double* W /* W[(k)*nbw + (j-j0)] = L[k,j]*d_j */, int64_t nbw) {
  const int64_t nb = j1 - j0;
  constexpr int64_t KB = 8, IB = 256;
  for (int64_t kb = k0; kb < k1; kb += KB) {
    const int64_t ke = std::min(k1, kb + KB);
    for (int64_t ib = kb; ib < nrow; ib += IB) {
      const int64_t ie = std::min(nrow, ib + IB);
      for (int64_t k = kb; k < ke; ++k) {
        double* c = Fm + k * ld;
        const double* wk = W + k * nbw;
        const int64_t is = std::max(ib, k);
        for (int64_t j = 0; j < nb; ++j) {
          const double a = wk[j];
          if (a == 0.0) continue;
          const double* lj = Fm + (j0 + j) * ld;
          for (int64_t i = is; i < ie; ++i) c[i] -= lj[i] * a;
        }
      }
    }
  }
}

Status factor_front(Ctx& C, int32_t s, int inner_threads) {
  const Symbolic& S = C.S;
  const int32_t f = S.snptr[s], l = S.snptr[s + 1] - 1;
  const int64_t w = l - f + 1;
  const int64_t u = S.colptr[l + 1] - S.colptr[l];
  const int64_t nf = w + u;
  const int32_t* U = S.rowidx.data() + S.colptr[l];
  std::vector<int32_t> frow(nf);
  for (int64_t t = 0; t < w; ++t) frow[t] = f + (int32_t)t;
  for (int64_t t = 0; t < u; ++t) frow[w + t] = U[t];
  std::unique_ptr<double[]> Fbuf(new (std::nothrow) double[(size_t)(nf * nf)]);
  if (!Fbuf) return E_HOST_OOM;
  double* Fm = Fbuf.get();
  std::memset(Fm, 0, sizeof(double) * (size_t)(nf * nf));
  auto pos = [&](int32_t row) -> int64_t {
    return std::lower_bound(frow.begin(), frow.end(), row) - frow.begin();
  };
  // original entries; r starts as each pivot's own conductance to the ground
  std::vector<double> r(nf, 0.0);
  for (int64_t t = 0; t < w; ++t) {
    const int32_t j = f + (int32_t)t;
    r[t] = C.agnd[j];
    for (int64_t p = C.aptr[j]; p < C.aptr[j + 1]; ++p) Fm[t * nf + pos(C.arow[p])] += C.aval[p];
  }
  // extend-add children
  for (int32_t c : C.children[s]) {
    std::vector<double>& Uc = C.upd[c];
    const int32_t lc = S.snptr[c + 1] - 1;
    const int64_t uc = S.colptr[lc + 1] - S.colptr[lc];
    const int32_t* Ur = S.rowidx.data() + S.colptr[lc];
    std::vector<int64_t> map(uc);
    int64_t q = 0;
    for (int64_t p = 0; p < uc; ++p) {
      while (frow[q] != Ur[p]) ++q;
      map[p] = q;
    }
    for (int64_t b = 0; b < uc; ++b) {
      double* dst = Fm + map[b] * nf;
      const double* src = Uc.data() + b * uc;
      for (int64_t a = b; a < uc; ++a) dst[map[a]] += src[a];
    }
    const std::vector<double>& Rc = C.updr[c];
    for (int64_t a = 0; a < uc; ++a) r[map[a]] += Rc[a];
    std::vector<double>().swap(Uc);
    std::vector<double>().swap(C.updr[c]);
  }
  // blocked right-looking L D L^T on the first w columns
  constexpr int64_t NB = 32;
  std::vector<double> W;
  for (int64_t j0 = 0; j0 < w; j0 += NB) {
    const int64_t j1 = std::min(w, j0 + NB);
    for (int64_t j = j0; j < j1; ++j) {
      double* cj = Fm + j * nf;
      // the pivot as a sum of nonnegative terms (see the header); the
      // updated diagonal entry cj[j] is not used
      double off = 0.0;
      for (int64_t i = j + 1; i < nf; ++i) off -= cj[i];
      const double d = r[j] + off;
      if (!(d > 0.0) || !std::isfinite(d) || !(off >= 0.0)) {
        std::lock_guard<std::mutex> g(C.err_mu);
        C.err_msg = "non-positive pivot at column " + std::to_string(f + j);
        return E_NOT_SPD;
      }
      C.F.D[f + j] = d;
      const double inv = 1.0 / d;
      for (int64_t i = j + 1; i < nf; ++i) cj[i] *= inv;
      // the remaining rows' conductances to the ground through node j
      for (int64_t i = j + 1; i < nf; ++i) r[i] -= cj[i] * r[j];
      for (int64_t k = j + 1; k < j1; ++k) {
        const double a = cj[k] * d;
        double* ck = Fm + k * nf;
        for (int64_t i = k; i < nf; ++i) ck[i] -= cj[i] * a;
      }
    }
    if (j1 < nf) {
      const int64_t nbw = j1 - j0;
      W.assign((size_t)(nf * nbw), 0.0);
      for (int64_t k = j1; k < nf; ++k)
        for (int64_t j = j0; j < j1; ++j) W[k * nbw + (j - j0)] = Fm[j * nf + k] * C.F.D[f + j];
      const int64_t ncols = nf - j1;
      const int64_t CB = 64;
      const int64_t nblk = (ncols + CB - 1) / CB;
      if (inner_threads > 1 && ncols >= 256) {
        parallel_for(nblk, inner_threads, [&](int64_t b) {
          const int64_t k0 = j1 + b * CB, k1 = std::min(nf, k0 + CB);
          trailing_update(Fm, nf, nf, j0, j1, k0, k1, W.data(), nbw);
        });
      } else {
        trailing_update(Fm, nf, nf, j0, j1, j1, nf, W.data(), nbw);
      }
    }
  }
  // write L columns (rows ascending: the rest of the supernode, then U)
  for (int64_t t = 0; t < w; ++t) {
    const int32_t j = f + (int32_t)t;
    double* dst = C.F.Lx.data() + S.colptr[j];
    const double* src = Fm + t * nf;
    for (int64_t i = t + 1; i < nf; ++i) dst[i - t - 1] = src[i];
  }
  // update matrix for the parent
  if (u > 0 && C.snpar[s] >= 0) {
    std::vector<double>& Us = C.upd[s];
    Us.assign((size_t)(u * u), 0.0);
    for (int64_t b = 0; b < u; ++b)
      for (int64_t a = b; a < u; ++a) Us[b * u + a] = Fm[(w + b) * nf + (w + a)];
    C.updr[s].assign(r.begin() + w, r.end());
  }
  return OK;
}

}  // namespace

Status ldlt_numeric(const SymCsr& A, const std::vector<double>& gnd, const Symbolic& S, int threads,
                    Numeric& F) {
  const int32_t N = S.N;
  if (threads <= 0) threads = default_threads();
  // permuted strict-lower columns of A
  std::vector<int64_t> aptr(N + 1, 0);
  for (int32_t j = 0; j < N; ++j) {
    const int32_t r = S.perm[j];
    int64_t c = 0;
    for (int64_t p = A.ptr[r]; p < A.ptr[r + 1]; ++p) c += S.iperm[A.idx[p]] > j;
    aptr[j + 1] = aptr[j] + c;
  }
  std::vector<int32_t> arow(aptr[N]);
  std::vector<double> aval(aptr[N]), agnd(N);
  for (int32_t j = 0; j < N; ++j) {
    const int32_t r = S.perm[j];
    agnd[j] = gnd[r];
    int64_t q = aptr[j];
    for (int64_t p = A.ptr[r]; p < A.ptr[r + 1]; ++p) {
      const int32_t i = S.iperm[A.idx[p]];
      if (i > j) { arow[q] = i; aval[q++] = A.val[p]; }
    }
  }
  F.Lx.assign(S.colptr[N], 0.0);
  F.D.assign(N, 0.0);
  Ctx C{S, aptr, arow, aval, agnd, {}, {}, {}, {}, {}, F, {}, OK, {}};
  const int32_t ns = (int32_t)S.snptr.size() - 1;
  C.sn_of.resize(N);
  for (int32_t s = 0; s < ns; ++s)
    for (int32_t j = S.snptr[s]; j < S.snptr[s + 1]; ++j) C.sn_of[j] = s;
  C.snpar.assign(ns, -1);
  C.children.assign(ns, {});
  for (int32_t s = 0; s < ns; ++s) {
    const int32_t l = S.snptr[s + 1] - 1;
    if (S.parent[l] >= 0) {
      C.snpar[s] = C.sn_of[S.parent[l]];
      C.children[C.snpar[s]].push_back(s);
    }
  }
  C.upd.assign(ns, {});
  C.updr.assign(ns, {});
  // work per supernode and per subtree (supernodes are in postorder)
  std::vector<double> work(ns), sub(ns);
  double total = 0;
  for (int32_t s = 0; s < ns; ++s) {
    const double w = S.snptr[s + 1] - S.snptr[s];
    const int32_t l = S.snptr[s + 1] - 1;
    const double u = (double)(S.colptr[l + 1] - S.colptr[l]);
    work[s] = w * u * u + w * w * u + w * w * w / 3.0 + 4.0 * (w + u);
    total += work[s];
  }
  for (int32_t s = 0; s < ns; ++s) {
    sub[s] += work[s];
    if (C.snpar[s] >= 0) sub[C.snpar[s]] += sub[s];
  }
  // parallel subtrees: maximal subtrees with work below a share of the total
  const double cap = threads > 1 ? total / (4.0 * threads) : 1e300;
  std::vector<char> in_par(ns, 0);
  std::vector<int32_t> roots;
  for (int32_t s = ns - 1; s >= 0; --s) {
    const int32_t p = C.snpar[s];
    const bool parent_par = p >= 0 && in_par[p];
    if (parent_par) { in_par[s] = 1; continue; }
    if (sub[s] <= cap) { in_par[s] = 1; roots.push_back(s); }
  }
  std::sort(roots.begin(), roots.end(), [&](int32_t a, int32_t b) { return sub[a] > sub[b]; });
  // each root's subtree is the contiguous supernode range ending at it
  std::vector<int32_t> sfirst(ns);
  for (int32_t s = 0; s < ns; ++s) sfirst[s] = s;
  for (int32_t s = 0; s < ns; ++s)
    if (C.snpar[s] >= 0) sfirst[C.snpar[s]] = std::min(sfirst[C.snpar[s]], sfirst[s]);
  parallel_for((int64_t)roots.size(), threads, [&](int64_t k) {
    const int32_t r = roots[k];
    for (int32_t s = sfirst[r]; s <= r; ++s) {
      if (C.err != OK) return;
      Status st = factor_front(C, s, 1);
      if (st != OK) {
        std::lock_guard<std::mutex> g(C.err_mu);
        if (C.err == OK) C.err = st;
        return;
      }
    }
  });
  if (C.err != OK) { set_error(C.err_msg.empty() ? "factorization failed" : C.err_msg); return C.err; }
  for (int32_t s = 0; s < ns; ++s) {
    if (in_par[s]) continue;
    Status st = factor_front(C, s, threads);
    if (st != OK) { set_error(C.err_msg.empty() ? "factorization failed" : C.err_msg); return st; }
  }
  return OK;
}

}  // namespace peers
