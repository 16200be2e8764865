// Symbolic analysis of the factor (Lemma 1, Definition 2, Theorems 1-2).
//
// For the permuted grounded Laplacian A = P L_r P^T = L D L^T:
//  * the elimination tree: parent(i) = min{k > i : L_ki != 0};
//  * a postorder of that tree (children in ascending index), so every subtree
//    is the contiguous index range [first(j), j]. Because edges of the factor
//    graph H run from a row to strictly smaller indices (Theorem 1) and row j
//    reaches exactly subtree(j) (Lemma 1, Theorem 2), descending index order
//    inside [first(j), j] is a topological order of row j's traversal;
//  * the strict-lower pattern of L by row subtrees: row k of L holds every
//    node on the tree paths from i (A_ki != 0, i < k) up to k;
//  * depths (root depth 1), fundamental supernodes (consecutive columns i,
//    i+1 with parent(i) = i+1, i+1 having one child, and
//    colcount(i) = colcount(i+1) + 1) and the sweep's FMA count
//    F = sum over L_ki != 0 of depth(k).
#include <algorithm>
#include <numeric>

#include "host.h"

namespace peers {

namespace {

// rows[new k] = new i < k with A_ki != 0
void lower_rows(const SymCsr& A, const std::vector<int32_t>& perm, const std::vector<int32_t>& iperm,
                std::vector<int64_t>& ptr, std::vector<int32_t>& idx) {
  const int32_t N = A.n;
  ptr.assign(N + 1, 0);
  for (int32_t k = 0; k < N; ++k) {
    int32_t r = perm[k];
    int64_t c = 0;
    for (int64_t p = A.ptr[r]; p < A.ptr[r + 1]; ++p) c += iperm[A.idx[p]] < k;
    ptr[k + 1] = ptr[k] + c;
  }
  idx.resize(ptr[N]);
  for (int32_t k = 0; k < N; ++k) {
    int32_t r = perm[k];
    int64_t q = ptr[k];
    for (int64_t p = A.ptr[r]; p < A.ptr[r + 1]; ++p) {
      int32_t i = iperm[A.idx[p]];
      if (i < k) idx[q++] = i;
    }
  }
}

}  // namespace

void etree_of(const SymCsr& A, const std::vector<int32_t>& perm, const std::vector<int32_t>& iperm,
              std::vector<int32_t>& parent) {
  const int32_t N = A.n;
  std::vector<int64_t> ptr;
  std::vector<int32_t> idx;
  lower_rows(A, perm, iperm, ptr, idx);
  parent.assign(N, -1);
  std::vector<int32_t> anc(N, -1);
  for (int32_t k = 0; k < N; ++k) {
    for (int64_t p = ptr[k]; p < ptr[k + 1]; ++p) {
      int32_t r = idx[p];
      while (r != -1 && r < k) {
        int32_t nxt = anc[r];
        anc[r] = k;
        if (nxt == -1) { parent[r] = k; break; }
        r = nxt;
      }
    }
  }
}

Status symbolic_analyze(const SymCsr& A, const std::vector<int32_t>& order, Symbolic& S) {
  const int32_t N = A.n;
  S.N = N;
  if ((int32_t)order.size() != N) { set_error("ordering has the wrong length"); return E_INVALID_ARG; }
  std::vector<int32_t> iperm0(N, -1);
  for (int32_t k = 0; k < N; ++k) {
    int32_t r = order[k];
    if (r < 0 || r >= N || iperm0[r] != -1) { set_error("ordering is not a permutation"); return E_INVALID_ARG; }
    iperm0[r] = k;
  }
  std::vector<int32_t> parent0;
  etree_of(A, order, iperm0, parent0);
  // postorder: children in ascending index, roots in ascending index
  std::vector<int32_t> head(N, -1), next(N, -1), post;
  post.reserve(N);
  for (int32_t i = N - 1; i >= 0; --i) {
    if (parent0[i] >= 0) { next[i] = head[parent0[i]]; head[parent0[i]] = i; }
  }
  std::vector<int32_t> stk;
  for (int32_t r = 0; r < N; ++r) {
    if (parent0[r] != -1) continue;
    stk.push_back(r);
    while (!stk.empty()) {
      int32_t v = stk.back();
      int32_t c = head[v];
      if (c != -1) {
        head[v] = next[c];
        stk.push_back(c);
      } else {
        stk.pop_back();
        post.push_back(v);
      }
    }
  }
  S.perm.resize(N);
  for (int32_t k = 0; k < N; ++k) S.perm[k] = order[post[k]];
  S.iperm.assign(N, -1);
  for (int32_t k = 0; k < N; ++k) S.iperm[S.perm[k]] = k;
  etree_of(A, S.perm, S.iperm, S.parent);

  // factor pattern by row subtrees: count, then fill (rows ascending per column)
  std::vector<int64_t> rptr;
  std::vector<int32_t> ridx;
  lower_rows(A, S.perm, S.iperm, rptr, ridx);
  std::vector<int32_t> mark(N, -1);
  std::vector<int64_t> cnt(N, 0);
  for (int32_t k = 0; k < N; ++k) {
    mark[k] = k;
    for (int64_t p = rptr[k]; p < rptr[k + 1]; ++p) {
      for (int32_t i = ridx[p]; mark[i] != k; i = S.parent[i]) {
        cnt[i]++;
        mark[i] = k;
      }
    }
  }
  S.colptr.assign(N + 1, 0);
  for (int32_t i = 0; i < N; ++i) S.colptr[i + 1] = S.colptr[i] + cnt[i];
  S.rowidx.resize(S.colptr[N]);
  std::vector<int64_t> fill(S.colptr.begin(), S.colptr.end() - 1);
  std::fill(mark.begin(), mark.end(), -1);
  for (int32_t k = 0; k < N; ++k) {
    mark[k] = k;
    for (int64_t p = rptr[k]; p < rptr[k + 1]; ++p) {
      for (int32_t i = ridx[p]; mark[i] != k; i = S.parent[i]) {
        S.rowidx[fill[i]++] = k;
        mark[i] = k;
      }
    }
  }
  // depths, first, supernodes, sweep cost
  S.depth.assign(N, 0);
  S.height = 0;
  for (int32_t i = N - 1; i >= 0; --i) {
    S.depth[i] = S.parent[i] < 0 ? 1 : S.depth[S.parent[i]] + 1;
    S.height = std::max(S.height, S.depth[i]);
  }
  S.first.resize(N);
  std::iota(S.first.begin(), S.first.end(), 0);
  for (int32_t i = 0; i < N; ++i)
    if (S.parent[i] >= 0) S.first[S.parent[i]] = std::min(S.first[S.parent[i]], S.first[i]);
  std::vector<int32_t> nchild(N, 0);
  for (int32_t i = 0; i < N; ++i)
    if (S.parent[i] >= 0) nchild[S.parent[i]]++;
  S.snptr.clear();
  S.snptr.push_back(0);
  for (int32_t i = 0; i + 1 < N; ++i) {
    bool join = S.parent[i] == i + 1 && nchild[i + 1] == 1 && cnt[i] == cnt[i + 1] + 1;
    if (!join) S.snptr.push_back(i + 1);
  }
  if (N > 0) S.snptr.push_back(N);
  S.max_sn_width = 0;
  for (size_t s = 0; s + 1 < S.snptr.size(); ++s)
    S.max_sn_width = std::max(S.max_sn_width, S.snptr[s + 1] - S.snptr[s]);
  double f = 0;
  for (int64_t p = 0; p < S.colptr[N]; ++p) f += S.depth[S.rowidx[p]];
  S.f_sweep = f;
  return OK;
}

}  // namespace peers
