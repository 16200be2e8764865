// Nested-dissection orderings (Section II-D, Definition 1 and Lemma 2).
//
// A separator C splits a node set into parts A and B with no edge between
// them; A and B are ordered first (recursively) and C last. With O(n^alpha)
// separators this bounds nnz(L) and the elimination-tree height h, which
// sets the cost of the implicit sweep (Theorem 4: W = O(n^alpha nnz(L))).
//
// Two separator sources:
//  * coordinates (meshes, point clouds): split at the median of the widest
//    coordinate; the separator is the smaller of the two boundary layers;
//  * the graph alone: a breadth-first level structure from a pseudo-peripheral
//    node, split at the median level, keeping only level nodes that touch the
//    next level.
// METIS is not available; these are written here.
#include <algorithm>
#include <array>
#include <numeric>

#include "host.h"

namespace peers {

namespace {

struct Task {
  bool emit;
  std::vector<int32_t> nodes;
};

void sort_by_coords(std::vector<int32_t>& v, const double* X) {
  std::sort(v.begin(), v.end(), [X](int32_t a, int32_t b) {
    for (int d = 0; d < 3; ++d) {
      double xa = X[3 * (int64_t)a + d], xb = X[3 * (int64_t)b + d];
      if (xa != xb) return xa < xb;
    }
    return a < b;
  });
}

}  // namespace

void nd_order_coords(const SymCsr& A, const double* X, int leaf, std::vector<int32_t>& order) {
  const int32_t N = A.n;
  order.clear();
  order.reserve(N);
  if (leaf < 4) leaf = 4;
  std::vector<int8_t> side(N, -1);
  std::vector<Task> stack;
  {
    Task t{false, std::vector<int32_t>(N)};
    std::iota(t.nodes.begin(), t.nodes.end(), 0);
    stack.push_back(std::move(t));
  }
  std::vector<double> vals;
  while (!stack.empty()) {
    Task t = std::move(stack.back());
    stack.pop_back();
    std::vector<int32_t>& S = t.nodes;
    if (t.emit) {
      order.insert(order.end(), S.begin(), S.end());
      continue;
    }
    if ((int)S.size() <= leaf) {
      sort_by_coords(S, X);
      order.insert(order.end(), S.begin(), S.end());
      continue;
    }
    std::array<double, 3> lo{1e300, 1e300, 1e300}, hi{-1e300, -1e300, -1e300};
    for (int32_t s : S)
      for (int d = 0; d < 3; ++d) {
        double x = X[3 * (int64_t)s + d];
        lo[d] = std::min(lo[d], x);
        hi[d] = std::max(hi[d], x);
      }
    int ax = 0;
    for (int d = 1; d < 3; ++d)
      if (hi[d] - lo[d] > hi[ax] - lo[ax]) ax = d;
    if (!(hi[ax] > lo[ax])) {
      sort_by_coords(S, X);
      order.insert(order.end(), S.begin(), S.end());
      continue;
    }
    vals.resize(S.size());
    for (size_t k = 0; k < S.size(); ++k) vals[k] = X[3 * (int64_t)S[k] + ax];
    size_t mid = (S.size() - 1) / 2;
    std::nth_element(vals.begin(), vals.begin() + mid, vals.end());
    double med = vals[mid];
    std::vector<int32_t> low, high;
    low.reserve(S.size() / 2 + 1);
    high.reserve(S.size() / 2 + 1);
    for (int32_t s : S) (X[3 * (int64_t)s + ax] <= med ? low : high).push_back(s);
    if (high.empty()) {
      low.clear();
      for (int32_t s : S) (X[3 * (int64_t)s + ax] < med ? low : high).push_back(s);
    }
    if (low.empty() || high.empty()) {
      sort_by_coords(S, X);
      order.insert(order.end(), S.begin(), S.end());
      continue;
    }
    for (int32_t s : low) side[s] = 0;
    for (int32_t s : high) side[s] = 1;
    std::vector<int32_t> lowB, lowI, highB, highI;
    for (int32_t s : low) {
      bool b = false;
      for (int64_t p = A.ptr[s]; p < A.ptr[s + 1] && !b; ++p) b = side[A.idx[p]] == 1;
      (b ? lowB : lowI).push_back(s);
    }
    for (int32_t s : high) {
      bool b = false;
      for (int64_t p = A.ptr[s]; p < A.ptr[s + 1] && !b; ++p) b = side[A.idx[p]] == 0;
      (b ? highB : highI).push_back(s);
    }
    for (int32_t s : S) side[s] = -1;
    Task sep{true, {}}, p1{false, {}}, p2{false, {}};
    if (lowB.size() <= highB.size()) {
      sep.nodes = std::move(lowB);
      p1.nodes = std::move(lowI);
      p2.nodes = std::move(high);
    } else {
      sep.nodes = std::move(highB);
      p1.nodes = std::move(low);
      p2.nodes = std::move(highI);
    }
    sort_by_coords(sep.nodes, X);
    stack.push_back(std::move(sep));
    if (!p2.nodes.empty()) stack.push_back(std::move(p2));
    if (!p1.nodes.empty()) stack.push_back(std::move(p1));
  }
}

void nd_order_graph(const SymCsr& A, int leaf, std::vector<int32_t>& order) {
  const int32_t N = A.n;
  order.clear();
  order.reserve(N);
  if (leaf < 4) leaf = 4;
  std::vector<int32_t> stamp(N, -1), level(N, -1), queue;
  int32_t cur = 0;
  std::vector<Task> stack;
  {
    Task t{false, std::vector<int32_t>(N)};
    std::iota(t.nodes.begin(), t.nodes.end(), 0);
    stack.push_back(std::move(t));
  }
  // breadth-first search inside the stamped set; returns the last node reached
  auto bfs = [&](int32_t src, int32_t st) -> int32_t {
    queue.clear();
    queue.push_back(src);
    level[src] = 0;
    int32_t lastv = src;
    for (size_t h = 0; h < queue.size(); ++h) {
      int32_t v = queue[h];
      lastv = v;
      for (int64_t p = A.ptr[v]; p < A.ptr[v + 1]; ++p) {
        int32_t u = A.idx[p];
        if (stamp[u] == st && level[u] < 0) {
          level[u] = level[v] + 1;
          queue.push_back(u);
        }
      }
    }
    return lastv;
  };
  while (!stack.empty()) {
    Task t = std::move(stack.back());
    stack.pop_back();
    std::vector<int32_t>& S = t.nodes;
    if (t.emit || (int)S.size() <= leaf) {
      order.insert(order.end(), S.begin(), S.end());
      continue;
    }
    const int32_t st = cur++;
    for (int32_t s : S) { stamp[s] = st; level[s] = -1; }
    // connected components of S: order each separately
    bfs(S[0], st);
    if (queue.size() < S.size()) {
      std::vector<int32_t> comp(queue.begin(), queue.end()), rest;
      for (int32_t s : S)
        if (level[s] < 0) rest.push_back(s);
      for (int32_t s : S) stamp[s] = -1;
      stack.push_back(Task{false, std::move(rest)});
      stack.push_back(Task{false, std::move(comp)});
      continue;
    }
    // pseudo-peripheral start: two sweeps
    int32_t a = S[0];
    for (int it = 0; it < 2; ++it) {
      for (int32_t s : S) level[s] = -1;
      a = bfs(a, st);
    }
    for (int32_t s : S) level[s] = -1;
    bfs(a, st);
    int32_t maxl = 0;
    for (int32_t s : S) maxl = std::max(maxl, level[s]);
    if (maxl < 2) {
      order.insert(order.end(), S.begin(), S.end());
      for (int32_t s : S) stamp[s] = -1;
      continue;
    }
    std::vector<int64_t> cnt(maxl + 2, 0);
    for (int32_t s : S) cnt[level[s]]++;
    int64_t acc = 0;
    int32_t ls = 1;
    for (int32_t l = 0; l <= maxl; ++l) {
      acc += cnt[l];
      if (2 * acc >= (int64_t)S.size()) { ls = l; break; }
    }
    ls = std::max(1, std::min(ls, maxl - 1));
    std::vector<int32_t> low, high, sep;
    for (int32_t s : S) {
      int32_t l = level[s];
      if (l < ls) low.push_back(s);
      else if (l > ls) high.push_back(s);
      else {
        bool touches = false;
        for (int64_t p = A.ptr[s]; p < A.ptr[s + 1] && !touches; ++p) {
          int32_t u = A.idx[p];
          touches = stamp[u] == st && level[u] == ls + 1;
        }
        (touches ? sep : low).push_back(s);
      }
    }
    for (int32_t s : S) stamp[s] = -1;
    stack.push_back(Task{true, std::move(sep)});
    if (!high.empty()) stack.push_back(Task{false, std::move(high)});
    if (!low.empty()) stack.push_back(Task{false, std::move(low)});
  }
}

}  // namespace peers
