// Graph ingest and grounding (Section II-A, eq 1).
//
// L_G = sum over edges of w_ij (1_i - 1_j)(1_i - 1_j)^T: a self-loop adds
// nothing and parallel edges add up. Grounding node g deletes its row and
// column; the reduced matrix L_r is SPD iff the graph is connected. L_r is
// kept as its off-diagonal entries and, per node, its conductance to the
// ground (the row sum of L_r); the factorization forms every pivot from
// these, so the diagonal itself is never needed. Conductances to the ground
// are sums of edges of very different size and are accumulated with
// Neumaier's compensated summation.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "host.h"

namespace peers {

namespace {

struct Kahan {
  double s = 0, c = 0;
  void add(double x) {
    double t = s + x;
    if (std::fabs(s) >= std::fabs(x)) c += (s - t) + x; else c += (x - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};

int32_t find_root(std::vector<int32_t>& p, int32_t x) {
  while (p[x] != x) {
    p[x] = p[p[x]];
    x = p[x];
  }
  return x;
}

}  // namespace

Status ingest(int64_t n, int64_t m, const int32_t* eu, const int32_t* ev, const double* w,
              int32_t ground, Ingested& out) {
  if (n < 1 || m < 0 || n > (int64_t)INT32_MAX) { set_error("n must be in [1, 2^31) and m >= 0"); return E_INVALID_ARG; }
  if (m > 0 && (!eu || !ev || !w)) { set_error("null edge array"); return E_INVALID_ARG; }
  if (ground < 0 || ground >= n) { set_error("ground node out of range"); return E_NODE_RANGE; }
  for (int64_t e = 0; e < m; ++e) {
    if (eu[e] < 0 || eu[e] >= n || ev[e] < 0 || ev[e] >= n) {
      set_error("edge " + std::to_string(e) + " has an endpoint outside [0, n)");
      return E_NODE_RANGE;
    }
    if (!(w[e] > 0.0) || !std::isfinite(w[e])) {
      set_error("edge " + std::to_string(e) + " has a conductance that is not finite and positive");
      return E_WEIGHT;
    }
  }
  // connectivity of the original graph (the ground included)
  {
    std::vector<int32_t> p(n);
    std::iota(p.begin(), p.end(), 0);
    int64_t comps = n;
    for (int64_t e = 0; e < m; ++e) {
      int32_t a = find_root(p, eu[e]), b = find_root(p, ev[e]);
      if (a != b) { p[std::max(a, b)] = std::min(a, b); --comps; }
    }
    if (comps != 1) {
      set_error("graph is not connected (" + std::to_string(comps) + " components): the grounded Laplacian is singular");
      return E_DISCONNECTED;
    }
  }
  out.n = n;
  out.m = m;
  out.ground = ground;
  const int32_t N = (int32_t)(n - 1);
  out.N = N;
  auto red = [ground](int32_t x) { return x < ground ? x : x - 1; };

  std::vector<Kahan> gg(N);
  // off-diagonal coordinate list, both triangles
  std::vector<int64_t> cnt(N + 1, 0);
  int64_t self = 0;
  for (int64_t e = 0; e < m; ++e) {
    int32_t a = eu[e], b = ev[e];
    if (a == b) { ++self; continue; }
    if (a != ground && b != ground) { cnt[red(a) + 1]++; cnt[red(b) + 1]++; }
    if (a == ground) gg[red(b)].add(w[e]);
    if (b == ground) gg[red(a)].add(w[e]);
  }
  out.self_loops = self;
  out.gnd.resize(N);
  for (int32_t i = 0; i < N; ++i) out.gnd[i] = gg[i].value();
  for (int32_t i = 0; i < N; ++i) cnt[i + 1] += cnt[i];
  std::vector<int32_t> col(cnt[N]);
  std::vector<double> val(cnt[N]);
  std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
  for (int64_t e = 0; e < m; ++e) {
    int32_t a = eu[e], b = ev[e];
    if (a == b || a == ground || b == ground) continue;
    int32_t ra = red(a), rb = red(b);
    col[fill[ra]] = rb; val[fill[ra]++] = -w[e];
    col[fill[rb]] = ra; val[fill[rb]++] = -w[e];
  }
  // sort each row by column and merge parallel edges
  SymCsr& A = out.A;
  A.n = N;
  A.ptr.assign(N + 1, 0);
  A.idx.clear();
  A.val.clear();
  A.idx.reserve(cnt[N]);
  A.val.reserve(cnt[N]);
  std::vector<std::pair<int32_t, double>> row;
  for (int32_t i = 0; i < N; ++i) {
    row.clear();
    for (int64_t p = cnt[i]; p < cnt[i + 1]; ++p) row.emplace_back(col[p], val[p]);
    std::sort(row.begin(), row.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
    size_t k = 0;
    while (k < row.size()) {
      Kahan s;
      int32_t c = row[k].first;
      while (k < row.size() && row[k].first == c) s.add(row[k++].second);
      A.idx.push_back(c);
      A.val.push_back(s.value());
    }
    A.ptr[i + 1] = (int64_t)A.idx.size();
  }
  return OK;
}

}  // namespace peers
