// Algorithm 8, step 1: ground the graph, reorder it, analyse and factor L_r.
// Each phase is timed separately (the paper's T_Chol covers ordering and
// factorization; here they are reported apart from the device sweep).
#include <algorithm>

#include "graph_handle.h"

namespace peers {

Status build_graph(int64_t n, int64_t m, const int32_t* eu, const int32_t* ev, const double* w, int32_t ground,
                   const peers_graph_opts& o, GraphHandle& G) {
  double t0 = now_s();
  Status st = ingest(n, m, eu, ev, w, ground, G.ing);
  if (st != OK) return st;
  G.eu.assign(eu, eu + m);
  G.ev.assign(ev, ev + m);
  const int32_t N = G.ing.N;
  double t1 = now_s();
  std::vector<int32_t> order;
  const int leaf = o.leaf_size > 0 ? o.leaf_size : 64;
  G.store64 = o.store_offsets_64 != 0;
  G.sweep_only = o.sweep_only != 0;
  int ordering = o.ordering;
  if (ordering == PEERS_ORDER_AUTO) ordering = o.coords ? PEERS_ORDER_COORD : PEERS_ORDER_GRAPH;
  if (ordering == PEERS_ORDER_COORD) {
    if (!o.coords) { set_error("coordinate ordering needs coords"); return E_INVALID_ARG; }
    std::vector<double> X((size_t)N * 3);
    for (int64_t x = 0; x < n; ++x) {
      if (x == ground) continue;
      const int64_t r = x < ground ? x : x - 1;
      for (int d = 0; d < 3; ++d) {
        const double c = o.coords[3 * x + d];
        if (!(c == c)) { set_error("coordinate is NaN"); return E_INVALID_ARG; }
        X[3 * r + d] = c;
      }
    }
    nd_order_coords(G.ing.A, X.data(), leaf, order);
  } else if (ordering == PEERS_ORDER_GRAPH) {
    nd_order_graph(G.ing.A, leaf, order);
  } else if (ordering == PEERS_ORDER_GIVEN) {
    if (!o.given_order) { set_error("given ordering is null"); return E_INVALID_ARG; }
    order.resize(N);
    for (int32_t k = 0; k < N; ++k) {
      const int32_t x = o.given_order[k];
      if (x < 0 || x >= n || x == ground) { set_error("given ordering has an invalid id"); return E_NODE_RANGE; }
      order[k] = x < ground ? x : x - 1;
    }
  } else {
    set_error("unknown ordering");
    return E_INVALID_ARG;
  }
  double t2 = now_s();
  st = symbolic_analyze(G.ing.A, order, G.sym);
  if (st != OK) return st;
  double t3 = now_s();
  G.numeric_on_device = o.numeric_on_device != 0;
  G.numeric_ready = !G.numeric_on_device;
  if (!G.numeric_on_device) {
    st = ldlt_numeric(G.ing.A, G.ing.gnd, G.sym, o.threads, G.num);
    if (st != OK) return st;
  }
  double t4 = now_s();

  peers_graph_stats& s = G.stats;
  s.n = n;
  s.m = m;
  s.N = N;
  s.nnz_l = G.sym.colptr.empty() ? 0 : G.sym.colptr[N];
  s.height = G.sym.height;
  s.n_supernodes = G.sym.snptr.empty() ? 0 : (int32_t)G.sym.snptr.size() - 1;
  s.max_sn_width = G.sym.max_sn_width;
  s.n_roots = 0;
  for (int32_t i = 0; i < N; ++i) s.n_roots += G.sym.parent[i] < 0;
  s.self_loops = G.ing.self_loops;
  s.f_sweep = G.sym.f_sweep;
  double acc = 0;
  for (int64_t e = 0; e < m; ++e) {
    if (eu[e] == ev[e]) continue;
    int32_t a = eu[e] == ground ? -1 : G.sym.iperm[eu[e] < ground ? eu[e] : eu[e] - 1];
    int32_t b = ev[e] == ground ? -1 : G.sym.iperm[ev[e] < ground ? ev[e] : ev[e] - 1];
    int32_t lo = (a < 0) ? b : (b < 0 ? a : std::min(a, b));
    acc += G.sym.depth[lo];
  }
  s.acc_terms = acc;
  s.t_ingest = t1 - t0;
  s.t_order = t2 - t1;
  s.t_symbolic = t3 - t2;
  s.t_numeric = t4 - t3;
  return OK;
}

}  // namespace peers
