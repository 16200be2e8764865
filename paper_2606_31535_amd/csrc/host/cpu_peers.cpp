// The paper's own shared-memory scheme on the host CPU, for comparison with
// the device sweep (it is not used by any device entry point).
//
// Algorithm 8: every thread walks the rows j = 0 .. N-1 and claims a row by
// compare-and-swap on a shared flag; a claimed row is computed by
// Algorithm 6 with thread-local state (visitation marks vis, in-degrees d,
// saved in-degrees ld, row values v, a queue), its query contributions are
// added to the thread's own answers by Algorithm 7, and the answers of all
// threads are summed at the end.
//
// Algorithm 6 for row j, with the state (vis, d) holding the reach set of a
// row whose reach set is contained in S_j:
//   1. symbolic update (Algorithm 3): depth-first search from j over the
//      factor graph H (edge s -> t for every L_st != 0, s > t), counting each
//      edge into d_t and expanding only nodes not yet visited;
//   2. numeric phase in topological order: v_j = D_j^{-1/2} (1 / L_jj of the
//      paper's L L^T factor), and for each dequeued s and edge s -> t,
//      v_t += (-L_st) v_s (the paper's w~_{s,t} for a unit L), recording the
//      in-degree before the decrement in ld_t and queueing t when d_t reaches
//      zero; afterwards d is restored from ld;
//   3. for every edge i -> j (i in the pattern of column j: an ancestor of j
//      whose reach set contains S_j) whose row is still unclaimed, claim it,
//      compute it from the current state, and roll the state back to S_j by
//      Algorithm 5 (remove i, decrement the in-degrees of its targets, and
//      remove recursively every node whose in-degree drops to zero, except j).
// Algorithm 7 for row j: flag the nodes of S_j; for every query (u, w) at a
// flagged node u, add (v_u - v_w)^2 if w is flagged and u > w, or v_u^2 if w
// is not flagged (w outside S_j, or the ground). Flags and row values are
// cleared after the row (the listing leaves that implicit).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

#include "../../../include/peers_cpu.h"
#include "graph_handle.h"

namespace peers {

namespace {

struct Shared {
  int32_t N = 0;
  // H out-edges of s: columns t < s with L_st != 0, and -L_st (rows of L)
  std::vector<int64_t> optr;
  std::vector<int32_t> ocol;
  std::vector<double> oval;
  // H in-edges of j: rows i > j with L_ij != 0 (the pattern of column j)
  const int64_t* colptr = nullptr;
  const int32_t* rowidx = nullptr;
  std::vector<double> isd;  // D^{-1/2}
  // query graph: for node u, its queries (partner node or -1, answer index)
  std::vector<int64_t> qptr;
  std::vector<int32_t> qadj;
  std::vector<int64_t> qid;
  int64_t q = 0;
  std::unique_ptr<std::atomic<int32_t>[]> cal;  // -1 = unclaimed, else the thread
};

struct Local {
  std::vector<uint8_t> vis, c;
  std::vector<int32_t> d, ld, queue, stack;
  std::vector<int64_t> it;
  std::vector<double> v, ans;
  int64_t rows = 0;
};

// Algorithm 3 from node j on the persisted state (explicit stack).
void symbolic_dfs(const Shared& S, Local& L, int32_t j) {
  if (L.vis[j]) return;
  L.vis[j] = 1;
  L.stack.clear();
  L.stack.push_back(j);
  L.it[j] = S.optr[j];
  while (!L.stack.empty()) {
    const int32_t i = L.stack.back();
    if (L.it[i] == S.optr[i + 1]) {
      L.stack.pop_back();
      continue;
    }
    const int32_t k = S.ocol[L.it[i]++];
    L.d[k]++;
    if (!L.vis[k]) {
      L.vis[k] = 1;
      L.it[k] = S.optr[k];
      L.stack.push_back(k);
    }
  }
}

// Algorithm 5: remove i and everything only it reaches, stopping at o.
void rollback(const Shared& S, Local& L, int32_t i, int32_t o) {
  L.stack.clear();
  L.stack.push_back(i);
  L.vis[i] = 0;
  while (!L.stack.empty()) {
    const int32_t x = L.stack.back();
    L.stack.pop_back();
    for (int64_t p = S.optr[x]; p < S.optr[x + 1]; ++p) {
      const int32_t k = S.ocol[p];
      if (--L.d[k] == 0 && k != o) {
        L.vis[k] = 0;
        L.stack.push_back(k);
      }
    }
  }
}

// Algorithm 6 (steps 1 and 2) and Algorithm 7 for row j.
void row(const Shared& S, Local& L, int32_t j) {
  symbolic_dfs(S, L, j);
  int64_t head = 0, tail = 0;
  L.queue[0] = j;
  L.v[j] = S.isd[j];
  while (head <= tail) {
    const int32_t s = L.queue[head++];
    const double vs = L.v[s];
    for (int64_t p = S.optr[s]; p < S.optr[s + 1]; ++p) {
      const int32_t t = S.ocol[p];
      L.v[t] += S.oval[p] * vs;
      L.ld[t] = std::max(L.ld[t], L.d[t]);
      if (--L.d[t] == 0) L.queue[++tail] = t;
    }
  }
  for (int64_t x = 0; x <= tail; ++x) {
    const int32_t u = L.queue[x];
    L.d[u] = L.ld[u];
    L.ld[u] = 0;
    L.c[u] = 1;
  }
  // Algorithm 7
  for (int64_t x = 0; x <= tail; ++x) {
    const int32_t u = L.queue[x];
    const double vu = L.v[u];
    for (int64_t p = S.qptr[u]; p < S.qptr[u + 1]; ++p) {
      const int32_t w = S.qadj[p];
      if (w >= 0 && L.c[w]) {
        if (u > w) {
          const double t = vu - L.v[w];
          L.ans[S.qid[p]] += t * t;
        }
      } else {
        L.ans[S.qid[p]] += vu * vu;
      }
    }
  }
  for (int64_t x = 0; x <= tail; ++x) {
    const int32_t u = L.queue[x];
    L.c[u] = 0;
    L.v[u] = 0.0;
  }
  L.rows++;
}

// Algorithm 6 with its step 3: the ancestors reached from j through H's
// in-edges, claimed and computed incrementally, each rolled back to S_j.
void row_and_ancestors(Shared& S, Local& L, int32_t j, int32_t p) {
  struct Frame { int32_t j; int64_t e; };
  std::vector<Frame> st;
  row(S, L, j);
  st.push_back({j, S.colptr[j]});
  while (!st.empty()) {
    Frame& f = st.back();
    if (f.e == S.colptr[f.j + 1]) {
      const int32_t done = f.j;
      st.pop_back();
      if (!st.empty()) rollback(S, L, done, st.back().j);
      continue;
    }
    const int32_t i = S.rowidx[f.e++];
    int32_t expect = -1;
    if (S.cal[i].load(std::memory_order_relaxed) == -1 &&
        S.cal[i].compare_exchange_strong(expect, p, std::memory_order_acq_rel)) {
      row(S, L, i);
      st.push_back({i, S.colptr[i]});
    }
  }
  // back to the empty state: the row j itself
  rollback(S, L, j, -1);
}

}  // namespace

}  // namespace peers

using namespace peers;

extern "C" {

peers_status peers_cpu_query(peers_graph g, int64_t q, const int32_t* qu, const int32_t* qv, int32_t threads,
                             double* R_out, peers_cpu_stats* stats) {
  if (!g || q < 0 || (q > 0 && (!qu || !qv || !R_out))) { set_error("null argument"); return PEERS_E_INVALID_ARG; }
  const GraphHandle& G = *reinterpret_cast<GraphHandle*>(g);
  std::lock_guard<std::mutex> lk(G.num_mu);  // the factor stays as it is while it is read
  if (!G.numeric_ready) {
    set_error("the factor of this graph is formed on the device by its first peers_factor_upload");
    return PEERS_E_UNSUPPORTED;
  }
  const double t0 = now_s();
  try {
    Shared S;
    const int32_t N = G.sym.N;
    S.N = N;
    S.q = q;
    const int64_t nnz = G.sym.colptr[N];
    // rows of L (H out-edges), by counting sort over the column storage
    S.optr.assign(N + 1, 0);
    for (int64_t p = 0; p < nnz; ++p) S.optr[G.sym.rowidx[p] + 1]++;
    for (int32_t i = 0; i < N; ++i) S.optr[i + 1] += S.optr[i];
    S.ocol.resize(nnz);
    S.oval.resize(nnz);
    {
      std::vector<int64_t> fill(S.optr.begin(), S.optr.end() - 1);
      for (int32_t t = 0; t < N; ++t)
        for (int64_t p = G.sym.colptr[t]; p < G.sym.colptr[t + 1]; ++p) {
          const int32_t s = G.sym.rowidx[p];
          S.ocol[fill[s]] = t;
          S.oval[fill[s]++] = -G.num.Lx[p];
        }
    }
    S.colptr = G.sym.colptr.data();
    S.rowidx = G.sym.rowidx.data();
    S.isd.resize(N);
    for (int32_t i = 0; i < N; ++i) S.isd[i] = 1.0 / std::sqrt(G.num.D[i]);
    // query graph in elimination indices (ground -1)
    const int32_t gnd = G.ing.ground;
    auto pidx = [&](int32_t x) -> int32_t { return x == gnd ? -1 : G.sym.iperm[x < gnd ? x : x - 1]; };
    std::vector<int32_t> a(q), b(q);
    S.qptr.assign(N + 1, 0);
    for (int64_t k = 0; k < q; ++k) {
      if (qu[k] < 0 || qu[k] >= G.ing.n || qv[k] < 0 || qv[k] >= G.ing.n) {
        set_error("query " + std::to_string(k) + " has a node id outside [0, n)");
        return PEERS_E_NODE_RANGE;
      }
      a[k] = pidx(qu[k]);
      b[k] = pidx(qv[k]);
      if (qu[k] == qv[k]) continue;  // R = 0
      if (a[k] >= 0) S.qptr[a[k] + 1]++;
      if (b[k] >= 0) S.qptr[b[k] + 1]++;
    }
    for (int32_t i = 0; i < N; ++i) S.qptr[i + 1] += S.qptr[i];
    S.qadj.resize(S.qptr[N]);
    S.qid.resize(S.qptr[N]);
    {
      std::vector<int64_t> fill(S.qptr.begin(), S.qptr.end() - 1);
      for (int64_t k = 0; k < q; ++k) {
        if (qu[k] == qv[k]) continue;
        if (a[k] >= 0) { S.qadj[fill[a[k]]] = b[k]; S.qid[fill[a[k]]++] = k; }
        if (b[k] >= 0) { S.qadj[fill[b[k]]] = a[k]; S.qid[fill[b[k]]++] = k; }
      }
    }
    S.cal.reset(new std::atomic<int32_t>[N > 0 ? N : 1]);
    for (int32_t i = 0; i < N; ++i) S.cal[i].store(-1, std::memory_order_relaxed);
    const int P = threads > 0 ? threads : default_threads();
    std::vector<Local> locals(P);
    const double t1 = now_s();
    auto worker = [&](int p) {
      Local& L = locals[p];
      L.vis.assign(N, 0);
      L.c.assign(N, 0);
      L.d.assign(N, 0);
      L.ld.assign(N, 0);
      L.queue.assign(N > 0 ? N : 1, 0);
      L.it.assign(N, 0);
      L.v.assign(N, 0.0);
      L.ans.assign(q, 0.0);
      for (int32_t j = 0; j < N; ++j) {
        int32_t expect = -1;
        if (S.cal[j].load(std::memory_order_relaxed) != -1) continue;
        if (!S.cal[j].compare_exchange_strong(expect, p, std::memory_order_acq_rel)) continue;
        row_and_ancestors(S, L, j, p);
      }
    };
    std::vector<std::thread> th;
    for (int p = 1; p < P; ++p) th.emplace_back(worker, p);
    worker(0);
    for (auto& t : th) t.join();
    // Algorithm 8 step 3: the threads' answers, summed in thread order
    for (int64_t k = 0; k < q; ++k) {
      double s = 0.0;
      for (int p = 0; p < P; ++p) s += locals[p].ans[k];
      R_out[k] = s;
    }
    const double t2 = now_s();
    if (stats) {
      *stats = peers_cpu_stats{};
      stats->threads = P;
      stats->t_setup_s = t1 - t0;
      stats->t_rows_s = t2 - t1;
      for (int p = 0; p < P; ++p) stats->rows += locals[p].rows;
    }
    return PEERS_OK;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return PEERS_E_HOST_OOM;
  }
}

}  // extern "C"
