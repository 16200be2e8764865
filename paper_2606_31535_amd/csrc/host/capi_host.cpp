// Host half of the C ABI: graph creation (ingest, ordering, symbolic, numeric),
// statistics, exports and error reporting.
#include <cstring>
#include <new>
#include <string>
#include <thread>

#include "../../../include/peers.h"
#include "graph_handle.h"

namespace peers {

namespace {
thread_local std::string g_err;
}

void set_error(const std::string& msg) { g_err = msg; }
const char* last_error() { return g_err.c_str(); }

int default_threads() {
  unsigned h = std::thread::hardware_concurrency();
  return h ? (int)std::min(h, 64u) : 4;
}

}  // namespace peers

using namespace peers;

extern "C" {

const char* peers_last_error(void) { return peers::last_error(); }

const char* peers_status_string(peers_status st) {
  switch (st) {
    case PEERS_OK: return "ok";
    case PEERS_E_INVALID_ARG: return "invalid argument";
    case PEERS_E_NODE_RANGE: return "node id out of range";
    case PEERS_E_WEIGHT: return "conductance not finite and positive";
    case PEERS_E_DISCONNECTED: return "graph not connected";
    case PEERS_E_NOT_SPD: return "grounded Laplacian not positive definite";
    case PEERS_E_HOST_OOM: return "host out of memory";
    case PEERS_E_OVER_BUDGET: return "device HBM budget exceeded";
    case PEERS_E_HIP: return "HIP runtime error";
    case PEERS_E_BUSY: return "server queue full";
    case PEERS_E_CANCELLED: return "cancelled";
    case PEERS_E_TIMEOUT: return "timed out";
    case PEERS_E_UNSUPPORTED: return "unsupported";
    default: return "internal error";
  }
}

peers_status peers_graph_create(int64_t n, int64_t m, const int32_t* eu, const int32_t* ev, const double* w,
                                int32_t ground, const peers_graph_opts* opts, peers_graph* out) {
  if (!out) { set_error("out is null"); return PEERS_E_INVALID_ARG; }
  *out = nullptr;
  peers_graph_opts o{};
  if (opts) o = *opts;
  try {
    auto* G = new GraphHandle();
    Status st = build_graph(n, m, eu, ev, w, ground, o, *G);
    if (st != OK) { delete G; return (peers_status)st; }
    *out = reinterpret_cast<peers_graph>(G);
    return PEERS_OK;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return PEERS_E_HOST_OOM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return PEERS_E_INTERNAL;
  }
}

peers_status peers_graph_stats_get(peers_graph g, peers_graph_stats* out) {
  if (!g || !out) { set_error("null argument"); return PEERS_E_INVALID_ARG; }
  const GraphHandle& G = *reinterpret_cast<GraphHandle*>(g);
  std::lock_guard<std::mutex> lk(G.num_mu);
  *out = G.stats;
  return PEERS_OK;
}

peers_status peers_graph_export_symbolic(peers_graph g, int32_t* perm, int32_t* parent, int64_t* colptr,
                                         int32_t* rowidx, int32_t* snptr) {
  if (!g) { set_error("null graph"); return PEERS_E_INVALID_ARG; }
  const GraphHandle& G = *reinterpret_cast<GraphHandle*>(g);
  const Symbolic& S = G.sym;
  const int32_t N = S.N;
  if (perm)
    for (int32_t k = 0; k < N; ++k) {
      const int32_t r = S.perm[k];
      perm[k] = r < G.ing.ground ? r : r + 1;  // reduced id -> original id
    }
  if (parent && N) std::memcpy(parent, S.parent.data(), sizeof(int32_t) * N);
  if (colptr) std::memcpy(colptr, S.colptr.data(), sizeof(int64_t) * (N + 1));
  if (rowidx && !S.rowidx.empty()) std::memcpy(rowidx, S.rowidx.data(), sizeof(int32_t) * S.rowidx.size());
  if (snptr) std::memcpy(snptr, S.snptr.data(), sizeof(int32_t) * S.snptr.size());
  return PEERS_OK;
}

peers_status peers_graph_export_factor(peers_graph g, double* Lx, double* D) {
  if (!g) { set_error("null graph"); return PEERS_E_INVALID_ARG; }
  const GraphHandle& G = *reinterpret_cast<GraphHandle*>(g);
  std::lock_guard<std::mutex> lk(G.num_mu);
  if (!G.numeric_ready) {
    set_error("the factor of this graph is formed on the device by its first peers_factor_upload");
    return PEERS_E_UNSUPPORTED;
  }
  if (Lx && !G.num.Lx.empty()) std::memcpy(Lx, G.num.Lx.data(), sizeof(double) * G.num.Lx.size());
  if (D && !G.num.D.empty()) std::memcpy(D, G.num.D.data(), sizeof(double) * G.num.D.size());
  return PEERS_OK;
}

void peers_graph_destroy(peers_graph g) { delete reinterpret_cast<GraphHandle*>(g); }

}  // extern "C"
