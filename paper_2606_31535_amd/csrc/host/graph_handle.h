// The host graph handle: ingest + ordering + symbolic + numeric results and the
// statistics reported through the C ABI.
#pragma once

#include <mutex>

#include "../../../include/peers.h"
#include "host.h"

namespace peers {

struct GraphHandle {
  Ingested ing;
  Symbolic sym;
  Numeric num;
  peers_graph_stats stats{};
  std::vector<int32_t> eu, ev;  // the input edge list (all-edge queries in input order)
  bool store64 = false;         // peers_graph_opts::store_offsets_64
  bool sweep_only = false;      // peers_graph_opts::sweep_only
  // numeric factor formed on the device by the first upload (num is filled
  // then, from the device's result); num_mu orders that upload against other
  // uploads of the graph and against readers of num and stats
  bool numeric_on_device = false;
  bool numeric_ready = true;
  mutable std::mutex num_mu;
};

Status build_graph(int64_t n, int64_t m, const int32_t* eu, const int32_t* ev, const double* w, int32_t ground,
                   const peers_graph_opts& o, GraphHandle& G);

}  // namespace peers
