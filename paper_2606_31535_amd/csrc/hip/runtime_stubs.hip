// Batched and served entry points (filled in by the batch/server runtime).
#include "../../../include/peers.h"
#include "../host/host.h"

using namespace peers;

extern "C" {
peers_status peers_server_start(peers_device, const peers_server_opts*, peers_server*) { return PEERS_E_UNSUPPORTED; }
peers_status peers_server_submit(peers_server, peers_factor, int64_t, const int32_t*, const int32_t*, double*,
                                 uint64_t*) { return PEERS_E_UNSUPPORTED; }
peers_status peers_server_wait(peers_server, uint64_t, int64_t, peers_status*) { return PEERS_E_UNSUPPORTED; }
peers_status peers_server_stats_get(peers_server, peers_server_stats*) { return PEERS_E_UNSUPPORTED; }
peers_status peers_server_stop(peers_server) { return PEERS_E_UNSUPPORTED; }
}
