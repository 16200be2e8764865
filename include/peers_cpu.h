/*
 * peers_cpu.h -- the paper's own shared-memory scheme on the host CPU, for
 * comparison with the device sweep of peers.h. No device entry point calls
 * it: it exists so that the same host can time the paper's method beside
 * the GPU path on the same graph.
 *
 * Algorithm 8 (parallel row computation with compare-and-swap row claims,
 * thread-local answers summed at the end), Algorithm 6 (incremental
 * symbolic update by the depth-first search of Algorithm 3, numeric phase in
 * topological order, moves to the rows of ancestors with state rollback by
 * Algorithm 5), Algorithm 7 (query answers updated from each row). The factor
 * is the graph handle's host L D L^T; row j of Z = D^{-1/2} L^{-1} is formed
 * with v_j = D_j^{-1/2} and weights -L_st (the paper's 1/L_jj and
 * -L_st/L_tt for its L L^T factor).
 */
#ifndef PEERS_CPU_H_
#define PEERS_CPU_H_

#include "peers.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t threads;     /* threads used */
  int64_t rows;        /* rows computed (each row of Z exactly once: N) */
  double t_setup_s;    /* factor graph and query graph construction */
  double t_rows_s;     /* row computation and the final reduction */
} peers_cpu_stats;

/* R_out[k] for q pairs (qu[k], qv[k]) of original ids (pairs with u == v
 * give +0.0, pairs with the ground use eq 12's grounded cases). threads <= 0:
 * all hardware threads. Per-thread memory is O(n) (the listing's arrays).
 * The per-query sums run in whatever order the threads claimed the rows, so
 * results can differ from run to run in the last bits.
 * Errors: INVALID_ARG, NODE_RANGE, HOST_OOM. */
peers_status peers_cpu_query(peers_graph g, int64_t q, const int32_t* qu, const int32_t* qv, int32_t threads,
                             double* R_out, peers_cpu_stats* stats);

#ifdef __cplusplus
}
#endif

#endif /* PEERS_CPU_H_ */
