/*
 * peers.h -- C ABI of libpeers: exact effective resistances on MI355X (gfx950)
 * by the implicit-inverse sweep of Chen, Gan, Yang and Yu, "PEERS: A Parallel
 * and Exact Effective Resistance Solver via Implicit Inversion and Augmented
 * Symbolic Analysis".
 *
 * Problem statement (Section II-A, eq 1-4; Algorithm 8 inputs/outputs):
 *   a weighted undirected graph G = (V, E, w) with n nodes and m edges, a ground
 *   node g, and a query set of node pairs (u, v); the result for query k is the
 *   effective resistance R_uv = (e_u - e_v)^T L_r^{-1} (e_u - e_v), where L_r is
 *   the Laplacian L_G with g's row and column deleted and e_g := 0 (eq 4).
 *   The answer array is indexed by query number (the query graph's edge
 *   weights are answer indices, Section III-G).
 *
 * Method: L_r is ordered by nested dissection and factored on the host as
 *   P L_r P^T = L D L^T (Algorithm 8 step 1). The device never forms L^{-1}: the
 *   rows of Z = D^{-1/2} L^{-1} are produced implicitly by sweeping
 *   elimination-tree paths (eq 11, Section III-C) and every query accumulates
 *   its contributions (Z_ju - Z_jv)^2 as the rows pass (eq 12, Algorithm 7).
 *
 * Conventions for every function:
 *   - Return value: peers_status; 0 (PEERS_OK) on success, negative on error.
 *     Nothing aborts or throws. peers_last_error() gives a thread-local message.
 *   - Input arrays are borrowed for the duration of the call only; the library
 *     copies what it keeps. Handles are owned by the library and released only
 *     by the matching destroy/release/close/stop call.
 *   - Node ids are 0-based int32 in [0, n). Floating point is IEEE FP64
 *     throughout (host preparation and device sweep).
 *   - hip_stream is a hipStream_t (NULL = the null stream). Device calls are
 *     stream-ordered: they return after enqueueing; the caller synchronizes.
 */
#ifndef PEERS_H_
#define PEERS_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PEERS_OK = 0,
  PEERS_E_INVALID_ARG = -1,   /* null pointer, bad size, bad option */
  PEERS_E_NODE_RANGE = -2,    /* a node id (edge endpoint, ground, query endpoint) outside [0, n) */
  PEERS_E_WEIGHT = -3,        /* a conductance that is not finite and > 0 */
  PEERS_E_DISCONNECTED = -4,  /* the graph is not connected: L_r is singular */
  PEERS_E_NOT_SPD = -5,       /* a non-positive pivot in L D L^T */
  PEERS_E_HOST_OOM = -6,      /* host allocation failed */
  PEERS_E_OVER_BUDGET = -7,   /* the device HBM budget would be exceeded; nothing was admitted */
  PEERS_E_HIP = -8,           /* a HIP runtime error (message in peers_last_error) */
  PEERS_E_BUSY = -9,          /* the server queue is full */
  PEERS_E_CANCELLED = -10,    /* the request was cancelled or the server stopped */
  PEERS_E_TIMEOUT = -11,      /* a wait timed out; the request is still pending */
  PEERS_E_UNSUPPORTED = -12,  /* the operation is not available for this input */
  PEERS_E_INTERNAL = -99
} peers_status;

typedef struct peers_graph_s* peers_graph;   /* host: ordering, symbolic, L D L^T; immutable */
typedef struct peers_device_s* peers_device; /* one GPU with an HBM budget */
typedef struct peers_factor_s* peers_factor; /* one graph's sweep data resident in HBM */
typedef struct peers_server_s* peers_server; /* asynchronous request server */

/* Ordering choices (nested dissection, Section II-D, Lemma 2). */
enum {
  PEERS_ORDER_AUTO = 0,  /* coordinates if given, else graph bisection */
  PEERS_ORDER_COORD = 1, /* coordinate bisection; needs coords */
  PEERS_ORDER_GRAPH = 2, /* breadth-first level-structure bisection */
  PEERS_ORDER_GIVEN = 3  /* caller's elimination order (given_order) */
};

typedef struct {
  int32_t ordering;           /* PEERS_ORDER_*; 0 = auto */
  const double* coords;       /* optional n x 3 row-major point coordinates, original ids */
  const int32_t* given_order; /* PEERS_ORDER_GIVEN: n-1 original ids (ground excluded), elimination order */
  int32_t threads;            /* host threads for the factorization; 0 = all hardware threads */
  int32_t leaf_size;          /* nested-dissection leaf size; 0 = 64 */
  int32_t store_offsets_64;   /* 1: the sweep addresses the top store with 64-bit offsets even
                                 when 32-bit ones suffice (they are used above 4 GB); for tests */
  int32_t numeric_on_device;  /* 1: the numeric L D L^T is formed on the GPU by the first
                                 peers_factor_upload of the graph (bottom subtrees, then the
                                 top chains level by level with FP64 matrix-core products);
                                 until then peers_graph_export_factor returns UNSUPPORTED and
                                 t_numeric is 0; afterwards t_numeric is the device time.
                                 Uploads of such a graph from several threads run one at a
                                 time; the first forms the factor, the others reuse it */
  int32_t sweep_only;         /* 1: the sweep sums every row of every bottom query (no dense
                                 sums of the rows above bottom subtrees); for tests */
} peers_graph_opts;

typedef struct {
  int64_t n, m;            /* as given */
  int64_t N;               /* n - 1: order of L_r */
  int64_t nnz_l;           /* strict-lower nonzeros of L */
  int32_t height;          /* elimination-tree height h (root depth 1) */
  int32_t n_supernodes;    /* fundamental supernodes */
  int32_t max_sn_width;
  int32_t n_roots;         /* elimination-forest roots (> 1 when the ground is a cut node) */
  int64_t self_loops;
  double f_sweep;          /* sweep FMAs: sum over L_ki != 0 of depth(k) (the work of Theorem 4, Part I) */
  double acc_terms;        /* all-edge accumulation terms: sum over edges of depth(lower endpoint) */
  double t_ingest, t_order, t_symbolic, t_numeric; /* host preparation seconds */
} peers_graph_stats;

/* Build the host factor of a graph (Algorithm 8 step 1: ground, reorder, factor).
 * eu, ev: m endpoint ids; w: m conductances (> 0, finite). Self-loops are
 * accepted and ignored (they do not enter L_G, eq 1); parallel edges add.
 * ground: the grounded node g. opts may be NULL (defaults).
 * Errors: INVALID_ARG, NODE_RANGE, WEIGHT, DISCONNECTED, NOT_SPD, HOST_OOM. */
peers_status peers_graph_create(int64_t n, int64_t m, const int32_t* eu, const int32_t* ev,
                                const double* w, int32_t ground, const peers_graph_opts* opts,
                                peers_graph* out);
peers_status peers_graph_stats_get(peers_graph g, peers_graph_stats* out);
/* Symbolic structures (Lemma 1, Definition 2), caller-allocated from the stats:
 * perm[N]: original id eliminated i-th; parent[N] (-1 at roots); colptr[N+1] and
 * rowidx[nnz_l]: strict-lower pattern of L in CSC with rows ascending;
 * snptr[n_supernodes+1]: fundamental supernode column ranges. Any pointer may be NULL. */
peers_status peers_graph_export_symbolic(peers_graph g, int32_t* perm, int32_t* parent, int64_t* colptr,
                                         int32_t* rowidx, int32_t* snptr);
/* Numeric factor: Lx[nnz_l] aligned with rowidx, D[N] pivots. Either may be NULL.
 * Every pivot is formed as a sum of nonnegative terms (the node's conductance
 * to the ground plus its off-diagonal Schur magnitudes), so L and D carry
 * small relative errors entry by entry. Errors: UNSUPPORTED when the graph
 * was created with numeric_on_device and has not been uploaded yet. */
peers_status peers_graph_export_factor(peers_graph g, double* Lx, double* D);
void peers_graph_destroy(peers_graph g);

/* Open GPU `ordinal` (HIP device index). hbm_budget_bytes caps what factors
 * and per-call work buffers may hold (0 = 90% of the device memory). */
peers_status peers_device_open(int32_t ordinal, uint64_t hbm_budget_bytes, peers_device* out);
void peers_device_close(peers_device d);
/* Bytes currently held on the device by this library, and the budget. */
peers_status peers_device_usage(peers_device d, uint64_t* used, uint64_t* budget);
/* Change the HBM budget (0 = 90% of the device memory). Later reservations
 * (uploads, per-call workspaces, server batch arenas) are checked against the
 * new value; nothing already held is freed. Errors: OVER_BUDGET when the
 * library already holds more than the new budget (the budget is unchanged). */
peers_status peers_device_set_budget(peers_device d, uint64_t hbm_budget_bytes);

/* Upload a graph's sweep data to HBM (the factor in the device layout, the
 * schedule and the resident edge-query plan). Errors: OVER_BUDGET, HIP. */
peers_status peers_factor_upload(peers_device d, peers_graph g, void* hip_stream, peers_factor* out);
void peers_factor_release(peers_factor f);
/* Device bytes of a resident factor and its per-call workspace bound. */
peers_status peers_factor_footprint(peers_factor f, uint64_t* resident_bytes, uint64_t* workspace_bytes);

enum {
  PEERS_OUT_DEVICE = 1u,    /* R_out is a device pointer (else host memory) */
  PEERS_IN_DEVICE = 2u,     /* qu/qv are device pointers (peers_query only) */
  PEERS_SYNC = 4u,          /* synchronize the stream before returning */
  PEERS_PROFILE = 8u        /* record per-phase HIP event times (peers_factor_timings) */
};

/* Per-phase device times of the last sweep on this factor, recorded with HIP
 * events on the caller's stream when the sweep ran with PEERS_PROFILE set
 * (milliseconds; 0 for phases that did not run). */
typedef struct {
  double top_ms;      /* top tree: separator chains (dense blocks) */
  double bottom_ms;   /* bottom subtrees: path sweep with register path stacks */
  double finish_ms;   /* ordered window reduction, top-node queries, zero pairs, non-ancestor pairs */
  double total_ms;
  int32_t top_launches;
  int32_t bottom_launches;
  /* Algorithmic work of the all-edge sweep, per phase: 2 flops per FMA of
   * eq 11 (sum over L_ki != 0 of depth(k), restricted to the phase's columns)
   * plus 3 flops per accumulation term of eq 12 (one subtraction, one FMA:
   * sum over the pairs whose lower endpoint is in the phase of its depth). */
  double top_flops;     /* chain rows and chain-level products (eq 11 only) */
  double bottom_flops;  /* bottom subtrees: eq 11 and the fused eq 12 terms there */
  double top_bytes;     /* algorithmic HBM bytes of the top phase */
  double bottom_bytes;  /* algorithmic HBM bytes of the bottom phase */
  double finish_flops;  /* eq 12 terms of pairs whose lower endpoint is a top node */
  /* Host seconds spent when the factor was uploaded (peers_factor_upload):
   * the device layout of the factor (chains, blocks, subtree records), the
   * resident all-edge query plan, allocation and host-to-device copies, and
   * forming L_CC^{-1} and B_C = -L_{U,C} L_CC^{-1} on the device. */
  double t_layout_s, t_edge_plan_s, t_transfer_s, t_transform_s;
} peers_sweep_timings;
peers_status peers_factor_timings(peers_factor f, peers_sweep_timings* out);

/* Columns of Z = D^{-1/2} L^{-1} exactly as one sweep forms them (Section
 * III-C eq 11; Lemma 3 equates these implicit rows with triangular
 * substitution), for checking the sweep's intermediate values against an
 * independent inverse of the factor. For node x = nodes[i] (an original id,
 * not the ground) with elimination index p and depth dp (root depth 1), row i
 * of Z_out gets Z_out[i * ld + d] = Z[a_d(p), p] for d < dp, where a_d(p) is
 * p's ancestor at depth d + 1 (so d = dp - 1 holds the diagonal D_p^{-1/2}),
 * and zeros for dp <= d < ld. Columns of bottom-subtree nodes are staged by a
 * sweep that runs only the subtrees holding them; top columns come from the
 * top store. Z_out: host memory, k * ld doubles; ld at least the elimination
 * tree height. Synchronous.
 * Errors: INVALID_ARG (null, ld below the height, a ground node), NODE_RANGE,
 * OVER_BUDGET, HIP. */
peers_status peers_factor_export_columns(peers_factor f, int64_t k, const int32_t* nodes, int64_t ld,
                                         double* Z_out, void* hip_stream);

/* All-edge effective resistances (Section III-G, eq 12): R_out[e] for every
 * input edge e in input order (m values; self-loops give +0.0). */
peers_status peers_query_all_edges(peers_factor f, double* R_out, uint32_t flags, void* hip_stream);

/* Node-to-ground resistances (eq 4 with t = g; eq 12 cases 2-3): R_out[x] =
 * R_{x,g} = (L_r^{-1})_xx for every original id x, in id order (n values;
 * R_out[g] = +0.0). This is the "weak link" screen of a power grid grounded
 * at its supply: every node's resistance to the source. Their sum is
 * trace(L_r^{-1}). The plan (one pair per node, accumulated at that node
 * during the sweep) is built on the first call and kept with the factor.
 * Output host or device (PEERS_OUT_DEVICE); stream-ordered like
 * peers_query_all_edges. Errors: INVALID_ARG, OVER_BUDGET, HIP. */
peers_status peers_query_all_to_ground(peers_factor f, double* R_out, uint32_t flags, void* hip_stream);

/* Resistances for q arbitrary pairs given in original ids (eq 4 and eq 12):
 * pairs with u == v give +0.0, pairs with the ground use the grounded case.
 * A pair whose endpoints are ancestor-related in the elimination tree is
 * accumulated at its lower endpoint during the sweep; any other pair is split
 * at the lowest common ancestor c of its endpoints (rows above c are shared by
 * both columns, rows below are not):
 *   R = sum_{d < depth(c)} (z_u[d] - z_v[d])^2 + sum_{d >= depth(c)} (z_u[d]^2 + z_v[d]^2),
 * with the bottom-subtree columns staged during the sweep. Only the subtrees
 * that hold an endpoint are swept. qu, qv: q ids each (host, or device with
 * PEERS_IN_DEVICE); R_out: q doubles (host, or device with PEERS_OUT_DEVICE),
 * in query order. Blocks until the results are in R_out (host output) or
 * enqueued (device output without PEERS_SYNC).
 * Errors: NODE_RANGE for an id outside [0, n); OVER_BUDGET when the plan and
 * workspace do not fit the device budget; INVALID_ARG when the pairs whose
 * lower endpoint lies in a bottom subtree need more than 4 GB of query
 * records (about 178M such pairs; split the request). */
peers_status peers_query(peers_factor f, int64_t q, const int32_t* qu, const int32_t* qv, double* R_out,
                         uint32_t flags, void* hip_stream);

/* peers_query for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, kernels and results (bit for bit) as peers_query, but the
 * call allocates no device memory: its query plan, launch layout, partial
 * sums, staged columns and (for host output) result staging go into one
 * fixed 64 MiB device array that each GPU holds from first use until the
 * process ends. Calls through this entry point are serialized per GPU: each
 * holds the array until its work has finished, and returns only then
 * (host or device output). PEERS_PROFILE is not supported (INVALID_ARG).
 * Errors: as peers_query, and OVER_BUDGET when the request needs more than
 * the array holds (about 64 MiB of plan, partial sums and staging: e.g. tens
 * of thousands of edge pairs, or about a thousand non-ancestor pairs on a
 * 1M-node factor; split such requests or use peers_query). */
peers_status peers_query_noalloc(peers_factor f, int64_t q, const int32_t* qu, const int32_t* qv, double* R_out,
                                 uint32_t flags, void* hip_stream);

/* Spectral sparsification by effective resistances (Section II-B,
 * Algorithm 1): q independent draws of an edge with probability
 * p_e proportional to w_e R_e; an edge drawn c_e times gets the weight
 * c_e w_e / (q p_e). Inputs: m edges' conductances w and resistances R (host,
 * or device with PEERS_IN_DEVICE: typically R straight from
 * peers_query_all_edges with PEERS_OUT_DEVICE). Outputs: count[m] (int32)
 * and w_new[m] (0 for edges never drawn), host or device (PEERS_OUT_DEVICE).
 * How the draws are made, so that any implementation can reproduce them:
 *   k_e = floor(2^s * fl(w_e * R_e)), s = 61 - ceil(log2 m), K = sum of k_e,
 *   p_e = k_e / K (integer weights: the prefix sums are exact);
 *   draw i (0 <= i < q) takes the first output word x of Philox4x64-10
 *   (Salmon, Moraes, Dror, Shaw, SC 2011) at counter (i, 0, 0, 0) and key
 *   (seed, 0) and picks the edge e with C_{e-1} <= floor(x K / 2^64) < C_e,
 *   C the inclusive prefix sums of k;
 *   w_new_e = c_e * w_e * (K / (q * k_e)) in FP64, in that order.
 * Synchronous. Errors: INVALID_ARG (m < 1, q outside [0, 2^31 - 1], some
 * w_e R_e not finite or outside [0, 2], or every k_e zero), OVER_BUDGET,
 * HIP. */
peers_status peers_sparsify(peers_device d, int64_t m, const double* w, const double* R, int64_t q, uint64_t seed,
                            int32_t* count, double* w_new, uint32_t flags, void* hip_stream);

/* Batched form (many graphs of uneven size): the sweeps of nb resident
 * factors on one device run as one sequence of grouped launches, one launch
 * per step of the sweep covering that step of every factor, captured as a HIP
 * graph. Each result is bit-identical to the same query run alone
 * (peers_query / peers_query_all_edges on that factor).
 *   f[i]: distinct factors on device d; qu[i]/qv[i]: q[i] pairs of original
 *   ids (host, or device with PEERS_IN_DEVICE), or NULL for all edges of
 *   factor i (q[i] ignored, R_out[i] gets m_i values in edge order);
 *   R_out[i]: host, or device with PEERS_OUT_DEVICE.
 * The first call for a set of factors and outputs times the candidate
 * schedules of the bottom step (subtree work items to workgroups) and keeps
 * the fastest, remembered per device under a signature of the batch's
 * structure (factor sizes, tree height, top-tree shape and GEMM tiles per
 * chain level, bottom work items, query entries; for pair batches the
 * counts that depend on the pairs to within a factor of two), so batches of
 * the same structure skip the timing;
 * all-edge batches keep their captured graph and replay it on
 * later calls with the same factors and outputs (released factors and grown
 * workspaces drop it). Blocks until done unless every entry is all-edge with
 * device output and PEERS_SYNC is not set.
 * Errors: INVALID_ARG (null, duplicate factor, factor of another device, a
 * plan over the query-record limit of peers_query), NODE_RANGE, OVER_BUDGET. */
peers_status peers_batch_query(peers_device d, int32_t nb, const peers_factor* f, const int64_t* q,
                               const int32_t* const* qu, const int32_t* const* qv, double* const* R_out,
                               uint32_t flags, void* hip_stream);

/* What the last batch on this device ran. */
typedef struct {
  int32_t factors;
  int32_t stages;            /* grouped launches in the captured graph */
  int64_t bottom_items;      /* bottom work items (subtree task x 4 windows) */
  int32_t schedule;          /* bottom schedule chosen by the autotuner */
  int32_t candidates;
  double candidate_ms[8];    /* measured bottom-step time of each candidate */
  char schedule_name[96];
  int32_t graph_reused;      /* 1 if the call replayed a cached graph */
  double last_ms;            /* graph execution time of the call (0 if not synchronized) */
  int32_t schedule_cached;   /* 1 if the schedule came from the signature memo (no timing) */
  uint64_t signature;        /* structure signature the schedule is remembered under */
} peers_batch_info;
peers_status peers_batch_last_info(peers_device d, peers_batch_info* out);

/* Served form: thread-safe asynchronous requests with continuous batching. */
typedef struct {
  int32_t max_batch_pairs;  /* work cap per device batch (0 = 1<<20 pairs) */
  int32_t max_wait_us;      /* longest a request waits for batch-mates (0 = 200 us) */
  int32_t queue_capacity;   /* pending requests before PEERS_E_BUSY (0 = 4096) */
  int32_t streams;          /* device streams in flight (0 = 2) */
} peers_server_opts;

typedef struct {
  uint64_t submitted, completed, rejected, batches;
  double p50_us, p99_us, max_us;   /* submit -> result latency */
  double resistances_per_s;        /* completed pairs / busy wall time */
  uint64_t memory_waits;           /* batches put back in the queue until memory freed up */
  uint64_t arena_bytes;            /* device bytes the streams' batch arenas hold now */
  uint64_t pending;                /* requests waiting in the queue now */
} peers_server_stats;

/* Start a server on device d. One worker thread forms batches from the
 * queue; each batch runs on one of `streams` HIP streams with its own arena
 * (query plans, launch layout, partial slots, staging and results), reserved
 * against the device's HBM budget when the batch is formed. A batch that does
 * not fit while other batches run waits at the head of the queue until one
 * completes; idle streams give their arenas back to the budget. */
peers_status peers_server_start(peers_device d, const peers_server_opts* opts, peers_server* out);
/* Enqueue q pairs (original ids) against a resident factor. The ids are
 * copied. R_out (host, length q) is written by the library when the request's
 * batch completes: it must stay valid until peers_server_wait returns for the
 * ticket with a finished status, or until peers_server_cancel returns.
 * peers_factor_release waits for the factor's queued and running requests.
 * Errors: INVALID_ARG, NODE_RANGE, BUSY (queue_capacity requests already
 * wait), CANCELLED (the server is stopping). */
peers_status peers_server_submit(peers_server s, peers_factor f, int64_t q, const int32_t* qu,
                                 const int32_t* qv, double* R_out, uint64_t* ticket);
/* Wait for a ticket; timeout_us < 0 waits forever. On PEERS_OK, *result gets
 * the request's status (PEERS_OK: R_out holds the results; OVER_BUDGET: it
 * cannot fit even an idle device; CANCELLED) and the ticket is retired.
 * PEERS_E_TIMEOUT: the request is still queued or running and may still
 * write R_out; wait again or cancel it. Several threads may wait on one
 * ticket. */
peers_status peers_server_wait(peers_server s, uint64_t ticket, int64_t timeout_us, peers_status* result);
/* Cancel a request. After this returns the library never writes the
 * request's R_out: a queued request leaves the queue, a running one finishes
 * without its results being copied out; either way its status becomes
 * PEERS_E_CANCELLED (a request that had already finished keeps its status).
 * The ticket stays valid for peers_server_wait. Errors: INVALID_ARG (unknown
 * ticket). */
peers_status peers_server_cancel(peers_server s, uint64_t ticket);
peers_status peers_server_stats_get(peers_server s, peers_server_stats* out);
peers_status peers_server_stop(peers_server s);

const char* peers_status_string(peers_status st);
const char* peers_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PEERS_H_ */
