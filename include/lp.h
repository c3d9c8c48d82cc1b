/*
 * lp.h - C ABI of the MI355X (gfx950) neighbourhood-based link predictor.
 *
 * Implements the prediction of Sahu, "A Fast Parallel Approach for
 * Neighborhood-based Link Prediction by Disregarding Large Hubs"
 * (arXiv 2401.11415): for every source vertex a, two-hop accumulation of the
 * common neighbours it shares with each second-order vertex c (Section 4.1),
 * optionally disregarding intermediates whose degree exceeds a hub limit
 * (DLH, Section 4.2), scoring by one of nine local measures (Section 3.1),
 * and selection of the top-scoring predicted edges (Section 4.1.6 and the
 * merging phase of Algorithm 1).
 *
 * Conventions for every entry point
 *  - Vertex ids are int32 in [0, n); a graph is simple and undirected, given
 *    as CSR with every row sorted ascending and both arc directions present.
 *  - Every call returns an lp_status; on failure it writes no partial output,
 *    sets *out_count (where there is one) to 0, and records a message that
 *    lp_last_error() returns on the same thread.
 *  - "Device or host pointer": either memory type is accepted; the library
 *    checks with hipPointerGetAttributes and copies as needed.
 *  - Work is enqueued on hip_stream (a hipStream_t; NULL = the null stream).
 *    lp_predict and lp_query return after the stream has finished the call.
 *  - A graph is not thread-safe: a second call on the same graph while one is
 *    running on another thread returns LP_ERR_BUSY.
 *  - No C++ exception crosses this boundary.
 */
#ifndef LP_H
#define LP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lp_graph lp_graph; /* opaque; owns all device memory of one graph */

typedef enum {
  LP_OK = 0,
  LP_ERR_INVALID_ARGUMENT = 1, /* a scalar argument or pointer is out of its domain */
  LP_ERR_INVALID_GRAPH = 2,    /* the CSR violates the conventions above */
  LP_ERR_OUT_OF_MEMORY = 3,    /* device memory exhausted; the graph stays usable */
  LP_ERR_DEVICE = 4,           /* a HIP runtime call failed */
  LP_ERR_BUSY = 5              /* the graph is in use by another thread */
} lp_status;

/* The nine measures of Section 3.1 (equations CN ... RA).  With h the number
 * of explored common neighbours and d_v the observed degree:
 *   CN  h                      JC  h / (d_a + d_c - h)   (union, Section 4.1.2)
 *   SI  h / (d_a + d_c)        SC  h / sqrt(d_a * d_c)
 *   HP  h / min(d_a, d_c)      HD  h / max(d_a, d_c)
 *   LHN h / (d_a * d_c)
 *   AA  sum over explored common neighbours b of 1 / ln(d_b)
 *   RA  sum over explored common neighbours b of 1 / d_b
 * Scores are evaluated in FP64 and returned rounded to FP32 (Section 5.1:
 * 32-bit floats for scores). */
typedef enum {
  LP_CN = 0, LP_JC = 1, LP_SI = 2, LP_SC = 3, LP_HP = 4,
  LP_HD = 5, LP_LHN = 6, LP_AA = 7, LP_RA = 8
} lp_measure;

/* hub_limit value meaning "no limit": every intermediate is explored, i.e.
 * the improved baseline IBase (Section 4.4 treats IBase as L_H = infinity). */
#define LP_HUB_NONE INT64_MAX

/* lp_graph_create flags */
#define LP_VALIDATE 1u /* check sortedness, duplicates, self-loops and symmetry */

/*
 * Copy a CSR graph to the device and build the resident structures
 * (degree-ordered relabelling and per-arc two-hop bookkeeping).  The input is
 * the observed graph of Section 5.1: simple and undirected (self-loops
 * removed, each edge present in both directions) with 32-bit vertex ids.
 *   n        number of vertices, 0 <= n <= INT32_MAX.
 *   offsets  n+1 int64, offsets[0] == 0, non-decreasing, offsets[n] = arcs
 *            (twice the undirected edge count, < 2^32).  Device or host pointer.
 *   indices  offsets[n] int32 neighbour ids.  Device or host pointer.
 *   flags    0 or LP_VALIDATE.
 *   out      receives the new graph; unchanged on failure.
 * Ownership: the inputs are copied; the caller keeps them.  Offsets and index
 * ranges are always checked (LP_ERR_INVALID_GRAPH); LP_VALIDATE adds the
 * semantic checks.  Results on a graph that breaks the conventions without
 * LP_VALIDATE are unspecified (but memory-safe).
 */
lp_status lp_graph_create(int64_t n, const int64_t *offsets, const int32_t *indices,
                          uint32_t flags, lp_graph **out);

/* Release every device allocation of g.  NULL is accepted. */
lp_status lp_graph_destroy(lp_graph *g);

/* Number of vertices and arcs, and the device bytes the graph holds. */
lp_status lp_graph_info(const lp_graph *g, int64_t *n, int64_t *arcs, int64_t *max_degree,
                        int64_t *device_bytes);

/*
 * Whole-graph link prediction (Algorithm 1, predictLinks).
 *   m                measure.
 *   hub_limit        L_H: an intermediate b is explored iff d_b <= hub_limit
 *                    (Section 4.2.1); LP_HUB_NONE gives IBase.  Must be >= 0.
 *   k                N_P, the maximum number of edges to predict, >= 0.
 *   score_threshold  S_th: only pairs whose FP32 score is strictly greater are
 *                    predicted (Algorithm 1, scoring phase); finite and >= 0.
 *   out_a, out_c     k int32 each: predicted edges (a, c) with a < c, original
 *                    vertex ids.  Device or host pointers, caller-owned.
 *   out_score        k float: FP32 scores.  Device or host pointer.
 *   out_count        host pointer; receives k' = min(k, number of candidates).
 * Candidates are unordered non-adjacent pairs with at least one explored common
 * neighbour (Sections 4.1.1 and 4.1.4).  Rows are written in the order
 * (score desc, a asc, c asc), which fixes one of the equally correct answers
 * when scores tie (Section 4.2.3 notes that ties make the choice arbitrary).
 */
lp_status lp_predict(lp_graph *g, lp_measure m, int64_t hub_limit, int64_t k,
                     float score_threshold, int32_t *out_a, int32_t *out_c, float *out_score,
                     int64_t *out_count, void *hip_stream);

/*
 * Per-vertex recommendation (the ranked candidate list of Section 3: the
 * top-k links for one vertex).  For each sources[i], its candidates are every
 * c != s that is not a neighbour of s and shares at least one explored common
 * neighbour with s; the top k_q by (score desc, c asc) are returned.
 *   sources          n_sources int32 vertex ids (repeats allowed).  Device or
 *                    host pointer.
 *   k_q              > 0, results per source.
 *   out_c, out_score n_sources * k_q entries; row i holds out_count[i] results.
 *   out_count        n_sources int32.  Device or host pointer.
 */
lp_status lp_query(lp_graph *g, const int32_t *sources, int64_t n_sources, lp_measure m,
                   int64_t hub_limit, int32_t k_q, float score_threshold, int32_t *out_c,
                   float *out_score, int32_t *out_count, void *hip_stream);

/*
 * lp_query without device allocation, for callers that cannot allocate
 * device memory during the call: applications that capture HIP graphs on
 * other streams meanwhile, tight serving loops, hosts that forbid hipMalloc
 * after start-up.  (The call itself reads the plan back to the host, so it
 * cannot be recorded into a HIP graph.)
 * Arguments, results and errors are those of lp_query; results are identical
 * to lp_query's on the same inputs.  Every piece of device scratch comes from
 * one array of about 90 MB that the library holds per device until the
 * process ends; the first call on a device looks its address up (nothing is
 * allocated then either).  Inputs and outputs stay the caller's.
 * Limits of the fixed scratch (LP_ERR_INVALID_ARGUMENT beyond them, with
 * nothing written; the graph and the scratch stay usable):
 *   n_sources <= 4096, n_sources * k_q <= 2^20, the sources' two-hop path
 *   bound (the sum over sources of the wedges they may explore) <= 2^21, and
 *   a source above the LDS capacity only when 12 * n <= 32 MiB.
 * The scratch is shared by every graph on the device and keeps the last
 * call's contents; a call clears what it needs.  One call per device at a
 * time: a call that starts while another is running on the same device
 * (from another thread) returns LP_ERR_BUSY instead of racing on it.  The
 * call does not take g's own busy flag, and returns after the stream has
 * finished its work, like lp_query.
 */
lp_status lp_query_static(lp_graph *g, const int32_t *sources, int64_t n_sources, lp_measure m,
                          int64_t hub_limit, int32_t k_q, float score_threshold, int32_t *out_c,
                          float *out_score, int32_t *out_count, void *hip_stream);

/*
 * Order-independent digest of the whole candidate set for hub limit L (the
 * prediction orientation, unordered pairs): out[0] = number of candidates,
 * out[1] = sum of h, out[2] = sum over candidates of mix64(a, c, h) modulo
 * 2^64 with original ids a < c, out[3] = wedges explored.  mix64 is the
 * SplitMix64 finaliser of ((a << 32) | c) XOR (h * 0x9E3779B97F4A7C15).
 * Used to verify exact counts at sizes where the candidate set cannot be
 * listed.  out is a host pointer to 4 uint64.
 */
lp_status lp_fingerprint(lp_graph *g, int64_t hub_limit, uint64_t *out, void *hip_stream);

/* Tuning knobs of the scheduler; 0 keeps the default.  Values apply to later
 * calls on g (host pointer; copied).
 *   lds_wedge_cap: T = U + d_a (wedges plus degree of a source) above which a
 *     source uses the global-memory accumulator instead of an LDS table
 *     (default 65536); in lp_predict and lp_fingerprint a source keeps an LDS
 *     table (in partitions) while its keys, at most min(T, ids above its own),
 *     fit the cap and T is at most 4 times it;
 *   global_slots: workgroups of the global-memory path, each holding a dense
 *     accumulator of 12 bytes per vertex (default: one per compute unit; the
 *     pool of each workspace is also kept within an eighth of the device
 *     memory);
 *   sample_budget: wedge budget of the sampling pass that sets the top-k
 *     filter threshold (default: about 0.1% of the call's wedges, clamped to
 *     [2^20, 2^22]; a negative value disables sampling); the sample also
 *     takes at least one in 1024 of the sources with wedges, whatever the
 *     budget;
 *   bucket_max[b]: upper bound of T for the scheduling buckets tiny, small,
 *     mid1, mid2, mid3 (defaults 32, 256, 1024, 2048, 4096, the table sizes
 *     the kernels are built for; a value may only lower its default, moving
 *     sources to the next bucket);
 *   batch_sources[2]: sources sharing one 256-lane workgroup in the tiny
 *     bucket (48 or 32; 48 needs fewer than 2^26 vertices, else 32 is used)
 *     and in the small bucket (8 or 4).
 *   kernel_shape[2]: the kernel of the small and mid1 buckets in the
 *     prediction orientation: 1 batches (several sources share a workgroup
 *     and one LDS table), 2 one source per 64-lane wave (small only), 3 one
 *     source per 128-lane workgroup, 4 one source per 256-lane workgroup;
 *     0 keeps the default (batches).
 *   scratch_limit: largest single device scratch allocation a call on g may
 *     make, in bytes (0: none); a call that needs more returns
 *     LP_ERR_OUT_OF_MEMORY, as when the device runs out, and g stays usable.
 * Results do not depend on the knobs.  Errors: LP_ERR_INVALID_ARGUMENT for
 * NULL arguments, negative lds_wedge_cap or global_slots, a bucket_max
 * outside [0, its default], another batch_sources value, a kernel_shape
 * outside [0, 4] (2 for the mid1 bucket) or a negative scratch_limit; g then
 * keeps its previous knobs. */
typedef struct {
  int64_t lds_wedge_cap;
  int64_t global_slots;
  int64_t sample_budget;
  int64_t bucket_max[5];
  int64_t batch_sources[2];
  int64_t kernel_shape[2];
  int64_t scratch_limit;
} lp_tuning;
lp_status lp_set_tuning(lp_graph *g, const lp_tuning *t);

/* Work done by the accumulation launches of one scheduling bucket during a
 * call, summed over the call's launches of that bucket in one kind of pass
 * (the main pass and any repeat of it; the sampling pass is kept apart).
 * Sources whose LDS table overflowed are counted under the global bucket,
 * which re-runs them.  AA / RA with a threshold: a source of the tiny, small
 * or mid1 bucket whose explored arcs' weights sum below the threshold has no
 * key that can reach it; such sources are skipped whole and not counted.  Times are HIP events on the stream of each launch
 * (sampling-pass launches run concurrently on internal streams). */
typedef struct {
  uint64_t launches;    /* kernel launches */
  uint64_t sources;     /* sources completed */
  uint64_t first_order; /* sum of the sources' degrees d_a */
  uint64_t arcs;        /* explored arcs a -> b that lead to at least one wedge */
  uint64_t wedges;      /* two-hop paths a - b - c accumulated */
  uint64_t candidates;  /* distinct non-adjacent pairs accumulated (without a threshold:
                           all of them; with one, a source skips the ids its degree
                           bound rules out for any count) */
  double ms;            /* device time of the launches */
} lp_bucket_stats;

/* Statistics of the last lp_predict / lp_fingerprint / lp_query on g (host
 * pointer).  For lp_query, wedges is the plan's upper bound, appended the
 * candidates written for the final sort, and only the main-pass launch
 * counters and times are filled. */
typedef struct {
  uint64_t wedges;            /* two-hop paths accumulated */
  uint64_t sources;           /* sources with at least one wedge */
  uint64_t bucket_sources[8]; /* sources per scheduling bucket */
  uint64_t appended;          /* candidates written to the selection buffer */
  uint64_t retries;           /* extra passes after a threshold estimate missed */
  double ms_plan, ms_accumulate, ms_select, ms_total; /* device time per phase */
  lp_bucket_stats bucket[8];  /* per bucket (tiny, small, mid1, mid2, mid3, large, global),
                                 then "split": AA / RA sources whose sums do not fit a
                                 packed 64-bit slot, run afterwards with 12-byte tables;
                                 the main pass, or the only pass without sampling */
  lp_bucket_stats sampled[8]; /* the sampling pass that estimates the top-k threshold */
} lp_stats;
lp_status lp_last_stats(const lp_graph *g, lp_stats *out);

/* Several graphs in one call (the batched form of Algorithm 1): g holds the
 * disjoint union of ngraphs graphs, graph i owning the original ids
 * [vstart[i], vstart[i+1]) (vstart[0] = 0, non-decreasing, vstart[ngraphs] =
 * n; no edge may join two graphs).  Every accumulation launch covers all the
 * graphs; thresholds and top-k are per graph.  Graph i gets what lp_predict
 * returns for it alone with k = k[i] (ids as in g): its rows start at output
 * offset sum_{j<i} k[j], out_count[i] = k'_i, and rows beyond k'_i in its
 * range are left untouched.  vstart, k, out_count: host arrays; out_a, out_c,
 * out_score: sum(k) entries, device or host.  Errors: LP_ERR_INVALID_GRAPH if
 * an edge joins two graphs, LP_ERR_INVALID_ARGUMENT for bad vstart / k. */
lp_status lp_predict_multi(lp_graph *g, int64_t ngraphs, const int64_t *vstart, const int64_t *k,
                           lp_measure m, int64_t hub_limit, float score_threshold, int32_t *out_a,
                           int32_t *out_c, float *out_score, int64_t *out_count, void *hip_stream);

/* ---------------------------------------------------------------------------
 * Serving: a request loop over the per-source query (lp_query), for the
 * recommendation use the paper describes in Section 1.  A server keeps the
 * graph resident and runs up to `slots` batches at once, each on its own HIP
 * stream with its own device scratch (candidate buffers, tables, sort space).
 * Requests queue until a slot is free; a free slot takes the oldest request
 * and every other queued request with the same measure, hub limit, k_q and
 * threshold whose sources, two-hop paths and device scratch still fit the
 * caps below, and runs them as one query.  The path count of a source s under
 * hub limit L is the sum of d_b over its neighbours b with d_b <= L: the
 * wedges it explores, which bound its candidates (computed for all vertices
 * on the first request with a given L and kept).  A batch's device
 * scratch is 24 bytes per path (candidates and sort space), the per-source
 * records and outputs, and 12 bytes per vertex for each source whose paths
 * plus degree exceed the LDS capacity (a dense global accumulator; at most as
 * many as a workspace holds).  A request above any cap runs alone.  Each request's result equals lp_query on that request alone.
 * Requests that arrive while batches run join the next batch of the slot that
 * frees first, so work of several requests overlaps on the device.
 * By default a batch runs as a replayed HIP graph: the first batch of a
 * shape (kind of request; source, candidate and dense-accumulator capacities
 * in coarse classes) records the whole query, with every count read on the
 * device, into a graph of its slot; later batches of that shape copy their
 * sources in and replay it, with no host round trip between the copies.  A
 * batch that outgrows the candidate capacity recorded for its kind runs on
 * host launches, and the kind's capacity grows.  Results do not depend on
 * the path taken.
 * ------------------------------------------------------------------------- */
typedef struct lp_server lp_server;

typedef struct {
  int32_t slots;             /* concurrent batches, 1..8 (0: 2) */
  int64_t max_batch_sources; /* sources per batch (0: 16384) */
  int64_t max_batch_paths;   /* two-hop paths per batch (0: 2^27) */
  int64_t max_batch_bytes;   /* device scratch per batch (0: an eighth of the device
                                memory divided among the slots) */
  int64_t host_launches;     /* nonzero: every batch is launched from the host, as
                                lp_query does, instead of replaying captured HIP graphs */
} lp_server_config;

typedef struct {
  lp_status status;        /* of the batch that served the request */
  uint64_t batch;          /* batch id (in launch order, from 1) */
  uint32_t batch_requests; /* requests served by that batch */
  uint32_t replayed;       /* how that batch ran: 1 as a replayed HIP graph; 0 launched
                              from the host (by configuration, or a shape beyond the
                              scratch budget); 2 from the host after the replay
                              outgrew the capacities recorded for its kind (the
                              next batches get more); 3 from the host after a
                              failed capture or replay */
  uint64_t batch_sources;  /* sources in that batch */
  uint64_t batch_bytes;    /* that batch's device scratch bound (bytes) */
  double queue_ms;         /* submit -> batch start (host clock) */
  double run_ms;           /* batch start -> results written */
  double total_ms;         /* submit -> results written */
} lp_request_info;

/* g must outlive the server; while a server exists, lp_query / lp_predict on g
 * from other threads stay allowed (they use the graph's own scratch). */
lp_status lp_server_create(lp_graph *g, const lp_server_config *cfg, lp_server **out);
/* Finishes every submitted request, then frees the server (not the graph). */
lp_status lp_server_destroy(lp_server *s);
/* Queue a request.  sources (original ids, host memory) is copied.  out_c and
 * out_score (n_sources * k_q entries, row i = i-th source, best first) and
 * out_count (n_sources) are host buffers that the server writes before the
 * request completes; they must stay valid until lp_server_wait returns for the
 * ticket.  Invalid arguments or a source outside [0, n) fail here. */
lp_status lp_server_submit(lp_server *s, const int32_t *sources, int64_t n_sources, lp_measure m,
                           int64_t hub_limit, int32_t k_q, float score_threshold, int32_t *out_c,
                           float *out_score, int32_t *out_count, uint64_t *ticket);
/* Wait for a request (timeout_ms < 0: no limit).  Returns the request's
 * status; LP_ERR_BUSY if it is still running at the timeout.  Each ticket can
 * be waited for successfully once (LP_ERR_INVALID_ARGUMENT afterwards). */
lp_status lp_server_wait(lp_server *s, uint64_t ticket, int64_t timeout_ms, lp_request_info *info);

/* Human-readable name of a status, and the detail of the last failure on the
 * calling thread ("" if none).  Both return static / thread-local storage. */
const char *lp_status_string(lp_status s);
const char *lp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LP_H */
