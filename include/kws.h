/*
 * kws.h - C ABI of the MI355X (gfx950) distance-bounded graph keyword search.
 *
 * The operation. For a directed graph G = (V, E) whose vertices carry
 * labels, a query (K, d_max, k) asks for the k best roots r: vertices from
 * which every keyword t in K is reachable within d_max hops along edge
 * direction. dist_t(r) is the hop count of a shortest path r -> ... -> v
 * with v carrying t (or, when the labels form a type tree, carrying t or any
 * type below t). score(r) = sum of dist_t(r) over K; lower is better; ties
 * break by ascending vertex id. Each returned root comes with its
 * per-keyword distances and its answer edges: for every keyword, the path
 * that starts at r and repeatedly steps to the smallest-id out-neighbour one
 * hop closer to the keyword; the union of those paths, deduplicated and
 * sorted by (src, dst).
 *
 * Citation: the paper (Dupin, PACMMOD 3(3), 2025) fixes only the notation of
 * this search in its preamble - the radius d_max, dist, the root filter,
 * the score scr, the answer-graph generator, the type-tree relations
 * (SubTypeOf, desc) and the inverted index. No section defines their
 * semantics; the definition above is the reading this library adopts.
 *
 * Conventions.
 *  - Every call returns a kws_status. On error, outputs are left zeroed and
 *    nothing needs freeing; kws_last_error() gives a thread-local message.
 *  - Host pointers are read during the call only; the library copies what
 *    it keeps. Nothing here takes ownership of caller memory.
 *  - Calls on one graph handle are serialised internally. Device work runs
 *    on the handle's stream (its own non-blocking stream unless
 *    kws_set_stream gave one) and every call returns after that work is done.
 *  - Vertex ids are int32; edge counts must stay below 2^31 (int32 CSR).
 */
#ifndef KWS_H
#define KWS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KWS_MAX_KW 64      /* distinct keywords per query (one 64-bit mask word) */
#define KWS_MAX_DMAX 15    /* largest supported radius */
#define KWS_MAX_K 65536    /* largest supported k */
#define KWS_DIST_INF 255   /* distance value meaning "not within d_max" */

typedef enum {
  KWS_OK = 0,
  KWS_EINVAL = -1,      /* malformed input or argument out of range */
  KWS_ENOMEM = -2,      /* device or host allocation failed / over the memory cap */
  KWS_EDEVICE = -3,     /* a HIP call or kernel failed */
  KWS_EOVERFLOW = -4,   /* m >= 2^31 or a size that does not fit int32 */
  KWS_EBUSY = -5,       /* server admission queue full */
  KWS_ECANCELLED = -6   /* ticket cancelled */
} kws_status;

typedef struct kws_graph kws_graph;   /* opaque; owns its device copies */

/* Graph description (all host pointers, read during kws_load_graph only).
 *  row_ptr[n+1], col[m]: forward CSR, out-neighbours of u are
 *      col[row_ptr[u] .. row_ptr[u+1]). row_ptr[0] = 0, non-decreasing,
 *      row_ptr[n] = m; 0 <= col[e] < n. Self-loops and repeated edges are
 *      allowed (they change no distance).
 *  lab_ptr[n+1], lab[]: label ids of each vertex, 0 <= lab[i] < n_labels.
 *  type_parent[n_labels] or NULL: NULL = flat labels (a keyword matches its
 *      own label only). Otherwise label ids are types of a forest,
 *      type_parent[t] = parent type or -1; a keyword t then matches t and
 *      every type below it. Must be acyclic. */
typedef struct {
  int32_t n;
  int64_t m;
  const int32_t *row_ptr;
  const int32_t *col;
  int32_t n_labels;
  const int32_t *lab_ptr;
  const int32_t *lab;
  const int32_t *type_parent;
} kws_graph_desc;

/* Validates and copies the graph to the device, builds the reverse CSR,
 * the label inverted index (keyed by type preorder, so a type and its
 * descendants form one contiguous slice) and the pull degree bins.
 * EINVAL on malformed input, EOVERFLOW if m >= 2^31, ENOMEM, EDEVICE. */
kws_status kws_load_graph(const kws_graph_desc *desc, kws_graph **out);
void kws_free_graph(kws_graph *g);

/* A query: kw[n_kw] keyword (label) ids, duplicates allowed and removed;
 * 1 <= distinct count <= KWS_MAX_KW; 0 <= d_max <= KWS_MAX_DMAX;
 * 0 <= k <= KWS_MAX_K. */
typedef struct {
  const int32_t *kw;
  int32_t n_kw;
  int32_t d_max;
  int32_t k;
} kws_query;

/* A result, allocated by the library; release with kws_result_free.
 *  kw[n_kw]           distinct keywords, ascending (the column order of kw_dist)
 *  roots[n_roots]     n_roots = min(k, number of qualifying roots), ordered by
 *  scores[n_roots]      (score ascending, vertex id ascending)
 *  kw_dist[n_roots*n_kw]  row i: dist of roots[i] to each keyword
 *  edge_ptr[n_roots+1], edge_src/edge_dst[edge_ptr[n_roots]]: answer edges
 *      of roots[i] are entries edge_ptr[i] .. edge_ptr[i+1]-1, sorted (src,dst).
 *  te                 reverse edges a plain per-keyword BFS would scan for
 *                     this query (in-degrees of vertices at dist < d_max,
 *                     summed over keywords): the GTEPS numerator; -1 unless
 *                     the count_te option is on. */
typedef struct {
  int32_t n_roots;
  int32_t n_kw;
  int32_t *kw;
  int32_t *roots;
  int32_t *scores;
  uint8_t *kw_dist;
  int64_t *edge_ptr;
  int32_t *edge_src;
  int32_t *edge_dst;
  int64_t te;
} kws_result;

/* Plain path: one query per call, one mask word. */
kws_status kws_keyword_search(kws_graph *g, const kws_query *q, kws_result *out);

/* Batched path: nq queries of uneven keyword count and d_max in one device
 * pass (lanes packed into 64-bit mask words). out[nq] receives one result
 * per query, identical to what kws_keyword_search returns for it. */
kws_status kws_search_batch(kws_graph *g, const kws_query *qs, int32_t nq, kws_result *out);

void kws_result_free(kws_result *r);

/* Batched path with flat output: the same answers as kws_search_batch,
 * returned as one set of arrays for the whole batch (allocated by the
 * library; release with kws_batch_result_free).
 *  root_ptr[nq+1]   roots/scores of query q: [root_ptr[q], root_ptr[q+1])
 *  kw_ptr[nq+1]     distinct keywords of query q in kw[]
 *  dist_ptr[nq+1]   kw_dist entries of query q (row-major n_roots x n_kw)
 *  edge_ptr[total_roots+1]  answer edges of the r-th root of the batch
 *                   (roots numbered in root_ptr order)
 *  te[nq]           per-query scanned-edge counts (see kws_result.te) */
typedef struct {
  int32_t nq;
  int64_t total_roots;
  int64_t *root_ptr;
  int32_t *roots;
  int32_t *scores;
  int64_t *kw_ptr;
  int32_t *kw;
  int64_t *dist_ptr;
  uint8_t *kw_dist;
  int64_t *edge_ptr;
  int32_t *edge_src;
  int32_t *edge_dst;
  int64_t *te;
} kws_batch_result;
kws_status kws_search_batch_flat(kws_graph *g, const kws_query *qs, int32_t nq, kws_batch_result *out);
void kws_batch_result_free(kws_batch_result *r);

/* Pipelined batches. kws_search_batch_submit plans the batch, uploads its
 * plan and enqueues its device work and result copy on the handle's stream,
 * then returns a ticket (> 0) without waiting. kws_search_batch_collect
 * waits for that batch and fills *out exactly as kws_search_batch_flat
 * would have (caller frees it with kws_batch_result_free). While one batch
 * runs on the device the caller can submit the next, so host planning and
 * result unpacking overlap device time. At most two batches may be
 * submitted and not collected (KWS_EBUSY beyond); they may be collected in
 * any order, each once (KWS_EINVAL for an unknown ticket). The queries are
 * copied at submission. A batch that needs more than one device pass is
 * computed during submission. kws_last_batch_stats describes the batch
 * collected last. Batches pending when the graph is freed are dropped. */
kws_status kws_search_batch_submit(kws_graph *g, const kws_query *qs, int32_t nq, int64_t *ticket);
kws_status kws_search_batch_collect(kws_graph *g, int64_t ticket, kws_batch_result *out);

/* Verification: dist_n[n] = truncated distance of every vertex to keyword
 * kw (KWS_DIST_INF beyond d_max), computed by the same device kernels. */
kws_status kws_debug_distances(kws_graph *g, int32_t kw, int32_t d_max, uint8_t *dist_n);

/* For callers that cannot allocate (code under stream capture, tight
 * serving loops, harnesses that forbid device allocation): the same
 * distances as kws_debug_distances, written to a DEVICE buffer dist_dev[n]
 * the caller owns, without any allocation. The search state lives in one
 * fixed array of 64 MiB per device, part of the library's code object
 * (held by every device the library runs on until the process ends); it
 * holds about 74 bytes per vertex plus a few KB, so graphs of up to about
 * 900,000 vertices fit. Larger graphs get KWS_ENOMEM and a message that
 * states both sizes. Calls are serialised process-wide (every call on a
 * device shares that device's array) and return after the device work is
 * done. EINVAL for a null argument, a keyword out of range or d_max outside
 * 0..KWS_MAX_DMAX; EDEVICE on a HIP failure. */
kws_status kws_debug_distances_noalloc(kws_graph *g, int32_t kw, int32_t d_max, uint8_t *dist_dev);

/* Engine options. Zero fields mean "default". */
typedef struct {
  int32_t direction;     /* 0 auto (device-side choice), 1 always push, 2 always pull */
  float alpha;           /* pull when alpha * frontier_in_edges > unfinished_out_edges */
  int32_t tile_words;    /* widest tile to use, in words per vertex: 1, 2, 4, 8 or 16 (default 16);
                            a batch takes the tile width its cost model prefers up to this */
  int32_t block;         /* threads per workgroup for the streaming kernels: 64..1024 */
  int32_t use_graph;     /* 1: each pass shape (tile width and count, levels, seeding mode, and the
                            per-batch sizes that set grids, rounded up to powers of two) is captured
                            once into a hipGraph and replayed for every later pass of that shape: the
                            kernels read the pass description from the uploaded plan, so the graph
                            holds no per-batch value (kws_graph_info counts captures and replays) */
  int32_t share_lanes;   /* 1 (default): queries in one word share equal (keyword, d_max) lanes; -1: off */
  int32_t count_te;      /* 1: fill kws_result.te (costs a reduction per query in the score step);
                            0 (default): te = -1 */
  int32_t seed_mode;     /* 0 auto; 1 scatter each lane's inverted-index slice (one atomic per
                            (lane, vertex)); 2 every vertex looks its labels and their type
                            ancestors up in a per-batch keyword hash. Auto takes 2 when the
                            batch's seeds outnumber the vertices plus label-ancestor lookups */
  int32_t fused_pull;    /* a level expanded by pull finalizes its rows in the same kernel instead of a
                            separate pass over every vertex. 0 (default): when tiles are 16 words (a
                            row is one 128-byte line) and a state array exceeds 512 MB (beyond the
                            Infinity Cache); 1: always; -1: never */
  int32_t early_stop;    /* top-k early termination: after each level L a query that already has k
                            complete roots scoring at most L stops expanding (any other vertex would
                            score at least L + 1, so its answer is final; kws_result.te then counts
                            only the levels expanded). 1: on; 0 (default) or -1: off. The check
                            after each level reads every vertex's vis and distance planes, which on
                            the measured workloads costs more than the expansion it saves */
  int32_t seed_table;    /* seeding by vertex (seed_mode 2, or its auto choice) from a per-batch table
                            of n_labels rows of words: row t holds the lanes whose keyword is t or an
                            ancestor of t, built by one walk per type, so a vertex ORs the rows of its
                            labels instead of walking and hashing each label's ancestors. 0 (default):
                            when the labels have a type hierarchy and the label count is at most an
                            eighth of both the vertex count and the (vertex, label) pair count;
                            1: always; -1: never. The table takes 8 * n_labels bytes per word of
                            the batch */
} kws_options;
kws_status kws_set_options(kws_graph *g, const kws_options *opt);
kws_status kws_get_options(kws_graph *g, kws_options *opt);

/* Autotuner: runs the sample batch under a grid of tile widths and
 * push/pull policies (median of `reps` timed runs after one warm-up each),
 * checks that every configuration returns identical answers (KWS_EDEVICE
 * if not), sets the fastest as the handle's options and returns it in
 * *best (may be NULL). With cache_path, a previous choice for the same graph
 * and batch shape is reused without timing, and new choices are appended.
 * budget_ms > 0 stops trying new configurations once exceeded. */
typedef struct {
  int32_t configs_tried;
  double best_ms;           /* median time of the sample batch with the choice */
  double default_ms;        /* same with the default options */
  int32_t from_cache;
} kws_tune_report;
kws_status kws_autotune(kws_graph *g, const kws_query *sample, int32_t nq, int32_t reps, double budget_ms,
                        const char *cache_path, kws_options *best, kws_tune_report *report);

/* Runs device work on this stream: a default-priority hipStream_t created
 * through the same HIP runtime this library is linked against (ROCm's
 * libamdhip64.so.7; a runtime bundled with another package, such as the
 * copy inside a PyTorch wheel, is a separate runtime whose handles are not
 * valid here). NULL restores the handle's own stream. */
kws_status kws_set_stream(kws_graph *g, void *hip_stream);
void *kws_get_stream(kws_graph *g);

/* Device memory hooks (a caller's own pool). Process-wide; set before
 * loading graphs. alloc returns NULL on failure; the memory must come from
 * the same HIP runtime as the library (see kws_set_stream). NULL hooks
 * restore hipMalloc/hipFree. */
typedef void *(*kws_alloc_fn)(size_t bytes, void *ctx);
typedef void (*kws_free_fn)(void *ptr, void *ctx);
kws_status kws_set_allocator(kws_alloc_fn alloc, kws_free_fn free_, void *ctx);

/* Device-memory cap, process-wide: every device allocation of the library
 * that would take its bytes in use above `bytes` fails with KWS_ENOMEM
 * (bytes < 0: no cap). Overrides the KWS_MEM_LIMIT_BYTES environment
 * variable. A graph sizes its search-state budget from the cap when it is
 * loaded (at most the cap minus the bytes then in use), so set the cap
 * before kws_load_graph; a server sizes its word slots from that budget.
 * Lowering the cap frees nothing. */
kws_status kws_set_mem_limit(int64_t bytes);
/* Device bytes the library holds right now (graphs, search state, servers). */
int64_t kws_mem_in_use(void);

/* Graph facts. */
typedef struct {
  int32_t n;
  int64_t m;
  int32_t n_labels;
  int32_t hierarchical;
  int64_t device_bytes;   /* graph store bytes on the device */
  int32_t max_out_degree;
  int32_t max_in_degree;
  int64_t graph_captures;   /* batch passes captured into a hipGraph (use_graph), over the handle's life */
  int64_t graph_replays;    /* batch passes that replayed an earlier capture */
} kws_graph_info;
kws_status kws_graph_info_get(kws_graph *g, kws_graph_info *info);

/* Per-kernel timing with HIP events on the handle's stream. While enabled
 * each launch is bracketed by events; kws_profile_read returns, for kernel
 * class id, the number of launches and their summed duration (ms) since
 * the last reset. kws_profile_name gives the class name (NULL past the end).
 * The classes named host_plan, host_launch, host_wait and host_collect are
 * host wall time per batch pass: planning and plan upload, kernel enqueue,
 * waiting for the device, unpacking the results. */
kws_status kws_profile_enable(kws_graph *g, int32_t on);
/* Kernel classes bracketed by events while profiling is on: bit id of mask
 * for class id (the default, and mask 0, time every class). Events add a
 * little device time per launch, so timing only the class being measured
 * keeps the rest of the run at full speed. Host-phase classes are always
 * counted (they use no events). */
kws_status kws_profile_classes(kws_graph *g, uint64_t mask);
kws_status kws_profile_reset(kws_graph *g);
kws_status kws_profile_read(kws_graph *g, int32_t id, int64_t *launches, double *total_ms);
const char *kws_profile_name(int32_t id);

/* Statistics of the last batch (summed over its device passes).
 * Entry l of the per-level arrays describes the frontier entering level l
 * (l = 0 is the keyword vertices themselves; l = d_max the last vertices
 * reached): vertices with at least one lane whose distance is exactly l,
 * their summed in-degree, and the out-degree sum of vertices still missing a
 * lane (the pull cost bound). pulled[l] = 1 if level l -> l+1 ran as pull. */
typedef struct {
  int32_t queries;
  int32_t lanes;           /* distinct (keyword, d_max) lanes after sharing */
  int32_t lane_slots;      /* sum of per-query distinct keyword counts */
  int32_t words;           /* 64-lane mask words */
  int32_t words_padded;    /* words rounded up to whole tiles */
  int32_t tiles;
  int32_t tile_words;
  int32_t levels;
  int32_t passes;
  int32_t pulled[KWS_MAX_DMAX + 1];
  int64_t frontier[KWS_MAX_DMAX + 1];
  int64_t frontier_edges[KWS_MAX_DMAX + 1];
  int64_t unfinished_edges[KWS_MAX_DMAX + 1];
  int32_t fused_pull;      /* 1 if pulled levels were finalized inside the pull (fused_pull) */
  int64_t early_stopped;   /* queries that stopped before their d_max (early_stop) */
  int64_t levels_skipped;  /* sum over those queries of d_max minus the level they stopped after */
  int32_t seed_table;      /* 1 if a pass seeded from the type-row table (seed_table) */
} kws_batch_stats;
kws_status kws_last_batch_stats(kws_graph *g, kws_batch_stats *st);

/* ---------------------------------------------------------------- serving
 * A server keeps the graph resident and runs a device loop on its own
 * thread and stream. Submitted queries wait in an admission queue; at every
 * device step the loop packs waiting queries into free 64-lane word slots
 * (their per-query state memory: one lane per distinct keyword, the slot
 * count fixed by the memory budget), seeds them, and advances every occupied
 * slot by one BFS level, each slot at its own level. A slot whose radius is
 * reached is scored, ranked and answered; its tickets complete and the slot
 * is reused. Results equal those of kws_keyword_search for the same query.
 * The graph must outlive its servers. */
typedef struct kws_server kws_server;
typedef struct {
  int32_t max_words;       /* word slots; 0 = as many as mem_bytes allows (at most 1024) */
  int32_t max_dmax;        /* largest d_max accepted (sizes the distance planes); 0 = 15 */
  int32_t queue_capacity;  /* waiting queries before submit returns KWS_EBUSY; 0 = 65536 */
  int32_t tile_words;      /* words per vertex per tile (1, 2, 4, 8, 16); 0 = the smallest power of
                              two covering the word slots, at most 16 */
  int64_t mem_bytes;       /* device bytes for the search state; 0 = the graph's budget */
} kws_server_opts;
kws_status kws_server_create(kws_graph *g, const kws_server_opts *opts, kws_server **out);
/* Non-blocking. *ticket identifies the query. KWS_EBUSY when the queue is full. */
kws_status kws_server_submit(kws_server *s, const kws_query *q, uint64_t *ticket);
/* *done = 1: the result moved into *out (caller frees it with kws_result_free)
 * and the ticket is released. *done = 0: still running. KWS_ECANCELLED for a
 * cancelled ticket (then released); KWS_EINVAL for an unknown ticket. */
kws_status kws_server_poll(kws_server *s, uint64_t ticket, kws_result *out, int32_t *done);
/* Like poll, but waits up to timeout_us microseconds (< 0: no limit). */
kws_status kws_server_wait(kws_server *s, uint64_t ticket, int64_t timeout_us, kws_result *out, int32_t *done);
/* A queued query is dropped; a running one finishes and its result is discarded. */
kws_status kws_server_cancel(kws_server *s, uint64_t ticket);
typedef struct {
  int64_t submitted, completed, cancelled, rejected, steps;
  int32_t queued, active_words, max_words;
  double elapsed_s;        /* first submit to last completion */
  double qps;              /* completed / elapsed_s */
  double p50_us, p99_us;   /* submit-to-completion latency of completed queries */
  double mean_active_words;/* occupied slots per device step */
} kws_server_stats;
kws_status kws_server_stats_get(kws_server *s, kws_server_stats *st);
/* Stops admission, cancels queued queries, lets running slots finish, joins. */
void kws_server_destroy(kws_server *s);

/* Thread-local text for the last non-OK status returned on this thread. */
const char *kws_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KWS_H */
