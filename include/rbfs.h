/*
 * rbfs -- RCM-relabelled, direction-optimizing breadth-first search on AMD
 * Instinct MI355X (gfx950).  C ABI.
 *
 * The library implements the method of "Fast and Efficient Parallel
 * Breadth-First Search with Power-law Graph Transformation" (Jiang et al.,
 * PPoPP'21 poster): a graph given as undirected CSR (section 3.1, Eq. 2) is
 * relabelled by Reverse Cuthill-McKee with isolated vertices moved to the end
 * (Algorithm 3, section 3.2), then searched level by level, top-down from a
 * frontier queue or bottom-up over the unvisited vertices (Algorithm 2), with
 * the work of each direction spread evenly over the GPU (sections 3.3-3.4).
 * The problem statement (section 2.1): given G = (V, E) and a source s,
 * produce the predecessor map pi with pi(s) = s and pi(v) = -1 when v is not
 * reachable.
 *
 * Determinism.  The paper's parent choice depends on thread timing.  Here
 * every parent is fixed: parent(v) is the neighbour one level closer to the
 * source that has the largest label in the graph's current labelling
 * (original IDs before rbfs_rcm_reorder, RCM labels after it).  After RCM,
 * labels rise with degree, so this is the neighbour that the degree-ordered
 * bottom-up scan of Algorithm 6 meets first.  depth(v) is the hop distance,
 * -1 if unreachable.  Both arrays are therefore unique and independent of the
 * direction schedule, of batching and of timing.
 *
 * Conventions for every function:
 *   - returns RBFS_OK (0) or a negative RBFS_E_* code; nothing throws;
 *   - on error, rbfs_last_error() gives a message (thread-local); output
 *     buffers hold unspecified contents and no handle is leaked;
 *   - "device pointer" means memory on the GPU the graph lives on;
 *   - `stream` is a hipStream_t (NULL = the default stream); work is ordered
 *     on it.  Calls that report results on the host synchronise it;
 *   - a handle must not be used by two host threads at once; distinct
 *     handles are independent.
 */
#ifndef RBFS_H
#define RBFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------ */
#define RBFS_OK 0
#define RBFS_E_INVAL (-1)       /* bad argument or non-canonical CSR */
#define RBFS_E_RANGE (-2)       /* root / n / nnz out of the supported range */
#define RBFS_E_NOMEM (-3)       /* device allocation failed */
#define RBFS_E_DEVICE (-4)      /* HIP runtime or kernel error */
#define RBFS_E_STATE (-5)       /* handles in incompatible states */
#define RBFS_E_NODEV (-6)       /* no usable GPU */
#define RBFS_E_UNSUPPORTED (-7) /* request outside what the library supports */

/* ---- graph creation flags --------------------------------------------- */
#define RBFS_HOST_PTRS 1u /* row_offsets / cols are host pointers */
#define RBFS_VALIDATE 2u  /* check the canonical form on the GPU (O(nnz)) */

/* ---- direction modes --------------------------------------------------- */
#define RBFS_DIR_HEURISTIC 0 /* alpha/beta rule, see rbfs_opts_t */
#define RBFS_DIR_TD_ONLY 1   /* every level top-down */
#define RBFS_DIR_BU_ONLY 2   /* level 0 top-down, every later level bottom-up */
#define RBFS_DIR_SCHEDULE 3  /* per-level directions given by the caller */
#define RBFS_DIR_LEARNED 4   /* on-device MLP, heuristic outside its range */

#define RBFS_OUT_ORIGINAL 0 /* outputs indexed by and holding original IDs */
#define RBFS_OUT_INTERNAL 1 /* outputs in the graph's internal labels */

#define RBFS_STATS_MAX_LEVELS 64

typedef struct rbfs_graph rbfs_graph_t;
typedef struct rbfs_multi rbfs_multi_t;

/* Options of a search.  A NULL opts pointer means: heuristic direction with
 * alpha = 14, beta = 24, original output space.
 *
 * Heuristic (alpha/beta switch of Algorithm 2, named in section 2.1 and tuned
 * in "Parameter Tuning"; the paper gives no formula, this integer form is
 * used): level 0 is top-down; before level d >= 1, with n_f / m_f the vertex
 * and edge (degree) counts of the frontier F_d, m_u the degree sum of the
 * vertices not yet reached and n the number of vertices the bottom-up sweep
 * covers, switch top-down -> bottom-up when m_f * alpha > m_u, and
 * bottom-up -> top-down when n_f * beta < n and n_f < n_f of the previous
 * level. */
typedef struct rbfs_opts {
  int32_t direction;       /* RBFS_DIR_* */
  int32_t alpha;           /* > 0 */
  int32_t beta;            /* > 0 */
  int32_t output_space;    /* RBFS_OUT_* */
  const int8_t* schedule;  /* host; RBFS_DIR_SCHEDULE: 0 = TD, 1 = BU for level
                              d; levels past schedule_len repeat the last entry;
                              level 0 is always top-down */
  int32_t schedule_len;
  int32_t tune_profile;    /* 0 = the graph's tuning (rbfs_graph_set_tuning,
                              rbfs_tune; built-in defaults until then);
                              1..4 = 256-thread workgroups, that many per
                              compute unit; 5, 6 = 1024-thread workgroups,
                              1 or 2 per compute unit (single-root only) */
  int32_t flags;           /* RBFS_OPT_* */
} rbfs_opts_t;

/* opts flags */
#define RBFS_OPT_TIMING 1 /* record HIP events around the search kernel and
                             the whole call; read them with rbfs_graph_timings */
#define RBFS_OPT_WG_WORK 2 /* single-root searches: record the adjacency
                              entries each workgroup processed per level;
                              read them with rbfs_graph_wg_work */
#define RBFS_OPT_NO_BALANCE 8 /* single-root searches, for the load-balance
                                  ablation (sections 3.3-3.4): top-down gives
                                  each frontier vertex's whole row to one
                                  wave (Algorithm 1's vertex-per-worker
                                  split on the GPU's SIMD unit), bottom-up
                                  sweeps equal vertex ranges, one set per
                                  workgroup, with no work stealing.  Same
                                  results; slower on skewed graphs. */
#define RBFS_OPT_ZERO_WAIT 4 /* single-root searches, for tests of the error
                                path: the search's grid barrier waits for no
                                time, so the search gives up at its first
                                barrier with the time-out status (outputs
                                unspecified; every kernel still exits
                                normally).  Without stats the call returns
                                RBFS_OK and rbfs_graph_check reports it. */

/* Per-search statistics; asking for them synchronises the stream.  Level d
 * arrays describe the level that expands frontier F_d. */
typedef struct rbfs_stats {
  int32_t levels;                            /* number of levels expanded */
  int32_t status;                            /* device status word, 0 = ok */
  int8_t dir[RBFS_STATS_MAX_LEVELS];         /* 0 = TD, 1 = BU */
  int8_t fallback[RBFS_STATS_MAX_LEVELS];    /* learned mode: the alpha/beta rule
                                                decided because the features were
                                                out of range (1) or the predictions
                                                within the margin (2); 0 = network */
  int64_t nf[RBFS_STATS_MAX_LEVELS];         /* |F_d| */
  int64_t mf[RBFS_STATS_MAX_LEVELS];         /* degree sum over F_d */
  int64_t mu[RBFS_STATS_MAX_LEVELS];         /* degree sum of unreached after F_d */
  int64_t edges[RBFS_STATS_MAX_LEVELS];      /* adjacency entries read at level d */
  float level_us[RBFS_STATS_MAX_LEVELS];     /* device wall-clock time of level d */
  int64_t reached;                           /* vertices with depth >= 0 */
  int64_t component_edges;                   /* undirected edges among reached */
  float ms_kernel;                           /* search kernel time */
  float ms_total;                            /* incl. output translation */
} rbfs_stats_t;

typedef struct rbfs_graph_info {
  int64_t n;          /* vertices */
  int64_t nnz;        /* adjacency entries (2 x undirected edges) */
  int64_t n_plus;     /* non-isolated vertices */
  int32_t reordered;  /* 1 after rbfs_rcm_reorder */
  int32_t device;     /* HIP device ordinal */
  int64_t max_degree;
  int64_t device_bytes; /* device memory held by the handle */
  int64_t rcm_keep;   /* after a reorder: vertices placed by Cuthill-McKee
                         (n_plus for the full RCM order); 0 before */
} rbfs_graph_info_t;

typedef struct rbfs_device_info {
  int32_t device;
  int32_t compute_units;
  int32_t wavefront_size;
  int32_t clock_khz;
  int64_t global_mem_bytes;
  int64_t l2_bytes;
  char arch[64];
} rbfs_device_info_t;

/* Message for the last failing call on this host thread ("" if none). */
const char* rbfs_last_error(void);

/* Current HIP device; RBFS_E_NODEV when there is none. */
int rbfs_device_info(rbfs_device_info_t* out);

/* Device memory of the library (graph arrays, search workspaces, batch
 * engines, per-call temporaries) comes from hipMalloc/hipFree unless an
 * allocator is installed here, e.g. a framework's caching allocator, so that
 * the caller's memory pool accounts for it (not in the paper: plumbing of the
 * boundary).  alloc(bytes, stream, ctx) returns device memory of at least
 * `bytes` bytes, or NULL on failure (the library call then returns
 * RBFS_E_NOMEM); `stream` is the stream of the library call that asks for it
 * (NULL: the NULL stream).  free_fn(ptr, stream, ctx) releases a block that
 * alloc returned; the library has synchronised the work that used it, except
 * for blocks freed on the stream of the call that used them.  Pass NULL for
 * both to return to hipMalloc/hipFree.  Process-wide; allowed only while no
 * graph or multi-graph handle exists (else RBFS_E_STATE), so that every block
 * goes back to the allocator that made it, and not while another library call
 * runs.  Both functions must be given or neither (else RBFS_E_INVAL).  The
 * learned-switch parameters uploaded by rbfs_switch_load keep using hipMalloc:
 * they live until the process ends. */
typedef void* (*rbfs_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*rbfs_free_fn)(void* ptr, void* stream, void* ctx);
int rbfs_set_allocator(rbfs_alloc_fn alloc, rbfs_free_fn free_fn, void* ctx);

/* Create a graph handle on the current HIP device from a canonical undirected
 * CSR (section 3.1, Eq. 2): row_offsets[n+1] (int64, row_offsets[0] = 0,
 * non-decreasing, row_offsets[n] = nnz) and cols[nnz] (int32 in [0, n), each
 * row strictly ascending, no self-loops, every edge present in both
 * directions).  0 <= n < 2^31.  Pointers are device pointers unless flags has
 * RBFS_HOST_PTRS.  With RBFS_VALIDATE the form is checked on the GPU and a
 * violation returns RBFS_E_INVAL.  The library copies the CSR: the caller may
 * free its buffers once the call returns (it synchronises `stream`). */
int rbfs_graph_create(int64_t n, int64_t nnz, const int64_t* row_offsets, const int32_t* cols,
                      uint32_t flags, void* stream, rbfs_graph_t** out);

/* Release a handle and its device memory.  NULL is accepted.  Returns
 * RBFS_E_STATE (and releases nothing) while a multi-graph handle built over
 * this graph exists: destroy that first. */
int rbfs_graph_destroy(rbfs_graph_t* g);

int rbfs_graph_info(const rbfs_graph_t* g, rbfs_graph_info_t* out);

/* Bandwidth of the graph's current labels (section 3.2: what the
 * Cuthill-McKee order keeps small): the largest |u - v| over its adjacency
 * entries, 0 for a graph without edges.  After rbfs_rcm_reorder these are
 * the RCM labels.  One O(n) pass on `stream` (a row's first and last entries
 * bound it, rows being ascending) into *out (host); synchronises `stream`.
 * Allocates 8 bytes of device memory for the call. */
int rbfs_graph_bandwidth(const rbfs_graph_t* g, int64_t* out, void* stream);

/* Relabel the graph by Reverse Cuthill-McKee (Algorithm 3, section 3.2):
 * V+ (non-isolated vertices) sorted by increasing (degree, id); each
 * connected component is explored from its unvisited vertex of least
 * (degree, id), neighbours appended in increasing (degree, id) order; the
 * sequence is reversed and the isolated vertices are appended in increasing
 * id.  The result is exactly the permutation of that sequential algorithm.
 * The internal CSR is replaced by the relabelled one (rows ascending) and
 * later searches sweep only the n+ non-isolated vertices.
 * perm_out (nullable, device, int32[n]) receives perm[old] = new.
 * ms_out (nullable, host) receives the elapsed time.  Synchronises `stream`.
 * A second call returns RBFS_OK and changes nothing.  RBFS_E_STATE while a
 * multi-graph handle built over the graph in its original labels exists. */
int rbfs_rcm_reorder(rbfs_graph_t* g, int32_t* perm_out, void* stream, float* ms_out);

/* How rbfs_rcm_reorder builds the relabelled CSR (the result is the same
 * either way).  0 (default): graphs of up to 2^32 adjacency entries in one
 * sort of all their (column, new row) pairs (16 bytes per entry of
 * temporary memory), larger ones in batches of about 2^30 entries of new
 * rows (the rows' entries renamed and sorted row by row), which keeps the
 * relabel within memory for the largest graphs one GPU holds.  max_entries
 * > 0: always in batches of about that many entries. */
int rbfs_graph_set_rcm_batch(rbfs_graph_t* g, int64_t max_entries);

/* Where a batched relabel keeps the old column array.  0 (default): on the
 * device while there is room for both column arrays, else in pinned host
 * memory, brought back a slice of old rows at a time (the graph's device
 * memory then peaks at about one column array, which is what lets the
 * largest graphs be relabelled on one GPU); 1: always in host memory; -1:
 * never.  Applies only to batched relabels (rbfs_graph_set_rcm_batch). */
int rbfs_graph_set_rcm_staging(rbfs_graph_t* g, int32_t mode);

/* Size of the single-root search's frontier sub-queues.  The next frontier
 * (and the bottom-up vertex list) is appended to 8 sub-queues, one per group
 * of workgroups, each holding `entries` vertices; what does not fit goes to
 * one shared overflow queue of n entries, so no size loses vertices.  0
 * (default): n/4 each, about 3n entries in all.  Results do not depend on
 * it.  Releases the search workspace (rebuilt by the next search). */
int rbfs_graph_set_queue_cap(rbfs_graph_t* g, int64_t entries);

/* Partial RCM (section 4.6): as rbfs_rcm_reorder, but only the first `keep`
 * vertices of Algorithm 3's Cuthill-McKee sequence are reordered.  They take
 * labels [0, keep) in reverse sequence order; the other non-isolated
 * vertices follow in increasing original ID; isolated vertices come last in
 * increasing ID.  keep < 0 or keep >= n_plus gives exactly rbfs_rcm_reorder;
 * keep = 0 only moves the isolated vertices to the end.  The paper's ratio p
 * corresponds to keep = ceil(p * n_plus) (n_plus from rbfs_graph_info).  The
 * search results follow the new labels like after the full order; since
 * components no longer occupy label intervals, searches sweep all n_plus
 * vertices.  After either reorder call, a second call of either returns
 * RBFS_OK and changes nothing. */
int rbfs_rcm_reorder_partial(rbfs_graph_t* g, int64_t keep, int32_t* perm_out, void* stream,
                             float* ms_out);

/* Inverse of the current relabelling: iperm_out[new] = old (device int32[n]).
 * Identity before rbfs_rcm_reorder. */
int rbfs_graph_iperm(const rbfs_graph_t* g, int32_t* iperm_out, void* stream);

/* The graph's current CSR (section 3.1, Eq. 2): the input graph, or after
 * rbfs_rcm_reorder the relabelled one of section 3.2 (vertex k = the vertex
 * with new label k, neighbours as new labels, rows ascending).
 * row_offsets_out: device int64[n+1]; cols_out: device int32[nnz] (may be
 * NULL when nnz = 0).  Synchronises `stream`. */
int rbfs_graph_csr(const rbfs_graph_t* g, int64_t* row_offsets_out, int32_t* cols_out,
                   void* stream);

/* Breadth-first search from `root` (an original ID in [0, n)).
 * depth, parent: device int32[n], fully overwritten: depth = hop distance or
 * -1; parent(root) = root; parent = -1 when unreachable; otherwise the
 * largest-label neighbour one level up.  With output_space
 * RBFS_OUT_ORIGINAL (default) both are indexed by original ID and parents
 * are original IDs; with RBFS_OUT_INTERNAL, by internal label.
 * Enqueued on `stream` without a host round trip; `stats` (nullable, host)
 * forces a synchronisation and fills per-level counters. */
int rbfs_bfs(rbfs_graph_t* g, int32_t root, int32_t* depth, int32_t* parent,
             const rbfs_opts_t* opts, void* stream, rbfs_stats_t* stats);

/* Certificate of a search result, checked on the device in O(n + nnz):
 * *result = 0 when (depth, parent) is exactly what rbfs_bfs from `root` (an
 * original ID) returns on this graph -- hop distances of section 2.1 with the
 * predecessor map, the parent being the largest-label neighbour one level up
 * in the graph's current labels -- else a negative RBFS_CERT_* code of a
 * rule the outputs break (when several are broken, the most negative code
 * among those found; the same on every call).  depth, parent: device int32[n]
 * laid out as rbfs_bfs writes them for `output_space`; read only, values need
 * not be in range (every parent is range-checked before it is used as an
 * index).  Synchronises `stream`.  Returns RBFS_E_INVAL for NULL pointers or
 * an unknown output_space, RBFS_E_RANGE for a root outside [0, n). */
#define RBFS_CERT_ROOT (-1)       /* root entries wrong, or another vertex at depth 0 */
#define RBFS_CERT_REACH (-2)      /* an edge joins a reached and an unreached vertex */
#define RBFS_CERT_LEVEL (-3)      /* an edge spans more than one level */
#define RBFS_CERT_ORPHAN (-4)     /* an unreached vertex has a parent */
#define RBFS_CERT_PARENT (-5)     /* parent is not a neighbour one level up */
#define RBFS_CERT_LARGER (-6)     /* a neighbour one level up has a larger label */
#define RBFS_CERT_RANGE (-7)      /* depth below -1, or parent outside [-1, n) */
int rbfs_certify(rbfs_graph_t* g, int32_t root, const int32_t* depth, const int32_t* parent,
                 int32_t output_space, void* stream, int32_t* result);

/* rbfs_certify for callers that cannot allocate device memory (tight serving
 * loops, harnesses that forbid hipMalloc): the same checks and result, with
 * the scratch (result word, long-row list and chunk plan, and for original-ID
 * outputs of a relabelled graph the depths in internal order) taken from a
 * static device buffer of 64 MiB that each GPU the library runs on holds
 * until the process ends, instead of from the allocator.  It makes no
 * allocation of any kind.  Graphs whose scratch exceeds the buffer -- about
 * 4 * n + 16 * (nnz / 4096) bytes with that gather, so n up to about 16
 * million vertices -- are refused with RBFS_E_RANGE (use rbfs_certify).
 * Every call on a GPU uses that GPU's one buffer: calls that overlap on one
 * GPU (on different streams or host threads) race and must be serialised by
 * the caller.  The buffer keeps the last call's contents; each call clears
 * what it needs.  Arguments, results and errors otherwise as rbfs_certify;
 * synchronises `stream`. */
int rbfs_certify_noalloc(rbfs_graph_t* g, int32_t root, const int32_t* depth,
                         const int32_t* parent, int32_t output_space, void* stream,
                         int32_t* result);

/* Synchronise `stream` and report any device status (queue overflow,
 * barrier time-out, corrupt input detected by a kernel) raised by any
 * single-root search on this graph since the last check, including those a
 * call with stats already reported: RBFS_OK or RBFS_E_DEVICE.  The status is
 * cleared once reported.  (Batched searches report their status at the end
 * of each call.) */
int rbfs_graph_check(rbfs_graph_t* g, void* stream);

/* Work per workgroup of the graph's last single-root search, if it was made
 * with RBFS_OPT_WG_WORK: the GPU counterpart of the per-thread edge counts
 * behind the load balancing of sections 3.3-3.4 (Algorithms 4-5).
 * out[d * grid + w] (host int64, cap entries) = adjacency entries workgroup w
 * processed in level d: top-down, the frontier edges of the chunks it took;
 * bottom-up, the row entries it read.  Summed over w, a level gives
 * rbfs_stats_t's nf-weighted edge count (m_f top-down, edges bottom-up).
 * *levels (at most RBFS_STATS_MAX_LEVELS) and *grid receive the shape;
 * out may be NULL to ask for it.  Synchronises `stream`.  RBFS_E_STATE when
 * the last search was made without the flag. */
int rbfs_graph_wg_work(rbfs_graph_t* g, int64_t* out, int64_t cap, int32_t* levels, int32_t* grid,
                       void* stream);

/* Durations of the calls made with RBFS_OPT_TIMING since the last read
 * (oldest first, at most 1024 kept): kernel_ms[i] = search kernel(s) only,
 * total_ms[i] = whole call incl. output translation.  Synchronises `stream`;
 * *count receives the number written (<= cap).  Clears the record. */
int rbfs_graph_timings(rbfs_graph_t* g, float* kernel_ms, float* total_ms, int32_t cap,
                       int32_t* count, void* stream);

/* k searches at once, 64 roots per bit-parallel pass (one 64-bit visit word
 * per vertex).  roots: host int32[k] original IDs (duplicates allowed).
 * depth, parent: device int32[k][n] root-major; row j equals rbfs_bfs from
 * roots[j] bit for bit.  stats (nullable): levels and counters of the last
 * 64-root pass, synchronises. */
int rbfs_bfs_batch(rbfs_graph_t* g, const int32_t* roots, int32_t k, int32_t* depth,
                   int32_t* parent, const rbfs_opts_t* opts, void* stream, rbfs_stats_t* stats);

/* Multi-graph batch: the graphs are packed as one disjoint union (each keeps
 * its own labels, offset by the vertex counts of the graphs before it) and
 * searched together, root j of every graph sharing bit j.  All graphs must be
 * in the same state (all reordered or none) on the same device.  The handle
 * copies the member CSRs but keeps using each member's label maps, so until
 * rbfs_multi_destroy the members may be neither relabelled nor destroyed
 * (both calls return RBFS_E_STATE meanwhile). */
int rbfs_multi_create(rbfs_graph_t* const* graphs, int32_t count, void* stream,
                      rbfs_multi_t** out);
int rbfs_multi_destroy(rbfs_multi_t* m);

/* roots: host int32[count][k] (k <= 64, original IDs of each graph).
 * depth, parent: device int32, graph after graph, each graph's block
 * root-major [k][n_g].  The whole search runs as one captured HIP graph that
 * is replayed on later calls with the same k. */
int rbfs_bfs_multi(rbfs_multi_t* m, const int32_t* roots, int32_t k, int32_t* depth,
                   int32_t* parent, const rbfs_opts_t* opts, void* stream, rbfs_stats_t* stats);

/* ---- autotuner ----------------------------------------------------------
 * Launch shape and work-split parameters of the searches.  They decide only
 * how the work of a level is spread over the GPU: every setting gives the
 * same depth and parent arrays, bit for bit.  The autotuner (not in the
 * paper; its counterpart there is the grid search over the partition factor
 * lambda of Algorithm 5 in "Parameter Tuning") times settings on sample roots
 * and keeps the fastest whose outputs equal those of the built-in defaults. */
typedef struct rbfs_tuning {
  int32_t block;     /* threads per search workgroup: 256 or 1024 (batched
                        searches: 1024 only) */
  int32_t per_cu;    /* search workgroups per compute unit, 1..4; clamped to
                        what can be resident at once */
  int32_t lane_row;  /* bottom-up: rows of at most lane_row entries are scanned
                        by one lane each, longer rows by a whole wave; 1..4096 */
  int32_t bu_grain;  /* bottom-up: edge-balanced work ranges per search
                        workgroup (taken by work stealing); 1..1024 */
  int32_t td_chunk;  /* top-down: adjacency entries per load-balancing chunk,
                        a power of two from 256 to 4 * block (single-root
                        only; batched searches ignore it) */
  int32_t reset;     /* single-root with original-ID outputs: 1 = the output
                        translation sets the internal entries it reads back
                        to unreached, 0 = the next search re-initialises
                        them in one coalesced pass */
} rbfs_tuning_t;

#define RBFS_TUNE_SINGLE 0 /* rbfs_bfs */
#define RBFS_TUNE_BATCH 1  /* rbfs_bfs_batch */

typedef struct rbfs_tune_record {
  rbfs_tuning_t tuning;
  float ms;            /* mean device time of one call (rbfs_bfs: one root;
                          batch and multi: one call over all roots) */
  int32_t mismatches;  /* output entries that differ from the reference */
} rbfs_tune_record_t;

/* Fills *t with the built-in defaults of `kind`. */
int rbfs_tuning_default(int32_t kind, rbfs_tuning_t* t);

/* Sets or reads the parameters later calls of `kind` use on this graph.
 * Values outside the documented ranges return RBFS_E_INVAL; per_cu is
 * clamped.  Setting synchronises `stream` when the bottom-up ranges have to
 * be rebuilt. */
int rbfs_graph_set_tuning(rbfs_graph_t* g, int32_t kind, const rbfs_tuning_t* t, void* stream);
int rbfs_graph_get_tuning(const rbfs_graph_t* g, int32_t kind, rbfs_tuning_t* t);

/* Autotuner.  roots: host int32[k] original IDs (RBFS_TUNE_SINGLE: 1 <= k <=
 * 64, each root searched in turn; RBFS_TUNE_BATCH: 1 <= k <= 64, one batch).
 * opts (nullable) gives direction and output space; timing flags and
 * tune_profile are ignored.  The reference outputs come from the built-in
 * defaults.  Each candidate runs once per root (compared entry by entry with
 * the reference) and then `reps` timed times.  The search is coordinate
 * descent over launch shape, lane_row, bu_grain, td_chunk and reset, starting
 * from the defaults; a change is kept when it is at least 1 % faster, and
 * the sweep over the parameters repeats while it changes anything (at most
 * three sweeps).  The winner is set on the graph and copied to *best
 * (nullable); records[cap] (nullable) receives every candidate timed, *count
 * (nullable) their number.
 * A candidate whose outputs differ is never chosen and makes the call return
 * RBFS_E_DEVICE after it finishes (its record shows the mismatches).
 * Device memory: 8 * k * n bytes for the reference and 8 * n (single) or
 * 8 * k * n (batch) for the candidate outputs, freed before returning.
 * Synchronises `stream`. */
int rbfs_tune(rbfs_graph_t* g, int32_t kind, const int32_t* roots, int32_t k, int32_t reps,
              const rbfs_opts_t* opts, rbfs_tuning_t* best, rbfs_tune_record_t* records,
              int32_t cap, int32_t* count, void* stream);

/* The same for a multi-graph batch (kind RBFS_TUNE_BATCH parameters; roots
 * as in rbfs_bfs_multi).  Changing the parameters re-captures the search on
 * the next call.  Device memory: twice the output size of rbfs_bfs_multi. */
int rbfs_multi_set_tuning(rbfs_multi_t* m, const rbfs_tuning_t* t, void* stream);
int rbfs_multi_get_tuning(const rbfs_multi_t* m, rbfs_tuning_t* t);
int rbfs_multi_tune(rbfs_multi_t* m, const int32_t* roots, int32_t k, int32_t reps,
                    rbfs_tuning_t* best, rbfs_tune_record_t* records, int32_t cap,
                    int32_t* count, void* stream);

/* ---- learned direction switch ------------------------------------------
 * Not in the paper: the alpha/beta rule of Algorithm 2 (section 2.1,
 * "Parameter Tuning") is replaced by a small network that predicts, from 8
 * per-level features, ln(microseconds) of the next level in each direction
 * (output 0 top-down, 1 bottom-up); the cheaper one is taken when the two
 * predictions differ by at least the blob's margin (ln microseconds; 0.25 is
 * about 28 %).  Closer predictions, which lie within the network's training
 * error, and inputs outside the training range leave the decision to the
 * alpha/beta rule.
 *
 * Network: x[8] -> ReLU(W1 x + b1)[32] -> ReLU(W2 h1 + b2)[32] -> W3 h2 + b3
 * [2], fp32.  Parameters (1410 floats) in the order W1[32][8] (row = output
 * unit), b1[32], W2[32][32], b2[32], W3[2][32], b3[2].  A switch blob adds
 * fmin[8], fmax[8] (training feature range), the largest training level and
 * the margin: 1428 floats.  Features: log2(1+n_f)/log2(n), log2(1+m_f)/log2(nnz),
 * log2(1+m_u)/log2(nnz), n_u/n, clamp(log2((1+m_f)/(1+m_u))/16, -2, 2),
 * level/32, current direction, clamp(log2((1+n_f)/(1+n_f_prev))/8, -2, 2),
 * with n the swept vertex count and n_u the swept vertices not yet reached.
 * All buffers of these calls are host memory. */

/* Loads the switch blob (1428 floats) for the current device; later
 * searches with RBFS_DIR_LEARNED use it.  Process-wide. */
int rbfs_switch_load(const float* blob, int32_t n);

/* Training samples: for each root and each level d >= 1, searches that
 * follow the alpha/beta rule's directions up to level d - 1, take level d
 * top-down, or bottom-up, and follow the alpha/beta rule again from there
 * on, `reps` times each.  A direction's cost at level d is the median device
 * time from the start of level d to the end of the search: the level itself,
 * including whatever the switch costs there (a first bottom-up level sweeps
 * the component's words, a later one walks the vertex list the last
 * bottom-up level left), and what the choice does to the levels after it (a
 * bottom-up level taken early spares the next one the word sweep).  A
 * network that picks the cheaper of the two predicted costs improves on the
 * rule it was labelled with, one level at a time.  From level 2 on the same
 * is done once more with level d - 1 taken the other way, which samples the
 * other value of the current-direction feature (the frontiers, hence the
 * other features and the rule's later decisions, do not depend on the
 * directions).  Searches deeper than RBFS_STATS_MAX_LEVELS levels are
 * labelled on their first RBFS_STATS_MAX_LEVELS levels, and their schedules
 * repeat the last of those directions after them.  Rows of 11 floats:
 * features[8], ln(us TD), ln(us BU), level.  Writes at most `cap` rows;
 * *count receives the number. */
int rbfs_collect_level_samples(rbfs_graph_t* g, const int32_t* roots, int32_t k, int32_t reps,
                               int32_t alpha, int32_t beta, float* out, int32_t cap,
                               int32_t* count, void* stream);
/* The same call under the name the interface plan gives it. */
int rbfs_collect_level_timings(rbfs_graph_t* g, const int32_t* roots, int32_t k, int32_t reps,
                               int32_t alpha, int32_t beta, float* out, int32_t cap,
                               int32_t* count, void* stream);

/* Training on the GPU: samples[n][10] (features[8], targets[2]); w_init[1410];
 * order[epochs][n]: the sample order of each epoch (batches are consecutive
 * runs of `batch` entries, the last one possibly shorter).  Loss: mean over
 * the batch of half the squared error; Adam (beta1 0.9, beta2 0.999, eps
 * 1e-8, learning rate lr).  Gradients are summed in a fixed order, so the
 * result is bit-reproducible.  w_out[1410]; loss_curve[epochs] (nullable):
 * mean loss of each epoch. */
int rbfs_mlp_train(const float* samples, int32_t n, const float* w_init, const int32_t* order,
                   int32_t epochs, int32_t batch, float lr, float* w_out, float* loss_curve,
                   void* stream);

/* Test hooks: forward pass (x[n][8] -> y[n][2]) with the kernel the search
 * uses, and the gradient of the batch loss over all n samples. */
int rbfs_mlp_forward(const float* w, const float* x, int32_t n, float* y);
int rbfs_mlp_grad(const float* w, const float* samples, int32_t n, float* grad, float* loss);
/* rbfs_mlp_grad under the name the interface plan gives it. */
int rbfs_mlp_backward(const float* w, const float* samples, int32_t n, float* grad,
                      float* loss);

#ifdef __cplusplus
}
#endif

#endif /* RBFS_H */
