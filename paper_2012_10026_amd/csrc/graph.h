// Graph handle layout and the host entry points of the passes (RCM, BFS,
// batched BFS).  Internal to the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/rbfs.h"
#include "prim.h"

namespace rbfs {

// Edges per chunk of the edge-balanced frontier expansion.
constexpr int kChunkShift = 10;
constexpr int kChunkEdges = 1 << kChunkShift;  // largest top-down chunk
constexpr int kMinChunkShift = 8;               // smallest (tunable)
// Single-root top-down step: frontier edges per thread and round.  Their
// column, bitmap, pair and atomic accesses are issued together, so each thread
// keeps kTdK independent chains in flight; a chunk holds at most kTdK * block
// entries.
constexpr int kTdK = 4;

// Slack entries after a graph's column array: the bottom-up row scans read
// aligned groups of 4 entries and may read up to 7 entries past a row's end.
constexpr int kColPad = 16;

// Device memory of graphs, engines, workspaces and call temporaries: hipMalloc
// and hipFree, or the allocator installed with rbfs_set_allocator.  stream is
// the stream the memory will be used on (NULL: the NULL stream).
hipError_t dev_malloc(void** p, size_t bytes, hipStream_t stream = nullptr);
template <class T>
hipError_t dev_malloc(T** p, size_t bytes, hipStream_t stream = nullptr) {
  return dev_malloc(reinterpret_cast<void**>(p), bytes, stream);
}
void dev_free(void* p, hipStream_t stream = nullptr);
// Live graph and multi-graph handles (the allocator may change only at 0).
void live_handles_add(int d);

// Built-in defaults of the tunable parameters and their check.
rbfs_tuning_t default_tuning(int kind);
bool tuning_valid(int kind, const rbfs_tuning_t& t, std::string* why);

// Edge-balanced ranges of 64-vertex words over [0, n_sweep): about
// nnz / nparts_want adjacency entries and at most
// max(min_words, W / nparts_want + 1) words each (W = number of words).
// Allocates *bounds (n_part + 1 entries, device); synchronises `stream`.
int build_edge_ranges(const int64_t* off, int64_t n_sweep, int64_t nnz, int64_t nparts_want,
                      int64_t min_words, int32_t** bounds, int32_t* n_part, hipStream_t stream);

struct BfsCtl;
struct MsCtl;
struct Graph;

// Workspace of the single-root search (sized for n_sweep vertices).
struct BfsWork {
  int64_t n_sweep = 0;
  uint64_t* dp = nullptr;       // packed (depth << 32 | ~parent) per swept vertex
  uint64_t* vis = nullptr;      // reached before the current level
  uint64_t* front = nullptr;    // three rotating frontier bitmaps
  int32_t* qv[2] = {nullptr, nullptr};
  int64_t* qe[2] = {nullptr, nullptr};
  int32_t* chunk[2] = {nullptr, nullptr};
  int64_t chunk_cap = 0;
  int chunk_shift = 0;          // log2 of the chunk length the tables are sized for
  int64_t qcap = 0;             // entries of each sub-queue / sub-list (then the overflow one)
  int32_t* bu_part = nullptr;
  int32_t n_part = 0;
  int32_t part_grain = 0;       // bu_grain the ranges were built for
  int32_t part_grid = 0;        // grid size the ranges were built for
  unsigned long long* wctr = nullptr;  // range counters: 3 x max_grid x 16
  int max_grid = 0;
  int32_t* vl[2] = {nullptr, nullptr};  // bottom-up vertex lists (n_sweep each)
  int32_t* top = nullptr;       // largest-label neighbour of each swept vertex
  // original-ID outputs after RCM (built at the first such search): the
  // layout of the three output passes, whose staging arrays are the frontier
  // queues (idle once the search kernel has finished): pass A writes pairs
  // to qe[0] and original IDs to qv[0], pass B to qe[1] and qv[1]
  int64_t* owstart = nullptr;   // first position of each window (windows + 1)
  int64_t* ogA = nullptr;       // pass-A run of each (tile, bucket), tile-major
  int64_t ontiles = 0;          // pass-A tiles
  int32_t* ocnt_w = nullptr;    // ... in each window
  int32_t* ochunk = nullptr;    // first pass-B chunk of each bucket (buckets + 1)
  int64_t onwin = 0;            // windows
  int ona = 0, oas = 0;         // buckets; windows per bucket = 2^oas
  int onchunk = 0;              // pass-B chunks
  BfsCtl* ctl = nullptr;
  bool clean = false;           // every pair holds the unreached value
  uint32_t base = 0;            // depth-field base of the last search (see bfs.hip)
  bool base_valid = false;
  int grid = 0;                 // persistent grid size
  int max_per_cu = 1;           // resident 1024-thread workgroups per CU
  int max_per_cu_256 = 1;       // resident 256-thread workgroups per CU
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
  int64_t* wg_work = nullptr;   // RBFS_OPT_WG_WORK: [level][grid] entries per workgroup
  int wg_grid = 0;              // grid of the recorded search
  bool wg_valid = false;        // the last search recorded wg_work
};

// Bit-parallel multi-root search engine over one "union" graph: a single
// graph (off/cols/oid point at the graph's arrays) or a packed disjoint union
// of several graphs (uoff/ucols/uoid owned here).
struct MsEngine {
  const int64_t* off = nullptr;
  const int32_t* cols = nullptr;
  const int32_t* oid = nullptr;   // internal -> original ID, null = identity
  int64_t* uoff = nullptr;        // owned union CSR (multi-graph)
  int32_t* ucols = nullptr;
  int32_t* uoid = nullptr;
  int64_t n_sweep = 0;
  int64_t nnz = 0;
  uint64_t* vis = nullptr;
  uint64_t* front = nullptr;      // 3 x n_sweep words
  uint64_t* dp = nullptr;         // [n_sweep][64] packed (depth << 32 | ~parent)
  int32_t* qv[2] = {nullptr, nullptr};
  int64_t* qe[2] = {nullptr, nullptr};
  int32_t* chunk[2] = {nullptr, nullptr};
  int64_t chunk_cap = 0;
  int32_t* bu_part = nullptr;
  int32_t n_part = 0;
  unsigned long long* wctr = nullptr;  // range counters: 3 x max_grid x 16
  int max_grid = 0;
  MsCtl* ctl = nullptr;
  int ngraphs = 1;
  rbfs_tuning_t tune{};           // parameters in use (kind RBFS_TUNE_BATCH)
  int max_per_cu = 1;             // resident search workgroups per CU
  int compute_units = 0;
  int32_t* roots_dev = nullptr;   // 64 union IDs per graph, then 64 original IDs per graph
  int32_t* roots_host = nullptr;  // pinned staging for the original IDs (64 per graph)
  int grid = 0;
  int64_t wall_rate_khz = 100000;
  hipGraphExec_t gexec = nullptr; // captured multi-graph search
  // depth-field base of the packed pairs (see the single-root search): a
  // single-graph engine lowers it every batch and its outputs leave the
  // pairs in place; a captured (multi-graph) one keeps it fixed and clears
  // the pairs it translates, since a replay cannot change kernel arguments
  uint32_t base = 0xFFFFFFFFu;
  bool base_valid = true;         // every pair below the base's run holds all ones
  bool fixed_base = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

int ms_engine_setup(MsEngine* m, int compute_units, int64_t wall_rate_khz, hipStream_t stream);
// Applies batch parameters (rebuilds the bottom-up ranges when the grain or
// grid changes and drops a captured search).
int ms_apply_tuning(MsEngine* m, const rbfs_tuning_t& t, hipStream_t stream);
void ms_engine_free(MsEngine* m);
int ms_enqueue_search(MsEngine* m, int32_t k, int32_t nroots, int mode, int alpha, int beta,
                      hipStream_t stream);
int ms_enqueue_translate(MsEngine* m, int64_t n_g, const int32_t* perm, int64_t n_sweep_g,
                         int64_t ubase, int32_t k, const int32_t* roots_orig_dev,
                         int32_t* out_dep, int32_t* out_par, hipStream_t stream);
int ms_enqueue_roots(const int32_t* roots_orig_dev, int32_t k, const int32_t* perm,
                     int64_t n_sweep, int64_t ubase, int32_t* roots_union, hipStream_t stream);
int ms_read_stats(MsEngine* m, hipStream_t stream, void* stats);
int ms_build_union(MsEngine* m, const struct Graph* const* gs, int count, hipStream_t stream);

// Ring of event triples (start, after search kernel, end) for timed calls.
struct TimingRing {
  static constexpr int kCap = 1024;
  hipEvent_t ev[kCap][3];
  int created = 0;
  int count = 0;
  hipError_t next(hipEvent_t** out);
  void destroy();
};

struct Graph {
  int device = 0;
  int64_t n = 0, nnz = 0;
  int64_t n_plus = 0;      // non-isolated vertices
  int64_t n_sweep = 0;     // vertices the searches cover: n_plus after RCM, else n
  int64_t max_degree = 0;
  int reordered = 0;
  int64_t rcm_keep = 0;    // after RCM: vertices of the Cuthill-McKee sequence reordered
  int64_t* off = nullptr;  // internal CSR
  int32_t* cols = nullptr;
  int32_t* perm = nullptr;   // original -> internal (after RCM)
  int32_t* iperm = nullptr;  // internal -> original
  int32_t* comp_bounds = nullptr;  // after RCM: component intervals, ascending (n_comp + 1)
  int64_t n_comp = 0;
  BfsWork* bfs = nullptr;
  MsEngine* ms = nullptr;
  rbfs_tuning_t tune_single{};  // parameters of rbfs_bfs
  rbfs_tuning_t tune_batch{};   // parameters of rbfs_bfs_batch
  Scratch scratch;
  TimingRing timing;
  int compute_units = 0;
  int64_t wall_rate_khz = 100000;
  size_t bytes = 0;
  // multi-graph handles built over this graph: they keep its perm, n and
  // n_sweep, so while any exists the graph may be neither relabelled nor
  // destroyed
  int multi_refs = 0;
  // relabel batch size of rbfs_rcm_reorder (entries; 0 = automatic)
  int64_t rcm_batch = 0;
  // relabel with the old columns in host memory: 0 = when the device is short
  // of memory, 1 = always (with batches), -1 = never
  int rcm_stage = 0;
  // single-root search: entries of each frontier sub-queue (0 = automatic)
  int64_t queue_cap = 0;
};

// Sticky error text for the calling thread.
void set_error(const std::string& msg);

// keep < 0 or >= n+: the full RCM order; otherwise the partial order that
// reorders only the first `keep` vertices of the Cuthill-McKee sequence.
int rcm_reorder_impl(Graph* g, hipStream_t stream, float* ms_out, int64_t keep = -1);
int validate_csr_impl(Graph* g, hipStream_t stream);
int bfs_impl(Graph* g, int32_t root, int32_t* depth, int32_t* parent, int mode, int alpha,
             int beta, const int8_t* sched, int sched_len, int out_space, int flags,
             int tune_profile, hipStream_t stream, void* stats);
int bfs_batch_impl(Graph* g, const int32_t* roots, int32_t k, int32_t* depth, int32_t* parent,
                   int mode, int alpha, int beta, int out_space, int flags,
                   hipStream_t stream, void* stats);
int bfs_apply_tuning(Graph* g, hipStream_t stream);
void free_bfs_work(Graph* g);
int bfs_wg_work(Graph* g, int64_t* out, int64_t cap, int32_t* levels, int32_t* grid,
                hipStream_t stream);
void free_ms_work(Graph* g);

}  // namespace rbfs
