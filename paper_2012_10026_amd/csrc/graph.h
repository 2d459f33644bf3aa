// Graph handle layout and the host entry points of the passes (RCM, BFS,
// batched BFS).  Internal to the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "prim.h"

namespace rbfs {

// Edges per chunk of the edge-balanced frontier expansion.
constexpr int kChunkEdges = 1024;

struct BfsCtl;
struct MsCtl;

// Workspace of the single-root search (sized for n_sweep vertices).
struct BfsWork {
  int64_t n_sweep = 0;
  int32_t* depth = nullptr;     // internal depth (translate mode)
  uint32_t* parent = nullptr;   // internal parent (translate mode)
  uint64_t* vis = nullptr;      // reached before the current level
  uint64_t* front = nullptr;    // three rotating frontier bitmaps
  int32_t* qv[2] = {nullptr, nullptr};
  int64_t* qe[2] = {nullptr, nullptr};
  int32_t* chunk[2] = {nullptr, nullptr};
  int64_t chunk_cap = 0;
  int32_t* bu_part = nullptr;
  int32_t n_part = 0;
  BfsCtl* ctl = nullptr;
  bool clean = false;           // depth/parent hold -1 everywhere
  int grid = 0;                 // persistent grid size
  int max_per_cu = 1;           // resident workgroups per CU (occupancy)
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
};

// Workspace of the 64-root bit-parallel search.
struct MsWork {
  int64_t n_sweep = 0;
  uint64_t* seen = nullptr;
  uint64_t* front[2] = {nullptr, nullptr};
  int32_t* dep = nullptr;       // [n_sweep][64] internal, vertex-major
  int32_t* par = nullptr;       // [n_sweep][64]
  MsCtl* ctl = nullptr;
  int32_t* roots_dev = nullptr; // 64 internal roots
  int grid = 0;
};

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
  int64_t* off = nullptr;  // internal CSR
  int32_t* cols = nullptr;
  int32_t* perm = nullptr;   // original -> internal (after RCM)
  int32_t* iperm = nullptr;  // internal -> original
  BfsWork* bfs = nullptr;
  MsWork* ms = nullptr;
  Scratch scratch;
  TimingRing timing;
  int compute_units = 0;
  int64_t wall_rate_khz = 100000;
  size_t bytes = 0;
};

// Sticky error text for the calling thread.
void set_error(const std::string& msg);

int rcm_reorder_impl(Graph* g, hipStream_t stream, float* ms_out);
int validate_csr_impl(Graph* g, hipStream_t stream);
int bfs_impl(Graph* g, int32_t root, int32_t* depth, int32_t* parent, int mode, int alpha,
             int beta, const int8_t* sched, int sched_len, int out_space, int flags,
             int tune_profile, hipStream_t stream, void* stats);
int bfs_batch_impl(Graph* g, const int32_t* roots, int32_t k, int32_t* depth, int32_t* parent,
                   int mode, int alpha, int beta, int out_space, int flags,
                   hipStream_t stream, void* stats);
void free_bfs_work(Graph* g);
void free_ms_work(Graph* g);

}  // namespace rbfs
