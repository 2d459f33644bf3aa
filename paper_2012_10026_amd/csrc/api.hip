// C ABI of librbfs: argument checking, handle lifetime, CSR validation and
// dispatch to the passes.  Nothing here computes any part of the search.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rbfs.h"
#include "common.h"
#include "graph.h"
#include "switch.h"

#include "handles.h"

namespace rbfs {

static thread_local std::string t_last_error;

void set_error(const std::string& msg) { t_last_error = msg; }

hipError_t TimingRing::next(hipEvent_t** out) {
  *out = nullptr;
  if (count >= kCap) return hipSuccess;  // full: the call is not recorded
  while (created <= count) {
    for (int j = 0; j < 3; ++j) {
      hipError_t e = hipEventCreate(&ev[created][j]);
      if (e != hipSuccess) return e;
    }
    ++created;
  }
  *out = ev[count++];
  return hipSuccess;
}

void TimingRing::destroy() {
  for (int i = 0; i < created; ++i)
    for (int j = 0; j < 3; ++j) (void)hipEventDestroy(ev[i][j]);
  created = 0;
  count = 0;
}

int bfs_check_status(Graph* g, hipStream_t stream);

namespace {

constexpr int kVBadOffsets = 1, kVColRange = 2, kVSelfLoop = 4, kVUnsorted = 8,
              kVAsymmetric = 16;

// The degree maximum and the non-isolated count are reduced per wave over
// the wave's whole grid-stride share: one atomic per wave on each of the two
// words, and few waves (the launch uses kFoldBlocks workgroups).
__global__ void check_offsets_kernel(const int64_t* off, int64_t n, int64_t nnz, int* flags,
                                     unsigned long long* maxdeg, unsigned long long* nonzero) {
  int64_t dmax = 0, nz = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = off[v], b = off[v + 1];
    if (a < 0 || b < a || b > nnz) {
      atomicOr(flags, kVBadOffsets);
      continue;
    }
    if (b > a) {
      dmax = (b - a) > dmax ? (b - a) : dmax;
      ++nz;
    }
  }
  dmax = wave_max(dmax);
  nz = wave_sum(nz);
  if (lane_id() == 0 && nz > 0) {
    atomicMax(maxdeg, (unsigned long long)dmax);
    atomicAdd(nonzero, (unsigned long long)nz);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && (off[0] != 0 || off[n] != nnz))
    atomicOr(flags, kVBadOffsets);
}

// Largest |u - v| over the adjacency entries: rows are ascending, so a row's
// first and last entries bound it.
__global__ void bandwidth_kernel(const int64_t* off, const int32_t* cols, int64_t n,
                                 unsigned long long* out) {
  unsigned long long best = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = off[v], e = off[v + 1];
    if (e > b) {
      const int64_t lo = v - cols[b], hi = (int64_t)cols[e - 1] - v;
      const int64_t m = lo > hi ? lo : hi;
      if (m > 0 && (unsigned long long)m > best) best = (unsigned long long)m;
    }
  }
  if (best) atomicMax(out, best);
}

__global__ void check_cols_kernel(const int32_t* cols, int64_t nnz, int64_t n, int* flags) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = cols[e];
    if (c < 0 || c >= n) atomicOr(flags, kVColRange);
  }
}

// Canonical form: rows strictly ascending, no self-loops, (w, v) present for
// every (v, w).  Requires valid offsets and column range.
__global__ __launch_bounds__(kBlock) void check_canonical_kernel(const int64_t* off,
                                                                 const int32_t* cols, int64_t n,
                                                                 int* flags) {
  const int64_t nwords = ceil_div(n, kWave);
  for (int64_t word = (int64_t)blockIdx.x * kWavesPerBlock + wave_id(); word < nwords;
       word += (int64_t)gridDim.x * kWavesPerBlock) {
    word_edges(off, cols, n, word, [&](int64_t v, int32_t w, int64_t e) {
      if (w == v) atomicOr(flags, kVSelfLoop);
      if (e > off[v] && cols[e - 1] >= w) atomicOr(flags, kVUnsorted);
      int64_t lo = off[w], hi = off[w + 1];
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (cols[mid] < v) lo = mid + 1; else hi = mid;
      }
      if (lo >= off[w + 1] || cols[lo] != v) atomicOr(flags, kVAsymmetric);
    });
  }
}

int grid_for(int64_t work) {
  int64_t b = ceil_div(work, kBlock);
  if (b < 1) b = 1;
  if (b > (1 << 20)) b = 1 << 20;
  return (int)b;
}

int device_ok() {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
    set_error("no HIP device");
    return RBFS_E_NODEV;
  }
  return 0;
}

}  // namespace

#define API_CHECK(x)                                                            \
  do {                                                                          \
    hipError_t e_ = (x);                                                        \
    if (e_ != hipSuccess) {                                                     \
      set_error(std::string(#x) + ": " + hipGetErrorString(e_));                \
      rc = (e_ == hipErrorOutOfMemory) ? RBFS_E_NOMEM : RBFS_E_DEVICE;          \
      goto fail;                                                                \
    }                                                                           \
  } while (0)

// ---- device memory: hipMalloc/hipFree or the caller's allocator
namespace {
std::mutex s_alloc_mu;
rbfs_alloc_fn s_alloc = nullptr;
rbfs_free_fn s_free = nullptr;
void* s_alloc_ctx = nullptr;
std::atomic<long long> s_live{0};
}  // namespace

hipError_t dev_malloc(void** p, size_t bytes, hipStream_t stream) {
  if (!s_alloc) return hipMalloc(p, bytes);
  *p = s_alloc(bytes > 0 ? bytes : 1, (void*)stream, s_alloc_ctx);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}

void dev_free(void* p, hipStream_t stream) {
  if (!p) return;
  if (s_free) s_free(p, (void*)stream, s_alloc_ctx);
  else (void)hipFree(p);
}

void live_handles_add(int d) { s_live += d; }

static int graph_setup(Graph* g, uint32_t flags, hipStream_t stream) {
  int rc = 0;
  int* d_flags = nullptr;
  unsigned long long* d_stats = nullptr;
  int hflags = 0;
  unsigned long long hstats[2] = {0, 0};
  const int64_t n = g->n, nnz = g->nnz;
  API_CHECK(rbfs::dev_malloc(&d_flags, sizeof(int)));
  API_CHECK(rbfs::dev_malloc(&d_stats, 2 * sizeof(unsigned long long)));
  API_CHECK(hipMemsetAsync(d_flags, 0, sizeof(int), stream));
  API_CHECK(hipMemsetAsync(d_stats, 0, 2 * sizeof(unsigned long long), stream));
  hipLaunchKernelGGL(check_offsets_kernel,
                     dim3((unsigned)std::min<int64_t>(grid_for(n), kFoldBlocks)), dim3(kBlock),
                     0, stream, g->off, n,
                     nnz, d_flags, d_stats, d_stats + 1);
  API_CHECK(hipGetLastError());
  if (nnz > 0) {
    hipLaunchKernelGGL(check_cols_kernel, dim3(grid_for(nnz)), dim3(kBlock), 0, stream, g->cols,
                       nnz, n, d_flags);
    API_CHECK(hipGetLastError());
  }
  API_CHECK(hipMemcpyAsync(&hflags, d_flags, sizeof(int), hipMemcpyDeviceToHost, stream));
  API_CHECK(hipMemcpyAsync(hstats, d_stats, sizeof(hstats), hipMemcpyDeviceToHost, stream));
  API_CHECK(hipStreamSynchronize(stream));
  if (hflags) {
    set_error(hflags & kVBadOffsets ? "row_offsets not monotone / not ending at nnz"
                                    : "column index out of range");
    rc = RBFS_E_INVAL;
    goto fail;
  }
  if ((flags & RBFS_VALIDATE) && n > 0) {
    const int64_t nwords = ceil_div(n, kWave);
    const int64_t blocks = std::min<int64_t>(ceil_div(nwords, kWavesPerBlock), 1 << 18);
    hipLaunchKernelGGL(check_canonical_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, stream,
                       g->off, g->cols, n, d_flags);
    API_CHECK(hipGetLastError());
    API_CHECK(hipMemcpyAsync(&hflags, d_flags, sizeof(int), hipMemcpyDeviceToHost, stream));
    API_CHECK(hipStreamSynchronize(stream));
    if (hflags) {
      std::string m = "non-canonical CSR:";
      if (hflags & kVSelfLoop) m += " self-loop";
      if (hflags & kVUnsorted) m += " row not strictly ascending";
      if (hflags & kVAsymmetric) m += " missing reverse edge";
      set_error(m);
      rc = RBFS_E_INVAL;
      goto fail;
    }
  }
  g->max_degree = (int64_t)hstats[0];
  g->n_plus = (int64_t)hstats[1];
fail:
  if (d_flags) (void)rbfs::dev_free(d_flags);
  if (d_stats) (void)rbfs::dev_free(d_stats);
  return rc;
}

}  // namespace rbfs

using rbfs::Graph;
using rbfs::set_error;

extern "C" {

const char* rbfs_last_error(void) { return rbfs::t_last_error.c_str(); }

int rbfs_device_info(rbfs_device_info_t* out) {
  if (!out) {
    set_error("rbfs_device_info: out is NULL");
    return RBFS_E_INVAL;
  }
  int rc = rbfs::device_ok();
  if (rc) return rc;
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) {
    set_error("hipGetDeviceProperties failed");
    return RBFS_E_DEVICE;
  }
  memset(out, 0, sizeof(*out));
  out->device = dev;
  out->compute_units = p.multiProcessorCount;
  out->wavefront_size = p.warpSize;
  out->clock_khz = p.clockRate;
  out->global_mem_bytes = (int64_t)p.totalGlobalMem;
  out->l2_bytes = p.l2CacheSize;
  strncpy(out->arch, p.gcnArchName, sizeof(out->arch) - 1);
  return RBFS_OK;
}

int rbfs_set_allocator(rbfs_alloc_fn alloc, rbfs_free_fn free_fn, void* ctx) {
  if ((alloc == nullptr) != (free_fn == nullptr)) {
    set_error("rbfs_set_allocator: give both functions or neither");
    return RBFS_E_INVAL;
  }
  std::lock_guard<std::mutex> lock(rbfs::s_alloc_mu);
  if (rbfs::s_live.load() != 0) {
    set_error("rbfs_set_allocator: graph or multi-graph handles still exist");
    return RBFS_E_STATE;
  }
  rbfs::s_alloc = alloc;
  rbfs::s_free = free_fn;
  rbfs::s_alloc_ctx = alloc ? ctx : nullptr;
  return RBFS_OK;
}

int rbfs_graph_create(int64_t n, int64_t nnz, const int64_t* row_offsets, const int32_t* cols,
                      uint32_t flags, void* stream_, rbfs_graph_t** out) {
  if (!out) {
    set_error("rbfs_graph_create: out is NULL");
    return RBFS_E_INVAL;
  }
  *out = nullptr;
  if (n < 0 || n >= 0x7FFFFFFFll || nnz < 0) {
    set_error("rbfs_graph_create: n must be in [0, 2^31-1) and nnz >= 0");
    return RBFS_E_RANGE;
  }
  if (!row_offsets || (nnz > 0 && !cols)) {
    set_error("rbfs_graph_create: NULL row_offsets or cols");
    return RBFS_E_INVAL;
  }
  if (flags & ~(RBFS_HOST_PTRS | RBFS_VALIDATE)) {
    set_error("rbfs_graph_create: unknown flags");
    return RBFS_E_INVAL;
  }
  if (flags & RBFS_HOST_PTRS) {
    if (row_offsets[0] != 0 || row_offsets[n] != nnz) {
      set_error("rbfs_graph_create: row_offsets[0] != 0 or row_offsets[n] != nnz");
      return RBFS_E_INVAL;
    }
  }
  int rc = rbfs::device_ok();
  if (rc) return rc;
  hipStream_t stream = (hipStream_t)stream_;
  rbfs_graph_t* h = new rbfs_graph_t();
  Graph* g = &h->g;
  hipDeviceProp_t p;
  const hipMemcpyKind kind =
      (flags & RBFS_HOST_PTRS) ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  int rate = 0;
  API_CHECK(hipGetDevice(&g->device));
  API_CHECK(hipGetDeviceProperties(&p, g->device));
  g->compute_units = p.multiProcessorCount;
  g->tune_single = rbfs::default_tuning(RBFS_TUNE_SINGLE);
  g->tune_batch = rbfs::default_tuning(RBFS_TUNE_BATCH);
  if (hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, g->device) == hipSuccess &&
      rate > 0)
    g->wall_rate_khz = rate;
  g->n = n;
  g->nnz = nnz;
  g->n_sweep = n;
  API_CHECK(rbfs::dev_malloc(&g->off, sizeof(int64_t) * (size_t)(n + 1)));
  // kColPad entries of slack: row scans read whole aligned 16-byte groups
  API_CHECK(rbfs::dev_malloc(&g->cols, sizeof(int32_t) * (size_t)(nnz + rbfs::kColPad)));
  g->bytes = sizeof(int64_t) * (size_t)(n + 1) + sizeof(int32_t) * (size_t)nnz;
  API_CHECK(hipMemcpyAsync(g->off, row_offsets, sizeof(int64_t) * (size_t)(n + 1), kind, stream));
  if (nnz > 0)
    API_CHECK(hipMemcpyAsync(g->cols, cols, sizeof(int32_t) * (size_t)nnz, kind, stream));
  rc = rbfs::graph_setup(g, flags, stream);
  if (rc) goto fail;
  rbfs::live_handles_add(1);
  *out = h;
  return RBFS_OK;
fail:
  if (g->off) (void)rbfs::dev_free(g->off);
  if (g->cols) (void)rbfs::dev_free(g->cols);
  delete h;
  return rc ? rc : RBFS_E_DEVICE;
}

int rbfs_graph_destroy(rbfs_graph_t* h) {
  if (!h) return RBFS_OK;
  Graph* g = &h->g;
  if (g->multi_refs > 0) {
    set_error("rbfs_graph_destroy: a multi-graph handle still uses this graph");
    return RBFS_E_STATE;
  }
  (void)hipSetDevice(g->device);
  // work still queued on any stream may use the memory released below
  (void)hipDeviceSynchronize();
  rbfs::free_bfs_work(g);
  rbfs::free_ms_work(g);
  g->scratch.release();
  g->timing.destroy();
  if (g->off) (void)rbfs::dev_free(g->off);
  if (g->cols) (void)rbfs::dev_free(g->cols);
  if (g->perm) (void)rbfs::dev_free(g->perm);
  if (g->iperm) (void)rbfs::dev_free(g->iperm);
  if (g->comp_bounds) (void)rbfs::dev_free(g->comp_bounds);
  delete h;
  rbfs::live_handles_add(-1);
  return RBFS_OK;
}

int rbfs_graph_info(const rbfs_graph_t* h, rbfs_graph_info_t* out) {
  if (!h || !out) {
    set_error("rbfs_graph_info: NULL argument");
    return RBFS_E_INVAL;
  }
  const Graph* g = &h->g;
  memset(out, 0, sizeof(*out));
  out->n = g->n;
  out->nnz = g->nnz;
  out->n_plus = g->n_plus;
  out->rcm_keep = g->reordered ? g->rcm_keep : 0;
  out->reordered = g->reordered;
  out->device = g->device;
  out->max_degree = g->max_degree;
  out->device_bytes = (int64_t)g->bytes;
  return RBFS_OK;
}

static int rcm_reorder_call(rbfs_graph_t* h, int64_t keep, int32_t* perm_out, void* stream_,
                            float* ms_out) {
  if (!h) {
    set_error("rbfs_rcm_reorder: NULL graph");
    return RBFS_E_INVAL;
  }
  Graph* g = &h->g;
  hipStream_t stream = (hipStream_t)stream_;
  if (hipSetDevice(g->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return RBFS_E_DEVICE;
  }
  int rc = 0;
  if (!g->reordered) {
    if (g->n == 0) {
      set_error("rbfs_rcm_reorder: empty graph");
      return RBFS_E_INVAL;
    }
    if (g->multi_refs > 0) {
      set_error("rbfs_rcm_reorder: a multi-graph handle uses this graph in its current labels");
      return RBFS_E_STATE;
    }
    rc = rbfs::rcm_reorder_impl(g, stream, ms_out, keep);
    if (rc) return rc;
  } else if (ms_out) {
    *ms_out = 0.f;
  }
  if (perm_out) {
    API_CHECK(hipMemcpyAsync(perm_out, g->perm, sizeof(int32_t) * (size_t)g->n,
                             hipMemcpyDeviceToDevice, stream));
    API_CHECK(hipStreamSynchronize(stream));
  }
  return RBFS_OK;
fail:
  return rc;
}

int rbfs_graph_set_rcm_batch(rbfs_graph_t* h, int64_t max_entries) {
  if (!h || max_entries < 0) {
    set_error("rbfs_graph_set_rcm_batch: NULL graph or negative size");
    return RBFS_E_INVAL;
  }
  h->g.rcm_batch = max_entries;
  return RBFS_OK;
}

int rbfs_graph_set_rcm_staging(rbfs_graph_t* h, int32_t mode) {
  if (!h || mode < -1 || mode > 1) {
    set_error("rbfs_graph_set_rcm_staging: NULL graph or mode outside [-1, 1]");
    return RBFS_E_INVAL;
  }
  h->g.rcm_stage = mode;
  return RBFS_OK;
}

int rbfs_graph_set_queue_cap(rbfs_graph_t* h, int64_t entries) {
  if (!h || entries < 0) {
    set_error("rbfs_graph_set_queue_cap: NULL graph or negative size");
    return RBFS_E_INVAL;
  }
  (void)hipSetDevice(h->g.device);
  (void)hipDeviceSynchronize();  // the workspace may still be in use
  h->g.queue_cap = entries;
  rbfs::free_bfs_work(&h->g);    // rebuilt with the new size by the next search
  return RBFS_OK;
}

int rbfs_rcm_reorder(rbfs_graph_t* h, int32_t* perm_out, void* stream, float* ms_out) {
  return rcm_reorder_call(h, -1, perm_out, stream, ms_out);
}

int rbfs_rcm_reorder_partial(rbfs_graph_t* h, int64_t keep, int32_t* perm_out, void* stream,
                             float* ms_out) {
  return rcm_reorder_call(h, keep, perm_out, stream, ms_out);
}

int rbfs_graph_iperm(const rbfs_graph_t* h, int32_t* iperm_out, void* stream_) {
  if (!h || !iperm_out) {
    set_error("rbfs_graph_iperm: NULL argument");
    return RBFS_E_INVAL;
  }
  const Graph* g = &h->g;
  hipStream_t stream = (hipStream_t)stream_;
  int rc = 0;
  if (!g->reordered) {
    std::string msg = "rbfs_graph_iperm: graph not reordered";
    set_error(msg);
    return RBFS_E_STATE;
  }
  API_CHECK(hipMemcpyAsync(iperm_out, g->iperm, sizeof(int32_t) * (size_t)g->n,
                           hipMemcpyDeviceToDevice, stream));
  API_CHECK(hipStreamSynchronize(stream));
  return RBFS_OK;
fail:
  return rc;
}

int rbfs_graph_csr(const rbfs_graph_t* h, int64_t* row_offsets_out, int32_t* cols_out,
                   void* stream_) {
  if (!h || !row_offsets_out || (!cols_out && h->g.nnz > 0)) {
    set_error("rbfs_graph_csr: NULL argument");
    return RBFS_E_INVAL;
  }
  const Graph* g = &h->g;
  hipStream_t stream = (hipStream_t)stream_;
  int rc = 0;
  API_CHECK(hipMemcpyAsync(row_offsets_out, g->off, sizeof(int64_t) * (size_t)(g->n + 1),
                           hipMemcpyDeviceToDevice, stream));
  if (g->nnz > 0)
    API_CHECK(hipMemcpyAsync(cols_out, g->cols, sizeof(int32_t) * (size_t)g->nnz,
                             hipMemcpyDeviceToDevice, stream));
  API_CHECK(hipStreamSynchronize(stream));
  return RBFS_OK;
fail:
  return rc;
}

int rbfs_graph_bandwidth(const rbfs_graph_t* h, int64_t* out, void* stream_) {
  if (!h || !out) {
    set_error("rbfs_graph_bandwidth: NULL argument");
    return RBFS_E_INVAL;
  }
  const Graph* g = &h->g;
  hipStream_t stream = (hipStream_t)stream_;
  int rc = 0;
  unsigned long long* d = nullptr;
  unsigned long long hv = 0;
  API_CHECK(hipSetDevice(g->device));
  API_CHECK(rbfs::dev_malloc(&d, sizeof(unsigned long long), stream));
  API_CHECK(hipMemsetAsync(d, 0, sizeof(unsigned long long), stream));
  if (g->n > 0 && g->nnz > 0) {
    const int64_t blocks =
        std::max<int64_t>(1, std::min<int64_t>(rbfs::ceil_div(g->n, rbfs::kBlock), 4096));
    hipLaunchKernelGGL(rbfs::bandwidth_kernel, dim3((unsigned)blocks), dim3(rbfs::kBlock), 0, stream, g->off,
                       g->cols, g->n, d);
    API_CHECK(hipGetLastError());
  }
  API_CHECK(hipMemcpyAsync(&hv, d, sizeof(hv), hipMemcpyDeviceToHost, stream));
  API_CHECK(hipStreamSynchronize(stream));
  rbfs::dev_free(d, stream);
  *out = (int64_t)hv;
  return RBFS_OK;
fail:
  if (d) {
    (void)hipStreamSynchronize(stream);
    rbfs::dev_free(d, stream);
  }
  return rc;
}

static int parse_opts(const rbfs_opts_t* o, int* mode, int* alpha, int* beta, int* out_space) {
  *mode = RBFS_DIR_HEURISTIC;
  *alpha = 14;
  *beta = 24;
  *out_space = RBFS_OUT_ORIGINAL;
  if (!o) return 0;
  if (o->direction < RBFS_DIR_HEURISTIC || o->direction > RBFS_DIR_LEARNED ||
      o->alpha <= 0 || o->beta <= 0 ||
      (o->output_space != RBFS_OUT_ORIGINAL && o->output_space != RBFS_OUT_INTERNAL)) {
    set_error("invalid rbfs_opts_t");
    return RBFS_E_INVAL;
  }
  *mode = o->direction;
  *alpha = o->alpha;
  *beta = o->beta;
  *out_space = o->output_space;
  return 0;
}

int rbfs_bfs(rbfs_graph_t* h, int32_t root, int32_t* depth, int32_t* parent,
             const rbfs_opts_t* opts, void* stream_, rbfs_stats_t* stats) {
  if (!h || !depth || !parent) {
    set_error("rbfs_bfs: NULL argument");
    return RBFS_E_INVAL;
  }
  Graph* g = &h->g;
  if (root < 0 || root >= g->n) {
    set_error("rbfs_bfs: root out of range");
    return RBFS_E_RANGE;
  }
  int mode, alpha, beta, out_space;
  int rc = parse_opts(opts, &mode, &alpha, &beta, &out_space);
  if (rc) return rc;
  if (hipSetDevice(g->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return RBFS_E_DEVICE;
  }
  return rbfs::bfs_impl(g, root, depth, parent, mode, alpha, beta,
                        opts ? opts->schedule : nullptr, opts ? opts->schedule_len : 0,
                        out_space, opts ? opts->flags : 0, opts ? opts->tune_profile : 0,
                        (hipStream_t)stream_, stats);
}

int rbfs_graph_wg_work(rbfs_graph_t* h, int64_t* out, int64_t cap, int32_t* levels,
                       int32_t* grid, void* stream) {
  if (!h || !levels || !grid || cap < 0 || (cap > 0 && !out)) {
    set_error("rbfs_graph_wg_work: bad arguments");
    return RBFS_E_INVAL;
  }
  return rbfs::bfs_wg_work(&h->g, out, cap, levels, grid, (hipStream_t)stream);
}

int rbfs_graph_timings(rbfs_graph_t* h, float* kernel_ms, float* total_ms, int32_t cap,
                       int32_t* count, void* stream_) {
  if (!h || !count || cap < 0 || (cap > 0 && (!kernel_ms || !total_ms))) {
    set_error("rbfs_graph_timings: bad arguments");
    return RBFS_E_INVAL;
  }
  Graph* g = &h->g;
  int rc = 0;
  const int nrec = g->timing.count;
  const int nout = nrec < cap ? nrec : cap;
  API_CHECK(hipStreamSynchronize((hipStream_t)stream_));
  for (int i = 0; i < nout; ++i) {
    API_CHECK(hipEventElapsedTime(&kernel_ms[i], g->timing.ev[i][0], g->timing.ev[i][1]));
    API_CHECK(hipEventElapsedTime(&total_ms[i], g->timing.ev[i][0], g->timing.ev[i][2]));
  }
  *count = nout;
  g->timing.count = 0;
  return RBFS_OK;
fail:
  g->timing.count = 0;
  return rc;
}

int rbfs_bfs_batch(rbfs_graph_t* h, const int32_t* roots, int32_t k, int32_t* depth,
                   int32_t* parent, const rbfs_opts_t* opts, void* stream_, rbfs_stats_t* stats) {
  if (!h || !roots || !depth || !parent || k < 1) {
    set_error("rbfs_bfs_batch: NULL argument or k < 1");
    return RBFS_E_INVAL;
  }
  Graph* g = &h->g;
  for (int32_t j = 0; j < k; ++j) {
    if (roots[j] < 0 || roots[j] >= g->n) {
      set_error("rbfs_bfs_batch: root out of range");
      return RBFS_E_RANGE;
    }
  }
  int mode, alpha, beta, out_space;
  int rc = parse_opts(opts, &mode, &alpha, &beta, &out_space);
  if (rc) return rc;
  if (mode == RBFS_DIR_SCHEDULE || mode == RBFS_DIR_LEARNED) {
    set_error("rbfs_bfs_batch: direction mode not supported for batches");
    return RBFS_E_UNSUPPORTED;
  }
  if (hipSetDevice(g->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return RBFS_E_DEVICE;
  }
  return rbfs::bfs_batch_impl(g, roots, k, depth, parent, mode, alpha, beta, out_space,
                              opts ? opts->flags : 0, (hipStream_t)stream_, stats);
}

int rbfs_multi_create(rbfs_graph_t* const* graphs, int32_t count, void* stream_,
                      rbfs_multi_t** out) {
  if (!graphs || !out || count < 1) {
    set_error("rbfs_multi_create: NULL argument or count < 1");
    return RBFS_E_INVAL;
  }
  *out = nullptr;
  for (int32_t i = 0; i < count; ++i) {
    if (!graphs[i]) {
      set_error("rbfs_multi_create: NULL graph");
      return RBFS_E_INVAL;
    }
    if (graphs[i]->g.device != graphs[0]->g.device ||
        graphs[i]->g.reordered != graphs[0]->g.reordered) {
      set_error("rbfs_multi_create: graphs differ in device or RCM state");
      return RBFS_E_STATE;
    }
  }
  if (hipSetDevice(graphs[0]->g.device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return RBFS_E_DEVICE;
  }
  hipStream_t stream = (hipStream_t)stream_;
  rbfs_multi_t* m = new rbfs_multi_t();
  m->device = graphs[0]->g.device;
  int64_t ub = 0, ob = 0;
  for (int32_t i = 0; i < count; ++i) {
    Graph* g = &graphs[i]->g;
    m->gs.push_back(g);
    m->ubase.push_back(ub);
    m->out_off.push_back(ob);
    ub += g->n_sweep;
    ob += g->n;
  }
  if (ub >= 0x7FFFFFFFll) {
    delete m;
    set_error("rbfs_multi_create: union too large");
    return RBFS_E_RANGE;
  }
  m->eng.ngraphs = count;
  m->eng.fixed_base = true;  // the search is captured and replayed
  std::vector<const Graph*> cg(m->gs.begin(), m->gs.end());
  int rc = rbfs::ms_build_union(&m->eng, cg.data(), count, stream);
  if (!rc) rc = rbfs::ms_engine_setup(&m->eng, graphs[0]->g.compute_units,
                                      graphs[0]->g.wall_rate_khz, stream);
  if (!rc && hipStreamCreateWithFlags(&m->own_stream, hipStreamNonBlocking) != hipSuccess) {
    set_error("rbfs_multi_create: stream creation failed");
    rc = RBFS_E_DEVICE;
  }
  if (rc) {
    rbfs::ms_engine_free(&m->eng);
    delete m;
    return rc;
  }
  for (Graph* g : m->gs) ++g->multi_refs;
  rbfs::live_handles_add(1);
  *out = m;
  return RBFS_OK;
}

int rbfs_multi_destroy(rbfs_multi_t* m) {
  if (!m) return RBFS_OK;
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  for (Graph* g : m->gs) --g->multi_refs;
  rbfs::ms_engine_free(&m->eng);
  if (m->own_stream) (void)hipStreamDestroy(m->own_stream);
  delete m;
  rbfs::live_handles_add(-1);
  return RBFS_OK;
}

// Enqueues the whole multi-graph search: roots upload, root mapping, the
// persistent search kernel and one output transpose per graph.
static int multi_enqueue(rbfs_multi_t* m, int32_t k, int32_t* depth, int32_t* parent, int mode,
                         int alpha, int beta, hipStream_t stream) {
  rbfs::MsEngine* e = &m->eng;
  const int G = (int)m->gs.size();
  int32_t* orig_dev = e->roots_dev + 64 * G;
  hipError_t he = hipMemcpyAsync(orig_dev, e->roots_host, sizeof(int32_t) * 64 * G,
                                 hipMemcpyHostToDevice, stream);
  if (he != hipSuccess) {
    set_error(std::string("rbfs_bfs_multi: roots upload: ") + hipGetErrorString(he));
    return RBFS_E_DEVICE;
  }
  for (int i = 0; i < G; ++i) {
    Graph* g = m->gs[i];
    int rc = rbfs::ms_enqueue_roots(orig_dev + 64 * i, k, g->reordered ? g->perm : nullptr,
                                    g->n_sweep, m->ubase[i], e->roots_dev + k * i, stream);
    if (rc) return rc;
  }
  int rc = rbfs::ms_enqueue_search(e, k, k * G, mode, alpha, beta, stream);
  if (rc) return rc;
  for (int i = 0; i < G; ++i) {
    Graph* g = m->gs[i];
    rc = rbfs::ms_enqueue_translate(e, g->n, g->reordered ? g->perm : nullptr, g->n_sweep,
                                    m->ubase[i], k, orig_dev + 64 * i,
                                    depth + (int64_t)k * m->out_off[i],
                                    parent + (int64_t)k * m->out_off[i], stream);
    if (rc) return rc;
  }
  return 0;
}

int rbfs_bfs_multi(rbfs_multi_t* m, const int32_t* roots, int32_t k, int32_t* depth,
                   int32_t* parent, const rbfs_opts_t* opts, void* stream_, rbfs_stats_t* stats) {
  if (!m || !roots || !depth || !parent || k < 1 || k > 64) {
    set_error("rbfs_bfs_multi: NULL argument or k outside [1, 64]");
    return RBFS_E_INVAL;
  }
  const int G = (int)m->gs.size();
  for (int i = 0; i < G; ++i)
    for (int32_t j = 0; j < k; ++j) {
      const int32_t r = roots[(int64_t)i * k + j];
      if (r < 0 || r >= m->gs[i]->n) {
        set_error("rbfs_bfs_multi: root out of range");
        return RBFS_E_RANGE;
      }
    }
  int mode, alpha, beta, out_space;
  int rc = parse_opts(opts, &mode, &alpha, &beta, &out_space);
  if (rc) return rc;
  if (out_space != RBFS_OUT_ORIGINAL || mode == RBFS_DIR_SCHEDULE || mode == RBFS_DIR_LEARNED) {
    set_error("rbfs_bfs_multi: unsupported options");
    return RBFS_E_UNSUPPORTED;
  }
  if (hipSetDevice(m->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return RBFS_E_DEVICE;
  }
  // stream capture is not possible on the legacy NULL stream: run on an own
  // stream then (the call synchronises before returning either way)
  hipStream_t stream = (hipStream_t)stream_;
  if (!stream) {
    if (hipStreamSynchronize(nullptr) != hipSuccess) {
      set_error("rbfs_bfs_multi: stream error");
      return RBFS_E_DEVICE;
    }
    stream = m->own_stream;
  }
  rbfs::MsEngine* e = &m->eng;
  // the pinned roots buffer is read by the (possibly captured) upload: make
  // sure the previous search has consumed it
  if (hipStreamSynchronize(stream) != hipSuccess) {
    set_error("rbfs_bfs_multi: stream error");
    return RBFS_E_DEVICE;
  }
  for (int i = 0; i < G; ++i)
    for (int32_t j = 0; j < k; ++j) e->roots_host[64 * i + j] = roots[(int64_t)i * k + j];
  const bool same = e->gexec && m->cap_k == k && m->cap_depth == depth &&
                    m->cap_parent == parent && m->cap_mode == mode && m->cap_alpha == alpha &&
                    m->cap_beta == beta && m->cap_stream == stream;
  if (!same) {
    if (e->gexec) (void)hipGraphExecDestroy(e->gexec);
    e->gexec = nullptr;
    hipGraph_t graph = nullptr;
    hipError_t he = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    if (he != hipSuccess) {
      set_error(std::string("rbfs_bfs_multi: begin capture: ") + hipGetErrorString(he));
      return RBFS_E_DEVICE;
    }
    rc = multi_enqueue(m, k, depth, parent, mode, alpha, beta, stream);
    he = hipStreamEndCapture(stream, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (he == hipSuccess) he = hipGraphInstantiate(&e->gexec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (he != hipSuccess) {
      e->gexec = nullptr;
      set_error(std::string("rbfs_bfs_multi: capture: ") + hipGetErrorString(he));
      return RBFS_E_DEVICE;
    }
    m->cap_k = k;
    m->cap_depth = depth;
    m->cap_parent = parent;
    m->cap_mode = mode;
    m->cap_alpha = alpha;
    m->cap_beta = beta;
    m->cap_stream = stream;
  }
  hipError_t he = hipGraphLaunch(e->gexec, stream);
  if (he != hipSuccess) {
    set_error(std::string("rbfs_bfs_multi: launch: ") + hipGetErrorString(he));
    return RBFS_E_DEVICE;
  }
  return rbfs::ms_read_stats(e, stream, stats);
}

int rbfs_collect_level_samples(rbfs_graph_t* h, const int32_t* roots, int32_t k, int32_t reps,
                               int32_t alpha, int32_t beta, float* out, int32_t cap,
                               int32_t* count, void* stream_) {
  if (!h || !roots || !out || !count || k < 1 || reps < 1 || cap < 0 || alpha <= 0 ||
      beta <= 0) {
    set_error("rbfs_collect_level_samples: bad arguments");
    return RBFS_E_INVAL;
  }
  Graph* g = &h->g;
  for (int32_t j = 0; j < k; ++j)
    if (roots[j] < 0 || roots[j] >= g->n) {
      set_error("rbfs_collect_level_samples: root out of range");
      return RBFS_E_RANGE;
    }
  if (hipSetDevice(g->device) != hipSuccess) {
    set_error("hipSetDevice failed");
    return RBFS_E_DEVICE;
  }
  hipStream_t stream = (hipStream_t)stream_;
  int rc = 0;
  int32_t *dd = nullptr, *dp = nullptr;
  int32_t cnt = 0;
  rbfs_stats_t sh, st;
  std::vector<float> t;
  int8_t sched[RBFS_STATS_MAX_LEVELS + 1];
  API_CHECK(rbfs::dev_malloc(&dd, sizeof(int32_t) * (size_t)(g->n > 0 ? g->n : 1)));
  API_CHECK(rbfs::dev_malloc(&dp, sizeof(int32_t) * (size_t)(g->n > 0 ? g->n : 1)));
  for (int32_t j = 0; j < k && cnt < cap; ++j) {
    rc = rbfs::bfs_impl(g, roots[j], dd, dp, RBFS_DIR_HEURISTIC, alpha, beta, nullptr, 0,
                        RBFS_OUT_INTERNAL, 0, 0, stream, &sh);
    if (rc) goto fail;
    {
      const int D = std::min(sh.levels, RBFS_STATS_MAX_LEVELS);
      long long reached = 1;
      for (int d = 1; d < D && cnt < cap; ++d) {
        reached += sh.nf[d];
        // the alpha/beta path up to level d - 1, and (from level 2 on) the same
        // path with level d - 1 flipped, so that both values of the current-
        // direction feature are sampled
        for (int variant = 0; variant < (d >= 2 ? 2 : 1) && cnt < cap; ++variant) {
          for (int i = 0; i < d; ++i) sched[i] = sh.dir[i];
          if (variant) sched[d - 1] = (int8_t)(1 - sched[d - 1]);
          float lab[2];
          for (int x = 0; x < 2; ++x) {
            sched[d] = (int8_t)x;
            // the levels after d follow the alpha/beta rule from direction x
            // (its inputs, the frontier sizes, do not depend on the directions)
            for (int e = d + 1; e < D; ++e)
              sched[e] = (int8_t)rbfs::heuristic_dir(sched[e - 1], sh.nf[e], sh.mf[e], sh.mu[e],
                                                     sh.nf[e - 1], g->n_sweep, alpha, beta);
            t.clear();
            for (int32_t r = 0; r < reps; ++r) {
              rc = rbfs::bfs_impl(g, roots[j], dd, dp, RBFS_DIR_SCHEDULE, alpha, beta, sched,
                                  std::max(D, d + 1), RBFS_OUT_INTERNAL, 0, 0, stream, &st);
              if (rc) goto fail;
              // the cost from level d to the end of the search
              const int De = std::min(st.levels, RBFS_STATS_MAX_LEVELS);
              float c2g = 0.f;
              for (int e = d; e < De; ++e) c2g += st.level_us[e];
              if (De > d) t.push_back(c2g);
            }
            if (t.empty()) break;
            std::sort(t.begin(), t.end());
            lab[x] = t[t.size() / 2];
          }
          if (t.empty()) continue;
          float* row = out + (int64_t)cnt * 11;
          rbfs::switch_features(row, sh.nf[d], sh.mf[d], sh.mu[d], g->n_sweep - reached,
                                sh.nf[d - 1], d, sched[d - 1], g->n_sweep, g->nnz);
          row[8] = logf(std::max(lab[0], 0.1f));
          row[9] = logf(std::max(lab[1], 0.1f));
          row[10] = (float)d;
          ++cnt;
        }
      }
    }
  }
  *count = cnt;
fail:
  if (dd) (void)rbfs::dev_free(dd);
  if (dp) (void)rbfs::dev_free(dp);
  return rc;
}

int rbfs_collect_level_timings(rbfs_graph_t* g, const int32_t* roots, int32_t k, int32_t reps,
                               int32_t alpha, int32_t beta, float* out, int32_t cap,
                               int32_t* count, void* stream) {
  return rbfs_collect_level_samples(g, roots, k, reps, alpha, beta, out, cap, count, stream);
}

int rbfs_graph_check(rbfs_graph_t* h, void* stream_) {
  if (!h) {
    set_error("rbfs_graph_check: NULL graph");
    return RBFS_E_INVAL;
  }
  return rbfs::bfs_check_status(&h->g, (hipStream_t)stream_);
}

}  // extern "C"
