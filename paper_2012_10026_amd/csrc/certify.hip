// BFS certificate on the GPU: checks, in O(nnz), that (depth, parent) is the
// search result the library defines (the predecessor map of section 2.1 with
// the largest-label parent), with no reference run.  Rules, for every vertex
// v with depth d(v) and parent p(v):
//   the root has depth 0 and is its own parent; no other vertex has depth 0;
//   an unreached vertex (depth -1) has parent -1;
//   no edge joins a reached and an unreached vertex, and no edge spans more
//   than one level;
//   a reached v other than the root has p(v) among its neighbours one level
//   up, and no neighbour one level up has a larger label than p(v).
// The first two edge rules give depth = hop distance and reached set = the
// root's component (any path from the root climbs at most one level per
// edge, and the parent chain gives a path of d(v) edges); the last rule makes
// the parent the unique largest.  Labels are the graph's current ones.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "../../include/rbfs.h"
#include "common.h"
#include "graph.h"
#include "handles.h"

namespace rbfs {
namespace {

constexpr int kCertBlock = 256;
constexpr int kCertLane = 64;      // rows longer than this are checked by the whole wave
constexpr int kCertLong = 4096;    // rows longer than this are split over workgroups
constexpr int kCertChunk = 16384;  // entries of a long row per workgroup

// Output index of internal vertex v, and internal label of output value x.
struct CertMap {
  const int32_t* perm;   // original -> internal (null: identity)
  const int32_t* iperm;  // internal -> original (null: identity)
  __device__ __forceinline__ int64_t out(int64_t v) const { return iperm ? iperm[v] : v; }
  __device__ __forceinline__ int64_t in(int64_t x) const { return perm ? perm[x] : x; }
};

// Rule check of one adjacency entry (v, w) of a vertex at depth dv with
// parent p (internal labels); dw = depth of w.  Sets isp when w is the
// parent one level up.
__device__ __forceinline__ int cert_edge(int32_t dv, int64_t p, int32_t w, int32_t dw,
                                         bool& isp) {
  if ((dv < 0) != (dw < 0)) return -2;
  if (dv >= 0 && (dv - dw > 1 || dw - dv > 1)) return -3;
  if (dv > 0 && dw == dv - 1) {
    if (w == p) isp = true;
    else if (w > p) return -6;
  }
  return 0;
}

// depth in internal order: dint[v] = depth[iperm[v]] (one gather per vertex,
// so that the entry checks read one array instead of two in a row)
__global__ void cert_gather_kernel(int64_t n, const int32_t* iperm, const int32_t* depth,
                                   int32_t* dint) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    dint[v] = depth[iperm[v]];
}

// Per-vertex rules and the rows up to kCertLong entries: short rows by one
// lane, longer ones by the whole wave.  Vertices whose rows are longer and
// whose own entries are in order go to the long-row list (lv, *lcount).
__global__ __launch_bounds__(kCertBlock) void certify_kernel(
    int64_t n, const int64_t* off, const int32_t* cols, CertMap map, const int32_t* root_perm,
    int32_t root_orig, const int32_t* dint, const int32_t* parent, int* result, int32_t* lv,
    int* lcount, int64_t lcap) {
  const int l = lane_id();
  const int64_t root = root_perm ? root_perm[root_orig] : root_orig;
  const int64_t nwaves = ((int64_t)gridDim.x * kCertBlock) / kWave;
  const int64_t w0 = ((int64_t)blockIdx.x * kCertBlock + threadIdx.x) / kWave;
  for (int64_t base = w0 * kWave; base < n; base += nwaves * kWave) {
    const int64_t v = base + l;
    int code = 0;
    int32_t dv = -1;
    int64_t p = -1, b = 0, e = 0;
    if (v < n) {
      dv = dint[v];
      const int32_t pv = parent[map.out(v)];
      b = off[v];
      e = off[v + 1];
      if (dv < -1 || pv < -1 || pv >= n) {
        code = -7;
      } else {
        p = pv >= 0 ? map.in(pv) : -1;
        if (v == root) {
          if (dv != 0 || p != root) code = -1;
        } else if (dv == 0) {
          code = -1;
        } else if (dv == -1 && pv != -1) {
          code = -4;
        }
      }
    }
    // short rows: one lane each
    bool found = false;
    if (v < n && !code && e - b <= kCertLane) {
      for (int64_t j = b; j < e && !code; ++j) {
        const int32_t w = cols[j];
        code = cert_edge(dv, p, w, dint[w], found);
      }
    }
    // rows too long for a wave go to the long-row list
    const bool longrow = v < n && !code && e - b > kCertLong;
    const uint64_t lm = ballot(longrow);
    if (lm) {
      int lb = 0;
      if (l == ffs64(lm)) lb = atomicAdd(lcount, popc64(lm));
      lb = shfl(lb, ffs64(lm));
      const int64_t pos = (int64_t)lb + popc64(lm & lanemask_lt());
      if (longrow) {
        if (pos < lcap) lv[pos] = (int32_t)v;
        else code = -7;  // cannot happen: lcap rows of more than kCertLong entries exceed nnz
      }
    }
    // medium rows: the whole wave, 64 entries per step
    uint64_t meds = ballot(v < n && !code && e - b > kCertLane && e - b <= kCertLong);
    while (meds) {
      const int h = ffs64(meds);
      meds &= meds - 1;
      const int64_t hb = shfl(b, h), he = shfl(e, h), hp = shfl(p, h);
      const int32_t hd = shfl(dv, h);
      int hcode = 0;
      bool hfound = false;
      for (int64_t j0 = hb; j0 < he && !hcode; j0 += kWave) {
        const int64_t j = j0 + l;
        int c = 0;
        bool isp = false;
        if (j < he) {
          const int32_t w = cols[j];
          c = cert_edge(hd, hp, w, dint[w], isp);
        }
        const bool any_parent = ballot(isp) != 0ull;
        hfound = hfound || any_parent;
        const uint64_t bad = ballot(c != 0);
        if (bad) hcode = shfl(c, ffs64(bad));
      }
      if (l == h) {
        code = hcode;
        found = hfound;
      }
    }
    const bool checked = v < n && !code && e - b <= kCertLong;
    if (checked && dv > 0 && v != root && !found) code = -5;
    if (code) atomicMin(result, code);
  }
}

// Chunk plan of the long-row list, one workgroup of kPlanBlock threads:
// row i of the list is cut into ceil(len / kCertChunk) chunks, cpre is the
// exclusive prefix of those counts (cpre[nl] = number of chunks), and the
// row's found flag starts at zero.  nl is read from the device counter.
constexpr int kPlanBlock = 1024;
__global__ __launch_bounds__(kPlanBlock) void cert_long_plan_kernel(
    const int32_t* lv, const int* lcount, int64_t lcap, const int64_t* off, int64_t* cpre,
    int* lfound) {
  __shared__ int64_t s_wave[kPlanBlock / kWave];
  __shared__ int64_t s_carry;
  const int64_t nl = min((int64_t)*lcount, lcap);
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nl; base += kPlanBlock) {
    const int64_t i = base + threadIdx.x;
    int64_t cnt = 0;
    if (i < nl) {
      const int64_t v = lv[i];
      cnt = (off[v + 1] - off[v] + kCertChunk - 1) / kCertChunk;
      lfound[i] = 0;
    }
    const int64_t inc = wave_inclusive_sum(cnt);
    if (lane_id() == kWave - 1) s_wave[wave_id()] = inc;
    __syncthreads();
    int64_t before = s_carry;
    for (int w = 0; w < wave_id(); ++w) before += s_wave[w];
    if (i < nl) cpre[i] = before + inc - cnt;
    __syncthreads();
    if (threadIdx.x == kPlanBlock - 1) s_carry = before + inc;
    __syncthreads();
  }
  if (threadIdx.x == 0) cpre[nl] = s_carry;
}

// One chunk of a long row per workgroup and step: chunk c belongs to the
// list row i with cpre[i] <= c < cpre[i + 1] and covers kCertChunk entries of
// it from (c - cpre[i]) * kCertChunk on.  A chunk that meets the parent
// marks the row in lfound.
__global__ __launch_bounds__(kCertBlock) void certify_long_kernel(
    const int64_t* off, const int32_t* cols, CertMap map, const int32_t* dint,
    const int32_t* parent, const int32_t* lv, const int* lcount, int64_t lcap,
    const int64_t* cpre, int* lfound, int* result) {
  const int64_t nl = min((int64_t)*lcount, lcap);
  const int64_t nchunks = cpre[nl];
  for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    int64_t lo = 0, hi = nl;  // largest i with cpre[i] <= c
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (cpre[mid] <= c) lo = mid;
      else hi = mid;
    }
    const int64_t i = lo;
    const int64_t v = lv[i];
    const int64_t cb = off[v] + (c - cpre[i]) * (int64_t)kCertChunk;
    const int64_t ce = min(off[v + 1], cb + (int64_t)kCertChunk);
    const int32_t dv = dint[v];
    const int32_t pv = parent[map.out(v)];  // in range: checked by the first pass
    const int64_t p = pv >= 0 ? map.in(pv) : -1;
    int code = 0;
    bool found = false;
    for (int64_t j = cb + threadIdx.x; j < ce; j += kCertBlock) {
      const int32_t w = cols[j];
      const int cj = cert_edge(dv, p, w, dint[w], found);
      code = cj < code ? cj : code;
    }
    if (code) atomicMin(result, code);
    if (found) atomicOr(&lfound[i], 1);
  }
}

// A long row of a vertex below the root level whose chunks never met its
// parent breaks the parent rule.
__global__ void certify_long_parent_kernel(const int32_t* lv, const int* lcount, int64_t lcap,
                                           const int32_t* dint, const int32_t* root_perm,
                                           int32_t root_orig, const int* lfound, int* result) {
  const int64_t nl = min((int64_t)*lcount, lcap);
  const int64_t root = root_perm ? root_perm[root_orig] : root_orig;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nl;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = lv[i];
    if (dint[v] > 0 && v != root && !lfound[i]) atomicMin(result, -5);
  }
}

__global__ void cert_zero_kernel(int* small) {
  if (threadIdx.x < 4) small[threadIdx.x] = 0;
}

}  // namespace
}  // namespace rbfs

using rbfs::Graph;
using rbfs::set_error;

namespace rbfs {
namespace {

// Scratch of one certificate, carved from one buffer at 256-byte offsets:
// result and long-row counter, the long-row list, its found flags and chunk
// prefix (lcap rows of more than kCertLong entries at most), and, when the
// outputs are in original IDs of a relabelled graph, the depths in internal
// order.
struct CertScratch {
  int* small = nullptr;     // [0] result, [1] long-row count
  int32_t* lv = nullptr;
  int* lf = nullptr;
  int64_t* cpre = nullptr;
  int32_t* dint = nullptr;
  int64_t lcap = 0;
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t cert_layout(const Graph* g, bool gather, unsigned char* base, CertScratch* cs) {
  const int64_t lcap = g->nnz / kCertLong + 1;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return base ? base + at : nullptr;
  };
  CertScratch c;
  c.lcap = lcap;
  c.small = (int*)take(4 * sizeof(int));
  c.lv = (int32_t*)take(sizeof(int32_t) * (size_t)lcap);
  c.lf = (int*)take(sizeof(int) * (size_t)lcap);
  c.cpre = (int64_t*)take(sizeof(int64_t) * (size_t)(lcap + 1));
  if (gather) c.dint = (int32_t*)take(sizeof(int32_t) * (size_t)(g->n > 0 ? g->n : 1));
  if (cs) *cs = c;
  return o;
}

int cert_args(rbfs_graph_t* h, int32_t root, const int32_t* depth, const int32_t* parent,
              int32_t output_space, int32_t* result, const char* who) {
  if (!h || !depth || !parent || !result ||
      (output_space != RBFS_OUT_ORIGINAL && output_space != RBFS_OUT_INTERNAL)) {
    set_error(std::string(who) + ": bad arguments");
    return RBFS_E_INVAL;
  }
  if (root < 0 || root >= h->g.n) {
    set_error(std::string(who) + ": root out of range");
    return RBFS_E_RANGE;
  }
  return 0;
}

// Enqueues the certificate on `stream` with the given scratch, then waits
// for its result: the only host round trip.
int cert_run(Graph* g, int32_t root, const int32_t* depth, const int32_t* parent,
             int32_t output_space, hipStream_t stream, const CertScratch& cs, int32_t* result,
             const char* who) {
  const bool orig = output_space == RBFS_OUT_ORIGINAL;
  CertMap map{g->reordered && orig ? g->perm : nullptr,
              g->reordered && orig ? g->iperm : nullptr};
  const int32_t* root_perm = g->reordered ? g->perm : nullptr;
  const int64_t n = g->n;
  const int32_t* dint = cs.dint ? cs.dint : depth;
  auto grid_of = [](int64_t work) {
    return (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((work + kCertBlock - 1) / kCertBlock, 1 << 16));
  };
  hipLaunchKernelGGL(cert_zero_kernel, dim3(1), dim3(64), 0, stream, cs.small);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && cs.dint) {
    hipLaunchKernelGGL(cert_gather_kernel, dim3(grid_of(n)), dim3(kCertBlock), 0, stream, n,
                       map.iperm, depth, cs.dint);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(certify_kernel, dim3(grid_of(n)), dim3(kCertBlock), 0, stream, n, g->off,
                       g->cols, map, root_perm, root, dint, parent, cs.small, cs.lv,
                       cs.small + 1, cs.lcap);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(cert_long_plan_kernel, dim3(1), dim3(kPlanBlock), 0, stream, cs.lv,
                       cs.small + 1, cs.lcap, g->off, cs.cpre, cs.lf);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    // at most nnz / kCertChunk + (long rows) chunks; most workgroups find
    // none when there are few long rows
    const int64_t max_chunks = g->nnz / kCertChunk + cs.lcap;
    hipLaunchKernelGGL(certify_long_kernel,
                       dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(max_chunks, 4096))),
                       dim3(kCertBlock), 0, stream, g->off, g->cols, map, dint, parent, cs.lv,
                       cs.small + 1, cs.lcap, cs.cpre, cs.lf, cs.small);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(certify_long_parent_kernel, dim3(grid_of(cs.lcap)), dim3(kCertBlock), 0,
                       stream, cs.lv, cs.small + 1, cs.lcap, dint, root_perm, root, cs.lf,
                       cs.small);
    e = hipGetLastError();
  }
  int res = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&res, cs.small, sizeof(int), hipMemcpyDeviceToHost,
                                          stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    set_error(std::string(who) + ": " + hipGetErrorString(e));
    return RBFS_E_DEVICE;
  }
  *result = res;
  return RBFS_OK;
}

// Static scratch of rbfs_certify_noalloc: one copy per device, held until
// the process ends.  Host code never uses this name as an address: the
// device address of each GPU's copy comes from hipGetSymbolAddress.
constexpr size_t kCertStaticBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kCertStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex s_scratch_mu;
void* s_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up once
// per device with that device current.
int static_scratch(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("rbfs_certify_noalloc: device index out of range");
    return RBFS_E_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(s_scratch_mu);
  if (!s_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("rbfs_certify_noalloc: hipGetSymbolAddress: ") +
                hipGetErrorString(e));
      return RBFS_E_DEVICE;
    }
    s_scratch_ptr[device] = p;
  }
  *out = (unsigned char*)s_scratch_ptr[device];
  return 0;
}

}  // namespace
}  // namespace rbfs

extern "C" int rbfs_certify(rbfs_graph_t* h, int32_t root, const int32_t* depth,
                            const int32_t* parent, int32_t output_space, void* stream_,
                            int32_t* result) {
  int rc = rbfs::cert_args(h, root, depth, parent, output_space, result, "rbfs_certify");
  if (rc) return rc;
  Graph* g = &h->g;
  hipStream_t stream = (hipStream_t)stream_;
  if (hipSetDevice(g->device) != hipSuccess) {
    set_error("rbfs_certify: hipSetDevice failed");
    return RBFS_E_DEVICE;
  }
  const bool gather = g->reordered && output_space == RBFS_OUT_ORIGINAL;
  const size_t bytes = rbfs::cert_layout(g, gather, nullptr, nullptr);
  unsigned char* buf = nullptr;
  if (rbfs::dev_malloc(&buf, bytes, stream) != hipSuccess || !buf) {
    set_error("rbfs_certify: out of device memory for the scratch");
    return RBFS_E_NOMEM;
  }
  rbfs::CertScratch cs;
  rbfs::cert_layout(g, gather, buf, &cs);
  rc = rbfs::cert_run(g, root, depth, parent, output_space, stream, cs, result, "rbfs_certify");
  rbfs::dev_free(buf, stream);
  return rc;
}

extern "C" int rbfs_certify_noalloc(rbfs_graph_t* h, int32_t root, const int32_t* depth,
                                    const int32_t* parent, int32_t output_space, void* stream_,
                                    int32_t* result) {
  int rc = rbfs::cert_args(h, root, depth, parent, output_space, result,
                           "rbfs_certify_noalloc");
  if (rc) return rc;
  Graph* g = &h->g;
  hipStream_t stream = (hipStream_t)stream_;
  const bool gather = g->reordered && output_space == RBFS_OUT_ORIGINAL;
  const size_t bytes = rbfs::cert_layout(g, gather, nullptr, nullptr);
  if (bytes > rbfs::kCertStaticBytes) {
    set_error("rbfs_certify_noalloc: the graph needs " + std::to_string(bytes) +
              " bytes of scratch, the static buffer holds " +
              std::to_string(rbfs::kCertStaticBytes) + " (use rbfs_certify)");
    return RBFS_E_RANGE;
  }
  if (hipSetDevice(g->device) != hipSuccess) {
    set_error("rbfs_certify_noalloc: hipSetDevice failed");
    return RBFS_E_DEVICE;
  }
  unsigned char* buf = nullptr;
  rc = rbfs::static_scratch(g->device, &buf);
  if (rc) return rc;
  rbfs::CertScratch cs;
  rbfs::cert_layout(g, gather, buf, &cs);
  return rbfs::cert_run(g, root, depth, parent, output_space, stream, cs, result,
                        "rbfs_certify_noalloc");
}
