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
#include <string>
#include <vector>

#include "../../include/rbfs.h"
#include "common.cuh"
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
    int64_t n, const int64_t* off, const int32_t* cols, CertMap map, int64_t root,
    const int32_t* dint, const int32_t* parent, int* result, int32_t* lv, int* lcount,
    int64_t lcap) {
  const int l = lane_id();
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

// Row bounds of the long-row list, for the host to cut them into chunks.
__global__ void cert_long_bounds_kernel(const int32_t* lv, int64_t nl, const int64_t* off,
                                        int64_t* lb) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nl;
       i += (int64_t)gridDim.x * blockDim.x) {
    lb[2 * i] = off[lv[i]];
    lb[2 * i + 1] = off[lv[i] + 1];
  }
}

// One chunk of a long row per workgroup: chunk c covers entries
// [cb[c], ce[c]) of long-row list entry ci[c].  A chunk that meets the
// parent marks the row in lfound.
__global__ __launch_bounds__(kCertBlock) void certify_long_kernel(
    const int32_t* cols, CertMap map, const int32_t* dint, const int32_t* parent,
    const int32_t* lv, const int32_t* ci, const int64_t* cb, const int64_t* ce,
    int64_t nchunks, int* lfound, int* result) {
  for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const int i = ci[c];
    const int64_t v = lv[i];
    const int32_t dv = dint[v];
    const int32_t pv = parent[map.out(v)];  // in range: checked by the first pass
    const int64_t p = pv >= 0 ? map.in(pv) : -1;
    int code = 0;
    bool found = false;
    for (int64_t j = cb[c] + threadIdx.x; j < ce[c]; j += kCertBlock) {
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
__global__ void certify_long_parent_kernel(const int32_t* lv, int64_t nl, const int32_t* dint,
                                           int64_t root, const int* lfound, int* result) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nl;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = lv[i];
    if (dint[v] > 0 && v != root && !lfound[i]) atomicMin(result, -5);
  }
}

}  // namespace
}  // namespace rbfs

using rbfs::Graph;
using rbfs::set_error;

extern "C" int rbfs_certify(rbfs_graph_t* h, int32_t root, const int32_t* depth,
                            const int32_t* parent, int32_t output_space, void* stream_,
                            int32_t* result) {
  if (!h || !depth || !parent || !result ||
      (output_space != RBFS_OUT_ORIGINAL && output_space != RBFS_OUT_INTERNAL)) {
    set_error("rbfs_certify: bad arguments");
    return RBFS_E_INVAL;
  }
  Graph* g = &h->g;
  if (root < 0 || root >= g->n) {
    set_error("rbfs_certify: root out of range");
    return RBFS_E_RANGE;
  }
  hipStream_t stream = (hipStream_t)stream_;
  const bool orig = output_space == RBFS_OUT_ORIGINAL;
  rbfs::CertMap map{g->reordered && orig ? g->perm : nullptr,
                    g->reordered && orig ? g->iperm : nullptr};
  int64_t root_int = root;
  if (g->reordered) {
    int32_t r = 0;
    hipError_t e = hipMemcpyAsync(&r, g->perm + root, sizeof(int32_t), hipMemcpyDeviceToHost,
                                  stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      set_error(std::string("rbfs_certify: ") + hipGetErrorString(e));
      return RBFS_E_DEVICE;
    }
    root_int = r;
  }
  const int64_t n = g->n;
  // scratch: result word, long-row counter and list, and (with a mapping)
  // the depths in internal order
  const bool gather = map.iperm != nullptr;
  int* d_small = nullptr;   // [0] result, [1] long-row count
  int32_t* d_lv = nullptr;  // long-row list: each holds more than kCertLong entries
  const int64_t lcap = g->nnz / rbfs::kCertLong + 1;
  int32_t* d_dint = nullptr;
  std::vector<void*> extra;
  auto release = [&]() {
    for (void* q : extra) rbfs::dev_free(q, stream);
    if (d_dint) rbfs::dev_free(d_dint, stream);
    if (d_lv) rbfs::dev_free(d_lv, stream);
    if (d_small) rbfs::dev_free(d_small, stream);
  };
  hipError_t e = rbfs::dev_malloc(&d_small, 2 * sizeof(int), stream);
  if (e == hipSuccess) e = rbfs::dev_malloc(&d_lv, sizeof(int32_t) * (size_t)lcap, stream);
  if (e == hipSuccess && gather)
    e = rbfs::dev_malloc(&d_dint, sizeof(int32_t) * (size_t)(n > 0 ? n : 1), stream);
  if (e != hipSuccess) {
    release();
    set_error(std::string("rbfs_certify: ") + hipGetErrorString(e));
    return RBFS_E_NOMEM;
  }
  const int32_t* dint = gather ? d_dint : depth;
  auto grid_of = [](int64_t work) {
    return (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((work + rbfs::kCertBlock - 1) / rbfs::kCertBlock, 1 << 16));
  };
  e = hipMemsetAsync(d_small, 0, 2 * sizeof(int), stream);
  if (e == hipSuccess && gather) {
    hipLaunchKernelGGL(rbfs::cert_gather_kernel, dim3(grid_of(n)), dim3(rbfs::kCertBlock), 0,
                       stream, n, map.iperm, depth, d_dint);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(rbfs::certify_kernel, dim3(grid_of(n)), dim3(rbfs::kCertBlock), 0, stream,
                       n, g->off, g->cols, map, root_int, dint, parent, d_small, d_lv,
                       d_small + 1, lcap);
    e = hipGetLastError();
  }
  int hs[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(hs, d_small, 2 * sizeof(int), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  const int64_t nl = hs[1];
  if (e == hipSuccess && nl > 0) {
    // long rows: chunk table from their bounds, one chunk per workgroup
    int64_t* d_lb = nullptr;
    std::vector<int64_t> hlb(2 * nl);
    e = rbfs::dev_malloc(&d_lb, sizeof(int64_t) * 2 * nl, stream);
    if (d_lb) extra.push_back(d_lb);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(rbfs::cert_long_bounds_kernel, dim3(grid_of(nl)), dim3(rbfs::kCertBlock),
                         0, stream, d_lv, nl, g->off, d_lb);
      e = hipGetLastError();
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(hlb.data(), d_lb, sizeof(int64_t) * 2 * nl, hipMemcpyDeviceToHost,
                         stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    std::vector<int32_t> ci;
    std::vector<int64_t> cb, ce;
    for (int64_t i = 0; e == hipSuccess && i < nl; ++i)
      for (int64_t j = hlb[2 * i]; j < hlb[2 * i + 1]; j += rbfs::kCertChunk) {
        ci.push_back((int32_t)i);
        cb.push_back(j);
        ce.push_back(std::min<int64_t>(hlb[2 * i + 1], j + rbfs::kCertChunk));
      }
    const int64_t nc = (int64_t)ci.size();
    int32_t* d_ci = nullptr;
    int64_t *d_cb = nullptr, *d_ce = nullptr;
    int* d_lf = nullptr;
    if (e == hipSuccess) e = rbfs::dev_malloc(&d_ci, sizeof(int32_t) * nc, stream);
    if (d_ci) extra.push_back(d_ci);
    if (e == hipSuccess) e = rbfs::dev_malloc(&d_cb, sizeof(int64_t) * nc, stream);
    if (d_cb) extra.push_back(d_cb);
    if (e == hipSuccess) e = rbfs::dev_malloc(&d_ce, sizeof(int64_t) * nc, stream);
    if (d_ce) extra.push_back(d_ce);
    if (e == hipSuccess) e = rbfs::dev_malloc(&d_lf, sizeof(int) * nl, stream);
    if (d_lf) extra.push_back(d_lf);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_ci, ci.data(), sizeof(int32_t) * nc, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_cb, cb.data(), sizeof(int64_t) * nc, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_ce, ce.data(), sizeof(int64_t) * nc, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemsetAsync(d_lf, 0, sizeof(int) * nl, stream);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(rbfs::certify_long_kernel,
                         dim3((unsigned)std::min<int64_t>(nc, 1 << 16)), dim3(rbfs::kCertBlock),
                         0, stream, g->cols, map, dint, parent, d_lv, d_ci, d_cb, d_ce, nc, d_lf,
                         d_small);
      e = hipGetLastError();
    }
    if (e == hipSuccess) {
      hipLaunchKernelGGL(rbfs::certify_long_parent_kernel, dim3(grid_of(nl)),
                         dim3(rbfs::kCertBlock), 0, stream, d_lv, nl, dint, root_int, d_lf,
                         d_small);
      e = hipGetLastError();
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(hs, d_small, sizeof(int), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
  }
  release();
  if (e != hipSuccess) {
    set_error(std::string("rbfs_certify: ") + hipGetErrorString(e));
    return RBFS_E_DEVICE;
  }
  const int res = hs[0];
  *result = res;
  return RBFS_OK;
}
