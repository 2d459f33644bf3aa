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

#include <string>

#include "../../include/rbfs.h"
#include "common.cuh"
#include "graph.h"
#include "handles.h"

namespace rbfs {
namespace {

constexpr int kCertBlock = 256;
constexpr int kCertLane = 64;  // rows longer than this are checked by the whole wave

// Output index of internal vertex v, and internal label of output value x.
struct CertMap {
  const int32_t* perm;   // original -> internal (null: identity)
  const int32_t* iperm;  // internal -> original (null: identity)
  __device__ __forceinline__ int64_t out(int64_t v) const { return iperm ? iperm[v] : v; }
  __device__ __forceinline__ int64_t in(int64_t x) const { return perm ? perm[x] : x; }
};

__global__ __launch_bounds__(kCertBlock) void certify_kernel(
    int64_t n, const int64_t* off, const int32_t* cols, CertMap map, int64_t root,
    const int32_t* depth, const int32_t* parent, int* result) {
  const int l = lane_id();
  const int64_t nwaves = ((int64_t)gridDim.x * kCertBlock) / kWave;
  const int64_t w0 = ((int64_t)blockIdx.x * kCertBlock + threadIdx.x) / kWave;
  for (int64_t base = w0 * kWave; base < n; base += nwaves * kWave) {
    const int64_t v = base + l;
    int code = 0;
    int32_t dv = -1;
    int64_t p = -1, b = 0, e = 0;
    if (v < n) {
      const int64_t ov = map.out(v);
      dv = depth[ov];
      const int32_t pv = parent[ov];
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
        const int32_t dw = depth[map.out(w)];
        if ((dv < 0) != (dw < 0)) code = -2;
        else if (dv >= 0 && (dv - dw > 1 || dw - dv > 1)) code = -3;
        else if (dv > 0 && dw == dv - 1) {
          if (w == p) found = true;
          else if (w > p) code = -6;
        }
      }
    }
    // long rows: the whole wave, 64 entries per step
    uint64_t longs = ballot(v < n && !code && e - b > kCertLane);
    while (longs) {
      const int h = ffs64(longs);
      longs &= longs - 1;
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
          const int32_t dw = depth[map.out(w)];
          if ((hd < 0) != (dw < 0)) c = -2;
          else if (hd >= 0 && (hd - dw > 1 || dw - hd > 1)) c = -3;
          else if (hd > 0 && dw == hd - 1) {
            if (w == hp) isp = true;
            else if (w > hp) c = -6;
          }
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
    if (v < n && !code && dv > 0 && v != root && !found) code = -5;
    if (code) atomicMin(result, code);
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
  int* d_res = nullptr;
  hipError_t e = rbfs::dev_malloc(&d_res, sizeof(int), stream);
  if (e != hipSuccess) {
    set_error(std::string("rbfs_certify: ") + hipGetErrorString(e));
    return RBFS_E_NOMEM;
  }
  e = hipMemsetAsync(d_res, 0, sizeof(int), stream);
  if (e == hipSuccess) {
    const int64_t waves = (g->n + rbfs::kWave - 1) / rbfs::kWave;
    const int64_t blocks = std::max<int64_t>(
        1, std::min<int64_t>((waves * rbfs::kWave + rbfs::kCertBlock - 1) / rbfs::kCertBlock, 1 << 16));
    hipLaunchKernelGGL(rbfs::certify_kernel, dim3((unsigned)blocks), dim3(rbfs::kCertBlock), 0,
                       stream, g->n, g->off, g->cols, map, root_int, depth, parent, d_res);
    e = hipGetLastError();
  }
  int res = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&res, d_res, sizeof(int), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  rbfs::dev_free(d_res, stream);
  if (e != hipSuccess) {
    set_error(std::string("rbfs_certify: ") + hipGetErrorString(e));
    return RBFS_E_DEVICE;
  }
  *result = res;
  return RBFS_OK;
}
