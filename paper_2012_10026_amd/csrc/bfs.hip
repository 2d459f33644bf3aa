// Single-root direction-optimizing BFS (Algorithm 2) as one persistent
// kernel: the level loop, both step kinds and the per-level direction
// decision run on the GPU with no host round trip.
//
// Labels are the graph's internal labels; the swept set is [0, n_sweep)
// (the non-isolated prefix after RCM).  parent(v) is the smallest-label
// neighbour one level up; both step kinds reach exactly that value:
//   top-down (Algorithm 1 / 4): for each frontier vertex u and neighbour w
//     not visited before this level, depth[w] is claimed with a CAS
//     (-1 -> d+1; the winner appends w to the next queue) and parent[w] is
//     lowered with atomicMin(u), so the minimum over all frontier neighbours
//     remains whatever the order;
//   bottom-up (Algorithm 2 lines 15-21 / Algorithm 5): each unvisited v scans
//     its row in increasing label order and stops at the first neighbour
//     that was visited at the start of the level.  For an unvisited v every
//     visited neighbour is in the current frontier, so that first hit is the
//     smallest-label frontier neighbour.
// The visited set is a bitmap.  Bottom-up reads the level-start bitmap and
// writes the next one (each 64-vertex word is owned by one wave, found bits
// come from one ballot: no atomics, the GPU form of the paper's cache-line
// blocks and of its visited |= next update outside the loop).  Top-down
// reads the bitmap to skip visited vertices and ORs the new vertices in after
// the level.
//
// Queues carry, besides the vertex, the exclusive prefix of degrees, which
// the appending wave obtains from one packed 64-bit atomic
// (count << eb | edges).  That prefix drives the edge-balanced top-down
// expansion of the next level without a separate scan.
// Bottom-up work is cut into edge-balanced ranges of words and handed out
// with an atomic counter (the fetch_add work stealing of Algorithm 5).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/rbfs.h"
#include "common.cuh"
#include "expand.cuh"
#include "graph.h"

namespace rbfs {

struct BfsCtl {
  GridBarrier bar;
  int level;
  int dir;
  int done;
  int pad0;
  unsigned long long qpack[2];
  long long nf, mf, mu, nf_prev;
  unsigned long long work;
  unsigned long long edges_level;
  long long reached, deg_reached;
  signed char hdir[RBFS_STATS_MAX_LEVELS];
  long long hnf[RBFS_STATS_MAX_LEVELS];
  long long hmf[RBFS_STATS_MAX_LEVELS];
  long long hmu[RBFS_STATS_MAX_LEVELS];
  long long hedges[RBFS_STATS_MAX_LEVELS];
};

namespace {

struct BfsParams {
  const int64_t* off;
  const int32_t* cols;
  const int32_t* perm;   // original -> internal, null when not reordered
  int64_t n_sweep;
  int64_t n_init;        // entries of depth/parent initialised by the kernel
  int64_t deg_total;     // degree sum over the swept set
  int32_t* depth;
  uint32_t* parent;
  uint64_t* vis[2];
  int32_t* qv[2];
  int64_t* qe[2];
  int32_t* chunk[2];
  int64_t chunk_cap;
  const int32_t* bu_part;
  int32_t n_part;
  int32_t root_orig;
  int32_t init;
  int32_t mode;
  int32_t alpha, beta;
  int32_t sched_len;
  int8_t sched[RBFS_STATS_MAX_LEVELS];
  int32_t eb;
  uint64_t timeout_ticks;
  BfsCtl* ctl;
};

__device__ __forceinline__ void wave_append(bool take, int32_t v, int64_t deg,
                                            unsigned long long* qpack, int eb, int32_t* qv,
                                            int64_t* qe, int32_t* chunk, int64_t chunk_cap,
                                            int64_t qcap, int* status) {
  const uint64_t m = ballot(take);
  if (m == 0) return;
  const int64_t d = take ? deg : 0;
  const int64_t inc = wave_inclusive_sum(d);
  const int64_t tot = shfl(inc, kWave - 1);
  const int leader = ffs64(m);
  unsigned long long old = 0;
  if (lane_id() == leader)
    old = atomicAdd(qpack, ((unsigned long long)popc64(m) << eb) + (unsigned long long)tot);
  old = shfl(old, leader);
  if (take) {
    const int64_t pos = (int64_t)(old >> eb) + popc64(m & lanemask_lt());
    const int64_t base = (int64_t)(old & ((1ull << eb) - 1ull)) + inc - d;
    if (pos >= qcap) {
      atomicOr(status, kStatusOverflow);
      return;
    }
    qv[pos] = v;
    qe[pos] = base;
    mark_chunks(chunk, chunk_cap, base, deg, (int32_t)pos);
  }
}

__device__ __forceinline__ int heuristic_dir(int dir, long long nf, long long mf, long long mu,
                                             long long nf_prev, long long n, int alpha,
                                             int beta) {
  if (dir == 0) return (mf * (long long)alpha > mu) ? 1 : 0;
  return (nf * (long long)beta < n && nf < nf_prev) ? 0 : 1;
}

// Runs on the last workgroup to reach the end-of-level barrier.
__device__ void decide(const BfsParams& P, int out_buf) {
  if (threadIdx.x != 0) return;
  BfsCtl* c = P.ctl;
  const unsigned long long pk = c->qpack[out_buf];
  const long long nf_new = (long long)(pk >> P.eb);
  const long long mf_new = (long long)(pk & ((1ull << P.eb) - 1ull));
  const int L = c->level;
  if (L < RBFS_STATS_MAX_LEVELS) c->hedges[L] = (long long)c->edges_level;
  const long long mu_new = c->mu - mf_new;
  int nd = c->dir;
  if (nf_new == 0) {
    c->done = 1;
  } else {
    switch (P.mode) {
      case RBFS_DIR_TD_ONLY: nd = 0; break;
      case RBFS_DIR_BU_ONLY: nd = 1; break;
      case RBFS_DIR_SCHEDULE: {
        int i = L + 1;
        if (i >= P.sched_len) i = P.sched_len - 1;
        nd = P.sched[i] ? 1 : 0;
        break;
      }
      default:
        nd = heuristic_dir(c->dir, nf_new, mf_new, mu_new, c->nf, P.n_sweep, P.alpha, P.beta);
    }
    if (L + 1 < RBFS_STATS_MAX_LEVELS) {
      c->hdir[L + 1] = (signed char)nd;
      c->hnf[L + 1] = nf_new;
      c->hmf[L + 1] = mf_new;
      c->hmu[L + 1] = mu_new;
    }
  }
  c->nf_prev = c->nf;
  c->nf = nf_new;
  c->mf = mf_new;
  c->mu = mu_new;
  c->dir = nd;
  c->level = L + 1;
  c->reached += nf_new;
  c->deg_reached += mf_new;
  c->qpack[out_buf ^ 1] = 0ull;  // the consumed queue is the next output
  c->work = 0ull;
  c->edges_level = 0ull;
}

__global__ __launch_bounds__(kBlock) void bfs_persistent_kernel(BfsParams P) {
  __shared__ ChunkLds s_chunk;
  BfsCtl* ctl = P.ctl;
  const int64_t gtid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t gsz = (int64_t)gridDim.x * kBlock;
  const int32_t root = P.perm ? P.perm[P.root_orig] : P.root_orig;
  const bool root_in = root < P.n_sweep;
  const int64_t W = ceil_div(P.n_sweep, kWave);
  const uint64_t emask = (1ull << P.eb) - 1ull;

  // ---- initialisation
  if (P.init) {
    for (int64_t i = gtid; i < P.n_init; i += gsz) {
      P.depth[i] = (i == root) ? 0 : -1;
      P.parent[i] = (i == root) ? (uint32_t)root : kNoParent;
    }
  }
  for (int64_t w = gtid; w < W; w += gsz)
    P.vis[0][w] = (root_in && w == (root >> 6)) ? (1ull << (root & 63)) : 0ull;
  if (gtid == 0) {
    const int64_t dr = root_in ? P.off[root + 1] - P.off[root] : 0;
    if (!P.init && root_in) {
      P.depth[root] = 0;
      P.parent[root] = (uint32_t)root;
    }
    ctl->level = 0;
    ctl->dir = 0;
    ctl->done = root_in ? 0 : 1;
    ctl->qpack[0] = root_in ? ((1ull << P.eb) | (unsigned long long)dr) : 0ull;
    ctl->qpack[1] = 0ull;
    ctl->nf = root_in ? 1 : 0;
    ctl->mf = dr;
    ctl->mu = P.deg_total - dr;
    ctl->nf_prev = 0;
    ctl->work = 0ull;
    ctl->edges_level = 0ull;
    ctl->reached = 1;
    ctl->deg_reached = dr;
    ctl->hdir[0] = 0;
    ctl->hnf[0] = ctl->nf;
    ctl->hmf[0] = dr;
    ctl->hmu[0] = ctl->mu;
    if (root_in) {
      P.qv[0][0] = root;
      P.qe[0][0] = 0;
      mark_chunks(P.chunk[0], P.chunk_cap, 0, dr, 0);
    }
  }
  if (!grid_barrier(&ctl->bar, P.timeout_ticks, [] {})) return;

  int cur = 0;  // queue buffer holding the current frontier
  int vc = 0;   // bitmap holding the level-start visited set
  for (;;) {
    const int done = ld_relaxed(&ctl->done);
    if (done) break;
    const int L = ld_relaxed(&ctl->level);
    const int dir = ld_relaxed(&ctl->dir);
    const int nb = cur ^ 1;
    const uint64_t* vis = P.vis[vc];
    if (dir == 0) {
      // ---- top-down step over frontier edges, chunk by chunk
      const unsigned long long pk = __hip_atomic_load(&ctl->qpack[cur], __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
      const int64_t nq = (int64_t)(pk >> P.eb);
      const int64_t E = (int64_t)(pk & emask);
      const int64_t nchunks = ceil_div(E, kChunkEdges);
      for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const bool ok = expand_chunk(s_chunk, c, E, P.qv[cur], P.qe[cur], nq, P.chunk[cur],
                                     nchunks, P.off, P.cols,
                                     [&](bool active, int32_t u, int32_t w) {
          bool win = false;
          int64_t dw = 0;
          if (active && !test_bit(vis, (uint32_t)w)) {
            int dcur = P.depth[w];
            if (dcur == -1) {
              const int old = atomicCAS(&P.depth[w], -1, L + 1);
              win = (old == -1);
            }
            if (P.parent[w] > (uint32_t)u) atomicMin(&P.parent[w], (uint32_t)u);
            if (win) dw = P.off[w + 1] - P.off[w];
          }
          wave_append(win, w, dw, &ctl->qpack[nb], P.eb, P.qv[nb], P.qe[nb], P.chunk[nb],
                      P.chunk_cap, P.n_sweep, &ctl->bar.status);
        });
        if (!ok) {
          if (threadIdx.x == 0) atomicOr(&ctl->bar.status, kStatusBadInput);
          break;
        }
      }
      if (threadIdx.x == 0 && blockIdx.x == 0) {
        __hip_atomic_fetch_add(&ctl->edges_level, (unsigned long long)E, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      }
      if (!grid_barrier(&ctl->bar, P.timeout_ticks, [&] { decide(P, nb); })) return;
      // new vertices join the visited bitmap
      int64_t nn = (int64_t)(__hip_atomic_load(&ctl->qpack[nb], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT) >> P.eb);
      if (nn > P.n_sweep) nn = P.n_sweep;
      uint64_t* visw = P.vis[vc];
      for (int64_t i = gtid; i < nn; i += gsz) {
        const int32_t w = P.qv[nb][i];
        atomicOr((unsigned long long*)&visw[w >> 6], 1ull << (w & 63));
      }
      if (!grid_barrier(&ctl->bar, P.timeout_ticks, [] {})) return;
    } else {
      // ---- bottom-up step over the swept words, edge-balanced ranges
      uint64_t* visn = P.vis[vc ^ 1];
      const int l = lane_id();
      int64_t examined = 0;
      for (;;) {
        unsigned long long p = 0;
        if (l == 0)
          p = __hip_atomic_fetch_add(&ctl->work, 1ull, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
        p = shfl(p, 0);
        if ((int64_t)p >= P.n_part) break;
        const int64_t k0 = P.bu_part[p], k1 = P.bu_part[p + 1];
        for (int64_t k = k0; k < k1; ++k) {
          const uint64_t curw = vis[k];
          const int64_t v = k * kWave + l;
          const bool valid = v < P.n_sweep;
          const bool unvis = valid && !((curw >> l) & 1ull);
          if (ballot(unvis) == 0) {
            if (l == 0) visn[k] = curw;
            continue;
          }
          int64_t b = 0, e = 0;
          if (unvis) {
            b = P.off[v];
            e = P.off[v + 1];
          }
          const bool hub = unvis && (e - b) > kLaneRow;
          bool found = false;
          int32_t par = 0;
          if (unvis && !hub) {
            for (int64_t j = b; j < e; ++j) {
              const int32_t w = P.cols[j];
              if (test_bit(vis, (uint32_t)w)) {
                found = true;
                par = w;
                examined += j - b + 1;
                break;
              }
            }
            if (!found) examined += e - b;
          }
          uint64_t hubs = ballot(hub);
          while (hubs) {
            const int h = ffs64(hubs);
            hubs &= hubs - 1;
            const int64_t hb = shfl(b, h), he = shfl(e, h);
            bool hf = false;
            int32_t hp = 0;
            int64_t scanned = he - hb;
            for (int64_t j0 = hb; j0 < he; j0 += kWave) {
              const int64_t j = j0 + l;
              int32_t w = 0;
              bool hit = false;
              if (j < he) {
                w = P.cols[j];
                hit = test_bit(vis, (uint32_t)w);
              }
              const uint64_t hm = ballot(hit);
              if (hm) {
                const int first = ffs64(hm);
                hp = shfl(w, first);
                hf = true;
                scanned = j0 - hb + first + 1;
                break;
              }
            }
            if (l == h) {
              found = hf;
              par = hp;
            }
            if (l == 0) examined += scanned;
          }
          const uint64_t fm = ballot(found);
          if (l == 0) visn[k] = curw | fm;
          if (found) {
            P.depth[v] = L + 1;
            P.parent[v] = (uint32_t)par;
          }
          wave_append(found, (int32_t)v, e - b, &ctl->qpack[nb], P.eb, P.qv[nb], P.qe[nb],
                      P.chunk[nb], P.chunk_cap, P.n_sweep, &ctl->bar.status);
        }
      }
      const int64_t ex = wave_sum(examined);
      if (l == 0 && ex)
        __hip_atomic_fetch_add(&ctl->edges_level, (unsigned long long)ex, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      if (!grid_barrier(&ctl->bar, P.timeout_ticks, [&] { decide(P, nb); })) return;
      vc ^= 1;
    }
    cur = nb;
  }
}

// Output in original IDs.  The internal arrays are read once and reset to
// their initial values, so the next search needs no initialisation pass.
__global__ void translate_kernel(int64_t n, const int32_t* perm, const int32_t* iperm,
                                 int64_t n_sweep, int32_t* depth_i, uint32_t* parent_i,
                                 int32_t* depth_o, int32_t* parent_o, int32_t root_orig) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t i = perm[v];
    int32_t d = -1, p = -1;
    if (i < n_sweep) {
      d = depth_i[i];
      const uint32_t pi = parent_i[i];
      if (d >= 0) {
        depth_i[i] = -1;
        parent_i[i] = kNoParent;
      }
      p = (pi >= (uint64_t)n_sweep) ? -1 : iperm[pi];
    } else if (v == root_orig) {
      d = 0;
      p = root_orig;
    }
    depth_o[v] = d;
    parent_o[v] = p;
  }
}

__global__ void reset_ctl_kernel(BfsCtl* c) {
  if (threadIdx.x == 0) {
    c->bar.count = 0;
    c->bar.gen = 0;
    c->bar.status = 0;
  }
}

// Edge-balanced word ranges over the swept set for the bottom-up step.
__global__ void bu_part_kernel(const int64_t* off, int64_t n_sweep, int64_t target,
                               int64_t nparts, int32_t* bounds) {
  const int64_t W = ceil_div(n_sweep, kWave);
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p <= nparts;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t want = p * target;
    int64_t lo = 0, hi = n_sweep;  // first vertex with off[v] >= want
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (off[mid] < want) lo = mid + 1; else hi = mid;
    }
    int64_t w = ceil_div(lo, kWave);
    if (p == nparts || w > W) w = W;
    bounds[p] = (int32_t)w;
  }
}


}  // namespace

void free_bfs_work(Graph* g) {
  BfsWork* w = g->bfs;
  if (!w) return;
  void* ps[] = {w->depth, w->parent, w->vis[0], w->vis[1], w->qv[0], w->qv[1], w->qe[0],
                w->qe[1], w->chunk[0], w->chunk[1], w->bu_part, w->ctl};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  if (w->ev0) (void)hipEventDestroy(w->ev0);
  if (w->ev1) (void)hipEventDestroy(w->ev1);
  if (w->ev2) (void)hipEventDestroy(w->ev2);
  delete w;
  g->bfs = nullptr;
}

#define BFS_CHECK(x)                                                            \
  do {                                                                          \
    hipError_t e_ = (x);                                                        \
    if (e_ != hipSuccess) {                                                     \
      set_error(std::string("bfs: ") + #x + ": " + hipGetErrorString(e_));      \
      return e_ == hipErrorOutOfMemory ? RBFS_E_NOMEM : RBFS_E_DEVICE;          \
    }                                                                           \
  } while (0)

static int ensure_bfs_work(Graph* g, hipStream_t stream) {
  if (g->bfs) return 0;
  BfsWork* w = new BfsWork();
  g->bfs = w;
  const int64_t ns = g->n_sweep > 0 ? g->n_sweep : 1;
  const int64_t W = ceil_div(ns, kWave);
  w->n_sweep = g->n_sweep;
  BFS_CHECK(hipMalloc(&w->depth, sizeof(int32_t) * ns));
  BFS_CHECK(hipMalloc(&w->parent, sizeof(uint32_t) * ns));
  for (int i = 0; i < 2; ++i) {
    BFS_CHECK(hipMalloc(&w->vis[i], sizeof(uint64_t) * W));
    BFS_CHECK(hipMalloc(&w->qv[i], sizeof(int32_t) * ns));
    BFS_CHECK(hipMalloc(&w->qe[i], sizeof(int64_t) * ns));
  }
  w->chunk_cap = ceil_div(g->nnz, kChunkEdges) + 2;
  for (int i = 0; i < 2; ++i) BFS_CHECK(hipMalloc(&w->chunk[i], sizeof(int32_t) * w->chunk_cap));
  BFS_CHECK(hipMalloc(&w->ctl, sizeof(BfsCtl)));
  BFS_CHECK(hipMemsetAsync(w->ctl, 0, sizeof(BfsCtl), stream));
  // bottom-up ranges: about 64K adjacency entries each, at most 256 words each
  const int64_t nnz_sweep = g->nnz;  // isolated vertices contribute no entries
  const int64_t target = std::max<int64_t>(4096, nnz_sweep / 16384 + 1);
  const int64_t nparts_e = std::max<int64_t>(1, ceil_div(nnz_sweep, target));
  int32_t* d_b = nullptr;
  BFS_CHECK(hipMalloc(&d_b, sizeof(int32_t) * (nparts_e + 1)));
  hipLaunchKernelGGL(bu_part_kernel, dim3((unsigned)ceil_div(nparts_e + 1, 256)), dim3(256), 0,
                     stream, g->off, g->n_sweep, target, nparts_e, d_b);
  BFS_CHECK(hipGetLastError());
  std::vector<int32_t> hb(nparts_e + 1);
  BFS_CHECK(hipMemcpyAsync(hb.data(), d_b, sizeof(int32_t) * (nparts_e + 1),
                           hipMemcpyDeviceToHost, stream));
  BFS_CHECK(hipStreamSynchronize(stream));
  (void)hipFree(d_b);
  std::vector<int32_t> parts;
  parts.push_back(0);
  for (int64_t p = 1; p <= nparts_e; ++p) {
    int32_t a = parts.back(), b = std::max(hb[p], a);
    while (b - a > 256) {
      a += 256;
      parts.push_back(a);
    }
    if (b > parts.back()) parts.push_back(b);
  }
  if (parts.back() != (int32_t)W) parts.push_back((int32_t)W);
  w->n_part = (int32_t)parts.size() - 1;
  BFS_CHECK(hipMalloc(&w->bu_part, sizeof(int32_t) * parts.size()));
  BFS_CHECK(hipMemcpyAsync(w->bu_part, parts.data(), sizeof(int32_t) * parts.size(),
                           hipMemcpyHostToDevice, stream));
  int per_cu = 0;
  BFS_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, bfs_persistent_kernel, kBlock,
                                                          0));
  if (per_cu < 1) per_cu = 1;
  if (per_cu > 4) per_cu = 4;
  w->grid = per_cu * g->compute_units;
  BFS_CHECK(hipEventCreate(&w->ev0));
  BFS_CHECK(hipEventCreate(&w->ev1));
  BFS_CHECK(hipEventCreate(&w->ev2));
  BFS_CHECK(hipStreamSynchronize(stream));
  w->clean = false;
  g->bytes += (sizeof(int32_t) * 2 + sizeof(int32_t) * 2 + sizeof(int64_t) * 2) * (size_t)ns +
              sizeof(uint64_t) * 2 * W + sizeof(int32_t) * 2 * w->chunk_cap;
  return 0;
}

int bfs_impl(Graph* g, int32_t root, int32_t* depth, int32_t* parent, int mode, int alpha,
             int beta, const int8_t* sched, int sched_len, int out_space, int flags,
             hipStream_t stream, void* stats_v) {
  rbfs_stats_t* stats = (rbfs_stats_t*)stats_v;
  int rc = ensure_bfs_work(g, stream);
  if (rc) return rc;
  BfsWork* w = g->bfs;
  const bool translate = g->reordered && out_space == RBFS_OUT_ORIGINAL;
  const int bits_n = bits_for(g->n_sweep + 2);
  const int eb = 64 - bits_n;
  if (eb < 40 && (g->nnz >> eb) != 0) {
    set_error("bfs: graph too large for the packed queue counter");
    return RBFS_E_UNSUPPORTED;
  }
  BfsParams P{};
  P.off = g->off;
  P.cols = g->cols;
  P.perm = g->reordered ? g->perm : nullptr;
  P.n_sweep = g->n_sweep;
  P.deg_total = g->nnz;
  if (translate) {
    P.depth = w->depth;
    P.parent = w->parent;
    P.init = w->clean ? 0 : 1;
    P.n_init = g->n_sweep;
  } else {
    P.depth = depth;
    P.parent = (uint32_t*)parent;
    P.init = 1;
    P.n_init = g->n;
  }
  for (int i = 0; i < 2; ++i) {
    P.vis[i] = w->vis[i];
    P.qv[i] = w->qv[i];
    P.qe[i] = w->qe[i];
    P.chunk[i] = w->chunk[i];
  }
  P.chunk_cap = w->chunk_cap;
  P.bu_part = w->bu_part;
  P.n_part = w->n_part;
  P.root_orig = root;
  P.mode = mode;
  P.alpha = alpha;
  P.beta = beta;
  P.sched_len = 0;
  if (mode == RBFS_DIR_SCHEDULE) {
    if (!sched || sched_len <= 0) {
      set_error("bfs: schedule mode needs a schedule");
      return RBFS_E_INVAL;
    }
    P.sched_len = std::min(sched_len, RBFS_STATS_MAX_LEVELS);
    for (int i = 0; i < P.sched_len; ++i) P.sched[i] = sched[i];
  }
  P.eb = eb;
  P.timeout_ticks = (uint64_t)g->wall_rate_khz * 1000ull * 4ull;  // 4 s
  P.ctl = w->ctl;

  hipEvent_t* tev = nullptr;
  if (flags & RBFS_OPT_TIMING) BFS_CHECK(g->timing.next(&tev));
  if (tev) BFS_CHECK(hipEventRecord(tev[0], stream));
  BFS_CHECK(hipEventRecord(w->ev0, stream));
  hipLaunchKernelGGL(reset_ctl_kernel, dim3(1), dim3(64), 0, stream, w->ctl);
  BFS_CHECK(hipGetLastError());
  hipLaunchKernelGGL(bfs_persistent_kernel, dim3(w->grid), dim3(kBlock), 0, stream, P);
  BFS_CHECK(hipGetLastError());
  BFS_CHECK(hipEventRecord(w->ev1, stream));
  if (tev) BFS_CHECK(hipEventRecord(tev[1], stream));
  if (translate) {
    const int64_t blocks = std::min<int64_t>(ceil_div(g->n, kBlock), 1 << 20);
    hipLaunchKernelGGL(translate_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, stream, g->n,
                       g->perm, g->iperm, g->n_sweep, w->depth, w->parent, depth, parent, root);
    BFS_CHECK(hipGetLastError());
    w->clean = true;
  }
  BFS_CHECK(hipEventRecord(w->ev2, stream));
  if (tev) BFS_CHECK(hipEventRecord(tev[2], stream));
  if (stats) {
    BfsCtl h;
    BFS_CHECK(hipMemcpyAsync(&h, w->ctl, sizeof(BfsCtl), hipMemcpyDeviceToHost, stream));
    BFS_CHECK(hipStreamSynchronize(stream));
    memset(stats, 0, sizeof(*stats));
    stats->levels = h.level;
    stats->status = h.bar.status;
    const int nl = std::min(h.level, RBFS_STATS_MAX_LEVELS);
    for (int i = 0; i < nl; ++i) {
      stats->dir[i] = h.hdir[i];
      stats->nf[i] = h.hnf[i];
      stats->mf[i] = h.hmf[i];
      stats->mu[i] = h.hmu[i];
      stats->edges[i] = h.hedges[i];
    }
    stats->reached = h.reached;
    stats->component_edges = h.deg_reached / 2;
    BFS_CHECK(hipEventElapsedTime(&stats->ms_kernel, w->ev0, w->ev1));
    BFS_CHECK(hipEventElapsedTime(&stats->ms_total, w->ev0, w->ev2));
    if (h.bar.status != 0) {
      w->clean = false;
      set_error("bfs: device status " + std::to_string(h.bar.status));
      return RBFS_E_DEVICE;
    }
  }
  return 0;
}

int bfs_check_status(Graph* g, hipStream_t stream) {
  if (!g->bfs) return 0;
  int st = 0;
  BFS_CHECK(hipMemcpyAsync(&st, &g->bfs->ctl->bar.status, sizeof(int), hipMemcpyDeviceToHost,
                           stream));
  BFS_CHECK(hipStreamSynchronize(stream));
  if (st != 0) {
    g->bfs->clean = false;
    set_error("bfs: device status " + std::to_string(st));
    return RBFS_E_DEVICE;
  }
  return 0;
}

}  // namespace rbfs
