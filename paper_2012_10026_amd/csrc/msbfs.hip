// Batched BFS: up to 64 roots searched together, one bit per root in a
// 64-bit word per vertex (multi-source BFS), as one persistent kernel.
//
// Row j of the result equals the single-root search from root j: depth is
// the hop distance and the parent of v for root j is the largest-label
// neighbour of v one level closer to root j.  For a vertex v still missing
// root j at level d, every neighbour that has bit j in the frontier F_d is at
// distance d from root j, so either step kind gives exactly those parents:
//   bottom-up: every vertex with missing bits scans its row in decreasing
//     label order until all of them are found, taking for each missing bit
//     the first neighbour whose frontier word has it (Algorithm 2's
//     bottom-up loop, per bit);
//   top-down: frontier vertices push their bits to their neighbours with
//     atomicOr, and for each bit the neighbour still misses propose
//     (depth, parent) = (d+1, u) with a 64-bit atomicMin on the neighbour's
//     packed word for that root (the complement of the parent in its low
//     half), so the largest label stays.
// Visited words, three rotating frontier word arrays, the per-wave staged
// frontier queue with degree prefix (edge-balanced top-down expansion) and
// the hierarchical grid barrier follow the single-root kernel.
//
// The kernel runs over a "union" graph: the graph itself for a batch, or the
// disjoint union of several graphs (each keeps its own labels, offset by the
// vertex counts of the graphs before it), where root j of every graph uses
// bit j; components never touch, so the bits never mix.
//
// Per-(vertex, root) results are packed 64-bit words (depth << 32 | ~parent,
// all ones = unreached), vertex-major ([v][64]), with parents as internal
// labels.  A tiled transpose through LDS turns them into the caller's
// root-major original-ID layout, maps the parents back, and resets the
// internal rows it reads.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/rbfs.h"
#include "common.h"
#include "expand.h"
#include "graph.h"

namespace rbfs {

struct alignas(128) MsCtl {
  GridBarrier bar;
  alignas(128) unsigned long long qpack[3][16];
  alignas(128) unsigned long long done_deg[3][16];  // degree of vertices completed
  alignas(128) unsigned long long edges[3][16];
  int levels;
  int pad;
  signed char hdir[RBFS_STATS_MAX_LEVELS];
  long long hnf[RBFS_STATS_MAX_LEVELS];
  long long hmf[RBFS_STATS_MAX_LEVELS];
  long long hmu[RBFS_STATS_MAX_LEVELS];
  long long hedges[RBFS_STATS_MAX_LEVELS];
  unsigned long long hts[RBFS_STATS_MAX_LEVELS + 1];
};

namespace {

constexpr int kMsStage = 256;
constexpr int kPullStep = 8;  // row entries a lane tests per step
constexpr int kMsBlock = 1024;
constexpr int kMsWaves = kMsBlock / kWave;

struct MsParams {
  const int64_t* off;
  const int32_t* cols;
  int64_t n_sweep;
  int64_t deg_total;
  uint64_t* vis;
  uint64_t* front[3];
  uint64_t* dp;            // [n_sweep][64] packed (depth field << 32 | ~parent), all ones = none
  uint32_t base;           // depth field of depth 0: base + depth (see the single-root search)
  int32_t* qv[2];
  int64_t* qe[2];
  int32_t* chunk[2];
  int64_t chunk_cap;
  const int32_t* bu_part;
  int32_t n_part;
  unsigned long long* wctr;  // BU range counters: 3 slots of wstride, 16 per workgroup
  int64_t wstride;
  const int32_t* roots;    // nroots internal (union) IDs, -1 when not swept;
                           // entry i is root (i mod k) of its graph (bit i mod k)
  int32_t nroots;
  int32_t k;
  uint64_t amask;
  int32_t mode, alpha, beta;
  int32_t eb;
  int32_t lane_row;      // rows longer than this are scanned by a whole wave
  uint64_t timeout_ticks;
  MsCtl* ctl;
};

struct MsStage {
  int32_t v[kMsWaves][kMsStage];
  int32_t d[kMsWaves][kMsStage];
  int32_t cnt[kMsWaves];
};


__device__ __forceinline__ void ms_flush(MsStage& st, const MsParams& P, int nq_idx,
                                         unsigned long long* qpack) {
  const int wv = wave_id(), l = lane_id();
  const int cnt = st.cnt[wv];
  if (cnt == 0) return;
  int64_t total = 0;
  for (int j0 = 0; j0 < cnt; j0 += kWave) {
    const int j = j0 + l;
    total += (j < cnt) ? (int64_t)st.d[wv][j] : 0;
  }
  total = wave_sum(total);
  unsigned long long old = 0;
  if (l == 0)
    old = atomicAdd(qpack, ((unsigned long long)cnt << P.eb) + (unsigned long long)total);
  old = shfl(old, 0);
  const int64_t pos0 = (int64_t)(old >> P.eb);
  int64_t ebase = (int64_t)(old & ((1ull << P.eb) - 1ull));
  if (pos0 + cnt > P.n_sweep) {
    if (l == 0) atomicOr(&P.ctl->bar.status, kStatusOverflow);
  } else {
    for (int j0 = 0; j0 < cnt; j0 += kWave) {
      const int j = j0 + l;
      const bool act = j < cnt;
      const int64_t d = act ? (int64_t)st.d[wv][j] : 0;
      const int64_t inc = wave_inclusive_sum(d);
      if (act) {
        const int64_t pos = pos0 + j;
        const int64_t base = ebase + inc - d;
        P.qv[nq_idx][pos] = st.v[wv][j];
        P.qe[nq_idx][pos] = base;
        mark_chunks(P.chunk[nq_idx], P.chunk_cap, base, d, (int32_t)pos);
      }
      ebase += shfl(inc, kWave - 1);
    }
  }
  __builtin_amdgcn_wave_barrier();
  if (l == 0) st.cnt[wv] = 0;
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void ms_stage(MsStage& st, bool take, int32_t v, int64_t deg,
                                         const MsParams& P, int nq_idx,
                                         unsigned long long* qpack) {
  const uint64_t m = ballot(take);
  if (m == 0) return;
  const int wv = wave_id();
  const int base = st.cnt[wv];
  __builtin_amdgcn_wave_barrier();
  if (take) {
    const int pos = base + popc64(m & lanemask_lt());
    st.v[wv][pos] = v;
    st.d[wv][pos] = (int32_t)deg;
  }
  if (lane_id() == 0) st.cnt[wv] = base + popc64(m);
  __builtin_amdgcn_wave_barrier();
  if (base + popc64(m) > kMsStage - kWave) ms_flush(st, P, nq_idx, qpack);
}

__device__ __forceinline__ uint64_t wave_or(uint64_t x) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) x |= __shfl_xor(x, off, kWave);
  return x;
}

__device__ __forceinline__ uint64_t wave_exclusive_or(uint64_t x) {
  const int l = lane_id();
  uint64_t inc = x;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint64_t t = __shfl_up(inc, off, kWave);
    if (l >= off) inc |= t;
  }
  const uint64_t ex = __shfl_up(inc, 1, kWave);
  return l == 0 ? 0ull : ex;
}

// Whole-wave scans of the long rows: every lane with hub = true holds vertex
// v (row cols[b, e)) missing root bits `miss`; each such row is scanned by the
// whole wave, 64 entries per step, where the first lane holding a bit
// (exclusive OR-scan) owns it.  Returns the bits found on the hub lanes.
// All lanes call.
__device__ __forceinline__ uint64_t ms_hub_pull(const MsParams& P, bool hub, int64_t v,
                                                int64_t b, int64_t e, uint64_t miss,
                                                const uint64_t* fcur, int d1,
                                                int64_t& examined) {
  const int l = lane_id();
  uint64_t found = 0;
  uint64_t hubs = ballot(hub && miss != 0);
  while (hubs) {
    const int h = ffs64(hubs);
    hubs &= hubs - 1;
    const int64_t hv = shfl(v, h);
    const int64_t hb0 = shfl(b, h), he = shfl(e, h);
    uint64_t hmiss = shfl(miss, h);
    uint64_t hfound = 0;
    int64_t scanned = 0;
    // downwards from the row's end, lane 0 on the highest entry
    for (int64_t j0 = he; j0 > hb0 && hmiss; j0 -= kWave) {
      const int64_t j = j0 - 1 - l;
      int32_t x = 0;
      uint64_t hb = 0;
      if (j >= hb0) {
        x = P.cols[j];
        hb = fcur[x] & hmiss;
      }
      const uint64_t mine = hb & ~wave_exclusive_or(hb);
      // the row's new pairs, written by the whole wave: lane r writes root
      // r's entry, once per lane that found something
      uint64_t ml = ballot(mine != 0ull);
      uint64_t* row = P.dp + hv * 64;
      while (ml) {
        const int sl = ffs64(ml);
        ml &= ml - 1;
        const uint64_t sm = shfl(mine, sl);
        const int32_t sx = shfl(x, sl);
        if ((sm >> l) & 1ull) row[l] = ((uint64_t)(uint32_t)d1 << 32) | (uint32_t)~(uint32_t)sx;
      }
      const uint64_t all = wave_or(hb);
      hmiss &= ~all;
      hfound |= all;
      scanned += (j0 - kWave > hb0 ? kWave : j0 - hb0);
    }
    if (l == h) found = hfound;
    if (l == 0) examined += scanned;
  }
  return found;
}

// Bottom-up pull over the vertices [v0, v1) with lane refill.  The vertices
// are taken 64 at a time (one coalesced load of their visited and frontier
// words, which also folds F_d into visited); those with missing root bits are
// handed to idle lanes, and a lane that finishes its vertex takes the next
// one at once, so a long row does not stall the other 63 lanes.  Each lane
// scans its row in decreasing label order, kPullStep entries per step, and
// records for every missing bit the first neighbour whose frontier word has
// it; rows longer than lane_row are scanned by the whole wave.  Vertices that
// found bits go to the next frontier; `done` gathers the degree of vertices
// that now have every root.
__device__ __forceinline__ void ms_pull_range(const MsParams& P, int64_t v0, int64_t v1,
                                              const uint64_t* fcur, uint64_t* fnext, int d1,
                                              int64_t& examined, int64_t& done, MsStage& st,
                                              int qn, unsigned long long* qpack) {
  const int l = lane_id();
  int64_t cb = v0;      // current 64-vertex chunk (same in every lane)
  uint64_t mch = 0;     // missing bits of vertex cb + l
  uint64_t cm = 0;      // chunk vertices not handed out yet (same in every lane)
  auto load_chunk = [&]() {
    const int64_t u = cb + l;
    mch = 0;
    if (u < v1) {
      const uint64_t vv = P.vis[u], fv = fcur[u];
      P.vis[u] = vv | fv;
      mch = P.amask & ~(vv | fv);
    }
    cm = ballot(mch != 0ull);
  };
  load_chunk();
  bool busy = false;
  int64_t v = 0, b = 0, j = 0, e = 0;
  uint64_t miss = 0, found = 0;
  for (;;) {
    // hand candidates to idle lanes, moving on to further chunks as needed
    bool fresh = false;
    for (;;) {
      const uint64_t idle = ballot(!busy && !fresh);
      if (idle == 0ull) break;
      if (cm == 0ull) {
        if (cb + kWave >= v1) break;
        cb += kWave;
        load_chunk();
        continue;
      }
      const int k = popc64(cm);
      const int r = popc64(idle & lanemask_lt());
      const bool take = !busy && !fresh && r < k;
      const int p = take ? nth_set_bit64(cm, r) : 0;
      const uint64_t mp = shfl(mch, p);
      if (take) {
        v = cb + p;
        miss = mp;
        found = 0;
        fresh = true;
      }
      const int given = k < popc64(idle) ? k : popc64(idle);
      cm = (given == k) ? 0ull : (cm & ~((1ull << nth_set_bit64(cm, given)) - 1ull));
    }
    if (fresh) {
      b = P.off[v];
      e = P.off[v + 1];
      j = e;
      busy = true;
    }
    const bool hub = fresh && (e - b) > P.lane_row;
    const uint64_t hf = ms_hub_pull(P, hub, v, b, e, miss, fcur, d1, examined);
    bool fin = false;
    // this step's hits: entry q of the lane's row gives the roots hrec[q]
    int32_t x[kPullStep];
    uint64_t hrec[kPullStep];
    int qmask = 0;
#pragma unroll
    for (int q = 0; q < kPullStep; ++q) {
      x[q] = 0;
      hrec[q] = 0ull;
    }
    if (hub) {
      found = hf;
      miss &= ~hf;
      fin = true;
    } else if (busy) {
      // entries j-1, j-2, .. downwards
      uint64_t fb[kPullStep];
#pragma unroll
      for (int q = 0; q < kPullStep; ++q) x[q] = (j - 1 - q >= b) ? P.cols[j - 1 - q] : 0;
#pragma unroll
      for (int q = 0; q < kPullStep; ++q) fb[q] = (j - 1 - q >= b) ? fcur[x[q]] : 0ull;
      int used = (j - b < kPullStep) ? (int)(j - b) : kPullStep;
#pragma unroll
      for (int q = 0; q < kPullStep; ++q) {
        const uint64_t hb = fb[q] & miss;
        if (hb) {
          hrec[q] = hb;
          qmask |= 1 << q;
          miss &= ~hb;
          found |= hb;
          if (miss == 0ull) used = q + 1;
        }
      }
      examined += used;
      j -= kPullStep;
      fin = miss == 0ull || j <= b;
    }
    // the packed pairs of the hits, written a row at a time by the whole
    // wave (lane r writes root r's entry): one store per hit covers up to
    // 64 roots of one vertex instead of one store per root
    uint64_t wl = ballot(qmask != 0);
    while (wl) {
      const int h = ffs64(wl);
      wl &= wl - 1;
      uint64_t* row = P.dp + shfl(v, h) * 64;
      const int qm = shfl(qmask, h);
#pragma unroll
      for (int q = 0; q < kPullStep; ++q) {
        if ((qm >> q) & 1) {
          const uint64_t hq = shfl(hrec[q], h);
          const int32_t hx = shfl(x[q], h);
          if ((hq >> l) & 1ull)
            row[l] = ((uint64_t)(uint32_t)d1 << 32) | (uint32_t)~(uint32_t)hx;
        }
      }
    }
    if (fin && found) fnext[v] = found;
    if (fin && miss == 0ull) done += e - b;
    ms_stage(st, fin && found != 0ull, (int32_t)v, e - b, P, qn, qpack);
    if (fin) busy = false;
    if (cm == 0ull && cb + kWave >= v1 && ballot(busy) == 0ull) break;
  }
}

__device__ __forceinline__ int ms_heuristic(int dir, long long nf, long long mf, long long mu,
                                            long long nf_prev, long long n, int alpha,
                                            int beta) {
  if (dir == 0) return (mf * (long long)alpha > mu) ? 1 : 0;
  return (nf * (long long)beta < n && nf < nf_prev) ? 0 : 1;
}

__global__ __launch_bounds__(kMsBlock) void msbfs_kernel(MsParams P) {
  __shared__ ChunkLds s_chunk;
  __shared__ MsStage s_st;
  MsCtl* ctl = P.ctl;
  const int64_t gtid = (int64_t)blockIdx.x * kMsBlock + threadIdx.x;
  const int64_t gsz = (int64_t)gridDim.x * kMsBlock;
  const uint64_t emask = (1ull << P.eb) - 1ull;
  const int l = lane_id();
  if (threadIdx.x < kMsWaves) s_st.cnt[threadIdx.x] = 0;

  for (int64_t i = gtid; i < P.n_sweep; i += gsz) {
    P.vis[i] = 0ull;
    P.front[0][i] = 0ull;
    P.front[1][i] = 0ull;
  }
  if (gtid == 0) {
    for (int r = 0; r < 2; ++r) {
      ctl->qpack[r][0] = 0ull;
      ctl->edges[r][0] = 0ull;
      ctl->done_deg[r][0] = 0ull;
    }
    ctl->hts[0] = (unsigned long long)wall_clock64();
  }
  if (threadIdx.x == 0)
    for (int r = 0; r < 3; ++r) P.wctr[r * P.wstride + blockIdx.x * 16] = 0ull;
  __syncthreads();
  if (!grid_sync(&ctl->bar, P.timeout_ticks)) return;

  // roots: level 0 frontier (one wave; duplicate roots share a vertex)
  if (blockIdx.x == 0 && threadIdx.x < kWave) {
    for (int i0 = 0; i0 < P.nroots; i0 += kWave) {
      const int i = i0 + l;
      int32_t r = -1;
      bool first = false;
      int64_t dg = 0;
      if (i < P.nroots) {
        r = P.roots[i];
        const int j = i % P.k;
        if (r >= 0) {
          const unsigned long long old =
              atomicOr((unsigned long long*)&P.front[0][r], 1ull << j);
          first = (old == 0ull);
          // depth 0, parent itself
          P.dp[(int64_t)r * 64 + j] = ((uint64_t)P.base << 32) | (uint32_t)~(uint32_t)r;
          dg = P.off[r + 1] - P.off[r];
        }
      }
      ms_stage(s_st, first, r, dg, P, 0, &ctl->qpack[0][0]);
    }
    ms_flush(s_st, P, 0, &ctl->qpack[0][0]);
  }
  if (!grid_sync(&ctl->bar, P.timeout_ticks)) return;

  long long nf, mf, mu;
  {
    const unsigned long long pk =
        __hip_atomic_load(&ctl->qpack[0][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    nf = (long long)(pk >> P.eb);
    mf = (long long)(pk & emask);
    mu = P.deg_total;
  }
  if (gtid == 0) {
    ctl->hdir[0] = 0;
    ctl->hnf[0] = nf;
    ctl->hmf[0] = mf;
    ctl->hmu[0] = mu;
  }
  int L = 0, dir = 0;
  while (nf > 0) {
    const int c3 = L % 3, n3 = (L + 1) % 3, z3 = (L + 2) % 3;
    const int qc = L & 1, qn = qc ^ 1;
    const uint64_t* fcur = P.front[c3];
    uint64_t* fnext = P.front[n3];
    unsigned long long* qpack = &ctl->qpack[n3][0];
    int64_t examined = 0, done = 0;
    for (int64_t i = gtid; i < P.n_sweep; i += gsz) P.front[z3][i] = 0ull;
    if (gtid == 0) {
      ctl->qpack[z3][0] = 0ull;
      ctl->edges[z3][0] = 0ull;
      ctl->done_deg[z3][0] = 0ull;
    }
    if (threadIdx.x == 0) P.wctr[z3 * P.wstride + blockIdx.x * 16] = 0ull;
    if (dir == 0) {
      // ---- top-down push.  Every frontier edge (u, w) carries the root bits
      // of u that w has not seen; for each, (L+1, u) is proposed with an
      // atomicMin on the bit's parent slot, so the largest label stays (the
      // rule of the single-root search), and the bits are ORed into w's next
      // frontier word.  The OR that completes w's root set adds w's degree to
      // the completed degree sum.
      for (int64_t i = gtid; i < nf; i += gsz) {
        const int32_t u = P.qv[qc][i];
        P.vis[u] |= fcur[u];
      }
      const int64_t E = mf;
      const int64_t nchunks = ceil_div(E, kChunkEdges);
      for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const bool ok = expand_chunk<kMsBlock>(s_chunk, c, E, P.qv[qc], P.qe[qc], nf,
                                               P.chunk[qc], nchunks, P.off, P.cols,
                                               [&](bool active, int32_t u, int32_t w) {
          bool first = false;
          int64_t dw = 0;
          if (active) {
            const uint64_t seen = P.vis[w] | fcur[w];
            const uint64_t cand = fcur[u] & P.amask & ~seen;
            if (cand) {
              // (L+1, u) proposed per bit: depth sits in the high half and
              // the complement of the parent in the low half, so the smallest
              // word is the largest-label parent of this level
              unsigned long long* row = (unsigned long long*)P.dp + (int64_t)w * 64;
              const unsigned long long prop = ((unsigned long long)(P.base + (uint32_t)(L + 1)) << 32) |
                                              (uint32_t)~(uint32_t)u;
              uint64_t bits = cand;
              while (bits) {
                const int j = ffs64(bits);
                bits &= bits - 1;
                if (row[j] > prop) atomicMin(&row[j], prop);  // stale reads are larger
              }
              if (cand & ~fnext[w]) {
                const unsigned long long old = atomicOr((unsigned long long*)&fnext[w], cand);
                const int64_t deg = P.off[w + 1] - P.off[w];
                if (old == 0ull) {
                  first = true;
                  dw = deg;
                }
                if (((seen | old) & P.amask) != P.amask &&
                    ((seen | old | cand) & P.amask) == P.amask)
                  done += deg;
              }
            }
          }
          ms_stage(s_st, first, w, dw, P, qn, qpack);
        });
        if (!ok) {
          if (threadIdx.x == 0) atomicOr(&ctl->bar.status, kStatusBadInput);
          break;
        }
      }
      ms_flush(s_st, P, qn, qpack);
      if (gtid == 0) examined = E;
    } else {
      // ---- bottom-up pull over edge-balanced vertex ranges
      RangeCursor cur;
      for (;;) {
        const int64_t part = next_range(P.wctr + c3 * P.wstride, P.n_part, cur);
        if (part < 0) break;
        const int64_t v0 = (int64_t)P.bu_part[part] * kWave;
        const int64_t v1 = std::min<int64_t>((int64_t)P.bu_part[part + 1] * kWave, P.n_sweep);
        ms_pull_range(P, v0, v1, fcur, fnext, (int)(P.base + (uint32_t)(L + 1)), examined, done,
                      s_st, qn, qpack);
      }
      ms_flush(s_st, P, qn, qpack);
    }
    block_fold_add(&ctl->edges[n3][0], examined);
    block_fold_add(&ctl->done_deg[n3][0], done);
    if (!grid_sync(&ctl->bar, P.timeout_ticks)) return;

    const unsigned long long pk =
        __hip_atomic_load(&ctl->qpack[n3][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const long long nf_new = (long long)(pk >> P.eb);
    const long long mf_new = (long long)(pk & emask);
    const long long mu_new =
        mu - (long long)__hip_atomic_load(&ctl->done_deg[n3][0], __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
    int nd = dir;
    if (P.mode == RBFS_DIR_TD_ONLY) nd = 0;
    else if (P.mode == RBFS_DIR_BU_ONLY) nd = 1;
    else nd = ms_heuristic(dir, nf_new, mf_new, mu_new, nf, P.n_sweep, P.alpha, P.beta);
    if (gtid == 0 && L < RBFS_STATS_MAX_LEVELS) {
      ctl->hedges[L] = (long long)ctl->edges[n3][0];
      ctl->hts[L + 1] = (unsigned long long)wall_clock64();
      if (L + 1 < RBFS_STATS_MAX_LEVELS && nf_new > 0) {
        ctl->hdir[L + 1] = (signed char)nd;
        ctl->hnf[L + 1] = nf_new;
        ctl->hmf[L + 1] = mf_new;
        ctl->hmu[L + 1] = mu_new;
      }
    }
    nf = nf_new;
    mf = mf_new;
    mu = mu_new;
    dir = nd;
    ++L;
  }
  if (gtid == 0) ctl->levels = L;
}

__global__ void ms_fill_kernel(uint64_t* a, int64_t n, uint64_t val) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = val;
}

__global__ void ms_reset_ctl_kernel(MsCtl* c) {
  int* p = (int*)&c->bar;
  for (int i = threadIdx.x; i < (int)(sizeof(GridBarrier) / sizeof(int)); i += blockDim.x)
    p[i] = 0;
}

// Root-major outputs, indexed by and holding original IDs, from the packed
// per-(vertex, root) pairs of the graph, as a tiled transpose through LDS.
// A workgroup takes 128 consecutive original IDs: each wave reads the packed
// internal rows of 16 of them (lane = root, one coalesced 512-byte row per
// vertex, reset to "none" as it goes), then writes 8 of the root rows
// (lane = vertex, 512-byte runs per row and array).  Parents go back to
// original IDs through oid.  The loads of each phase are issued together so
// that their latencies overlap.  Isolated vertices get -1; isolated roots
// are fixed up by ms_roots_fixup_kernel.
constexpr int kTrBlock = 512;  // 8 waves
constexpr int kTrTile = 128;   // vertices per tile

__global__ __launch_bounds__(kTrBlock) void ms_translate_kernel(
    int64_t n_g, const int32_t* perm, int64_t n_sweep_g, int64_t ubase, int32_t k, uint64_t* dp,
    uint32_t base, int64_t n_sweep_u, int clear, const int32_t* oid, int32_t* out_dep,
    int32_t* out_par) {
  constexpr int kWaves = kTrBlock / kWave;
  constexpr int kRows = kTrTile / kWaves;   // vertices per wave in the read phase
  constexpr int kRoots = kWave / kWaves;    // roots per wave in the write phase
  __shared__ uint64_t tile[kTrTile][kWave + 1];  // [vertex][root], padded
  const int wv = wave_id(), l = lane_id();
  for (int64_t v0 = (int64_t)blockIdx.x * kTrTile; v0 < n_g;
       v0 += (int64_t)gridDim.x * kTrTile) {
    // read phase: the wave's 16 internal rows are fetched together (lanes
    // 0..15 read the row numbers, then every lane reads its root's entry of
    // all 16 rows) so that their latencies overlap
    const int64_t vr = v0 + wv * kRows + (l & (kRows - 1));
    const int64_t ir = (vr < n_g) ? (perm ? (int64_t)perm[vr] : vr) : n_sweep_g;
    int64_t iv[kRows];
    uint64_t xv[kRows];
#pragma unroll
    for (int t = 0; t < kRows; ++t) iv[t] = shfl(ir, t);
#pragma unroll
    for (int t = 0; t < kRows; ++t)
      xv[t] = (l < k && iv[t] < n_sweep_g) ? dp[(ubase + iv[t]) * 64 + l] : ~0ull;
#pragma unroll
    for (int t = 0; t < kRows; ++t) {
      tile[wv * kRows + t][l] = xv[t];
      if (clear && l < k && iv[t] < n_sweep_g) dp[(ubase + iv[t]) * 64 + l] = ~0ull;
    }
    __syncthreads();
    // write phase: 8 roots per wave, lane = vertex, two halves of 64
#pragma unroll
    for (int h = 0; h < kTrTile / kWave; ++h) {
      const int vv = h * kWave + l;
      const int64_t v = v0 + vv;
      int32_t d[kRoots], p[kRoots];
#pragma unroll
      for (int t = 0; t < kRoots; ++t) {
        const uint64_t x = tile[vv][wv * kRoots + t];
        // written by this batch: its depth field lies within n_sweep of the base
        const uint32_t df = (uint32_t)(x >> 32) - base;
        const bool cur = (uint64_t)df <= (uint64_t)n_sweep_u;
        d[t] = cur ? (int32_t)df : -1;
        p[t] = cur ? (int32_t)~(uint32_t)x : -1;
      }
      if (oid) {
#pragma unroll
        for (int t = 0; t < kRoots; ++t)
          if (p[t] >= 0) p[t] = oid[p[t]];
      }
#pragma unroll
      for (int t = 0; t < kRoots; ++t) {
        const int j = wv * kRoots + t;
        if (j < k && v < n_g) {
          out_dep[(int64_t)j * n_g + v] = d[t];
          out_par[(int64_t)j * n_g + v] = p[t];
        }
      }
    }
    __syncthreads();
  }
}

// Union IDs of the roots (-1 for isolated roots, which are not swept).
__global__ void ms_roots_kernel(const int32_t* roots_orig, int32_t k, const int32_t* perm,
                                int64_t n_sweep, int64_t ubase, int32_t* roots_union) {
  const int j = threadIdx.x;
  if (j >= k) return;
  const int32_t r = roots_orig[j];
  const int64_t i = perm ? perm[r] : r;
  roots_union[j] = (i < n_sweep) ? (int32_t)(ubase + i) : -1;
}

__global__ void ms_roots_fixup_kernel(int64_t n_g, const int32_t* perm, int64_t n_sweep_g,
                                      const int32_t* roots_orig, int32_t k, int32_t* out_dep,
                                      int32_t* out_par) {
  const int j = threadIdx.x;
  if (j >= k) return;
  const int32_t r = roots_orig[j];
  const int64_t i = perm ? perm[r] : r;
  if (i >= n_sweep_g) {
    out_dep[(int64_t)j * n_g + r] = 0;
    out_par[(int64_t)j * n_g + r] = r;
  }
}

// union construction: shifted copies of one graph's internal CSR
__global__ void union_off_kernel(const int64_t* off, int64_t n_sweep, int64_t ubase,
                                 int64_t ebase, int64_t* uoff) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n_sweep;
       i += (int64_t)gridDim.x * blockDim.x)
    uoff[ubase + i] = ebase + off[i];
}

__global__ void union_cols_kernel(const int32_t* cols, int64_t nnz, int64_t ubase,
                                  int64_t ebase, int32_t* ucols) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x)
    ucols[ebase + e] = (int32_t)(ubase + cols[e]);
}

__global__ void union_oid_kernel(const int32_t* iperm, int64_t n_sweep, int64_t ubase,
                                 int32_t* uoid) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_sweep;
       i += (int64_t)gridDim.x * blockDim.x)
    uoid[ubase + i] = iperm ? iperm[i] : (int32_t)i;
}

int grid_blocks(int64_t work) {
  int64_t b = ceil_div(work, 256);
  if (b < 1) b = 1;
  if (b > (1 << 20)) b = 1 << 20;
  return (int)b;
}

}  // namespace

#define MS_CHECK(x)                                                             \
  do {                                                                          \
    hipError_t e_ = (x);                                                        \
    if (e_ != hipSuccess) {                                                     \
      set_error(std::string("bfs_batch: ") + #x + ": " + hipGetErrorString(e_)); \
      return e_ == hipErrorOutOfMemory ? RBFS_E_NOMEM : RBFS_E_DEVICE;          \
    }                                                                           \
  } while (0)

void ms_engine_free(MsEngine* m) {
  if (!m) return;
  void* ps[] = {m->uoff, m->ucols, m->uoid, m->vis, m->front, m->dp, m->qv[0],
                m->qv[1], m->qe[0], m->qe[1], m->chunk[0], m->chunk[1], m->bu_part, m->ctl,
                m->roots_dev, m->wctr};
  for (void* p : ps)
    if (p) (void)rbfs::dev_free(p);
  m->uoff = nullptr;
  m->ucols = nullptr;
  m->uoid = nullptr;
  m->vis = m->front = nullptr;
  m->dp = nullptr;
  m->qv[0] = m->qv[1] = m->chunk[0] = m->chunk[1] = m->bu_part = nullptr;
  m->qe[0] = m->qe[1] = nullptr;
  m->ctl = nullptr;
  m->roots_dev = nullptr;
  m->wctr = nullptr;
  if (m->roots_host) (void)hipHostFree(m->roots_host);
  m->roots_host = nullptr;
  if (m->gexec) (void)hipGraphExecDestroy(m->gexec);
  m->gexec = nullptr;
  if (m->ev0) (void)hipEventDestroy(m->ev0);
  if (m->ev1) (void)hipEventDestroy(m->ev1);
  m->ev0 = m->ev1 = nullptr;
}

void free_ms_work(Graph* g) {
  if (!g->ms) return;
  ms_engine_free(g->ms);
  delete g->ms;
  g->ms = nullptr;
}

// Sets up the engine's work buffers for an already described union graph
// (off, cols, oid, n_sweep, nnz filled in).
int ms_engine_setup(MsEngine* m, int compute_units, int64_t wall_rate_khz, hipStream_t stream) {
  const int64_t ns = m->n_sweep > 0 ? m->n_sweep : 1;
  MS_CHECK(rbfs::dev_malloc(&m->vis, sizeof(uint64_t) * ns));
  MS_CHECK(rbfs::dev_malloc(&m->front, sizeof(uint64_t) * 3 * ns));
  MS_CHECK(rbfs::dev_malloc(&m->dp, sizeof(uint64_t) * 64 * ns));
  for (int i = 0; i < 2; ++i) {
    MS_CHECK(rbfs::dev_malloc(&m->qv[i], sizeof(int32_t) * ns));
    MS_CHECK(rbfs::dev_malloc(&m->qe[i], sizeof(int64_t) * ns));
  }
  m->chunk_cap = ceil_div(m->nnz, kChunkEdges) + 2;
  for (int i = 0; i < 2; ++i) MS_CHECK(rbfs::dev_malloc(&m->chunk[i], sizeof(int32_t) * m->chunk_cap));
  MS_CHECK(rbfs::dev_malloc(&m->ctl, sizeof(MsCtl)));
  MS_CHECK(hipMemsetAsync(m->ctl, 0, sizeof(MsCtl), stream));
  MS_CHECK(rbfs::dev_malloc(&m->roots_dev, sizeof(int32_t) * 64 * 2 * m->ngraphs));
  MS_CHECK(hipHostMalloc(&m->roots_host, sizeof(int32_t) * 64 * (1 + m->ngraphs)));
  hipLaunchKernelGGL(ms_fill_kernel, dim3(grid_blocks(64 * ns)), dim3(256), 0, stream, m->dp,
                     64 * ns, ~0ull);
  MS_CHECK(hipGetLastError());
  int per_cu = 0;
  MS_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, msbfs_kernel, kMsBlock, 0));
  m->max_per_cu = per_cu < 1 ? 1 : per_cu;
  m->compute_units = compute_units;
  m->max_grid = 4 * compute_units;  // per_cu is at most 4
  MS_CHECK(rbfs::dev_malloc(&m->wctr, sizeof(unsigned long long) * 3 * 16 * (size_t)m->max_grid));
  MS_CHECK(hipEventCreate(&m->ev0));
  MS_CHECK(hipEventCreate(&m->ev1));
  MS_CHECK(hipStreamSynchronize(stream));
  m->wall_rate_khz = wall_rate_khz;
  return ms_apply_tuning(m, default_tuning(RBFS_TUNE_BATCH), stream);
}

int ms_apply_tuning(MsEngine* m, const rbfs_tuning_t& t, hipStream_t stream) {
  const int per = std::max(1, std::min(t.per_cu, m->max_per_cu));
  const int grid = per * m->compute_units;
  if (!m->bu_part || t.bu_grain != m->tune.bu_grain || grid != m->grid) {
    // edge-balanced vertex ranges (in 64-vertex units) for the bottom-up pull
    if (m->bu_part) (void)rbfs::dev_free(m->bu_part);
    m->bu_part = nullptr;
    m->n_part = 0;
    int rc = build_edge_ranges(m->uoff ? m->uoff : m->off, m->n_sweep, m->nnz,
                               (int64_t)t.bu_grain * grid, 1, &m->bu_part, &m->n_part, stream);
    if (rc) return rc;
  }
  m->grid = grid;
  m->tune = t;
  if (m->gexec) (void)hipGraphExecDestroy(m->gexec);
  m->gexec = nullptr;
  return 0;
}

// Enqueues one search of up to 64 roots (internal union IDs already in
// m->roots_dev): control reset + persistent kernel.
static uint64_t ms_base_step(const MsEngine* m) {
  return std::max<uint64_t>((uint64_t)m->n_sweep + 1, 1ull << 26);
}
static uint32_t ms_top_base(const MsEngine* m) {
  return (uint32_t)(0xFFFFFFFFull - ms_base_step(m));
}

int ms_enqueue_search(MsEngine* m, int32_t k, int32_t nroots, int mode, int alpha, int beta,
                      hipStream_t stream) {
  const int bits_n = bits_for(m->n_sweep + 2);
  const int eb = 64 - bits_n;
  if (((uint64_t)m->nnz >> eb) != 0) {
    set_error("bfs_batch: graph too large for the packed queue counter");
    return RBFS_E_UNSUPPORTED;
  }
  MsParams P{};
  P.off = m->uoff ? m->uoff : m->off;
  P.cols = m->ucols ? m->ucols : m->cols;
  P.n_sweep = m->n_sweep;
  P.deg_total = m->nnz;
  P.vis = m->vis;
  for (int i = 0; i < 3; ++i) P.front[i] = m->front + (size_t)i * (m->n_sweep > 0 ? m->n_sweep : 1);
  P.dp = m->dp;
  {
    // each batch lowers the base by at least n_sweep + 1; the all-ones state
    // (base 0xFFFFFFFF) is the start of a run
    const uint64_t step = ms_base_step(m);
    if (m->fixed_base) {
      P.base = ms_top_base(m);
    } else {
      if (m->base_valid && (uint64_t)m->base >= step) {
        P.base = (uint32_t)(m->base - step);
      } else {
        // a new run of bases: every pair back to all ones first
        hipLaunchKernelGGL(ms_fill_kernel, dim3(grid_blocks(64 * (m->n_sweep > 0 ? m->n_sweep : 1))),
                           dim3(256), 0, stream, m->dp, 64 * (m->n_sweep > 0 ? m->n_sweep : 1),
                           ~0ull);
        MS_CHECK(hipGetLastError());
        P.base = ms_top_base(m);
      }
      m->base = P.base;
      m->base_valid = true;
    }
  }
  for (int i = 0; i < 2; ++i) {
    P.qv[i] = m->qv[i];
    P.qe[i] = m->qe[i];
    P.chunk[i] = m->chunk[i];
  }
  P.chunk_cap = m->chunk_cap;
  P.bu_part = m->bu_part;
  P.n_part = m->n_part;
  P.wctr = m->wctr;
  P.wstride = 16 * (int64_t)m->max_grid;
  if (m->grid < 1 || m->grid > m->max_grid) {  // the range counters hold max_grid workgroups
    set_error("bfs_batch: launch grid outside the workspace");
    return RBFS_E_STATE;
  }
  P.roots = m->roots_dev;
  P.nroots = nroots;
  P.k = k;
  P.amask = (k >= 64) ? ~0ull : ((1ull << k) - 1ull);
  P.mode = mode;
  P.alpha = alpha;
  P.beta = beta;
  P.eb = eb;
  P.lane_row = m->tune.lane_row;
  P.timeout_ticks = (uint64_t)m->wall_rate_khz * 1000ull * 4ull;
  P.ctl = m->ctl;
  hipLaunchKernelGGL(ms_reset_ctl_kernel, dim3(1), dim3(256), 0, stream, m->ctl);
  MS_CHECK(hipGetLastError());
  hipLaunchKernelGGL(msbfs_kernel, dim3(m->grid), dim3(kMsBlock), 0, stream, P);
  MS_CHECK(hipGetLastError());
  return 0;
}

int ms_enqueue_translate(MsEngine* m, int64_t n_g, const int32_t* perm, int64_t n_sweep_g,
                         int64_t ubase, int32_t k, const int32_t* roots_orig_dev,
                         int32_t* out_dep, int32_t* out_par, hipStream_t stream) {
  const int64_t tiles = std::max<int64_t>(1, std::min<int64_t>(ceil_div(n_g, kTrTile), 1 << 20));
  hipLaunchKernelGGL(ms_translate_kernel, dim3((unsigned)tiles), dim3(kTrBlock), 0, stream, n_g,
                     perm, n_sweep_g, ubase, k, m->dp, m->fixed_base ? ms_top_base(m) : m->base,
                     m->n_sweep, m->fixed_base ? 1 : 0, m->uoid ? m->uoid : m->oid, out_dep,
                     out_par);
  MS_CHECK(hipGetLastError());
  hipLaunchKernelGGL(ms_roots_fixup_kernel, dim3(1), dim3(64), 0, stream, n_g, perm, n_sweep_g,
                     roots_orig_dev, k, out_dep, out_par);
  MS_CHECK(hipGetLastError());
  return 0;
}

int ms_read_stats(MsEngine* m, hipStream_t stream, void* stats_v) {
  rbfs_stats_t* stats = (rbfs_stats_t*)stats_v;
  MsCtl* h = new MsCtl;
  hipError_t e = hipMemcpyAsync(h, m->ctl, sizeof(MsCtl), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    delete h;
    MS_CHECK(e);
  }
  const int st = h->bar.status;
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->levels = h->levels;
    stats->status = st;
    const int nl = std::min(h->levels, RBFS_STATS_MAX_LEVELS);
    for (int i = 0; i < nl; ++i) {
      stats->dir[i] = h->hdir[i];
      stats->nf[i] = h->hnf[i];
      stats->mf[i] = h->hmf[i];
      stats->mu[i] = h->hmu[i];
      stats->edges[i] = h->hedges[i];
      stats->level_us[i] = (float)((double)(h->hts[i + 1] - h->hts[i]) * 1000.0 /
                                   (double)m->wall_rate_khz);
    }
  }
  delete h;
  if (st != 0) {
    m->base_valid = false;  // the next batch starts a new run of bases
    set_error("bfs_batch: device status " + std::to_string(st));
    return RBFS_E_DEVICE;
  }
  return 0;
}

static int ensure_ms(Graph* g, hipStream_t stream) {
  if (g->ms) return 0;
  MsEngine* m = new MsEngine();
  g->ms = m;
  m->off = g->off;
  m->cols = g->cols;
  m->oid = g->reordered ? g->iperm : nullptr;
  m->n_sweep = g->n_sweep;
  m->nnz = g->nnz;
  int rc = ms_engine_setup(m, g->compute_units, g->wall_rate_khz, stream);
  if (!rc) rc = ms_apply_tuning(m, g->tune_batch, stream);
  if (rc) return rc;
  g->bytes += sizeof(uint64_t) * 64 * (size_t)(g->n_sweep > 0 ? g->n_sweep : 1);
  return 0;
}


int ms_enqueue_roots(const int32_t* roots_orig_dev, int32_t k, const int32_t* perm,
                     int64_t n_sweep, int64_t ubase, int32_t* roots_union, hipStream_t stream) {
  hipLaunchKernelGGL(ms_roots_kernel, dim3(1), dim3(64), 0, stream, roots_orig_dev, k, perm,
                     n_sweep, ubase, roots_union);
  MS_CHECK(hipGetLastError());
  return 0;
}

// Packs the internal CSRs of the graphs into one union CSR: graph g's swept
// vertices occupy [ubase_g, ubase_g + n_sweep_g).
int ms_build_union(MsEngine* m, const Graph* const* gs, int count, hipStream_t stream) {
  int64_t ntot = 0, etot = 0;
  for (int i = 0; i < count; ++i) {
    ntot += gs[i]->n_sweep;
    etot += gs[i]->nnz;
  }
  m->n_sweep = ntot;
  m->nnz = etot;
  MS_CHECK(rbfs::dev_malloc(&m->uoff, sizeof(int64_t) * (ntot + 1)));
  MS_CHECK(rbfs::dev_malloc(&m->ucols, sizeof(int32_t) * (etot > 0 ? etot : 1)));
  MS_CHECK(rbfs::dev_malloc(&m->uoid, sizeof(int32_t) * (ntot > 0 ? ntot : 1)));
  int64_t ub = 0, eb = 0;
  for (int i = 0; i < count; ++i) {
    const Graph* g = gs[i];
    hipLaunchKernelGGL(union_off_kernel, dim3(grid_blocks(g->n_sweep + 1)), dim3(256), 0, stream,
                       g->off, g->n_sweep, ub, eb, m->uoff);
    if (g->nnz > 0)
      hipLaunchKernelGGL(union_cols_kernel, dim3(grid_blocks(g->nnz)), dim3(256), 0, stream,
                         g->cols, g->nnz, ub, eb, m->ucols);
    hipLaunchKernelGGL(union_oid_kernel, dim3(grid_blocks(g->n_sweep)), dim3(256), 0, stream,
                       g->reordered ? g->iperm : nullptr, g->n_sweep, ub, m->uoid);
    MS_CHECK(hipGetLastError());
    ub += g->n_sweep;
    eb += g->nnz;
  }
  MS_CHECK(hipStreamSynchronize(stream));
  return 0;
}

int bfs_batch_impl(Graph* g, const int32_t* roots, int32_t k, int32_t* depth, int32_t* parent,
                   int mode, int alpha, int beta, int out_space, int flags, hipStream_t stream,
                   void* stats) {
  (void)flags;
  if (out_space != RBFS_OUT_ORIGINAL) {
    set_error("bfs_batch: only original-ID output is supported");
    return RBFS_E_UNSUPPORTED;
  }
  int rc = ensure_ms(g, stream);
  if (rc) return rc;
  MsEngine* m = g->ms;
  int32_t* roots_orig_dev = m->roots_dev + 64 * m->ngraphs;
  for (int32_t j0 = 0; j0 < k; j0 += 64) {
    const int32_t kk = std::min<int32_t>(64, k - j0);
    memcpy(m->roots_host, roots + j0, sizeof(int32_t) * kk);
    hipError_t e = hipMemcpyAsync(roots_orig_dev, m->roots_host, sizeof(int32_t) * kk,
                                  hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);  // host buffer reused next pass
    MS_CHECK(e);
    rc = ms_enqueue_roots(roots_orig_dev, kk, g->reordered ? g->perm : nullptr, g->n_sweep, 0,
                          m->roots_dev, stream);
    if (!rc) rc = ms_enqueue_search(m, kk, kk, mode, alpha, beta, stream);
    if (!rc)
      rc = ms_enqueue_translate(m, g->n, g->reordered ? g->perm : nullptr, g->n_sweep, 0, kk,
                                roots_orig_dev, depth + (int64_t)j0 * g->n,
                                parent + (int64_t)j0 * g->n, stream);
    if (!rc && (stats || j0 + 64 < k)) rc = ms_read_stats(m, stream, stats);
    if (rc) return rc;
  }
  return ms_read_stats(m, stream, stats);
}

}  // namespace rbfs
