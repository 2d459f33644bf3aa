// Single-root direction-optimizing BFS (Algorithm 2) as one persistent
// kernel: the level loop, both step kinds and the per-level direction
// decision run on the GPU with no host round trip.
//
// Labels are the graph's internal labels; the swept set is [0, n_sweep)
// (the non-isolated prefix after RCM).  parent(v) is the largest-label
// neighbour one level up, reached the same way by both step kinds: a scan of
// v's row in decreasing label order that stops at the first neighbour in the
// current frontier F_d (any visited neighbour of a vertex first reached at
// level d+1 lies in F_d), or the maximum over all its frontier neighbours.
// After RCM labels rise with degree, so the downward scan meets the hubs
// first, as the degree-ordered bottom-up scan of Algorithm 6 does, and most
// rows stop after a few entries.  Depth and parent of a vertex are one 64-bit
// word, depth in the high half and the complement of the parent in the low
// half (unreached = all ones), so that ordering the words orders by depth
// first and then by decreasing parent label:
//   top-down (Algorithms 1 and 4): frontier edges (u, w) are spread evenly
//     over the GPU; every edge into a w unvisited at level start proposes
//     (d+1, u) with one 64-bit atomicMin: the smallest word, i.e. the
//     largest-label parent, stays, and the one proposal that finds w
//     unreached claims w and appends it;
//   bottom-up (the bottom-up step of Algorithm 2, Algorithm 5): every
//     unvisited v scans its own row; one wave owns a 64-vertex word, the
//     found bits come from one ballot and are stored without atomics (the GPU
//     form of the paper's cache-line blocks).
//
// Visited state: `vis` (reached before level d) plus three rotating frontier
// bitmaps: front[d % 3] = F_d, front[(d+1) % 3] receives F_{d+1}, and
// front[(d+2) % 3] (holding the dead F_{d-1}) is cleared for the next level.
// "Visited at the start of level d" is vis | F_d, so folding F_d into vis can
// happen during level d itself (the paper's visited |= next outside the
// loop), and every level needs exactly one grid barrier.
//
// Every workgroup keeps the level state (level, direction, |F|, degree sums)
// in registers and takes the direction decision itself from the one packed
// counter it reads after the barrier, so nothing runs serially inside the
// barrier.  Queue appends are staged per wave in LDS and published with one
// packed 64-bit atomic (count << eb | degree sum) per batch; the returned
// base gives both the queue position and the exclusive degree prefix that
// drives the edge-balanced top-down expansion of the next level.  Bottom-up
// work is cut into edge-balanced ranges of words; each workgroup owns a share
// behind its own counter and steals from the fullest others when done (the
// work stealing of Algorithm 5).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/rbfs.h"
#include "common.h"
#include "expand.h"
#include "graph.h"
#include "mlp_dev.h"
#include "switch.h"

namespace rbfs {

const float* switch_blob_device(int device);

// The next frontier (and the bottom-up vertex list) is split into kNQ
// sub-queues, one per group of workgroups (blockIdx mod kNQ, i.e. one per
// XCD), each behind its own packed counter: a single grid-wide counter
// serialises the appends of every wave on one address.
constexpr int kNQ = 8;
// ... plus one shared overflow sub-queue (and sub-list), index kNQ: a
// sub-queue holds qcap entries, and a flush that does not fit puts the rest
// there, so the queues need about 3 n entries in total instead of 8 n.
constexpr int kNQT = kNQ + 1;

struct alignas(128) BfsCtl {
  GridBarrier bar;
  alignas(128) unsigned long long qpack[3][kNQT][16];  // [rotation][sub-queue][0], own line each
  alignas(128) unsigned long long edges[3][16];     // entries read this level
  alignas(128) unsigned long long vlcnt[3][kNQT][16];  // vertices appended to each sub-list
  int levels;
  int sticky;  // statuses of the searches since the last rbfs_graph_check
  int sweep_lo, sweep_hi;  // bottom-up sweep: the root's component
  long long reached, deg_reached;
  signed char hdir[RBFS_STATS_MAX_LEVELS];
  signed char hood[RBFS_STATS_MAX_LEVELS];
  long long hnf[RBFS_STATS_MAX_LEVELS];
  long long hmf[RBFS_STATS_MAX_LEVELS];
  long long hmu[RBFS_STATS_MAX_LEVELS];
  long long hedges[RBFS_STATS_MAX_LEVELS];
  unsigned long long hts[RBFS_STATS_MAX_LEVELS + 1];
};

namespace {

constexpr int kStage = 384;  // staged appends per wave
constexpr int kListRange = 128;  // list vertices per bottom-up work range
constexpr int kScanStep = 8;    // row entries a lane tests per step (after the first)
static_assert(kScanStep == 8, "the row scan loads two aligned groups of 4 entries");
constexpr uint64_t kUnreached = ~0ull;  // packed pair of an unreached vertex

// Packed search state of a vertex: the depth field in the high half and the
// bitwise complement of the parent in the low half, so that the smallest
// word has the smallest depth and, within it, the largest parent label.
// The depth field is base + depth, with a base that each search lowers by
// at least n_sweep + 1: every word left by an earlier search then compares
// above every word of this one, as an unreached word does, so a search needs
// no initialisation pass until the base runs out.
__device__ __forceinline__ uint64_t pack_dp(uint32_t dfield, int32_t p) {
  return ((uint64_t)dfield << 32) | (uint32_t)~(uint32_t)p;
}
// True when word x was written by the search whose base is `base` (n_sweep
// bounds its depths).
__device__ __forceinline__ bool dp_current(uint64_t x, uint32_t base, int64_t n_sweep) {
  return (uint64_t)(uint32_t)((uint32_t)(x >> 32) - base) <= (uint64_t)n_sweep;
}
__device__ __forceinline__ int32_t dp_parent(uint64_t x) { return (int32_t)~(uint32_t)x; }

struct BfsParams {
  const int64_t* off;
  const int32_t* cols;
  const int32_t* perm;   // original -> internal, null when not reordered
  int64_t n_sweep;
  int64_t deg_total;     // degree sum over the swept set
  uint64_t* dp;          // packed (depth << 32 | ~parent) per swept vertex
  const int32_t* comp_bounds;  // component intervals (null: one interval)
  int64_t n_comp;
  uint64_t* vis;
  uint64_t* front[3];
  int32_t* qv[2];        // kNQ sub-queues of qcap entries each, then the overflow one
  int64_t* qe[2];
  int32_t* chunk[2];     // kNQ chunk tables of chunk_cap entries each
  int64_t chunk_cap;
  int64_t qcap;         // entries of each of the kNQ sub-queues (and sub-lists); the
                         // overflow one at index kNQ holds n_sweep
  const int32_t* bu_part;
  int32_t n_part;
  unsigned long long* wctr;  // BU range counters: 3 slots of wstride, 16 per workgroup
  int64_t wstride;
  int32_t* vl[2];            // vertex lists (kNQ sub-lists of qcap entries, overflow)
  const int32_t* top;        // largest-label neighbour of each swept vertex
  // the ablation without load balancing (RBFS_OPT_NO_BALANCE): top-down one
  // frontier vertex per thread, bottom-up equal vertex ranges per workgroup
  // with no stealing
  int32_t no_lb;
  int32_t root_orig;
  int32_t init;
  uint32_t base;         // depth field of depth 0 (see pack_dp)
  int32_t mode;
  int32_t alpha, beta;
  int32_t sched_len;
  int8_t sched[RBFS_STATS_MAX_LEVELS];
  int32_t eb;
  int32_t lane_row;      // bottom-up lane/wave split
  int32_t cshift;        // log2 of the top-down chunk length
  uint64_t timeout_ticks;
  const float* sw;       // learned-switch blob (RBFS_DIR_LEARNED)
  int64_t* wg_work;      // non-null: entries each workgroup processed, per level
  BfsCtl* ctl;
};

// LDS shared by the two step kinds: the chunk staging of the top-down
// expansion, or the coarse frontier summary of a sparse bottom-up level (a
// bit per 2^fs vertices).
template <int BLOCK>
union StepLds {
  static constexpr int kFiltWords = BLOCK >= 1024 ? 16384 : 4096;
  ChunkLdsB<kTdK * BLOCK> chunk;
  uint32_t filt[kFiltWords];
};

template <int WAVES>
struct StageLds {
  int32_t v[WAVES][kStage];
  int32_t d[WAVES][kStage];
  int32_t cnt[WAVES];
  uint64_t found[WAVES][kWave];  // bottom-up: found bits of the batch's words
  int32_t lv[WAVES][kStage];     // bottom-up: vertices left for the next list
  int32_t lcnt[WAVES];
};

// Publishes this wave's staged vertices to its sub-queue of the next
// frontier (qpack: the packed counters of the next level, one line per
// sub-queue).  The part that does not fit in the sub-queue's qcap entries
// goes to the overflow sub-queue (index kNQ), with its own count, degree
// prefix and chunk marks; the entries inside keep theirs, so the sub-queue
// holds exactly its first qcap positions (the next level clamps its count).
template <class ST>
__device__ __forceinline__ void flush_stage(ST& st, const BfsParams& P, int nq_idx,
                                            unsigned long long* qpack) {
  const int wv = wave_id(), l = lane_id();
  const int cnt = st.cnt[wv];
  if (cnt == 0) return;
  const int sq = (int)(blockIdx.x & (kNQ - 1));
  int64_t total = 0;
  for (int j0 = 0; j0 < cnt; j0 += kWave) {
    const int j = j0 + l;
    total += (j < cnt) ? (int64_t)st.d[wv][j] : 0;
  }
  total = wave_sum(total);
  unsigned long long old = 0;
  if (l == 0)
    old = atomicAdd(qpack + sq * 16,
                    ((unsigned long long)cnt << P.eb) + (unsigned long long)total);
  old = shfl(old, 0);
  const int64_t pos0 = (int64_t)(old >> P.eb);
  const int64_t ebase0 = (int64_t)(old & ((1ull << P.eb) - 1ull));
  // entries [0, kin) stay in the sub-queue, [kin, cnt) overflow
  const int kin = (int)std::max<int64_t>(0, std::min<int64_t>(cnt, P.qcap - pos0));
  int64_t pos1 = 0, ebase1 = 0, din = 0;
  if (kin < cnt) {
    for (int j0 = 0; j0 < kin; j0 += kWave) {
      const int j = j0 + l;
      din += (j < kin) ? (int64_t)st.d[wv][j] : 0;
    }
    din = wave_sum(din);
    unsigned long long o1 = 0;
    if (l == 0)
      o1 = atomicAdd(qpack + kNQ * 16, ((unsigned long long)(cnt - kin) << P.eb) +
                                           (unsigned long long)(total - din));
    o1 = shfl(o1, 0);
    pos1 = (int64_t)(o1 >> P.eb);
    ebase1 = (int64_t)(o1 & ((1ull << P.eb) - 1ull));
    if (pos1 + (cnt - kin) > P.n_sweep) {  // cannot happen: a level appends each vertex once
      if (l == 0) atomicOr(&P.ctl->bar.status, kStatusOverflow);
      __builtin_amdgcn_wave_barrier();
      if (l == 0) st.cnt[wv] = 0;
      __builtin_amdgcn_wave_barrier();
      return;
    }
  }
  int64_t run = 0;  // degree sum of the entries before this round
  for (int j0 = 0; j0 < cnt; j0 += kWave) {
    const int j = j0 + l;
    const bool act = j < cnt;
    const int64_t d = act ? (int64_t)st.d[wv][j] : 0;
    const int64_t inc = wave_inclusive_sum(d);
    if (act) {
      const int64_t g = run + inc - d;  // degree prefix inside this flush
      const bool in = j < kin;
      const int q = in ? sq : kNQ;
      const int64_t pos = in ? pos0 + j : pos1 + (j - kin);
      const int64_t base = in ? ebase0 + g : ebase1 + (g - din);
      P.qv[nq_idx][q * P.qcap + pos] = st.v[wv][j];
      P.qe[nq_idx][q * P.qcap + pos] = base;
      mark_chunks(P.chunk[nq_idx] + q * P.chunk_cap, P.chunk_cap, base, d, (int32_t)pos,
                  P.cshift);
    }
    run += shfl(inc, kWave - 1);
  }
  __builtin_amdgcn_wave_barrier();
  if (l == 0) st.cnt[wv] = 0;
  __builtin_amdgcn_wave_barrier();
}

// Stages the vertices of the lanes with take = true; flushes when full.
template <class ST>
__device__ __forceinline__ void stage(ST& st, bool take, int32_t v, int64_t deg,
                                      const BfsParams& P, int nq_idx,
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
  if (base + popc64(m) > kStage - kWave) flush_stage(st, P, nq_idx, qpack);
}

// Publishes this wave's staged list vertices to its sub-list (out: the
// sub-lists of cap entries each, then the overflow sub-list of n_sweep;
// count: their counters, one line each).  The part that does not fit goes
// to the overflow sub-list.
template <class ST>
__device__ __forceinline__ void flush_list(ST& st, int32_t* out, unsigned long long* count,
                                           int64_t cap, int64_t n_sweep, BfsCtl* ctl) {
  const int wv = wave_id(), l = lane_id();
  const int cnt = st.lcnt[wv];
  if (cnt == 0) return;
  const int sq = (int)(blockIdx.x & (kNQ - 1));
  unsigned long long base = 0;
  if (l == 0)
    base = __hip_atomic_fetch_add(count + sq * 16, (unsigned long long)cnt, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
  base = shfl(base, 0);
  const int kin = (int)std::max<int64_t>(0, std::min<int64_t>(cnt, cap - (int64_t)base));
  unsigned long long b1 = 0;
  if (kin < cnt) {
    if (l == 0)
      b1 = __hip_atomic_fetch_add(count + kNQ * 16, (unsigned long long)(cnt - kin),
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    b1 = shfl(b1, 0);
  }
  if ((int64_t)b1 + (cnt - kin) > n_sweep) {  // cannot happen: each vertex once per level
    if (l == 0) atomicOr(&ctl->bar.status, kStatusOverflow);
  } else {
    for (int j = l; j < cnt; j += kWave) {
      if (j < kin) out[sq * cap + (int64_t)base + j] = st.lv[wv][j];
      else out[kNQ * cap + (int64_t)b1 + (j - kin)] = st.lv[wv][j];
    }
  }
  __builtin_amdgcn_wave_barrier();
  if (l == 0) st.lcnt[wv] = 0;
  __builtin_amdgcn_wave_barrier();
}

// Stages the vertices of the lanes with take = true for the next list.
template <class ST>
__device__ __forceinline__ void stage_list(ST& st, bool take, int32_t v, int32_t* out,
                                           unsigned long long* count, int64_t cap,
                                           int64_t n_sweep, BfsCtl* ctl) {
  const uint64_t m = ballot(take);
  if (m == 0) return;
  const int wv = wave_id();
  const int base = st.lcnt[wv];
  __builtin_amdgcn_wave_barrier();
  if (take) st.lv[wv][base + popc64(m & lanemask_lt())] = v;
  if (lane_id() == 0) st.lcnt[wv] = base + popc64(m);
  __builtin_amdgcn_wave_barrier();
  if (base + popc64(m) > kStage - kWave) flush_list(st, out, count, cap, n_sweep, ctl);
}

// visited |= F_d for level d: through the queue (sub-queue sizes qcnt) when
// the frontier is small, else word by word.
__device__ __forceinline__ void fold_frontier(const BfsParams& P, int qc, long long nf,
                                              const uint64_t* fcur, int64_t W, int64_t gtid,
                                              int64_t gsz, const long long* qcnt) {
  if (nf * 8 < W) {
    for (int q = 0; q < kNQT; ++q) {
      const int32_t* qv = P.qv[qc] + q * P.qcap;
      for (int64_t i = gtid; i < qcnt[q]; i += gsz) {
        const int32_t u = qv[i];
        atomicOr((unsigned long long*)&P.vis[u >> 6], 1ull << (u & 63));
      }
    }
  } else {
    for (int64_t w = gtid; w < W; w += gsz) P.vis[w] |= fcur[w];
  }
}

// Lane-refilled first-hit scans.  `total` candidates are handed to the lanes
// in order, and a lane that finishes its candidate takes the next one at
// once, so a long row keeps only its own lane busy instead of stalling the
// other 63.  Each lane also holds the candidate after its current one with
// its row bounds already loaded, so taking it over costs no extra memory
// round trip.  Each row gets the same downward first-hit scan in steps over
// aligned groups of 4 entries (one 16-byte load each): one group on a row's
// first step, since rows facing a dense frontier mostly hit at once, two
// groups on later steps; the probes of a step are independent, so one pair
// of memory round trips covers them all.  Rows longer than lane_row are
// scanned by the whole wave in one go.  filt (LDS, used when use_filt) is a
// coarse summary of bits that rules out most probes when the frontier is
// sparse.
// cand(t)
// gives candidate t's vertex (t < 0: none), or -1 to skip it; it is called
// by all lanes.  done(fin, found, v, par, deg) is called by all lanes after
// every step; fin marks the lanes that finished a candidate in it.
template <class Cand, class Done>
__device__ __forceinline__ void refill_scan(int total, const int64_t* off, const int32_t* cols,
                                            const int32_t* top, const uint64_t* bits,
                                            const uint32_t* filt, bool use_filt, int fs,
                                            uint32_t hi0, int lane_row, int64_t& examined,
                                            Cand&& cand, Done&& done) {
  int next = 0;  // next candidate to hand out (same in every lane)
  bool busy = false, queued = false;
  int64_t v = 0, b = 0, j = 0, e = 0;  // current candidate
  int64_t vq = 0, bq = 0, eq = 0;      // queued candidate, bounds loaded
  int32_t t = 0, tq = 0;               // largest-label neighbours (with top)
  for (;;) {
    // take over the queued candidate
    bool fresh = false;
    if (!busy && queued) {
      v = vq;
      b = bq;
      e = eq;
      t = tq;
      j = e;
      busy = true;
      queued = false;
      fresh = true;
    }
    // queue the next one (its bounds arrive while this step runs)
    const uint64_t want = ballot(!queued);
    if (want != 0ull && next < total) {
      const int t = next + popc64(want & lanemask_lt());
      const int64_t c = cand((!queued && t < total) ? t : -1);
      next += popc64(want);
      if (c >= 0) {
        vq = c;
        bq = off[c];
        eq = off[c + 1];
        if (top) tq = top[c];
        queued = true;
      }
    }
    const bool hub = fresh && (e - b) > lane_row;
    bool found = false;
    int32_t par = 0;
    wave_hub_first_hit(hub, b, e, cols, bits, filt, use_filt, fs, hi0, found, par, examined);
    bool fin = hub;
    if (busy && !hub && j <= b) {
      fin = true;  // empty row
    } else if (busy && !hub && fresh && top) {
      // the row's highest entry from the dense copy: one probe and no
      // column load; against a dense frontier most rows end here
      examined += 1;
      if (probe_bit(bits, filt, use_filt, fs, hi0, (uint32_t)t)) {
        found = true;
        par = t;
        fin = true;
      } else {
        j = e - 1;
        fin = j <= b;
      }
    } else if (busy && !hub) {
      // entries below j, downwards, in aligned groups of 4: the group holding
      // entry j - 1 (w[0..3]) and, after a row's first step, the one below
      // it (w[4..7]) when it still holds entries of the row; entries from j
      // on (the next row) and below b (the previous row) are masked.  Reads
      // past the last row stay inside the column array's slack.  Positions
      // are kept relative to the top group: entry ga + r for r in [-4, 4).
      const int64_t ga = (j - 1) & ~(int64_t)3;
      const int rj = (int)(j - ga);                                // 1..4
      const int rb = (int)((b - ga > -8) ? b - ga : (int64_t)-8);  // row start
      const bool two = j != e && rb <= -1;
      int32_t w[kScanStep];
      bool h[kScanStep];
      {
        const int4 x = *(const int4*)(cols + ga);
        int4 y = make_int4(0, 0, 0, 0);
        if (two) y = *(const int4*)(cols + ga - 4);
        w[0] = x.x; w[1] = x.y; w[2] = x.z; w[3] = x.w;
        w[4] = y.x; w[5] = y.y; w[6] = y.z; w[7] = y.w;
      }
#pragma unroll
      for (int q = 0; q < kScanStep; ++q) {
        const int r = q < 4 ? q : q - 8;
        const bool in = (q < 4 || two) && r >= rb && r < rj;
        h[q] = in && probe_bit(bits, filt, use_filt, fs, hi0, (uint32_t)w[q]);
      }
      // the first hit downwards is the highest entry: visit the entries in
      // increasing position order (w[4..7], then w[0..3]), keep the last hit
      int hr = -9;
#pragma unroll
      for (int q = 4; q < kScanStep; ++q)
        if (h[q]) {
          hr = q - 8;
          par = w[q];
        }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (h[q]) {
          hr = q;
          par = w[q];
        }
      if (hr > -9) {
        found = true;
        fin = true;
        examined += rj - hr;
      } else {
        const int rlo = two ? -4 : 0;
        examined += rj - ((rlo > rb) ? rlo : rb);
        j = ga + rlo;
        fin = j <= b;
      }
    }
    done(fin, found, v, par, e - b);
    if (fin) busy = false;
    if (next >= total && ballot(busy || queued) == 0ull) break;
  }
}

// Sum of v over the workgroup, returned in thread 0 (0 elsewhere).  Every
// thread must call.
__device__ __forceinline__ int64_t block_sum(int64_t v) {
  __shared__ int64_t s_part[kMaxWaves];
  const int64_t w = wave_sum(v);
  if (lane_id() == 0) s_part[wave_id()] = w;
  __syncthreads();
  int64_t t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) t += s_part[i];
  __syncthreads();
  return t;
}

// LDS of the learned direction decision: wave 0's hidden layer and the
// decision it takes.  The network is read from the switch blob in global
// memory (5.7 KB, cache resident after the first level): an LDS copy made at
// kernel start costs the whole kernel registers.
struct LearnedLds {
  __align__(16) float h[kMlpHid];
  int dec[2];
};
struct NoLds {};

// WGW: record each workgroup's work per level (P.wg_work); LRN: learned
// direction decisions (RBFS_DIR_LEARNED).  Separate instantiations, so the
// searches that ask for neither run the kernel without that code.
template <int BLOCK, bool WGW, bool LRN>
__global__ __launch_bounds__(BLOCK) void bfs_persistent_kernel(BfsParams P) {
  constexpr int WAVES = BLOCK / kWave;
  __shared__ StepLds<BLOCK> s_step;
  __shared__ std::conditional_t<LRN, LearnedLds, NoLds> s_lrn;
  constexpr int kFiltBits = StepLds<BLOCK>::kFiltWords * 32;
  __shared__ StageLds<WAVES> s_st;
  // sizes of the current frontier's sub-queues and of the last vertex list's
  // sub-lists (the same in every workgroup)
  __shared__ long long s_qcnt[kNQT], s_qedg[kNQT], s_lcnt[kNQT];
  BfsCtl* ctl = P.ctl;
  const int64_t gtid = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const int64_t gsz = (int64_t)gridDim.x * BLOCK;
  const int32_t root = P.perm ? P.perm[P.root_orig] : P.root_orig;
  const bool root_in = root < P.n_sweep;
  const int64_t W = ceil_div(P.n_sweep, kWave);
  const uint64_t emask = (1ull << P.eb) - 1ull;
  int fs = 0;  // coarse summary: vertices per bit = 2^fs
  while ((((P.n_sweep - 1) >> fs) + 1) > kFiltBits) ++fs;
  const int l = lane_id();
  if (threadIdx.x < WAVES) {
    s_st.cnt[threadIdx.x] = 0;
    s_st.lcnt[threadIdx.x] = 0;
  }
  const int64_t dr = root_in ? P.off[root + 1] - P.off[root] : 0;

  if (threadIdx.x < kNQT) {  // F_0 = {root} sits in sub-queue 0
    s_qcnt[threadIdx.x] = (threadIdx.x == 0 && root_in) ? 1 : 0;
    s_qedg[threadIdx.x] = (threadIdx.x == 0) ? dr : 0;
    s_lcnt[threadIdx.x] = 0;
  }

  // ---- initialisation
  if (P.init) {
    for (int64_t i = gtid; i < P.n_sweep; i += gsz)
      P.dp[i] = (i == root) ? pack_dp(P.base, root) : kUnreached;
  }
  for (int64_t w = gtid; w < W; w += gsz) {
    P.vis[w] = 0ull;
    P.front[0][w] = (root_in && w == (root >> 6)) ? (1ull << (root & 63)) : 0ull;
    P.front[1][w] = 0ull;
  }
  if (gtid == 0) {
    if (!P.init && root_in) P.dp[root] = pack_dp(P.base, root);
    for (int r = 0; r < 2; ++r) {
      for (int q = 0; q < kNQT; ++q) {
        ctl->qpack[r][q][0] = 0ull;
        ctl->vlcnt[r][q][0] = 0ull;
      }
      ctl->edges[r][0] = 0ull;
    }
    ctl->hdir[0] = 0;
    ctl->hood[0] = 0;
    ctl->hnf[0] = 1;
    ctl->hmf[0] = dr;
    ctl->hmu[0] = P.deg_total - dr;
    ctl->hts[0] = (unsigned long long)wall_clock64();
    // the root's component [lo, hi): nothing outside it can be reached, so
    // the bottom-up sweep skips it (small components would otherwise be
    // rescanned in full at every bottom-up level)
    int64_t clo = 0, chi = P.n_sweep;
    if (P.comp_bounds && root_in) {
      int64_t a = 0, b = P.n_comp;  // last j with bounds[j] <= root
      while (b - a > 1) {
        const int64_t mid = (a + b) >> 1;
        if (P.comp_bounds[mid] <= root) a = mid; else b = mid;
      }
      clo = P.comp_bounds[a];
      chi = P.comp_bounds[a + 1];
    }
    ctl->sweep_lo = (int)clo;
    ctl->sweep_hi = (int)chi;
    if (root_in) {
      P.qv[0][0] = root;
      P.qe[0][0] = 0;
      mark_chunks(P.chunk[0], P.chunk_cap, 0, dr, 0, P.cshift);
    }
  }
  if (threadIdx.x == 0)
    for (int r = 0; r < 3; ++r) P.wctr[r * P.wstride + blockIdx.x * 16] = 0ull;
  __syncthreads();
  if (!grid_sync(&ctl->bar, P.timeout_ticks)) return;

  // bottom-up word range: the words of the root's component
  const int sweep_lo = __hip_atomic_load(&ctl->sweep_lo, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
  const int sweep_hi = __hip_atomic_load(&ctl->sweep_hi, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
  const int64_t kw_lo = sweep_lo >> 6, kw_hi = ceil_div(sweep_hi, kWave);

  // level state, identical in every workgroup
  int L = 0;
  int dir = 0;
  long long nf = root_in ? 1 : 0, mf = dr, mu = P.deg_total - dr;
  long long reached = 1, deg_reached = dr;
  // vertex list of the last bottom-up level: the sub-lists of vl[lsrc]
  // (s_lcnt entries each) hold the vertices of the root's component it left
  // unvisited, a superset of the unvisited ones (top-down levels only shrink
  // that set); -1 = none yet
  int lsrc = -1;
  while (nf > 0) {
    const int c3 = L % 3, n3 = (L + 1) % 3, z3 = (L + 2) % 3;
    const int qc = L & 1, qn = qc ^ 1;
    const uint64_t* fcur = P.front[c3];
    uint64_t* fnext = P.front[n3];
    unsigned long long* qpack = &ctl->qpack[n3][0][0];
    int64_t examined = 0;
    int64_t wg_td = 0;  // WGW, top-down: frontier edges of the chunks this workgroup took
    // clear what level L+1 will fill
    for (int64_t w = gtid; w < W; w += gsz) P.front[z3][w] = 0ull;
    if (gtid == 0) {
      for (int q = 0; q < kNQT; ++q) {
        ctl->qpack[z3][q][0] = 0ull;
        ctl->vlcnt[z3][q][0] = 0ull;
      }
      ctl->edges[z3][0] = 0ull;
    }
    if (threadIdx.x == 0) P.wctr[z3 * P.wstride + blockIdx.x * 16] = 0ull;
    if (dir == 0 && P.no_lb) {
      // ---- top-down without load balancing (Alg 1's split, one frontier
      // vertex per SIMD unit): frontier vertex j of the sub-queues taken one
      // after the other goes to wave j mod (grid waves), which walks its
      // whole row, 64 entries per step; a hub's row is not split further
      fold_frontier(P, qc, nf, fcur, W, gtid, gsz, s_qcnt);
      const int64_t nwaves = gsz / kWave;
      int64_t mine = 0;
      for (int64_t j = gtid / kWave; j < nf; j += nwaves) {
        int q = 0;
        int64_t i = j;
        while (i >= s_qcnt[q]) i -= s_qcnt[q++];
        const int32_t u = P.qv[qc][q * P.qcap + i];
        const int64_t rb = P.off[u], re = P.off[u + 1];
        for (int64_t e0 = rb; e0 < re; e0 += kWave) {
          const bool act = e0 + l < re;
          const int32_t w = act ? P.cols[e0 + l] : 0;
          bool claim = false;
          int64_t dw = 0;
          if (act && !(((P.vis[w >> 6] | fcur[w >> 6]) >> (w & 63)) & 1ull)) {
            const uint64_t prop = pack_dp(P.base + (uint32_t)(L + 1), u);
            // a claim: the word held was not written by this search
            if (P.dp[w] > prop)
              claim = (uint32_t)(atomicMin((unsigned long long*)&P.dp[w],
                                           (unsigned long long)prop) >> 32) >
                      P.base + (uint32_t)(L + 1);
            if (claim) {
              dw = P.off[w + 1] - P.off[w];
              atomicOr((unsigned long long*)&fnext[w >> 6], 1ull << (w & 63));
            }
          }
          stage(s_st, claim, w, dw, P, qn, qpack);
          mine += act ? 1 : 0;
        }
      }
      flush_stage(s_st, P, qn, qpack);
      if (WGW) wg_td = block_sum(mine);
      if (gtid == 0) examined = mf;
    } else if (dir == 0) {
      // ---- top-down
      fold_frontier(P, qc, nf, fcur, W, gtid, gsz, s_qcnt);
      // the chunks of the sub-queues, one after the other, taken from the
      // last: the vertices a row reaches are appended in ascending label
      // order (rows are expanded in ascending order), so this way higher
      // labels, whose proposals win, tend to propose first, and the pre-check
      // of the packed word drops more of the later proposals before their
      // atomic
      int64_t nchunks = 0;
      for (int q = 0; q < kNQT; ++q) nchunks += ceil_div(s_qedg[q], (int64_t)1 << P.cshift);
      for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        int q = 0;
        int64_t lc = nchunks - 1 - c, nq_ch = ceil_div(s_qedg[0], (int64_t)1 << P.cshift);
        while (lc >= nq_ch) {
          lc -= nq_ch;
          ++q;
          nq_ch = ceil_div(s_qedg[q], (int64_t)1 << P.cshift);
        }
        if (WGW && threadIdx.x == 0) {
          const int64_t e0 = lc << P.cshift;
          wg_td += std::min<int64_t>((int64_t)1 << P.cshift, s_qedg[q] - e0);
        }
        const bool ok = expand_chunk_batch<BLOCK, kTdK>(
            s_step.chunk, lc, s_qedg[q], P.qv[qc] + q * P.qcap, P.qe[qc] + q * P.qcap,
            s_qcnt[q], P.chunk[qc] + q * P.chunk_cap, nq_ch, P.off, P.cols, P.cshift,
            [&](const bool* act, const int32_t* u, const int32_t* w) {
          // w is a candidate if unvisited at level start; it then proposes
          // (L+1, u).  The smallest word stays, so the parent is the largest
          // label; only the first proposal finds w unreached and claims it.
          // A stale read of the word can only be larger than the stored one.
          uint64_t word[kTdK], cur[kTdK];
          bool cand[kTdK], claim[kTdK];
          int64_t dw[kTdK];
#pragma unroll
          for (int r = 0; r < kTdK; ++r)
            word[r] = act[r] ? (P.vis[w[r] >> 6] | fcur[w[r] >> 6]) : ~0ull;
#pragma unroll
          for (int r = 0; r < kTdK; ++r) {
            cand[r] = !((word[r] >> (w[r] & 63)) & 1ull);
            cur[r] = cand[r] ? P.dp[w[r]] : 0ull;
          }
#pragma unroll
          for (int r = 0; r < kTdK; ++r) {
            const uint64_t prop = pack_dp(P.base + (uint32_t)(L + 1), u[r]);
            claim[r] = false;
            // a claim: the word held was not written by this search
            if (cand[r] && cur[r] > prop)
              claim[r] = (uint32_t)(atomicMin((unsigned long long*)&P.dp[w[r]],
                                              (unsigned long long)prop) >> 32) >
                         P.base + (uint32_t)(L + 1);
          }
#pragma unroll
          for (int r = 0; r < kTdK; ++r) {
            dw[r] = 0;
            if (claim[r]) {
              dw[r] = P.off[w[r] + 1] - P.off[w[r]];
              atomicOr((unsigned long long*)&fnext[w[r] >> 6], 1ull << (w[r] & 63));
            }
          }
#pragma unroll
          for (int r = 0; r < kTdK; ++r) stage(s_st, claim[r], w[r], dw[r], P, qn, qpack);
        });
        if (!ok) {
          if (threadIdx.x == 0) atomicOr(&ctl->bar.status, kStatusBadInput);
          break;
        }
      }
      flush_stage(s_st, P, qn, qpack);
      if (gtid == 0) examined = mf;
    } else {
      // ---- bottom-up.  The first bottom-up level sweeps the component's
      // words in edge-balanced ranges; later ones walk only the vertex list
      // the previous one left (the paper's shrinking of the bottom-up
      // ranges), in ranges of kListRange vertices.  Rows are scanned with
      // lane refill.  The vertices a level leaves unvisited form the next
      // list.
      const bool listed = lsrc >= 0;
      const int32_t* vl_in = listed ? P.vl[lsrc] : nullptr;
      int32_t* vl_out = P.vl[listed ? (lsrc ^ 1) : 0];
      unsigned long long* vlcnt = &ctl->vlcnt[n3][0][0];
      // fold F_d into vis here: the list walk visits no words
      if (listed) fold_frontier(P, qc, nf, fcur, W, gtid, gsz, s_qcnt);
      // a sparse frontier: each workgroup builds the coarse summary of F_d
      // from the frontier queue, so that most row entries skip their probe
      const bool use_filt = (nf << fs) <= P.n_sweep;
      if (use_filt) {
        uint32_t* f = s_step.filt;
        for (int i = threadIdx.x; i < StepLds<BLOCK>::kFiltWords; i += BLOCK) f[i] = 0u;
        __syncthreads();
        for (int q = 0; q < kNQT; ++q) {
          const int32_t* qv = P.qv[qc] + q * P.qcap;
          for (int64_t i = threadIdx.x; i < s_qcnt[q]; i += BLOCK) {
            const uint32_t k = (uint32_t)qv[i] >> fs;
            atomicOr(&f[k >> 5], 1u << (k & 31));
          }
        }
        __syncthreads();
      }
      // a dense frontier: the exact bits of the highest labels (the hubs
      // after RCM, which most rows meet first) go to LDS for the probes
      uint32_t hi0 = 0xFFFFFFFFu;
      if (!use_filt) {
        constexpr int64_t kBits = (int64_t)StepLds<BLOCK>::kFiltWords * 32;
        const int64_t lo = P.n_sweep > kBits ? ((P.n_sweep - kBits + 63) & ~(int64_t)63) : 0;
        hi0 = (uint32_t)lo;
        const uint32_t* src = (const uint32_t*)fcur + (lo >> 5);
        const int nw = (int)((P.n_sweep - lo + 31) >> 5);
        for (int i = threadIdx.x; i < nw; i += BLOCK) s_step.filt[i] = src[i];
        __syncthreads();
      }
      int64_t nranges = P.n_part;
      if (listed) {
        nranges = 0;
        for (int q = 0; q < kNQT; ++q) nranges += ceil_div(s_lcnt[q], kListRange);
      }
      const int wv = wave_id();
      RangeCursor cur;
      for (;;) {
        const int64_t part = next_range(P.wctr + c3 * P.wstride, nranges, cur, !P.no_lb);
        if (part < 0) break;
        if (listed) {
          // range `part` of the sub-lists, one after the other
          int q = 0;
          int64_t lr = part, nq_r = ceil_div(s_lcnt[0], kListRange);
          while (lr >= nq_r) {
            lr -= nq_r;
            ++q;
            nq_r = ceil_div(s_lcnt[q], kListRange);
          }
          const int64_t i0 = q * P.qcap + lr * kListRange;
          const int total = (int)std::min<int64_t>(kListRange, s_lcnt[q] - lr * kListRange);
          refill_scan(
              total, P.off, P.cols, use_filt ? nullptr : P.top, fcur, s_step.filt, use_filt, fs,
              hi0, P.lane_row, examined,
              [&](int t) -> int64_t {
                if (t < 0) return -1;
                const int32_t u = vl_in[i0 + t];
                // reached since the list was made (by a top-down level)
                const uint64_t word = P.vis[u >> 6] | fcur[u >> 6];
                return ((word >> (u & 63)) & 1ull) ? -1 : (int64_t)u;
              },
              [&](bool fin, bool found, int64_t v, int32_t par, int64_t deg) {
                if (found) P.dp[v] = pack_dp(P.base + (uint32_t)(L + 1), par);
                wave_set_bits64(fnext, found, v);
                stage(s_st, found, (int32_t)v, deg, P, qn, qpack);
                stage_list(s_st, fin && !found, (int32_t)v, vl_out, vlcnt, P.qcap, P.n_sweep,
                           ctl);
              });
          continue;
        }
        // edge-balanced ranges, or without load balancing equal word counts
        const int64_t k0 = std::max<int64_t>(
            P.no_lb ? W * part / nranges : (int64_t)P.bu_part[part], kw_lo);
        const int64_t k1 = std::min<int64_t>(
            P.no_lb ? W * (part + 1) / nranges : (int64_t)P.bu_part[part + 1], kw_hi);
        // batches of 64 words: lane j loads word j (coalesced); the
        // unvisited vertices of the batch are handed to the lanes in order
        for (int64_t kb = k0; kb < k1; kb += kWave) {
          const int64_t kw = kb + l;
          uint64_t um = 0;
          if (kw < k1) {
            const uint64_t vk = P.vis[kw], fk = fcur[kw];
            P.vis[kw] = vk | fk;
            const int64_t v0 = kw * kWave;
            // vertices of this word inside [sweep_lo, sweep_hi)
            const uint64_t below = (v0 + kWave <= sweep_hi) ? ~0ull
                                   : ((1ull << (sweep_hi - v0)) - 1ull);
            const uint64_t above = (v0 >= sweep_lo) ? ~0ull : (~0ull << (sweep_lo - v0));
            um = ~(vk | fk) & below & above;
          }
          const int cnt = popc64(um);
          const int inc = (int)wave_inclusive_sum(cnt);
          const int total = shfl(inc, kWave - 1);
          s_st.found[wv][l] = 0ull;
          __builtin_amdgcn_wave_barrier();
          refill_scan(
              total, P.off, P.cols, use_filt ? nullptr : P.top, fcur, s_step.filt, use_filt, fs,
              hi0, P.lane_row, examined,
              [&](int t) -> int64_t {
                // the word holding the t-th unvisited vertex of the batch:
                // the first lane whose inclusive count exceeds t
                const int tt = t < 0 ? 0 : t;
                int jw = 0;
#pragma unroll
                for (int sft = 32; sft >= 1; sft >>= 1) {
                  const int probe = shfl(inc, jw + sft - 1);
                  if (probe <= tt) jw += sft;
                }
                const int excl = shfl(inc - cnt, jw);
                const uint64_t mj = shfl(um, jw);
                if (t < 0) return -1;
                return (kb + jw) * kWave + nth_set_bit64(mj, tt - excl);
              },
              [&](bool fin, bool found, int64_t v, int32_t par, int64_t deg) {
                if (found) {
                  atomicOr((unsigned long long*)&s_st.found[wv][(v >> 6) - kb],
                           1ull << (v & 63));
                  P.dp[v] = pack_dp(P.base + (uint32_t)(L + 1), par);
                }
                stage(s_st, found, (int32_t)v, deg, P, qn, qpack);
                stage_list(s_st, fin && !found, (int32_t)v, vl_out, vlcnt, P.qcap, P.n_sweep,
                           ctl);
              });
          __builtin_amdgcn_wave_barrier();
          const uint64_t fw = s_st.found[wv][l];
          if (kw < k1 && fw) fnext[kw] = fw;
        }
      }
      flush_list(s_st, vl_out, vlcnt, P.qcap, P.n_sweep, ctl);
      flush_stage(s_st, P, qn, qpack);
    }
    const int64_t wg_examined = block_fold_add(&ctl->edges[n3][0], examined);
    if (WGW && threadIdx.x == 0 && L < RBFS_STATS_MAX_LEVELS)
      P.wg_work[(int64_t)L * gridDim.x + blockIdx.x] = dir == 0 ? wg_td : wg_examined;
    if (!grid_sync(&ctl->bar, P.timeout_ticks)) return;

    // ---- next level: every workgroup decides the same way.  Sizes of the
    // next frontier's sub-queues (and of the new vertex list's sub-lists)
    if (threadIdx.x < kNQT) {
      const int q = threadIdx.x;
      const unsigned long long pk = __hip_atomic_load(&ctl->qpack[n3][q][0],
                                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      long long qc_n = (long long)(pk >> P.eb), qe_n = (long long)(pk & emask);
      if (q < kNQ && qc_n > P.qcap) {
        // the sub-queue overflowed: it holds its first qcap entries, whose
        // degree sum ends with the last one's
        const int64_t last = q * P.qcap + P.qcap - 1;
        const int32_t v = P.qv[qn][last];
        qc_n = P.qcap;
        qe_n = P.qe[qn][last] + (P.off[v + 1] - P.off[v]);
      }
      s_qcnt[q] = qc_n;
      s_qedg[q] = qe_n;
      if (dir == 1) {
        const long long lc_n = (long long)__hip_atomic_load(
            &ctl->vlcnt[n3][q][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_lcnt[q] = (q < kNQ && lc_n > P.qcap) ? P.qcap : lc_n;
      }
    }
    if constexpr (LRN) if (threadIdx.x < kWave) {
      // learned mode: wave 0, whose lanes wrote every sub-queue count, takes
      // the decision alone (the other waves read it after the barrier below).
      // Every workgroup evaluates the network on identical inputs with the
      // same fixed-order arithmetic, so all take the same decision.
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      long long nf_w = 0, mf_w = 0;
      for (int q = 0; q < kNQT; ++q) {
        nf_w += s_qcnt[q];
        mf_w += s_qedg[q];
      }
      const long long mu_w = mu - mf_w;
      float f[kMlpIn];
      switch_features(f, nf_w, mf_w, mu_w, P.n_sweep - (reached + nf_w), nf, L + 1, dir,
                      P.n_sweep, P.deg_total);
      int d = -1, fb = 0;  // fallback: 1 out of range, 2 predictions within the margin
      if (switch_ood(P.sw, f, L + 1)) {
        fb = 1;
      } else {
        float y0, y1;
        mlp_forward_wave<kMlpHid>(P.sw, P.sw + kOffW2, f, y0, y1, s_lrn.h);
        const float margin = P.sw[kOffMargin];
        d = (y0 - y1 >= margin) ? 1 : ((y1 - y0 >= margin) ? 0 : -1);
        if (d < 0) fb = 2;
      }
      if (fb) d = heuristic_dir(dir, nf_w, mf_w, mu_w, nf, P.n_sweep, P.alpha, P.beta);
      if (threadIdx.x == 0) {
        s_lrn.dec[0] = d;
        s_lrn.dec[1] = fb;
      }
    }
    __syncthreads();
    long long nf_new = 0, mf_new = 0;
    for (int q = 0; q < kNQT; ++q) {
      nf_new += s_qcnt[q];
      mf_new += s_qedg[q];
    }
    const long long mu_new = mu - mf_new;
    int nd = dir;
    int fallback = 0;  // learned mode: 1 out of range, 2 predictions within the margin
    switch (P.mode) {
      case RBFS_DIR_TD_ONLY: nd = 0; break;
      case RBFS_DIR_BU_ONLY: nd = 1; break;
      case RBFS_DIR_SCHEDULE: {
        int i = L + 1;
        if (i >= P.sched_len) i = P.sched_len - 1;
        nd = P.sched[i] ? 1 : 0;
        break;
      }
      case RBFS_DIR_LEARNED:
        if constexpr (LRN) {
          nd = s_lrn.dec[0];
          fallback = s_lrn.dec[1];
        }
        break;
      default:
        nd = heuristic_dir(dir, nf_new, mf_new, mu_new, nf, P.n_sweep, P.alpha, P.beta);
    }
    if (gtid == 0 && L < RBFS_STATS_MAX_LEVELS) {
      ctl->hedges[L] = (long long)ctl->edges[n3][0];
      ctl->hts[L + 1] = (unsigned long long)wall_clock64();
      if (L + 1 < RBFS_STATS_MAX_LEVELS && nf_new > 0) {
        ctl->hdir[L + 1] = (signed char)nd;
        ctl->hood[L + 1] = (signed char)fallback;
        ctl->hnf[L + 1] = nf_new;
        ctl->hmf[L + 1] = mf_new;
        ctl->hmu[L + 1] = mu_new;
      }
    }
    if (dir == 1) lsrc = (lsrc >= 0) ? (lsrc ^ 1) : 0;
    nf = nf_new;
    mf = mf_new;
    mu = mu_new;
    dir = nd;
    reached += nf_new;
    deg_reached += mf_new;
    ++L;
  }
  if (gtid == 0) {
    ctl->levels = root_in ? L : 1;
    ctl->reached = reached;
    ctl->deg_reached = deg_reached;
  }
}

// Outputs in internal labels (or of a graph that was not relabelled) from the
// packed pairs: output index v is the label itself.  Indices past the swept
// set are unreached, except an isolated root (perm_root: original -> internal
// of a relabelled graph).  With `reset`, reached pairs are set back to
// unreached, so the next search needs no initialisation pass (scattered
// 8-byte writes instead of one coalesced pass).
__global__ void output_kernel(int64_t n, const int32_t* perm_root, int64_t n_sweep, uint64_t* dp,
                              uint32_t base, int32_t* depth_o, int32_t* parent_o,
                              int32_t root_orig, int reset) {
  const int32_t root_out = perm_root ? perm_root[root_orig] : root_orig;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    int32_t d = -1, p = -1;
    if (v < n_sweep) {
      const uint64_t x = dp[v];
      if (reset && x != kUnreached) dp[v] = kUnreached;
      if (dp_current(x, base, n_sweep)) {
        d = (int32_t)((uint32_t)(x >> 32) - base);
        p = dp_parent(x);
      }
    } else if (v == root_out) {
      d = 0;
      p = root_out;
    }
    depth_o[v] = d;
    parent_o[v] = p;
  }
}

// ---- original-ID outputs of a relabelled graph in three coalesced passes.
// A random permutation of the 8-byte pairs costs one memory request per
// vertex as a gather (or scatter); this GPU serves such requests at about
// 50 G/s whatever the array size, so the vertices are moved in stages whose
// reads and writes are runs instead:
//   A: tile t of the swept labels (kOutTile of them, in label order) is
//      grouped in LDS by bucket (a range of 2^(kOutWin + as) original IDs)
//      and each group written as one run at its fixed place gA[a][t]
//      (unreached labels included, marked unreached);
//   B: each bucket's region is grouped the same way by window (2^kOutWin
//      original IDs), skipping unreached entries;
//   C: each window is assembled in LDS (unreached, then its entries) and
//      written out in original-ID order.
// Pass-A places come from the layout (counts of labels per tile and
// bucket), so no two workgroups contend for a counter; pass B reserves its
// runs in each window with one atomic per chunk and window.  Window w owns
// positions [wstart[w], wstart[w + 1]) of the pass-B arrays; cnt_w counts
// what a search put there, and pass C clears it for the next search.
constexpr int kOutWin = 13;                 // window: 8192 original IDs
constexpr int kOutWinSize = 1 << kOutWin;
constexpr int kOutThreads = 512;
constexpr int kOutPer = 8;                  // entries per thread and tile
constexpr int kOutTile = kOutThreads * kOutPer;
constexpr int kOutMaxKeys = 1024;           // buckets (A) or windows per bucket (B)

struct OutStage {
  uint64_t v[kOutTile];
  int32_t o[kOutTile];
  uint16_t key[kOutTile];
  int64_t start[kOutMaxKeys];  // where each key's run goes
  int32_t hist[kOutMaxKeys];
  int32_t scan[kOutMaxKeys];
};

// Groups a tile's entries by key in LDS and writes each key's group as one
// run at dest_of(key) + (reserved slot): every thread holds up to kOutPer
// entries (value, original ID, key, valid).
template <class DestOf, class Reserve>
__device__ __forceinline__ void out_group_write(OutStage& S, int nkeys, const uint64_t* v,
                                                const int32_t* o, const int* key,
                                                const bool* ok, uint64_t* dst_v,
                                                int32_t* dst_o, DestOf&& dest_of,
                                                Reserve&& reserve) {
  const int t = threadIdx.x;
  for (int k = t; k < nkeys; k += kOutThreads) S.hist[k] = 0;
  __syncthreads();
  int rank[kOutPer];
#pragma unroll
  for (int e = 0; e < kOutPer; ++e) rank[e] = ok[e] ? atomicAdd(&S.hist[key[e]], 1) : 0;
  __syncthreads();
  // exclusive scan of the counts (one wave per 64 keys, then the wave totals)
  if (t < kWave) {
    int64_t carry = 0;
    for (int k0 = 0; k0 < nkeys; k0 += kWave) {
      const int k = k0 + t;
      const int64_t c = k < nkeys ? S.hist[k] : 0;
      const int64_t inc = wave_inclusive_sum(c);
      if (k < nkeys) S.scan[k] = (int32_t)(carry + inc - c);
      carry += shfl(inc, kWave - 1);
    }
  }
  // each key's run start, read once per tile
  for (int k = t; k < nkeys; k += kOutThreads)
    if (S.hist[k] > 0) S.start[k] = dest_of(k) + reserve(k, S.hist[k]);
  __syncthreads();
  const int total = S.scan[nkeys - 1] + S.hist[nkeys - 1];
#pragma unroll
  for (int e = 0; e < kOutPer; ++e)
    if (ok[e]) {
      const int slot = S.scan[key[e]] + rank[e];
      S.v[slot] = v[e];
      S.o[slot] = o[e];
      S.key[slot] = (uint16_t)key[e];
    }
  __syncthreads();
  for (int k = t; k < total; k += kOutThreads) {
    const int kk = S.key[k];
    const int64_t d = S.start[kk] + (k - S.scan[kk]);
    dst_v[d] = S.v[k];
    dst_o[d] = S.o[k];
  }
  __syncthreads();
}

// Pass A: tile blockIdx.x of the swept labels, as (depth, parent's original
// ID) pairs, unreached ones marked.  With `reset`, every entry read is set
// to unreached (the next search then starts a new base with no
// initialisation pass).
__global__ __launch_bounds__(kOutThreads) void out_pass_a_kernel(
    int64_t n_sweep, int64_t ntiles, uint64_t* dp, uint32_t base, const int32_t* iperm, int as,
    int na, const int64_t* gA, uint64_t* av, int32_t* ao, int reset) {
  __shared__ OutStage S;
  const int64_t t0 = (int64_t)blockIdx.x * kOutTile;
  const int sh = kOutWin + as;
  uint64_t v[kOutPer];
  int32_t o[kOutPer];
  int key[kOutPer];
  bool ok[kOutPer];
#pragma unroll
  for (int e = 0; e < kOutPer; ++e) {
    const int64_t i = t0 + e * kOutThreads + threadIdx.x;
    ok[e] = i < n_sweep;
    v[e] = ok[e] ? dp[i] : kUnreached;
    o[e] = ok[e] ? iperm[i] : 0;
    if (reset && v[e] != kUnreached) dp[i] = kUnreached;
  }
#pragma unroll
  for (int e = 0; e < kOutPer; ++e) {
    key[e] = o[e] >> sh;
    v[e] = dp_current(v[e], base, n_sweep)
               ? pack_dp((uint32_t)(v[e] >> 32) - base, iperm[dp_parent(v[e])])
               : kUnreached;
  }
  out_group_write(
      S, na, v, o, key, ok, av, ao,
      [&](int a) { return gA[(int64_t)blockIdx.x * na + a]; },
      [&](int, int) { return 0; });
}

// Pass B: chunk c of bucket a (chunks: kOutTile entries of a bucket's
// region; chunk_start[a] = first chunk of bucket a) grouped by window.
__global__ __launch_bounds__(kOutThreads) void out_pass_b_kernel(
    int64_t nwin, int as, int na, const int64_t* wstart, const int32_t* chunk_start,
    const uint64_t* av, const int32_t* ao, int32_t* cnt_w, uint64_t* bv, int32_t* bo) {
  __shared__ OutStage S;
  // bucket of this chunk: the last a with chunk_start[a] <= blockIdx.x
  int a = 0, b = na;
  while (b - a > 1) {
    const int m = (a + b) >> 1;
    if (chunk_start[m] <= (int)blockIdx.x) a = m; else b = m;
  }
  const int64_t w0 = (int64_t)a << as;
  const int64_t c = (int64_t)blockIdx.x - chunk_start[a];
  const int64_t r0 = wstart[w0] + c * kOutTile;
  const int64_t r1 = std::min<int64_t>(r0 + kOutTile, wstart[std::min(w0 + (1 << as), nwin)]);
  uint64_t v[kOutPer];
  int32_t o[kOutPer];
  int key[kOutPer];
  bool ok[kOutPer];
#pragma unroll
  for (int e = 0; e < kOutPer; ++e) {
    const int64_t k = r0 + e * kOutThreads + threadIdx.x;
    v[e] = k < r1 ? av[k] : kUnreached;
    o[e] = k < r1 ? ao[k] : 0;
    ok[e] = v[e] != kUnreached;
    key[e] = (int)((o[e] >> kOutWin) - w0);
  }
  out_group_write(
      S, 1 << as, v, o, key, ok, bv, bo, [&](int w) { return wstart[w0 + w]; },
      [&](int w, int cnt) { return atomicAdd(&cnt_w[w0 + w], cnt); });
}

// Pass C: window w assembled in LDS and written in original-ID order; an
// isolated root gets depth 0 and itself as parent.  Clears the counters.
__global__ __launch_bounds__(kOutThreads) void out_pass_c_kernel(
    int64_t n, const int64_t* wstart, int32_t* cnt_w, const uint64_t* bv,
    const int32_t* bo, const int32_t* perm, int64_t n_sweep, int32_t root_orig,
    int32_t* depth_o, int32_t* parent_o) {
  __shared__ int32_t s_d[kOutWinSize], s_p[kOutWinSize];
  const int64_t w = blockIdx.x;
  const int64_t v0 = w << kOutWin;
  const int len = (int)std::min<int64_t>(kOutWinSize, n - v0);
  const int64_t rr = perm[root_orig] >= n_sweep ? root_orig - v0 : -1;
  for (int t = threadIdx.x; t < len; t += kOutThreads) {
    s_d[t] = t == rr ? 0 : -1;
    s_p[t] = t == rr ? root_orig : -1;
  }
  const int64_t k0 = wstart[w], k1 = k0 + cnt_w[w];
  __syncthreads();
  for (int64_t k = k0 + threadIdx.x; k < k1; k += kOutThreads) {
    const uint64_t x = bv[k];
    const int t = (int)(bo[k] - v0);
    s_d[t] = (int32_t)(x >> 32);
    s_p[t] = dp_parent(x);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < len; t += kOutThreads) {
    depth_o[v0 + t] = s_d[t];
    parent_o[v0 + t] = s_p[t];
  }
  if (threadIdx.x == 0) cnt_w[w] = 0;
}

// Layout of the three passes: swept labels per window, and per bucket and
// pass-A tile (bucket-major, for the scan that places the runs).
// Run places per (bucket, tile), bucket-major, to tile-major: a pass-A tile
// then reads its bucket places from one contiguous block.
__global__ void out_transpose_kernel(int64_t na, int64_t ntiles, const int64_t* in, int64_t* out) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < na * ntiles;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = j / na, a = j - t * na;
    out[j] = in[a * ntiles + t];
  }
}

__global__ void out_hist_kernel(int64_t n_sweep, const int32_t* iperm, int as, int64_t ntiles,
                                int32_t* hist_w, int32_t* hist_at) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_sweep;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t w = iperm[i] >> kOutWin;
    atomicAdd(&hist_w[w], 1);
    atomicAdd(&hist_at[(int64_t)(w >> as) * ntiles + i / kOutTile], 1);
  }
}

// Clears the barrier and status of the previous search; its status is kept
// in `sticky` until rbfs_graph_check reads it.
__global__ void reset_ctl_kernel(BfsCtl* c) {
  if (threadIdx.x == 0) c->sticky |= c->bar.status;
  __syncthreads();
  int* p = (int*)&c->bar;
  for (int i = threadIdx.x; i < (int)(sizeof(GridBarrier) / sizeof(int)); i += blockDim.x)
    p[i] = 0;
}

// top[v] = the largest label among v's neighbours (the row's last entry,
// rows being ascending); 0 for an empty row, which is never probed.
__global__ void top_kernel(const int64_t* off, const int32_t* cols, int64_t n, int32_t* top) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = off[v + 1];
    top[v] = e > off[v] ? cols[e - 1] : 0;
  }
}

__global__ void clear_status_kernel(BfsCtl* c) {
  if (threadIdx.x == 0) {
    c->sticky = 0;
    c->bar.status = 0;
  }
}

}  // namespace

int bfs_wg_work(Graph* g, int64_t* out, int64_t cap, int32_t* levels, int32_t* grid,
                hipStream_t stream) {
  BfsWork* w = g->bfs;
  if (!w || !w->wg_valid) {
    set_error("rbfs_graph_wg_work: the last search was not made with RBFS_OPT_WG_WORK");
    return RBFS_E_STATE;
  }
  int lv = 0;
  hipError_t e = hipMemcpyAsync(&lv, &w->ctl->levels, sizeof(int), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    set_error(std::string("rbfs_graph_wg_work: ") + hipGetErrorString(e));
    return RBFS_E_DEVICE;
  }
  lv = std::max(0, std::min(lv, (int)RBFS_STATS_MAX_LEVELS));
  const int64_t need = (int64_t)lv * w->wg_grid;
  *levels = lv;
  *grid = w->wg_grid;
  if (out && cap > 0 && need > 0) {
    e = hipMemcpy(out, w->wg_work, sizeof(int64_t) * (size_t)std::min(cap, need),
                  hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      set_error(std::string("rbfs_graph_wg_work: ") + hipGetErrorString(e));
      return RBFS_E_DEVICE;
    }
  }
  return 0;
}

// Resident workgroups per CU that every instantiation of one block size
// allows (at least 1).
template <int BLOCK>
static hipError_t min_per_cu(int* out) {
  const void* ks[] = {(const void*)bfs_persistent_kernel<BLOCK, false, false>,
                      (const void*)bfs_persistent_kernel<BLOCK, true, false>,
                      (const void*)bfs_persistent_kernel<BLOCK, false, true>,
                      (const void*)bfs_persistent_kernel<BLOCK, true, true>};
  int m = 1 << 30;
  for (const void* k : ks) {
    int c = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&c, k, BLOCK, 0);
    if (e != hipSuccess) return e;
    m = std::min(m, c);
  }
  *out = std::max(m, 1);
  return hipSuccess;
}

template <int BLOCK>
static void launch_search(bool wgw, bool lrn, int grid, hipStream_t stream, const BfsParams& P) {
  if (wgw && lrn)
    hipLaunchKernelGGL((bfs_persistent_kernel<BLOCK, true, true>), dim3(grid), dim3(BLOCK), 0,
                       stream, P);
  else if (wgw)
    hipLaunchKernelGGL((bfs_persistent_kernel<BLOCK, true, false>), dim3(grid), dim3(BLOCK), 0,
                       stream, P);
  else if (lrn)
    hipLaunchKernelGGL((bfs_persistent_kernel<BLOCK, false, true>), dim3(grid), dim3(BLOCK), 0,
                       stream, P);
  else
    hipLaunchKernelGGL((bfs_persistent_kernel<BLOCK, false, false>), dim3(grid), dim3(BLOCK), 0,
                       stream, P);
}

void free_bfs_work(Graph* g) {
  BfsWork* w = g->bfs;
  if (!w) return;
  void* ps[] = {w->dp,       w->vis,      w->front,   w->qv[0], w->qv[1], w->qe[0], w->qe[1],
                w->chunk[0], w->chunk[1], w->bu_part, w->ctl,   w->wctr,  w->vl[0], w->vl[1],
                w->wg_work,  w->top,   w->owstart, w->ogA, w->ocnt_w, w->ochunk};
  for (void* p : ps)
    if (p) (void)rbfs::dev_free(p);
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
  BFS_CHECK(rbfs::dev_malloc(&w->dp, sizeof(uint64_t) * ns));
  BFS_CHECK(rbfs::dev_malloc(&w->vis, sizeof(uint64_t) * W));
  BFS_CHECK(rbfs::dev_malloc(&w->front, sizeof(uint64_t) * 3 * W));
  // kNQ sub-queues (sub-lists) of qcap entries each, then the overflow one
  // of ns: a level appends each vertex at most once, so nothing is lost
  w->qcap = g->queue_cap > 0 ? g->queue_cap : (ns + 3) / 4 + kStage;
  const int64_t qlen = kNQ * w->qcap + ns;
  for (int i = 0; i < 2; ++i) BFS_CHECK(rbfs::dev_malloc(&w->vl[i], sizeof(int32_t) * qlen));
  BFS_CHECK(rbfs::dev_malloc(&w->top, sizeof(int32_t) * ns));
  {
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(ns, kBlock), 1 << 16));
    hipLaunchKernelGGL(top_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, stream, g->off,
                       g->cols, g->n_sweep, w->top);
    BFS_CHECK(hipGetLastError());
  }
  for (int i = 0; i < 2; ++i) {
    BFS_CHECK(rbfs::dev_malloc(&w->qv[i], sizeof(int32_t) * qlen));
    BFS_CHECK(rbfs::dev_malloc(&w->qe[i], sizeof(int64_t) * qlen));
  }
  // chunk tables for the tuned chunk length (rebuilt if a shorter one is set)
  BFS_CHECK(rbfs::dev_malloc(&w->ctl, sizeof(BfsCtl)));
  BFS_CHECK(hipMemsetAsync(w->ctl, 0, sizeof(BfsCtl), stream));
  // residency of every instantiation: the grid must fit each
  BFS_CHECK(min_per_cu<1024>(&w->max_per_cu));
  BFS_CHECK(min_per_cu<256>(&w->max_per_cu_256));
  w->grid = g->compute_units;
  w->max_grid = 4 * g->compute_units;  // per_cu is at most 4
  BFS_CHECK(rbfs::dev_malloc(&w->wctr, sizeof(unsigned long long) * 3 * 16 * (size_t)w->max_grid));
  BFS_CHECK(hipEventCreate(&w->ev0));
  BFS_CHECK(hipEventCreate(&w->ev1));
  BFS_CHECK(hipEventCreate(&w->ev2));
  BFS_CHECK(hipStreamSynchronize(stream));
  w->clean = false;
  g->bytes += sizeof(uint64_t) * (size_t)ns + sizeof(int32_t) * (size_t)ns +
              (sizeof(int32_t) * 2 + sizeof(int32_t) * 2 + sizeof(int64_t) * 2) * (size_t)qlen +
              sizeof(uint64_t) * 4 * W;
  return 0;
}

// Layout of the three output passes of a relabelled graph: the swept labels
// per window of original IDs and the pass-B chunks per bucket.  Synchronises
// `stream`.
static int ensure_out_layout(Graph* g, hipStream_t stream) {
  BfsWork* w = g->bfs;
  if (w->owstart) return 0;
  const int64_t ns = g->n_sweep;
  const int64_t nwin = ceil_div(g->n > 0 ? g->n : 1, (int64_t)kOutWinSize);
  const int as = std::max(0, bits_for(nwin) - 8);
  const int na = (int)ceil_div(nwin, (int64_t)1 << as);
  const int64_t ntiles = ceil_div(ns, (int64_t)kOutTile);
  const int64_t nat = (int64_t)na * ntiles;
  int32_t *hist_w = nullptr, *hist_at = nullptr;
  auto fail = [&](hipError_t e) {
    (void)hipStreamSynchronize(stream);
    if (hist_w) rbfs::dev_free(hist_w);
    if (hist_at) rbfs::dev_free(hist_at);
    for (void** q : {(void**)&w->owstart, (void**)&w->ogA, (void**)&w->ocnt_w, (void**)&w->ochunk})
      if (*q) {
        rbfs::dev_free(*q);
        *q = nullptr;
      }
    set_error(std::string("bfs: output layout: ") + hipGetErrorString(e));
    return RBFS_E_DEVICE;
  };
  hipError_t e = hipSuccess;
  if ((e = rbfs::dev_malloc(&w->owstart, sizeof(int64_t) * (size_t)(nwin + 1))) != hipSuccess)
    return fail(e);
  if ((e = rbfs::dev_malloc(&w->ogA, sizeof(int64_t) * (size_t)(nat + 1))) != hipSuccess)
    return fail(e);
  if ((e = rbfs::dev_malloc(&w->ocnt_w, sizeof(int32_t) * (size_t)nwin)) != hipSuccess)
    return fail(e);
  if ((e = rbfs::dev_malloc(&w->ochunk, sizeof(int32_t) * (size_t)(na + 1))) != hipSuccess)
    return fail(e);
  if ((e = rbfs::dev_malloc(&hist_w, sizeof(int32_t) * (size_t)nwin)) != hipSuccess)
    return fail(e);
  if ((e = rbfs::dev_malloc(&hist_at, sizeof(int32_t) * (size_t)std::max<int64_t>(nat, 1))) !=
      hipSuccess)
    return fail(e);
  if ((e = hipMemsetAsync(hist_w, 0, sizeof(int32_t) * (size_t)nwin, stream)) != hipSuccess ||
      (e = hipMemsetAsync(hist_at, 0, sizeof(int32_t) * (size_t)std::max<int64_t>(nat, 1),
                          stream)) != hipSuccess ||
      (e = hipMemsetAsync(w->ocnt_w, 0, sizeof(int32_t) * (size_t)nwin, stream)) != hipSuccess)
    return fail(e);
  if (ns > 0) {
    const unsigned blocks =
        (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(ns, kBlock), 1 << 16));
    hipLaunchKernelGGL(out_hist_kernel, dim3(blocks), dim3(kBlock), 0, stream, ns, g->iperm, as,
                       ntiles, hist_w, hist_at);
    if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  }
  // (the second scan may regrow the scratch the first one uses: wait between)
  {
    int64_t* tmp = nullptr;
    if ((e = rbfs::dev_malloc(&tmp, sizeof(int64_t) * (size_t)(nat + 1))) != hipSuccess)
      return fail(e);
    if ((e = scan_exclusive_i32(hist_w, w->owstart, nwin, g->scratch, stream)) == hipSuccess &&
        (e = hipStreamSynchronize(stream)) == hipSuccess &&
        (e = scan_exclusive_i32(hist_at, tmp, nat, g->scratch, stream)) == hipSuccess && nat > 0) {
      const unsigned blocks =
          (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(nat, kBlock), 1 << 16));
      hipLaunchKernelGGL(out_transpose_kernel, dim3(blocks), dim3(kBlock), 0, stream,
                         (int64_t)na, ntiles, tmp, w->ogA);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    rbfs::dev_free(tmp);
    if (e != hipSuccess) return fail(e);
  }
  std::vector<int64_t> ws((size_t)nwin + 1);
  if ((e = hipMemcpyAsync(ws.data(), w->owstart, sizeof(int64_t) * ws.size(),
                          hipMemcpyDeviceToHost, stream)) != hipSuccess ||
      (e = hipStreamSynchronize(stream)) != hipSuccess)
    return fail(e);
  std::vector<int32_t> chunk((size_t)na + 1);
  int64_t nc = 0;
  for (int a = 0; a < na; ++a) {
    chunk[a] = (int32_t)nc;
    const int64_t cap = ws[std::min<int64_t>((int64_t)(a + 1) << as, nwin)] - ws[(int64_t)a << as];
    nc += ceil_div(cap, (int64_t)kOutTile);
  }
  chunk[na] = (int32_t)nc;
  if ((e = hipMemcpyAsync(w->ochunk, chunk.data(), sizeof(int32_t) * chunk.size(),
                          hipMemcpyHostToDevice, stream)) != hipSuccess ||
      (e = hipStreamSynchronize(stream)) != hipSuccess)
    return fail(e);
  rbfs::dev_free(hist_w);
  rbfs::dev_free(hist_at);
  w->onwin = nwin;
  w->ona = na;
  w->oas = as;
  w->ontiles = ntiles;
  w->onchunk = (int)nc;
  g->bytes += sizeof(int64_t) * (size_t)(nwin + nat + 2) + sizeof(int32_t) * (size_t)(nwin + na + 1);
  return 0;
}

// Launch shape of the graph's single-root tuning, clamped to residency.
static void tuned_shape(const Graph* g, const BfsWork* w, int* block, int* grid) {
  const rbfs_tuning_t& t = g->tune_single;
  *block = t.block == 256 ? 256 : 1024;
  const int cap = *block == 256 ? w->max_per_cu_256 : w->max_per_cu;
  const int per = std::max(1, std::min(t.per_cu, cap));
  *grid = per * g->compute_units;
}

// (Re)builds the bottom-up ranges for the graph's tuning: bu_grain ranges
// per workgroup of the tuned grid.  Synchronises `stream` when it builds.
static int ensure_bfs_parts(Graph* g, hipStream_t stream) {
  BfsWork* w = g->bfs;
  // chunk tables for chunks of the tuned length: nnz / td_chunk + 2 entries
  // per sub-queue
  const int cs = bits_for(g->tune_single.td_chunk);
  if (!w->chunk[0] || cs < w->chunk_shift) {
    for (int i = 0; i < 2; ++i) {
      if (w->chunk[i]) (void)rbfs::dev_free(w->chunk[i]);
      w->chunk[i] = nullptr;
    }
    w->chunk_cap = ceil_div(g->nnz, (int64_t)1 << cs) + 2;
    for (int i = 0; i < 2; ++i)
      BFS_CHECK(rbfs::dev_malloc(&w->chunk[i], sizeof(int32_t) * kNQT * w->chunk_cap));
    w->chunk_shift = cs;
  }
  int block, grid;
  tuned_shape(g, w, &block, &grid);
  const int grain = g->tune_single.bu_grain;
  if (w->bu_part && w->part_grain == grain && w->part_grid == grid) return 0;
  if (w->bu_part) (void)rbfs::dev_free(w->bu_part);
  w->bu_part = nullptr;
  w->n_part = 0;
  int rc = build_edge_ranges(g->off, g->n_sweep, g->nnz, (int64_t)grain * grid, kWave,
                             &w->bu_part, &w->n_part, stream);
  if (rc) return rc;
  w->part_grain = grain;
  w->part_grid = grid;
  return 0;
}

int bfs_apply_tuning(Graph* g, hipStream_t stream) {
  if (!g->bfs) return 0;  // applied when the workspace is made
  return ensure_bfs_parts(g, stream);
}

int bfs_impl(Graph* g, int32_t root, int32_t* depth, int32_t* parent, int mode, int alpha,
             int beta, const int8_t* sched, int sched_len, int out_space, int flags,
             int tune_profile, hipStream_t stream, void* stats_v) {
  rbfs_stats_t* stats = (rbfs_stats_t*)stats_v;
  int rc = ensure_bfs_work(g, stream);
  if (!rc) rc = ensure_bfs_parts(g, stream);
  if (rc) return rc;
  BfsWork* w = g->bfs;
  const rbfs_tuning_t& tun = g->tune_single;
  const bool translate = g->reordered && out_space == RBFS_OUT_ORIGINAL;
  if (translate && (rc = ensure_out_layout(g, stream)) != 0) return rc;
  const int bits_n = bits_for(g->n_sweep + 2);
  const int eb = 64 - bits_n;
  if (((uint64_t)g->nnz >> eb) != 0) {
    set_error("bfs: graph too large for the packed queue counter");
    return RBFS_E_UNSUPPORTED;
  }
  BfsParams P{};
  P.off = g->off;
  P.cols = g->cols;
  P.perm = g->reordered ? g->perm : nullptr;
  P.n_sweep = g->n_sweep;
  P.deg_total = g->nnz;
  P.dp = w->dp;
  P.comp_bounds = g->reordered ? g->comp_bounds : nullptr;
  P.n_comp = g->n_comp;
  // the depth-field base: lowered by at least n_sweep + 1 per search, so that
  // every word an earlier search left compares above this one's; a new run
  // of bases starts from the top after a full initialisation, or when the
  // last output pass left every word unreached.  The step is at least 2^26,
  // so a run is at most 64 searches long whatever the graph.
  {
    const uint64_t step = std::max<uint64_t>((uint64_t)g->n_sweep + 1, 1ull << 26);
    const uint32_t top = (uint32_t)(0xFFFFFFFFull - step);
    if (w->clean) {
      P.init = 0;
      P.base = top;
    } else if (w->base_valid && (uint64_t)w->base >= step) {
      P.init = 0;
      P.base = (uint32_t)(w->base - step);
    } else {
      P.init = 1;
      P.base = top;
    }
    w->base = P.base;
    w->base_valid = true;
  }
  const int64_t W = ceil_div(g->n_sweep > 0 ? g->n_sweep : 1, kWave);
  P.vis = w->vis;
  for (int i = 0; i < 3; ++i) P.front[i] = w->front + (size_t)i * W;
  for (int i = 0; i < 2; ++i) {
    P.qv[i] = w->qv[i];
    P.qe[i] = w->qe[i];
    P.chunk[i] = w->chunk[i];
  }
  P.chunk_cap = w->chunk_cap;
  P.qcap = w->qcap;
  P.bu_part = w->bu_part;
  P.n_part = w->n_part;
  P.wctr = w->wctr;
  P.wstride = 16 * (int64_t)w->max_grid;
  P.vl[0] = w->vl[0];
  P.vl[1] = w->vl[1];
  P.top = w->top;
  P.no_lb = (flags & RBFS_OPT_NO_BALANCE) ? 1 : 0;
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
  P.lane_row = tun.lane_row;
  P.cshift = bits_for(tun.td_chunk);
  P.timeout_ticks = (uint64_t)g->wall_rate_khz * 1000ull * 4ull;  // 4 s
  if (flags & RBFS_OPT_ZERO_WAIT) P.timeout_ticks = 0;
  P.ctl = w->ctl;
  if (mode == RBFS_DIR_LEARNED) {
    P.sw = switch_blob_device(g->device);
    if (!P.sw) {
      set_error("bfs: learned direction needs weights (rbfs_switch_load)");
      return RBFS_E_STATE;
    }
  }

  if (flags & RBFS_OPT_WG_WORK) {
    if (!w->wg_work)
      BFS_CHECK(rbfs::dev_malloc(&w->wg_work, sizeof(int64_t) * RBFS_STATS_MAX_LEVELS *
                                                  (size_t)w->max_grid));
    P.wg_work = w->wg_work;
  }
  w->wg_valid = false;

  hipEvent_t* tev = nullptr;
  if (flags & RBFS_OPT_TIMING) BFS_CHECK(g->timing.next(&tev));
  if (tev) BFS_CHECK(hipEventRecord(tev[0], stream));
  BFS_CHECK(hipEventRecord(w->ev0, stream));
  hipLaunchKernelGGL(reset_ctl_kernel, dim3(1), dim3(256), 0, stream, w->ctl);
  BFS_CHECK(hipGetLastError());
  // launch shape: the graph's tuning, or a fixed profile (1..4: 256-thread
  // workgroups, that many per CU; 5, 6: 1024-thread, 1 or 2 per CU)
  int block, grid;
  tuned_shape(g, w, &block, &grid);
  if (tune_profile >= 1 && tune_profile <= 4) {
    block = 256;
    grid = std::min(tune_profile, w->max_per_cu_256) * g->compute_units;
  } else if (tune_profile == 5 || tune_profile == 6) {
    block = 1024;
    grid = std::min(tune_profile - 4, w->max_per_cu) * g->compute_units;
  }
  if (grid < 1 || grid > w->max_grid) {  // the range counters hold max_grid workgroups
    set_error("bfs: launch grid outside the workspace");
    return RBFS_E_STATE;
  }
  if (P.wg_work) {
    w->wg_grid = grid;
    w->wg_valid = true;
  }
  const bool lrn = mode == RBFS_DIR_LEARNED;
  if (block == 256)
    launch_search<256>(P.wg_work != nullptr, lrn, grid, stream, P);
  else
    launch_search<1024>(P.wg_work != nullptr, lrn, grid, stream, P);
  BFS_CHECK(hipGetLastError());
  BFS_CHECK(hipEventRecord(w->ev1, stream));
  if (tev) BFS_CHECK(hipEventRecord(tev[1], stream));
  if (translate) {
    if (w->ontiles > 0)
      hipLaunchKernelGGL(out_pass_a_kernel, dim3((unsigned)w->ontiles), dim3(kOutThreads), 0,
                         stream, g->n_sweep, w->ontiles, w->dp, P.base, g->iperm, w->oas, w->ona,
                         w->ogA, (uint64_t*)w->qe[0], w->qv[0], tun.reset ? 1 : 0);
    if (w->onchunk > 0)
      hipLaunchKernelGGL(out_pass_b_kernel, dim3((unsigned)w->onchunk), dim3(kOutThreads), 0,
                         stream, w->onwin, w->oas, w->ona, w->owstart, w->ochunk,
                         (const uint64_t*)w->qe[0], w->qv[0], w->ocnt_w, (uint64_t*)w->qe[1],
                         w->qv[1]);
    hipLaunchKernelGGL(out_pass_c_kernel, dim3((unsigned)w->onwin), dim3(kOutThreads), 0, stream,
                       g->n, w->owstart, w->ocnt_w, (const uint64_t*)w->qe[1], w->qv[1], g->perm,
                       g->n_sweep, root, depth, parent);
    BFS_CHECK(hipGetLastError());
  } else {
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(g->n, kBlock), 1 << 20));
    hipLaunchKernelGGL(output_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, stream, g->n,
                       g->reordered ? g->perm : nullptr, g->n_sweep, w->dp, P.base, depth, parent,
                       root, tun.reset ? 1 : 0);
    BFS_CHECK(hipGetLastError());
  }
  w->clean = tun.reset != 0;
  BFS_CHECK(hipEventRecord(w->ev2, stream));
  if (tev) BFS_CHECK(hipEventRecord(tev[2], stream));
  if (stats) {
    BfsCtl* h = new BfsCtl;
    hipError_t e = hipMemcpyAsync(h, w->ctl, sizeof(BfsCtl), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      delete h;
      BFS_CHECK(e);
    }
    memset(stats, 0, sizeof(*stats));
    stats->levels = h->levels;
    stats->status = h->bar.status;
    const int nl = std::min(h->levels, RBFS_STATS_MAX_LEVELS);
    for (int i = 0; i < nl; ++i) {
      stats->dir[i] = h->hdir[i];
      stats->fallback[i] = h->hood[i];
      stats->nf[i] = h->hnf[i];
      stats->mf[i] = h->hmf[i];
      stats->mu[i] = h->hmu[i];
      stats->edges[i] = h->hedges[i];
      stats->level_us[i] = (float)((double)(h->hts[i + 1] - h->hts[i]) * 1000.0 /
                                   (double)g->wall_rate_khz);
    }
    stats->reached = h->reached;
    stats->component_edges = h->deg_reached / 2;
    const int st = h->bar.status;
    delete h;
    BFS_CHECK(hipEventElapsedTime(&stats->ms_kernel, w->ev0, w->ev1));
    BFS_CHECK(hipEventElapsedTime(&stats->ms_total, w->ev0, w->ev2));
    if (st != 0) {
      w->clean = false;
      w->base_valid = false;  // the next search initialises every word
      set_error("bfs: device status " + std::to_string(st));
      return RBFS_E_DEVICE;
    }
  }
  return 0;
}

int bfs_check_status(Graph* g, hipStream_t stream) {
  if (!g->bfs) return 0;
  int st[2] = {0, 0};
  BFS_CHECK(hipMemcpyAsync(&st[0], &g->bfs->ctl->bar.status, sizeof(int),
                           hipMemcpyDeviceToHost, stream));
  BFS_CHECK(hipMemcpyAsync(&st[1], &g->bfs->ctl->sticky, sizeof(int), hipMemcpyDeviceToHost,
                           stream));
  BFS_CHECK(hipStreamSynchronize(stream));
  if ((st[0] | st[1]) != 0) {
    // reported once: the next check starts from a clear status
    hipLaunchKernelGGL(clear_status_kernel, dim3(1), dim3(64), 0, stream, g->bfs->ctl);
    BFS_CHECK(hipGetLastError());
    BFS_CHECK(hipStreamSynchronize(stream));
    g->bfs->clean = false;
    g->bfs->base_valid = false;
    set_error("bfs: device status " + std::to_string(st[0] | st[1]) +
              " raised by a search since the last check");
    return RBFS_E_DEVICE;
  }
  return 0;
}

}  // namespace rbfs
