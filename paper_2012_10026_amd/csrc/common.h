// Device helpers shared by the rbfs kernels: wave64 primitives, a grid
// barrier for persistent kernels, and the per-word edge walk used by
// several passes.  gfx950 (CDNA4): 64-lane wavefronts, 256 CUs in 8 XCDs.
#pragma once
#include <string.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rbfs {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
// grid of the grid-stride kernels that fold a shared counter once per wave
constexpr int kFoldBlocks = 2048;
constexpr uint32_t kNoParent = 0xFFFFFFFFu;

// status word bits (sticky, reported at the next synchronisation)
constexpr int kStatusTimeout = 1;
constexpr int kStatusOverflow = 2;
constexpr int kStatusBadInput = 4;

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }
__device__ __forceinline__ int wave_id() { return (int)(threadIdx.x / kWave); }

__device__ __forceinline__ uint64_t ballot(bool p) { return (uint64_t)__ballot((int)p); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }

// Position of the n-th set bit of m (0-based, n < popcount(m)).
__device__ __forceinline__ int nth_set_bit64(uint64_t m, int n) {
  int pos = 0;
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) {
    const uint64_t low = m & ((1ull << w) - 1ull);
    const int c = popc64(low);
    if (n >= c) {
      n -= c;
      m >>= w;
      pos += w;
    } else {
      m = low;
    }
  }
  return pos;
}

// index of the lowest set bit; x != 0
__device__ __forceinline__ int ffs64(uint64_t x) { return __ffsll((unsigned long long)x) - 1; }

template <class T>
__device__ __forceinline__ T shfl(T v, int src) {
  return __shfl(v, src, kWave);
}

// Inclusive prefix sum across the wave.
__device__ __forceinline__ int64_t wave_inclusive_sum(int64_t v) {
  const int l = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    int64_t t = __shfl_up(v, off, kWave);
    if (l >= off) v += t;
  }
  return v;
}

__device__ __forceinline__ int64_t wave_sum(int64_t v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ int64_t wave_max(int64_t v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const int64_t t = __shfl_xor(v, off, kWave);
    v = t > v ? t : v;
  }
  return v;
}

// Sums v over the workgroup and adds the total to *ctr with one atomic per
// workgroup: same-address atomics are served one after another (about
// 10 ns each), so one per wave of a full-GPU grid would cost tens of
// microseconds.  Returns the workgroup's total in thread 0 (0 elsewhere).
// Every thread of the workgroup must call it.
constexpr int kMaxWaves = 16;
__device__ __forceinline__ int64_t block_fold_add(unsigned long long* ctr, int64_t v) {
  __shared__ int64_t s_part[kMaxWaves];
  const int64_t w = wave_sum(v);
  if (lane_id() == 0) s_part[wave_id()] = w;
  __syncthreads();
  int64_t t = 0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) t += s_part[i];
    if (t)
      __hip_atomic_fetch_add(ctr, (unsigned long long)t, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  return t;
}

__device__ __forceinline__ uint64_t wave_or64(uint64_t x) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) x |= __shfl_xor(x, off, kWave);
  return x;
}

// Sets bit v of `words` for the lanes with take = true: one atomic per
// distinct word among them.  All lanes must call.
__device__ __forceinline__ void wave_set_bits64(uint64_t* words, bool take, int64_t v) {
  uint64_t pend = ballot(take);
  while (pend) {
    const int lead = ffs64(pend);
    const int64_t wl = shfl(v >> 6, lead);
    const bool mine = take && (v >> 6) == wl;
    const uint64_t bits = wave_or64(mine ? (1ull << (v & 63)) : 0ull);
    if (lane_id() == lead) atomicOr((unsigned long long*)&words[wl], bits);
    pend &= ~ballot(mine);
  }
}

__device__ __forceinline__ bool test_bit(const uint64_t* bits, uint32_t v) {
  return (bits[v >> 6] >> (v & 63)) & 1ull;
}

__device__ __forceinline__ uint64_t ld_relaxed(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_relaxed(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned ld_relaxed(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Grid barrier for a persistent kernel whose whole grid is resident.
//
// Arrival is counted in two stages: workgroups b with the same b mod 8 share
// a counter (each on its own 128-byte line, so arrivals proceed on eight
// addresses in parallel instead of serialising on one), and the last arrival
// of each group bumps the top counter; the last of those bumps the
// generation, which releases everyone.  The counters are never reset: no
// workgroup passes barrier k before every arrival at k has been counted, so
// each group counter advances by exactly its group size per barrier and the
// last arrival is the one that makes it a multiple of that size (the same
// for the top counter).  A reset would have to be ordered before the
// releasing increment at agent scope; without one, a fast workgroup's
// arrival at the next barrier could be wiped out by a late reset.  Each
// workgroup publishes its writes with one agent-scope release fence before
// arriving and takes one acquire fence after the release (polling itself is
// relaxed: an acquire per poll would invalidate the XCD's L2 while others
// still work).  A waiter gives up after `timeout_ticks` of the constant-rate
// wall clock, or as soon as the status word is non-zero, so the kernel always
// terminates; the status word then carries kStatusTimeout and the caller
// reports an error.  The counters start at zero for each launch.
struct GridBarrier {
  unsigned group[8][32];
  unsigned top;
  unsigned pad0[31];
  unsigned gen;
  unsigned pad1[31];
  int status;
  int pad2[31];
};

__device__ __forceinline__ bool grid_sync(GridBarrier* b, uint64_t timeout_ticks) {
  __shared__ bool s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned gen0 = __hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // publish this workgroup's writes
    const unsigned G = gridDim.x;
    const unsigned g = blockIdx.x & 7u;
    const unsigned ng = G < 8u ? G : 8u;
    const unsigned gsize = (G - g + 7u) / 8u;
    bool last = false;
    const unsigned old = __hip_atomic_fetch_add(&b->group[g][0], 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    if ((old + 1u) % gsize == 0u) {
      const unsigned o2 = __hip_atomic_fetch_add(&b->top, 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
      last = ((o2 + 1u) % ng == 0u);
    }
    if (last) {
      __hip_atomic_fetch_add(&b->gen, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const uint64_t t0 = wall_clock64();
      while (__hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen0) {
        if (__hip_atomic_load(&b->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
          break;
        if ((uint64_t)wall_clock64() - t0 > timeout_ticks) {
          __hip_atomic_fetch_or(&b->status, kStatusTimeout, __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ok = __hip_atomic_load(&b->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
  }
  __syncthreads();
  // the status as thread 0 read it, one read per workgroup
  return s_ok;
}

// ---------------------------------------------------------------------------
// Work ranges of one level, taken by whole waves.  The n ranges are cut into
// G regions (G = grid size); workgroup g owns region r(g) behind its own
// counter ctrs[16 * r] (one 128-byte line each), so only its own waves
// contend on it.  The 32 workgroups that share an XCD (workgroups are
// dispatched round-robin over the 8 XCDs) own adjacent regions, so an XCD
// works on one contiguous stretch of labels and its L2 sees their locality.
// A wave whose workgroup has drained its region steals: its lanes read up to
// 64 other counters per round trip, and it takes a range from a victim
// picked at random among those with at least two ranges left (the last one
// stays with its owner, so idle waves do not all queue on one counter).  It
// gives up after a few failed attempts; every range is still taken, since
// each workgroup drains its own region.  A counter is read before it is
// incremented, so a drained one costs a load and no atomic.

struct RangeCursor {
  int victim = -1;  // region stolen from last (-1: none)
  int fails = 0;    // failed steal attempts
  bool own_done = false;
};

__device__ __forceinline__ int region_of(int g, int G) {
  return (G % 8 == 0) ? (g % 8) * (G / 8) + g / 8 : g;
}

// Claims the next range of region r if at least min_left are left there.
// Only the value returned by this wave's own fetch-add is a claim.
__device__ __forceinline__ bool take_range(unsigned long long* ctrs, int64_t n, int G, int r,
                                           int64_t min_left, int64_t* out) {
  const int64_t lo = n * r / G, hi = n * (r + 1) / G;
  int64_t got = -1;
  if (lane_id() == 0) {
    unsigned long long* ctr = ctrs + (size_t)r * 16;
    const unsigned long long p =
        __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (hi - lo - (int64_t)p >= min_left) {
      const unsigned long long q =
          __hip_atomic_fetch_add(ctr, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (lo + (int64_t)q < hi) got = lo + (int64_t)q;
    }
  }
  got = shfl(got, 0);
  *out = got;
  return got >= 0;
}

// Next range for the calling wave (same value in every lane), or -1.
// steal = false: only the workgroup's own region (a static split).
__device__ __forceinline__ int64_t next_range(unsigned long long* ctrs, int64_t n,
                                              RangeCursor& c, bool steal = true) {
  constexpr int kMaxFails = 3;
  const int G = (int)gridDim.x;
  const int own = region_of((int)blockIdx.x, G);
  int64_t r;
  if (!c.own_done) {
    if (take_range(ctrs, n, G, own, 1, &r)) return r;
    c.own_done = true;
  }
  if (!steal) return -1;
  if (c.victim >= 0) {
    if (take_range(ctrs, n, G, c.victim, 2, &r)) return r;
    c.victim = -1;
  }
  const int l = lane_id();
  // per-wave pseudo-random choices
  uint32_t h = (uint32_t)(blockIdx.x * 64 + wave_id()) * 2654435761u + 0x9e3779b9u;
  while (c.fails < kMaxFails) {
    const int rounds = (G - 1 + kWave - 1) / kWave;
    int victim = -1;
    h = h * 1664525u + 1013904223u;
    for (int q = 0; q < rounds && victim < 0; ++q) {
      const int k = 1 + ((int)((h >> 8) % (uint32_t)rounds) + q) % rounds * kWave + l;
      bool cand = false;
      int v = 0;
      if (k < G) {
        v = (own + k) % G;
        const int64_t lo = n * v / G, hi = n * (v + 1) / G;
        const unsigned long long p = __hip_atomic_load(ctrs + (size_t)v * 16, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
        cand = hi - lo - (int64_t)p >= 2;
      }
      const uint64_t who = ballot(cand);
      if (who) {
        const int pick = nth_set_bit64(who, (int)((h >> 16) % (uint32_t)popc64(who)));
        victim = shfl(v, pick);
      }
    }
    if (victim < 0) return -1;  // nobody has ranges to spare
    if (take_range(ctrs, n, G, victim, 2, &r)) {
      c.victim = victim;
      return r;
    }
    ++c.fails;
  }
  return -1;
}

// The lanes with hub = true hold long rows cols[b, e); each is scanned by
// the whole wave, 64 entries per step, where the lowest hitting lane gives
// the first hit (in row order).  Sets found / par on the hub lanes; adds the
// entries read (up to and including the hit) to lane 0's `examined`.  All
// lanes must call.
// filt (LDS) holds, when use_filt, a coarse summary of bits, bit k set when
// any of the vertices [k << fs, (k + 1) << fs) is set, and entries it rules
// out skip the probe of bits; otherwise it holds the exact bits of the
// vertices from hi0 up (the highest labels), which are probed there.
__device__ __forceinline__ bool lds_bit(const uint32_t* filt, uint32_t k) {
  return (filt[k >> 5] >> (k & 31)) & 1u;
}

__device__ __forceinline__ bool probe_bit(const uint64_t* bits, const uint32_t* filt,
                                          bool use_filt, int fs, uint32_t hi0, uint32_t x) {
  if (x >= hi0) return lds_bit(filt, x - hi0);
  return (!use_filt || lds_bit(filt, x >> fs)) && test_bit(bits, x);
}

__device__ __forceinline__ void wave_hub_first_hit(bool hub, int64_t b, int64_t e,
                                                   const int32_t* cols, const uint64_t* bits,
                                                   const uint32_t* filt, bool use_filt,
                                                   int fs, uint32_t hi0,
                                                   bool& found, int32_t& par,
                                                   int64_t& examined) {
  const int l = lane_id();
  uint64_t hubs = ballot(hub);
  while (hubs) {
    const int h = ffs64(hubs);
    hubs &= hubs - 1;
    const int64_t hb = shfl(b, h), he = shfl(e, h);
    bool hf = false;
    int32_t hp = 0;
    int64_t scanned = he - hb;
    // downwards from the row's end, lane 0 on the highest entry
    for (int64_t j0 = he; j0 > hb; j0 -= kWave) {
      const int64_t j = j0 - 1 - l;
      int32_t w = 0;
      bool hit = false;
      if (j >= hb) {
        w = cols[j];
        hit = probe_bit(bits, filt, use_filt, fs, hi0, (uint32_t)w);
      }
      const uint64_t hm = ballot(hit);
      if (hm) {
        const int first = ffs64(hm);
        hp = shfl(w, first);
        hf = true;
        scanned = he - j0 + first + 1;
        break;
      }
    }
    if (l == h) {
      found = hf;
      par = hp;
    }
    if (l == 0) examined += scanned;
  }
}

// Rows of at most kLaneRow entries are scanned by one lane by default,
// longer rows by a whole wave (wave_hub_first_hit); the split is tunable.
constexpr int kLaneRow = 32;

// ---------------------------------------------------------------------------
// Edge walk over the rows of one 64-vertex word [64 k, 64 k + 64): rows of at
// most kLaneRow entries are walked by their own lane, longer rows by the whole
// wave (64 consecutive entries per step, coalesced).  f(v, w, e) is called
// once per adjacency entry e = (v, w).  All lanes of the wave must call it.

template <class F>
__device__ __forceinline__ void word_edges(const int64_t* off, const int32_t* cols, int64_t n,
                                           int64_t word, F&& f) {
  const int l = lane_id();
  const int64_t v = word * kWave + l;
  int64_t b = 0, e = 0;
  if (v < n) {
    b = off[v];
    e = off[v + 1];
  }
  const bool big = (e - b) > kLaneRow;
  if (!big) {
    for (int64_t j = b; j < e; ++j) f(v, cols[j], j);
  }
  uint64_t hubs = ballot(big);
  while (hubs) {
    const int h = ffs64(hubs);
    hubs &= hubs - 1;
    const int64_t vh = word * kWave + h;
    const int64_t hb = shfl(b, h), he = shfl(e, h);
    for (int64_t j = hb + l; j < he; j += kWave) f(vh, cols[j], j);
  }
}

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

__host__ __device__ inline int bits_for(int64_t n) {  // smallest b >= 1 with 2^b >= n
  int b = 1;
  while (b < 62 && ((int64_t)1 << b) < n) ++b;
  return b;
}

}  // namespace rbfs
