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
// generation, which releases everyone.  Each workgroup publishes its writes
// with one agent-scope release fence before arriving and takes one acquire
// fence after the release (polling itself is relaxed: an acquire per poll
// would invalidate the XCD's L2 while others still work).  A waiter gives up
// after `timeout_ticks` of the constant-rate wall clock, or as soon as the
// status word is non-zero, so the kernel always terminates; the status word
// then carries kStatusTimeout and the caller reports an error.
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
    if (old == gsize - 1u) {
      (void)__hip_atomic_exchange(&b->group[g][0], 0u, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // reset lands before top
      const unsigned o2 = __hip_atomic_fetch_add(&b->top, 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
      last = (o2 == ng - 1u);
    }
    if (last) {
      (void)__hip_atomic_exchange(&b->top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
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
  }
  __syncthreads();
  return __hip_atomic_load(&b->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
}

// ---------------------------------------------------------------------------
// First hit: each active lane holds a vertex whose row is cols[b, e); it
// finds the first entry w (in row order, i.e. increasing label) with bit w
// set in `bits`.  Rows of at most `lane_row` entries are scanned by their own
// lane; longer rows by the whole wave, 64 entries per step, where the lowest
// hitting lane is the first hit.  `examined` (per lane, summed later) counts
// the entries read up to and including the hit.  All lanes must call.
constexpr int kLaneRow = 32;  // default lane/wave split

__device__ __forceinline__ void wave_first_hit(bool active, int64_t b, int64_t e,
                                               const int32_t* cols, const uint64_t* bits,
                                               bool& found, int32_t& par, int64_t& examined,
                                               int lane_row = kLaneRow) {
  const int l = lane_id();
  found = false;
  par = 0;
  const bool hub = active && (e - b) > lane_row;
  if (active && !hub) {
    // four entries per step: the loads of a step are independent, so one
    // memory round trip covers four candidates
    int64_t hitj = e;
    for (int64_t j = b; j < e && hitj == e; j += 4) {
      int32_t w[4];
      bool h[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) w[q] = (j + q < e) ? cols[j + q] : 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) h[q] = (j + q < e) && test_bit(bits, (uint32_t)w[q]);
#pragma unroll
      for (int q = 3; q >= 0; --q)
        if (h[q]) {
          hitj = j + q;
          par = w[q];
        }
    }
    found = hitj < e;
    examined += found ? (hitj - b + 1) : (e - b);
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
        w = cols[j];
        hit = test_bit(bits, (uint32_t)w);
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
}

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
