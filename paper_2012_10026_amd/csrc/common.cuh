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
// Arrival counter plus generation number.  The last workgroup to arrive runs
// `last_fn` (with every workgroup's writes visible), resets the counter and
// bumps the generation, which releases the others.  A waiter gives up after
// `timeout_ticks` of the constant-rate wall clock, or as soon as the status
// word is non-zero, so the kernel always terminates; the status word then
// carries kStatusTimeout and the caller reports an error.
struct GridBarrier {
  unsigned count;
  unsigned gen;
  int status;
  unsigned pad;
};

template <class F>
__device__ __forceinline__ bool grid_barrier(GridBarrier* b, uint64_t timeout_ticks, F&& last_fn) {
  __shared__ unsigned s_last;
  __shared__ unsigned s_gen;
  __syncthreads();
  if (threadIdx.x == 0) {
    s_gen = __hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // publish this workgroup's writes
    unsigned old = __hip_atomic_fetch_add(&b->count, 1u, __ATOMIC_ACQ_REL,
                                          __HIP_MEMORY_SCOPE_AGENT);
    s_last = (old == gridDim.x - 1) ? 1u : 0u;
    if (s_last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  if (s_last) {
    last_fn();
    __syncthreads();
    if (threadIdx.x == 0) {
      __hip_atomic_store(&b->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(&b->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  } else if (threadIdx.x == 0) {
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(&b->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == s_gen) {
      if (__hip_atomic_load(&b->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
      if (wall_clock64() - t0 > timeout_ticks) {
        __hip_atomic_fetch_or(&b->status, kStatusTimeout, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return __hip_atomic_load(&b->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
}

// ---------------------------------------------------------------------------
// Edge walk over the rows of one 64-vertex word [64 k, 64 k + 64): rows of at
// most kLaneRow entries are walked by their own lane, longer rows by the whole
// wave (64 consecutive entries per step, coalesced).  f(v, w, e) is called
// once per adjacency entry e = (v, w).  All lanes of the wave must call it.
constexpr int kLaneRow = 32;

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
