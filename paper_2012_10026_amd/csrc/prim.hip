// Device-wide exclusive scan and stable LSD radix sort (64-bit keys).
//
// Scan: tiles of 2048 items (256 threads x 8); per-tile totals are scanned
// recursively, then each tile adds its offset.
//
// Radix sort: 8-bit digits.  Per pass, an upsweep counts digits per tile,
// the digit-major count table [digit][tile] is scanned, and a downsweep
// scatters each tile's keys in order.  Stability inside a tile comes from
// ranking one key per thread per round: lanes holding the same digit are
// found with eight ballots (one per digit bit), and earlier waves' counts of
// that digit come from LDS.
#include <hip/hip_runtime.h>

#include "common.h"
#include "graph.h"
#include "prim.h"

namespace rbfs {

hipError_t Scratch::get(size_t need, void** out) {
  if (need > bytes) {
    if (ptr) (void)rbfs::dev_free(ptr);
    ptr = nullptr;
    bytes = 0;
    size_t want = need + need / 4 + 256;
    hipError_t e = rbfs::dev_malloc(&ptr, want);
    if (e != hipSuccess) {
      ptr = nullptr;
      return e;
    }
    bytes = want;
  }
  *out = ptr;
  return hipSuccess;
}

void Scratch::release() {
  if (ptr) (void)rbfs::dev_free(ptr);
  ptr = nullptr;
  bytes = 0;
}

namespace {

constexpr int kScanItems = 8;
constexpr int64_t kScanTile = (int64_t)kBlock * kScanItems;

// Block-wide exclusive scan of one value per thread; returns the exclusive
// prefix, and the block total in *total.
__device__ __forceinline__ int64_t block_exclusive(int64_t v, int64_t* total) {
  __shared__ int64_t s_w[kWavesPerBlock];
  const int64_t inc = wave_inclusive_sum(v);
  if (lane_id() == kWave - 1) s_w[wave_id()] = inc;
  __syncthreads();
  int64_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kWavesPerBlock; ++w) {
    const int64_t x = s_w[w];
    if (w < wave_id()) base += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

template <class T>
__global__ __launch_bounds__(kBlock) void scan_reduce_kernel(const T* in, int64_t n,
                                                             int64_t* tile_sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int64_t i = base + (int64_t)j * kBlock + threadIdx.x;
    if (i < n) s += (int64_t)in[i];
  }
  int64_t tot;
  (void)block_exclusive(s, &tot);
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

// Exclusive scan of each tile plus its offset; thread t owns items
// [8t, 8t + 8) of the tile.  out has n + 1 entries; the last tile writes the
// total into out[n].
template <class T>
__global__ __launch_bounds__(kBlock) void scan_apply_kernel(const T* in, int64_t* out, int64_t n,
                                                            const int64_t* tile_offsets) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int64_t i = base + j;
    v[j] = (i < n) ? (int64_t)in[i] : 0;
    s += v[j];
  }
  int64_t tot;
  int64_t run = block_exclusive(s, &tot) + (tile_offsets ? tile_offsets[blockIdx.x] : 0);
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int64_t i = base + j;
    if (i < n) out[i] = run;
    run += v[j];
    if (i == n - 1) out[n] = run;
  }
}

size_t scan_scratch_bytes(int64_t n) {
  size_t b = 0;
  while (n > kScanTile) {
    int64_t nb = ceil_div(n, kScanTile);
    b += sizeof(int64_t) * (size_t)(2 * nb + 2);
    n = nb;
  }
  return b + 256;
}

template <class T>
hipError_t scan_impl(const T* in, int64_t* out, int64_t n, char* region, hipStream_t stream) {
  if (n <= 0) {
    return hipMemsetAsync(out, 0, sizeof(int64_t), stream);
  }
  const int64_t nb = ceil_div(n, kScanTile);
  if (nb == 1) {
    hipLaunchKernelGGL(scan_apply_kernel<T>, dim3(1), dim3(kBlock), 0, stream, in, out, n,
                       (const int64_t*)nullptr);
    return hipGetLastError();
  }
  int64_t* sums = (int64_t*)region;
  int64_t* offs = sums + nb;  // nb + 1 entries
  char* rest = (char*)(offs + nb + 1);
  hipLaunchKernelGGL(scan_reduce_kernel<T>, dim3((unsigned)nb), dim3(kBlock), 0, stream, in, n,
                     sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_impl<int64_t>(sums, offs, nb, rest, stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scan_apply_kernel<T>, dim3((unsigned)nb), dim3(kBlock), 0, stream, in, out,
                     n, (const int64_t*)offs);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// radix sort

constexpr int kRadixBits = 8;
constexpr int kDigits = 1 << kRadixBits;
constexpr int kSortItems = 16;
constexpr int64_t kSortTile = (int64_t)kBlock * kSortItems;

__global__ __launch_bounds__(kBlock) void radix_upsweep_kernel(const uint64_t* keys, int64_t n,
                                                               int shift, uint32_t* hist,
                                                               int64_t ntiles) {
  __shared__ uint32_t s_h[kDigits];
  s_h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll 4
  for (int j = 0; j < kSortItems; ++j) {
    const int64_t i = base + (int64_t)j * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&s_h[(keys[i] >> shift) & (kDigits - 1)], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = s_h[threadIdx.x];
}

// Scatter of one tile.  Each wave ranks its own quarter of the tile (16
// rounds of 64 consecutive keys) against a per-wave digit count in LDS, with
// no workgroup barrier between rounds; the counts of earlier waves are then
// added, the keys are placed in LDS grouped by digit (digit d's run starts at
// the tile's exclusive count of smaller digits), and written out run by run,
// so consecutive threads write consecutive positions of the same run.  Keys
// keep their tile order inside a digit: the sort is stable.
__global__ __launch_bounds__(kBlock) void radix_downsweep_kernel(const uint64_t* in,
                                                                 uint64_t* out, int64_t n,
                                                                 int shift,
                                                                 const int64_t* hist_scan,
                                                                 int64_t ntiles) {
  constexpr int kWaveKeys = kSortTile / kWavesPerBlock;  // keys per wave
  constexpr int kRounds = kWaveKeys / kWave;
  __shared__ int64_t s_base[kDigits];   // output start of this tile's digit-d keys
  __shared__ uint32_t s_loc[kDigits];   // start of digit d's run in the tile
  __shared__ uint32_t s_wcnt[kWavesPerBlock][kDigits];
  __shared__ uint64_t s_keys[kSortTile];
  const int t = threadIdx.x;
  const int l = lane_id();
  const int wv = wave_id();
  const int64_t hs = hist_scan[(int64_t)t * ntiles + blockIdx.x];
  s_base[t] = hs;
  const int64_t cnt_t = hist_scan[(int64_t)t * ntiles + blockIdx.x + 1] - hs;
  int64_t tot;
  const int64_t loc_t = block_exclusive(cnt_t, &tot);
  s_loc[t] = (uint32_t)loc_t;
#pragma unroll
  for (int w = 0; w < kWavesPerBlock; ++w) s_wcnt[w][t] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  const int tile_n = (int)((n - base) < kSortTile ? (n - base) : kSortTile);
  uint64_t key[kRounds];
  uint32_t dg[kRounds], rk[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int li = wv * kWaveKeys + r * kWave + l;
    key[r] = li < tile_n ? in[base + li] : 0ull;
  }
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int li = wv * kWaveKeys + r * kWave + l;
    const bool valid = li < tile_n;
    const uint32_t d = valid ? (uint32_t)((key[r] >> shift) & (kDigits - 1)) : 0u;
    uint64_t peers = ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = ballot(valid && bit);
      peers &= bit ? m : ~m;
    }
    const int rank = popc64(peers & lanemask_lt());
    const uint32_t before = valid ? s_wcnt[wv][d] : 0u;
    __builtin_amdgcn_wave_barrier();
    if (valid && rank == 0) s_wcnt[wv][d] = before + (uint32_t)popc64(peers);
    __builtin_amdgcn_wave_barrier();
    dg[r] = valid ? d : kDigits;  // kDigits marks an empty slot
    rk[r] = before + (uint32_t)rank;
  }
  __syncthreads();
  {  // counts of earlier waves: exclusive prefix over the waves, per digit
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) {
      const uint32_t c = s_wcnt[w][t];
      s_wcnt[w][t] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRounds; ++r)
    if (dg[r] < kDigits) s_keys[s_loc[dg[r]] + s_wcnt[wv][dg[r]] + rk[r]] = key[r];
  __syncthreads();
  for (int i = t; i < tile_n; i += kBlock) {
    const uint64_t k = s_keys[i];
    const uint32_t d = (uint32_t)((k >> shift) & (kDigits - 1));
    out[s_base[d] + (i - (int64_t)s_loc[d])] = k;
  }
}

}  // namespace

hipError_t scan_exclusive_i32(const int32_t* in, int64_t* out, int64_t n, Scratch& s,
                              hipStream_t stream) {
  void* region = nullptr;
  hipError_t e = s.get(scan_scratch_bytes(n), &region);
  if (e != hipSuccess) return e;
  return scan_impl<int32_t>(in, out, n, (char*)region, stream);
}

hipError_t scan_exclusive_i64(const int64_t* in, int64_t* out, int64_t n, Scratch& s,
                              hipStream_t stream) {
  void* region = nullptr;
  hipError_t e = s.get(scan_scratch_bytes(n), &region);
  if (e != hipSuccess) return e;
  return scan_impl<int64_t>(in, out, n, (char*)region, stream);
}

hipError_t radix_sort_u64(uint64_t** keys, uint64_t** alt, int64_t n, int begin_bit,
                          int end_bit, Scratch& s, hipStream_t stream) {
  if (n <= 1 || end_bit <= begin_bit) return hipSuccess;
  const int64_t ntiles = ceil_div(n, kSortTile);
  const int64_t nh = ntiles * kDigits;
  const size_t hist_bytes = sizeof(uint32_t) * (size_t)nh;
  const size_t hist_scan_bytes = sizeof(int64_t) * (size_t)(nh + 1);
  const size_t off2 = (hist_bytes + 255) / 256 * 256;
  const size_t off3 = off2 + (hist_scan_bytes + 255) / 256 * 256;
  void* region = nullptr;
  hipError_t e = s.get(off3 + scan_scratch_bytes(nh), &region);
  if (e != hipSuccess) return e;
  uint32_t* hist = (uint32_t*)region;
  int64_t* hist_scan = (int64_t*)((char*)region + off2);
  char* rest = (char*)region + off3;
  for (int shift = begin_bit; shift < end_bit; shift += kRadixBits) {
    hipLaunchKernelGGL(radix_upsweep_kernel, dim3((unsigned)ntiles), dim3(kBlock), 0, stream,
                       *keys, n, shift, hist, ntiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = scan_impl<uint32_t>(hist, hist_scan, nh, rest, stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(radix_downsweep_kernel, dim3((unsigned)ntiles), dim3(kBlock), 0, stream,
                       *keys, *alt, n, shift, (const int64_t*)hist_scan, ntiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    uint64_t* t = *keys;
    *keys = *alt;
    *alt = t;
  }
  return hipSuccess;
}

}  // namespace rbfs
