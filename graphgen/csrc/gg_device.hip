// Device generators: the same Kronecker and Chung-Lu tuples as the host
// generators (same counter-based draws), turned into the canonical undirected
// CSR on the GPU.  Used to build the large graphs quickly; the canonical CSR
// is unique for a tuple multiset, so it equals the host result bit for bit.
// The sort and unique steps use rocPRIM: this is input preparation, not part
// of the traversal library.
#include <string.h>
#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_select.hpp>
#include <stdint.h>
#include <stdio.h>
#include <string>
#include <algorithm>
#include <vector>

#include "gg_rng.h"

static thread_local std::string g_err;

#define GG_CHECK(x)                                                              \
  do {                                                                           \
    hipError_t e_ = (x);                                                         \
    if (e_ != hipSuccess) {                                                      \
      g_err = std::string(#x) + ": " + hipGetErrorString(e_);                    \
      goto fail;                                                                 \
    }                                                                            \
  } while (0)

namespace {

__global__ void kron_keys_kernel(gg_kron_t k, gg_perm_t p, int64_t m, int b, uint64_t* keys) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const uint64_t sentinel = (uint64_t)p.n << b;
  for (; e < m; e += stride) {
    uint32_t u0, v0;
    gg_kron_edge(k, e, &u0, &v0);
    uint64_t u = (uint64_t)gg_perm_apply(p, u0);
    uint64_t v = (uint64_t)gg_perm_apply(p, v0);
    if (u == v) {
      keys[2 * e] = sentinel;
      keys[2 * e + 1] = sentinel;
    } else {
      keys[2 * e] = (u << b) | v;
      keys[2 * e + 1] = (v << b) | u;
    }
  }
}

__global__ void cl_keys_kernel(uint64_t key, gg_perm_t p, const double* cdf, int64_t ncore,
                               int64_t m, int b, uint64_t* keys) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const uint64_t sentinel = (uint64_t)p.n << b;
  for (; e < m; e += stride) {
    uint64_t u = (uint64_t)gg_perm_apply(p, gg_cl_draw(key, 2 * (uint64_t)e, cdf, ncore));
    uint64_t v = (uint64_t)gg_perm_apply(p, gg_cl_draw(key, 2 * (uint64_t)e + 1, cdf, ncore));
    if (u == v) {
      keys[2 * e] = sentinel;
      keys[2 * e + 1] = sentinel;
    } else {
      keys[2 * e] = (u << b) | v;
      keys[2 * e + 1] = (v << b) | u;
    }
  }
}

// Number of Kronecker tuples (self-loops and duplicates included) whose two
// endpoints both have depth >= 0: the Graph500-style edge count of a search.
__global__ void kron_count_reached_kernel(gg_kron_t k, gg_perm_t p, int64_t m,
                                          const int32_t* depth, unsigned long long* count) {
  __shared__ unsigned long long s_sum[256];
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned long long c = 0;
  for (; e < m; e += stride) {
    uint32_t u0, v0;
    gg_kron_edge(k, e, &u0, &v0);
    const uint32_t u = gg_perm_apply(p, u0), v = gg_perm_apply(p, v0);
    c += (depth[u] >= 0 && depth[v] >= 0) ? 1ull : 0ull;
  }
  s_sum[threadIdx.x] = c;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s_sum[threadIdx.x] += s_sum[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(count, s_sum[0]);
}

// keys: sorted unique (row << b | col) with the sentinel possibly last.
__global__ void csr_from_keys_kernel(const uint64_t* keys, int64_t nnz, int64_t n, int b,
                                     int64_t* off, int32_t* cols) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const uint64_t mask = (1ull << b) - 1ull;
  for (; i <= nnz; i += stride) {
    int64_t s = (i < nnz) ? (int64_t)(keys[i] >> b) : n;
    int64_t prev = (i == 0) ? -1 : (int64_t)(keys[i - 1] >> b);
    for (int64_t v = prev + 1; v <= s; ++v) off[v] = i;
    if (i < nnz) cols[i] = (int32_t)(keys[i] & mask);
  }
}

// Directed keys per source bucket (source label >> bshift), self-loops left
// out: the sizes the range passes are planned from.
constexpr int kHistBuckets = 2048;
__global__ void kron_hist_kernel(gg_kron_t k, gg_perm_t p, int64_t m, int bshift,
                                 unsigned long long* hist) {
  __shared__ unsigned int s_h[kHistBuckets];
  for (int i = threadIdx.x; i < kHistBuckets; i += blockDim.x) s_h[i] = 0u;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) {
    uint32_t u0, v0;
    gg_kron_edge(k, e, &u0, &v0);
    const uint32_t u = gg_perm_apply(p, u0), v = gg_perm_apply(p, v0);
    if (u != v) {
      atomicAdd(&s_h[u >> bshift], 1u);
      atomicAdd(&s_h[v >> bshift], 1u);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kHistBuckets; i += blockDim.x)
    if (s_h[i]) atomicAdd(&hist[i], (unsigned long long)s_h[i]);
}

// The directed keys (u << b | v) whose source u lies in [r0, r1), appended
// at *count (order arbitrary: a sort follows); at most cap are written.
__global__ void kron_range_keys_kernel(gg_kron_t k, gg_perm_t p, int64_t m, int b, uint32_t r0,
                                       uint32_t r1, uint64_t* keys, unsigned long long* count,
                                       int64_t cap) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int lane = (int)(threadIdx.x & 63);
  for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x; e0 < m; e0 += stride) {
    const int64_t e = e0 + threadIdx.x;
    uint64_t key[2];
    int nk = 0;
    if (e < m) {
      uint32_t u0, v0;
      gg_kron_edge(k, e, &u0, &v0);
      const uint32_t u = gg_perm_apply(p, u0), v = gg_perm_apply(p, v0);
      if (u != v) {
        if (u >= r0 && u < r1) key[nk++] = ((uint64_t)u << b) | v;
        if (v >= r0 && v < r1) key[nk++] = ((uint64_t)v << b) | u;
      }
    }
    // one atomic per wave for its keys
    int incl = nk;
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o, 64);
      if (lane >= o) incl += t;
    }
    const int total = __shfl(incl, 63, 64);
    unsigned long long base = 0;
    if (lane == 63 && total > 0) base = atomicAdd(count, (unsigned long long)total);
    base = __shfl(base, 63, 64);
    for (int i = 0; i < nk; ++i) {
      const int64_t pos = (int64_t)base + incl - nk + i;
      if (pos < cap) keys[pos] = key[i];
    }
  }
}

// CSR rows [r0, r1) from sorted unique keys of sources in that range: row
// offsets relative to `base` (the entries of the rows before r0), columns
// written from cols[base] on.
__global__ void csr_range_kernel(const uint64_t* keys, int64_t nk, int64_t r0, int64_t r1, int b,
                                 int64_t base, int64_t* off, int32_t* cols) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const uint64_t mask = (1ull << b) - 1ull;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= nk; i += stride) {
    const int64_t s = (i < nk) ? (int64_t)(keys[i] >> b) : r1;
    const int64_t prev = (i == 0) ? r0 - 1 : (int64_t)(keys[i - 1] >> b);
    for (int64_t v = prev + 1; v <= s; ++v) off[v] = base + i;
    if (i < nk) cols[base + i] = (int32_t)(keys[i] & mask);
  }
}

int launch_blocks(int64_t work) {
  int64_t blocks = (work + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  return (int)blocks;
}

// Sort + unique + CSR assembly over 2m keys already in `keys`.
int64_t finish_csr(uint64_t* keys, int64_t m2, int64_t n, int b, int64_t* off, int32_t* cols,
                   int64_t cols_cap, hipStream_t stream) {
  uint64_t* keys2 = nullptr;
  void* tmp = nullptr;
  size_t tmp_bytes = 0, tmp2 = 0;
  int64_t* d_count = nullptr;
  int64_t h_count = 0, nnz = 0;
  uint64_t h_last = 0;
  const uint64_t sentinel = (uint64_t)n << b;
  GG_CHECK(hipMalloc(&keys2, sizeof(uint64_t) * (m2 > 0 ? m2 : 1)));
  GG_CHECK(hipMalloc(&d_count, sizeof(int64_t)));
  if (m2 > 0) {
    GG_CHECK(rocprim::radix_sort_keys(nullptr, tmp_bytes, keys, keys2, (size_t)m2, 0u,
                                      (unsigned)(2 * b + 1), stream));
    GG_CHECK(rocprim::unique(nullptr, tmp2, keys2, keys, d_count, (size_t)m2,
                             rocprim::equal_to<uint64_t>(), stream));
    if (tmp2 > tmp_bytes) tmp_bytes = tmp2;
    GG_CHECK(hipMalloc(&tmp, tmp_bytes));
    tmp2 = tmp_bytes;
    GG_CHECK(rocprim::radix_sort_keys(tmp, tmp2, keys, keys2, (size_t)m2, 0u,
                                      (unsigned)(2 * b + 1), stream));
    tmp2 = tmp_bytes;
    GG_CHECK(rocprim::unique(tmp, tmp2, keys2, keys, d_count, (size_t)m2,
                             rocprim::equal_to<uint64_t>(), stream));
    GG_CHECK(hipMemcpyAsync(&h_count, d_count, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    GG_CHECK(hipStreamSynchronize(stream));
    nnz = h_count;
    if (nnz > 0) {
      GG_CHECK(hipMemcpyAsync(&h_last, keys + (nnz - 1), sizeof(uint64_t),
                              hipMemcpyDeviceToHost, stream));
      GG_CHECK(hipStreamSynchronize(stream));
      if (h_last == sentinel) --nnz;
    }
  }
  if (nnz > cols_cap) {
    g_err = "cols capacity too small";
    goto fail;
  }
  hipLaunchKernelGGL(csr_from_keys_kernel, dim3(launch_blocks(nnz + 1)), dim3(256), 0, stream,
                     keys, nnz, n, b, off, cols);
  GG_CHECK(hipGetLastError());
  GG_CHECK(hipStreamSynchronize(stream));
  (void)hipFree(keys2);
  (void)hipFree(tmp);
  (void)hipFree(d_count);
  return nnz;
fail:
  if (keys2) (void)hipFree(keys2);
  if (tmp) (void)hipFree(tmp);
  if (d_count) (void)hipFree(d_count);
  return -4;
}

}  // namespace

extern "C" {

const char* gg_dev_last_error(void) { return g_err.c_str(); }

// Kronecker graph with m = edgefactor * 2^scale tuples, canonical CSR written
// to device buffers off (2^scale + 1) and cols (capacity cols_cap >= nnz).
// Returns nnz, or a negative value on error.
int64_t gg_dev_kron_csr(int scale, int64_t edgefactor, uint64_t seed, double A, double B,
                        double C, int64_t* off, int32_t* cols, int64_t cols_cap, void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (scale < 1 || scale > 30 || edgefactor < 0 || !off || !cols) {
    g_err = "bad arguments";
    return -1;
  }
  const int64_t n = (int64_t)1 << scale;
  const int64_t m = edgefactor * n;
  const int b = gg_bits_for(n);
  uint64_t* keys = nullptr;
  int64_t r;
  gg_kron_t k = gg_kron_make(seed, scale, A, B, C);
  gg_perm_t p = gg_perm_make(seed, n);
  GG_CHECK(hipMalloc(&keys, sizeof(uint64_t) * (2 * m > 0 ? 2 * m : 1)));
  hipLaunchKernelGGL(kron_keys_kernel, dim3(launch_blocks(m)), dim3(256), 0, stream, k, p, m, b,
                     keys);
  GG_CHECK(hipGetLastError());
  r = finish_csr(keys, 2 * m, n, b, off, cols, cols_cap, stream);
  (void)hipFree(keys);
  return r;
fail:
  if (keys) (void)hipFree(keys);
  return -4;
}

// The same CSR as gg_dev_kron_csr, built in passes over ranges of source
// labels so that the directed keys of one pass (at most max_pass_keys; 0 =
// as many as fit in 80 % of the free device memory with the sort buffers) fit in memory: each
// pass regenerates every tuple, keeps the keys whose source lies in its
// range, sorts and uniques them, and writes those rows.  The passes cover
// the labels in increasing order, so the result does not depend on how they
// are cut.  Returns nnz, or a negative value on error.
int64_t gg_dev_kron_csr_ranges(int scale, int64_t edgefactor, uint64_t seed, double A, double B,
                               double C, int64_t* off, int32_t* cols, int64_t cols_cap,
                               int64_t max_pass_keys, int64_t* passes_out, void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (scale < 1 || scale > 30 || edgefactor < 0 || !off || !cols || max_pass_keys < 0) {
    g_err = "bad arguments";
    return -1;
  }
  const int64_t n = (int64_t)1 << scale;
  const int64_t m = edgefactor * n;
  const int b = gg_bits_for(n);
  const int bshift = b > 11 ? b - 11 : 0;
  const int64_t nbk = ((n - 1) >> bshift) + 1;
  gg_kron_t k = gg_kron_make(seed, scale, A, B, C);
  gg_perm_t p = gg_perm_make(seed, n);
  unsigned long long* d_hist = nullptr;
  unsigned long long* d_count = nullptr;
  uint64_t *keys = nullptr, *keys2 = nullptr;
  void* tmp = nullptr;
  int64_t* d_nu = nullptr;
  std::vector<unsigned long long> hist(kHistBuckets, 0ull);
  int64_t kmax = max_pass_keys, total = 0, nnz = 0, passes = 0, maxb = 0;
  size_t tmp_bytes = 0;
  GG_CHECK(hipMalloc(&d_hist, sizeof(unsigned long long) * kHistBuckets));
  GG_CHECK(hipMalloc(&d_count, sizeof(unsigned long long)));
  GG_CHECK(hipMalloc(&d_nu, sizeof(int64_t)));
  GG_CHECK(hipMemsetAsync(d_hist, 0, sizeof(unsigned long long) * kHistBuckets, stream));
  hipLaunchKernelGGL(kron_hist_kernel, dim3(launch_blocks(m)), dim3(256), 0, stream, k, p, m,
                     bshift, d_hist);
  GG_CHECK(hipGetLastError());
  GG_CHECK(hipMemcpyAsync(hist.data(), d_hist, sizeof(unsigned long long) * kHistBuckets,
                          hipMemcpyDeviceToHost, stream));
  GG_CHECK(hipStreamSynchronize(stream));
  for (int64_t i = 0; i < nbk; ++i) {
    total += (int64_t)hist[i];
    maxb = std::max<int64_t>(maxb, (int64_t)hist[i]);
  }
  if (kmax == 0) {
    size_t fr = 0, tot = 0;
    GG_CHECK(hipMemGetInfo(&fr, &tot));
    // keys, sorted keys and the sort's temporary copy: 24 bytes a key
    kmax = std::min<int64_t>(total, (int64_t)((double)fr * 0.8 / (3 * sizeof(uint64_t))));
  }
  if (kmax < maxb) kmax = maxb;  // a pass holds at least one bucket
  if (kmax < 1) kmax = 1;
  GG_CHECK(hipMalloc(&keys, sizeof(uint64_t) * kmax));
  GG_CHECK(hipMalloc(&keys2, sizeof(uint64_t) * kmax));
  {
    size_t t1 = 0, t2 = 0;
    GG_CHECK(rocprim::radix_sort_keys(nullptr, t1, keys, keys2, (size_t)kmax, 0u,
                                      (unsigned)(2 * b), stream));
    GG_CHECK(rocprim::unique(nullptr, t2, keys2, keys, d_nu, (size_t)kmax,
                             rocprim::equal_to<uint64_t>(), stream));
    tmp_bytes = std::max(t1, t2);
    GG_CHECK(hipMalloc(&tmp, tmp_bytes > 0 ? tmp_bytes : 1));
  }
  for (int64_t i0 = 0; i0 < nbk;) {
    int64_t i1 = i0, cnt = 0;
    while (i1 < nbk && cnt + (int64_t)hist[i1] <= kmax) cnt += (int64_t)hist[i1++];
    const int64_t r0 = i0 << bshift, r1 = std::min<int64_t>(n, i1 << bshift);
    GG_CHECK(hipMemsetAsync(d_count, 0, sizeof(unsigned long long), stream));
    hipLaunchKernelGGL(kron_range_keys_kernel, dim3(launch_blocks(m)), dim3(256), 0, stream, k,
                       p, m, b, (uint32_t)r0, (uint32_t)r1, keys, d_count, kmax);
    GG_CHECK(hipGetLastError());
    int64_t nk = 0, nu = 0;
    if (cnt > 0) {
      size_t t = tmp_bytes;
      GG_CHECK(rocprim::radix_sort_keys(tmp, t, keys, keys2, (size_t)cnt, 0u, (unsigned)(2 * b),
                                        stream));
      t = tmp_bytes;
      GG_CHECK(rocprim::unique(tmp, t, keys2, keys, d_nu, (size_t)cnt,
                               rocprim::equal_to<uint64_t>(), stream));
      GG_CHECK(hipMemcpyAsync(&nu, d_nu, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    }
    GG_CHECK(hipMemcpyAsync(&nk, d_count, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    GG_CHECK(hipStreamSynchronize(stream));
    if (nk != cnt) {
      g_err = "range pass key count differs from its plan";
      goto fail;
    }
    if (nnz + nu > cols_cap) {
      g_err = "cols capacity too small";
      goto fail;
    }
    hipLaunchKernelGGL(csr_range_kernel, dim3(launch_blocks(nu + 1)), dim3(256), 0, stream, keys,
                       nu, r0, r1, b, nnz, off, cols);
    GG_CHECK(hipGetLastError());
    nnz += nu;
    ++passes;
    i0 = i1;
  }
  GG_CHECK(hipStreamSynchronize(stream));
  if (passes_out) *passes_out = passes;
  (void)hipFree(keys);
  (void)hipFree(keys2);
  (void)hipFree(tmp);
  (void)hipFree(d_hist);
  (void)hipFree(d_count);
  (void)hipFree(d_nu);
  return nnz;
fail:
  if (keys) (void)hipFree(keys);
  if (keys2) (void)hipFree(keys2);
  if (tmp) (void)hipFree(tmp);
  if (d_hist) (void)hipFree(d_hist);
  if (d_count) (void)hipFree(d_count);
  if (d_nu) (void)hipFree(d_nu);
  return -4;
}

// Tuples of the same Kronecker graph with both endpoints reached (depth:
// device int32[2^scale], indexed by vertex ID).  Returns the count, or a
// negative value on error.  Synchronises `stream`.
int64_t gg_dev_kron_count_reached(int scale, int64_t edgefactor, uint64_t seed, double A,
                                  double B, double C, const int32_t* depth, void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (scale < 1 || scale > 30 || edgefactor < 0 || !depth) {
    g_err = "bad arguments";
    return -1;
  }
  const int64_t n = (int64_t)1 << scale;
  const int64_t m = edgefactor * n;
  unsigned long long* d_count = nullptr;
  unsigned long long h_count = 0;
  gg_kron_t k = gg_kron_make(seed, scale, A, B, C);
  gg_perm_t p = gg_perm_make(seed, n);
  GG_CHECK(hipMalloc(&d_count, sizeof(unsigned long long)));
  GG_CHECK(hipMemsetAsync(d_count, 0, sizeof(unsigned long long), stream));
  hipLaunchKernelGGL(kron_count_reached_kernel, dim3(launch_blocks(m)), dim3(256), 0, stream, k,
                     p, m, depth, d_count);
  GG_CHECK(hipGetLastError());
  GG_CHECK(hipMemcpyAsync(&h_count, d_count, sizeof(h_count), hipMemcpyDeviceToHost, stream));
  GG_CHECK(hipStreamSynchronize(stream));
  (void)hipFree(d_count);
  return (int64_t)h_count;
fail:
  if (d_count) (void)hipFree(d_count);
  return -4;
}

// Chung-Lu graph: m tuples drawn from the host-built cumulative table
// (ncore entries), vertices relabelled over [0, n_total).
int64_t gg_dev_cl_csr(int64_t ncore, int64_t n_total, int64_t m, uint64_t seed,
                      const double* cdf_host, int64_t* off, int32_t* cols, int64_t cols_cap,
                      void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (ncore < 2 || n_total < ncore || n_total > 0x7FFFFFFFll || m < 0 || !cdf_host || !off ||
      !cols) {
    g_err = "bad arguments";
    return -1;
  }
  const int b = gg_bits_for(n_total);
  uint64_t* keys = nullptr;
  double* cdf = nullptr;
  int64_t r;
  gg_perm_t p = gg_perm_make(seed, n_total);
  uint64_t key = gg_key(seed, GG_STREAM_CL);
  GG_CHECK(hipMalloc(&cdf, sizeof(double) * ncore));
  GG_CHECK(hipMemcpy(cdf, cdf_host, sizeof(double) * ncore, hipMemcpyHostToDevice));
  GG_CHECK(hipMalloc(&keys, sizeof(uint64_t) * (2 * m > 0 ? 2 * m : 1)));
  hipLaunchKernelGGL(cl_keys_kernel, dim3(launch_blocks(m)), dim3(256), 0, stream, key, p, cdf,
                     ncore, m, b, keys);
  GG_CHECK(hipGetLastError());
  r = finish_csr(keys, 2 * m, n_total, b, off, cols, cols_cap, stream);
  (void)hipFree(keys);
  (void)hipFree(cdf);
  return r;
fail:
  if (keys) (void)hipFree(keys);
  if (cdf) (void)hipFree(cdf);
  return -4;
}

}  // extern "C"
