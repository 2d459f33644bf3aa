// Host generators: Kronecker and Chung-Lu edge tuples and the canonical
// undirected CSR built from them (self-loops dropped, both directions stored,
// each row strictly ascending, duplicates removed).  Multithreaded with
// std::thread; the result does not depend on the thread count.
#include <stdint.h>
#include <string.h>
#include <math.h>
#include <stdlib.h>
#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>

#include "gg_rng.h"

namespace {

template <class F>
void parallel_for(int64_t n, int nthreads, F f) {
  if (nthreads < 1) nthreads = 1;
  if (n < 4096 || nthreads == 1) { f(0, n); return; }
  std::vector<std::thread> ts;
  int64_t chunk = (n + nthreads - 1) / nthreads;
  for (int t = 0; t < nthreads; ++t) {
    int64_t b = t * chunk, e = std::min<int64_t>(n, b + chunk);
    if (b >= e) break;
    ts.emplace_back([=]() { f(b, e); });
  }
  for (auto& t : ts) t.join();
}

// Dynamic schedule over [0, n) in blocks of `grain` (rows of very different
// lengths).
template <class F>
void parallel_dynamic(int64_t n, int64_t grain, int nthreads, F f) {
  if (nthreads < 1) nthreads = 1;
  std::atomic<int64_t> next(0);
  auto worker = [&]() {
    for (;;) {
      int64_t b = next.fetch_add(grain);
      if (b >= n) break;
      f(b, std::min<int64_t>(n, b + grain));
    }
  };
  if (nthreads == 1) { worker(); return; }
  std::vector<std::thread> ts;
  for (int t = 0; t < nthreads; ++t) ts.emplace_back(worker);
  for (auto& t : ts) t.join();
}

}  // namespace

extern "C" {

uint64_t gg_host_draw(uint64_t seed, uint64_t stream, uint64_t ctr) {
  return gg_draw(gg_key(seed, stream), ctr);
}

int gg_perm_table(int64_t n, uint64_t seed, int32_t* out, int nthreads) {
  if (n <= 0 || n > 0x7FFFFFFFll || !out) return -1;
  gg_perm_t p = gg_perm_make(seed, n);
  parallel_for(n, nthreads, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) out[i] = (int32_t)gg_perm_apply(p, i);
  });
  return 0;
}

// Kronecker tuples for edge indices [e_begin, e_end), endpoints relabelled by
// the keyed permutation of [0, 2^scale).
int gg_kron_tuples(int scale, uint64_t seed, double A, double B, double C, int64_t e_begin,
                   int64_t e_end, int32_t* src, int32_t* dst, int nthreads) {
  if (scale < 1 || scale > 30 || e_end < e_begin || !src || !dst) return -1;
  gg_kron_t k = gg_kron_make(seed, scale, A, B, C);
  gg_perm_t p = gg_perm_make(seed, (int64_t)1 << scale);
  parallel_for(e_end - e_begin, nthreads, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      uint32_t u, v;
      gg_kron_edge(k, e_begin + i, &u, &v);
      src[i] = (int32_t)gg_perm_apply(p, u);
      dst[i] = (int32_t)gg_perm_apply(p, v);
    }
  });
  return 0;
}

// Chung-Lu weights w_i = c (i + i0)^(-1/(gamma-1)), i in [0, ncore), with
// w_0 = max_deg and mean weight mean_deg; i0 is found by bisection on the
// integral (Euler-Maclaurin) approximation of the weight sum, then the exact
// weights are summed in index order into the normalised cumulative table.
// params_out = {i0, c, realised weight sum}.
int gg_cl_cdf(int64_t ncore, double gamma, double mean_deg, double max_deg, double* cdf,
              double* params_out) {
  if (ncore < 2 || gamma <= 1.0 || !cdf) return -1;
  const double eta = 1.0 / (gamma - 1.0);
  const double N = (double)ncore;
  auto approx_mean = [&](double i0) {
    double integral;
    if (fabs(1.0 - eta) < 1e-12) integral = log((N + i0) / i0);
    else integral = (pow(N + i0, 1.0 - eta) - pow(i0, 1.0 - eta)) / (1.0 - eta);
    double s = integral + 0.5 * (pow(i0, -eta) + pow(N + i0, -eta));
    return max_deg * pow(i0, eta) * s / N;
  };
  double lo = 1e-6, hi = N;
  for (int it = 0; it < 300; ++it) {
    double mid = 0.5 * (lo + hi);
    if (approx_mean(mid) < mean_deg) lo = mid; else hi = mid;
  }
  double i0 = 0.5 * (lo + hi);
  double c = max_deg * pow(i0, eta);
  double acc = 0.0;
  for (int64_t i = 0; i < ncore; ++i) {
    acc += c * pow((double)i + i0, -eta);
    cdf[i] = acc;
  }
  double total = acc;
  for (int64_t i = 0; i < ncore; ++i) cdf[i] /= total;
  cdf[ncore - 1] = 1.0;
  if (params_out) { params_out[0] = i0; params_out[1] = c; params_out[2] = total; }
  return 0;
}

// Chung-Lu tuples for edge indices [e_begin, e_end): both endpoints drawn
// independently from the weight table, then relabelled by the keyed
// permutation of [0, n_total) (indices >= ncore are the isolated vertices).
int gg_cl_tuples(int64_t ncore, int64_t n_total, uint64_t seed, const double* cdf,
                 int64_t e_begin, int64_t e_end, int32_t* src, int32_t* dst, int nthreads) {
  if (ncore < 2 || n_total < ncore || n_total > 0x7FFFFFFFll || !cdf) return -1;
  uint64_t key = gg_key(seed, GG_STREAM_CL);
  gg_perm_t p = gg_perm_make(seed, n_total);
  parallel_for(e_end - e_begin, nthreads, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      uint64_t ei = (uint64_t)(e_begin + i);
      int64_t u = gg_cl_draw(key, 2 * ei, cdf, ncore);
      int64_t v = gg_cl_draw(key, 2 * ei + 1, cdf, ncore);
      src[i] = (int32_t)gg_perm_apply(p, u);
      dst[i] = (int32_t)gg_perm_apply(p, v);
    }
  });
  return 0;
}

// Canonical undirected CSR from m tuples over n vertices.  Returns nnz, or a
// negative value on bad arguments.  `cols` must hold 2*m entries.
int64_t gg_csr_from_tuples(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                           int64_t* off, int32_t* cols, int nthreads) {
  if (n <= 0 || n > 0x7FFFFFFFll || m < 0 || !off || (m > 0 && (!src || !dst || !cols)))
    return -1;
  for (int64_t i = 0; i < m; ++i) {
    if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) return -2;
  }
  std::vector<int64_t> cnt(n + 1, 0);
  int64_t* c = cnt.data();
  parallel_for(m, nthreads, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      if (src[i] == dst[i]) continue;
      __atomic_fetch_add(&c[src[i]], 1, __ATOMIC_RELAXED);
      __atomic_fetch_add(&c[dst[i]], 1, __ATOMIC_RELAXED);
    }
  });
  std::vector<int64_t> raw_off(n + 1, 0);
  for (int64_t v = 0; v < n; ++v) raw_off[v + 1] = raw_off[v] + cnt[v];
  const int64_t raw_n = raw_off[n];
  std::vector<int32_t> raw(raw_n > 0 ? raw_n : 1);
  std::vector<int64_t> cur(raw_off.begin(), raw_off.end());
  int64_t* cu = cur.data();
  int32_t* rw = raw.data();
  parallel_for(m, nthreads, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      int32_t u = src[i], v = dst[i];
      if (u == v) continue;
      rw[__atomic_fetch_add(&cu[u], 1, __ATOMIC_RELAXED)] = v;
      rw[__atomic_fetch_add(&cu[v], 1, __ATOMIC_RELAXED)] = u;
    }
  });
  // Sort and deduplicate each row; cnt[v] becomes the unique row length.
  parallel_dynamic(n, 4096, nthreads, [&](int64_t b, int64_t e) {
    for (int64_t v = b; v < e; ++v) {
      int32_t* r0 = rw + raw_off[v];
      int32_t* r1 = rw + raw_off[v + 1];
      std::sort(r0, r1);
      c[v] = std::unique(r0, r1) - r0;
    }
  });
  off[0] = 0;
  for (int64_t v = 0; v < n; ++v) off[v + 1] = off[v] + c[v];
  parallel_dynamic(n, 4096, nthreads, [&](int64_t b, int64_t e) {
    for (int64_t v = b; v < e; ++v) {
      if (c[v] > 0) memcpy(cols + off[v], rw + raw_off[v], sizeof(int32_t) * c[v]);
    }
  });
  return off[n];
}

}  // extern "C"
