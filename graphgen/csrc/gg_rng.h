// Seeded synthetic graph inputs: counter-based random numbers, a keyed vertex
// permutation, and the per-edge draws of the Kronecker (R-MAT style) and
// Chung-Lu generators.  Shared by the host and device generators so that both
// produce the same tuples.  Nothing here computes any part of RCM or BFS.
//
// Random numbers: the splitmix64 output mix (Steele, Lea and Flood, "Fast
// splittable pseudorandom number generators", OOPSLA 2014; constants as in
// Vigna's public-domain splitmix64.c) applied to a counter.  A draw is
// mix(mix(seed ^ stream * K) + (ctr + 1) * gamma), so every draw is a pure
// function of (seed, stream, counter) and the output does not depend on how
// the work is split over threads.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define GG_HD __host__ __device__ inline
#else
#define GG_HD inline
#endif

#define GG_GAMMA 0x9E3779B97F4A7C15ull
#define GG_STREAM_KRON 1ull
#define GG_STREAM_PERM 2ull
#define GG_STREAM_CL 3ull
#define GG_STREAM_ROOT 4ull

GG_HD uint64_t gg_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

GG_HD uint64_t gg_key(uint64_t seed, uint64_t stream) {
  return gg_mix64(seed ^ (stream * 0xD1B54A32D192ED03ull));
}

GG_HD uint64_t gg_draw(uint64_t key, uint64_t ctr) {
  return gg_mix64(key + (ctr + 1ull) * GG_GAMMA);
}

// Number of bits b with 2^b >= n (at least 1).
GG_HD int gg_bits_for(int64_t n) {
  int b = 1;
  while (b < 62 && ((int64_t)1 << b) < n) ++b;
  return b;
}

// Keyed bijection of [0, 2^b): four rounds of (multiply by an odd constant,
// xor-shift right, add a constant), each invertible modulo 2^b.
struct gg_perm_t {
  uint64_t mul[4];
  uint64_t add[4];
  uint64_t mask;
  int shift;
  int64_t n;
};

GG_HD gg_perm_t gg_perm_make(uint64_t seed, int64_t n) {
  gg_perm_t p;
  int b = gg_bits_for(n);
  p.mask = (b >= 64) ? ~0ull : ((1ull << b) - 1ull);
  p.shift = (b + 1) / 2;
  p.n = n;
  uint64_t key = gg_key(seed, GG_STREAM_PERM);
  for (int r = 0; r < 4; ++r) {
    uint64_t k = gg_draw(key, (uint64_t)r);
    p.mul[r] = k | 1ull;
    p.add[r] = k >> 32;
  }
  return p;
}

GG_HD uint64_t gg_perm_round(const gg_perm_t& p, uint64_t x) {
  for (int r = 0; r < 4; ++r) {
    x = (x * p.mul[r]) & p.mask;
    x ^= x >> p.shift;
    x = (x + p.add[r]) & p.mask;
  }
  return x;
}

// Bijection of [0, n) by cycle-walking the bijection of [0, 2^b): iterate
// until the value falls inside [0, n).  The orbit of x returns to x < n, so
// the loop ends, and the restriction is a bijection of [0, n).
GG_HD int64_t gg_perm_apply(const gg_perm_t& p, int64_t x) {
  uint64_t y = gg_perm_round(p, (uint64_t)x);
  while ((int64_t)y >= p.n) y = gg_perm_round(p, y);
  return (int64_t)y;
}

// Kronecker initiator thresholds on 32-bit uniform integers.
struct gg_kron_t {
  uint64_t key;
  int scale;
  uint32_t tA, tAB, tABC;
};

GG_HD uint32_t gg_threshold(double p) {
  double t = p * 4294967296.0 + 0.5;
  if (t >= 4294967295.0) return 0xFFFFFFFFu;
  if (t <= 0.0) return 0u;
  return (uint32_t)t;
}

GG_HD gg_kron_t gg_kron_make(uint64_t seed, int scale, double A, double B, double C) {
  gg_kron_t k;
  k.key = gg_key(seed, GG_STREAM_KRON);
  k.scale = scale;
  k.tA = gg_threshold(A);
  k.tAB = gg_threshold(A + B);
  k.tABC = gg_threshold(A + B + C);
  return k;
}

// Edge e: `scale` independent quadrant choices with probabilities
// (A, B, C, D); quadrant (row bit, column bit) = (0,0), (0,1), (1,0), (1,1).
// Returns the unpermuted endpoints.
GG_HD void gg_kron_edge(const gg_kron_t& k, int64_t e, uint32_t* u_out, uint32_t* v_out) {
  uint32_t u = 0, v = 0;
  const int words = (k.scale + 1) / 2;
  for (int w = 0; w < words; ++w) {
    uint64_t r64 = gg_draw(k.key, (uint64_t)e * (uint64_t)words + (uint64_t)w);
    for (int h = 0; h < 2; ++h) {
      int lvl = 2 * w + h;
      if (lvl >= k.scale) break;
      uint32_t r = (uint32_t)(h == 0 ? (r64 & 0xFFFFFFFFull) : (r64 >> 32));
      uint32_t rb, cb;
      if (r < k.tA) { rb = 0; cb = 0; }
      else if (r < k.tAB) { rb = 0; cb = 1; }
      else if (r < k.tABC) { rb = 1; cb = 0; }
      else { rb = 1; cb = 1; }
      u = (u << 1) | rb;
      v = (v << 1) | cb;
    }
  }
  *u_out = u;
  *v_out = v;
}

// Chung-Lu endpoint draw: index of the first cumulative weight strictly
// greater than a uniform double in [0, 1), clamped to the last index.
GG_HD int64_t gg_cl_draw(uint64_t key, uint64_t ctr, const double* cdf, int64_t ncore) {
  uint64_t r = gg_draw(key, ctr);
  double u = (double)(r >> 11) * (1.0 / 9007199254740992.0);
  int64_t lo = 0, hi = ncore;  // first index with cdf > u in [lo, hi)
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (cdf[mid] > u) hi = mid; else lo = mid + 1;
  }
  return lo < ncore ? lo : ncore - 1;
}
