// Learned direction switch: per-level features and the weight layout of the
// 8 -> 32 -> 32 -> 2 ReLU MLP that predicts ln(microseconds) of the next
// level in each direction (output 0: top-down, 1: bottom-up).
//
// Weight blob (fp32), in this order:
//   W1[32][8], b1[32], W2[32][32], b2[32], W3[2][32], b3[2]   (1410 values)
//   fmin[8], fmax[8]       feature range seen in training (inputs outside it,
//                          widened by 10 % of its width, fall back to the
//                          alpha/beta rule)
//   max_level              largest level seen in training (as a float)
//   margin                 the network decides only when its two predictions
//                          differ by at least this much (ln microseconds);
//                          closer ones leave the decision to the alpha/beta
//                          rule
#pragma once
#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__)
#define RBFS_HD __host__ __device__ inline
#else
#define RBFS_HD inline
#endif

namespace rbfs {

constexpr int kMlpIn = 8;
constexpr int kMlpHid = 32;
constexpr int kMlpOut = 2;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpHid * kMlpIn;     // 256
constexpr int kOffW2 = kOffB1 + kMlpHid;              // 288
constexpr int kOffB2 = kOffW2 + kMlpHid * kMlpHid;    // 1312
constexpr int kOffW3 = kOffB2 + kMlpHid;              // 1344
constexpr int kOffB3 = kOffW3 + kMlpOut * kMlpHid;    // 1408
constexpr int kMlpParams = kOffB3 + kMlpOut;          // 1410
constexpr int kOffFmin = kMlpParams;
constexpr int kOffFmax = kOffFmin + kMlpIn;
constexpr int kOffMaxLevel = kOffFmax + kMlpIn;
constexpr int kOffMargin = kOffMaxLevel + 1;
constexpr int kSwitchBlob = kOffMargin + 1;           // 1428

RBFS_HD float clampf_(float x, float lo, float hi) { return x < lo ? lo : (x > hi ? hi : x); }

// Features of the decision taken before level `level` (which will expand the
// frontier F_level):
//   nf, mf   vertices and degree sum of F_level
//   mu       degree sum of the vertices not reached yet
//   nu       number of swept vertices not reached yet
//   nf_prev  |F_{level-1}|
//   dir      direction used for level-1 (0 top-down, 1 bottom-up)
RBFS_HD void switch_features(float* f, long long nf, long long mf, long long mu, long long nu,
                             long long nf_prev, int level, int dir, long long n_sweep,
                             long long nnz) {
  const float lgn = log2f((float)(n_sweep > 2 ? n_sweep : 2));
  const float lge = log2f((float)(nnz > 2 ? nnz : 2));
  f[0] = log2f(1.0f + (float)nf) / lgn;
  f[1] = log2f(1.0f + (float)mf) / lge;
  f[2] = log2f(1.0f + (float)mu) / lge;
  f[3] = (float)nu / (float)(n_sweep > 1 ? n_sweep : 1);
  f[4] = clampf_(log2f((1.0f + (float)mf) / (1.0f + (float)mu)) / 16.0f, -2.0f, 2.0f);
  f[5] = (float)level / 32.0f;
  f[6] = (float)dir;
  f[7] = clampf_(log2f((1.0f + (float)nf) / (1.0f + (float)nf_prev)) / 8.0f, -2.0f, 2.0f);
}

// The alpha/beta rule (Algorithm 2's switch, integer form): the direction of
// the level that expands a frontier of nf vertices and mf edges, with mu
// edges of unreached vertices left, nf_prev the previous frontier's size, dir
// the previous level's direction (0 top-down, 1 bottom-up) and n the swept
// vertex count.
RBFS_HD int heuristic_dir(int dir, long long nf, long long mf, long long mu, long long nf_prev,
                          long long n, int alpha, int beta) {
  if (dir == 0) return (mf * (long long)alpha > mu) ? 1 : 0;
  return (nf * (long long)beta < n && nf < nf_prev) ? 0 : 1;
}

// True when a feature vector lies outside the widened training range.
RBFS_HD bool switch_ood(const float* blob, const float* f, int level) {
  if ((float)level > blob[kOffMaxLevel]) return true;
  for (int i = 0; i < kMlpIn; ++i) {
    const float lo = blob[kOffFmin + i], hi = blob[kOffFmax + i];
    const float pad = 0.1f * (hi - lo);
    if (f[i] < lo - pad || f[i] > hi + pad) return true;
  }
  return false;
}

}  // namespace rbfs
