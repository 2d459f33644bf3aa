// Wave-level forward pass of the direction-switch MLP, used inside the
// persistent search kernel.  Every lane returns the same outputs; the sums
// run in a fixed order, so every workgroup computes bit-identical values and
// takes the same decision.
#pragma once
#include "common.cuh"
#include "switch.h"

namespace rbfs {

// Value of x in lane k of the wave (k the same in every lane).
__device__ __forceinline__ float lane_value(float x, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), k));
}

__device__ __forceinline__ void mlp_forward_wave(const float* __restrict__ w, const float* f,
                                                 float& y0, float& y1) {
  const int j = lane_id() & 31;
  float a = w[kOffB1 + j];
#pragma unroll
  for (int k = 0; k < kMlpIn; ++k) a = fmaf(w[kOffW1 + j * kMlpIn + k], f[k], a);
  const float h1 = fmaxf(a, 0.0f);
  float c = w[kOffB2 + j];
#pragma unroll 8
  for (int k = 0; k < kMlpHid; ++k) c = fmaf(w[kOffW2 + j * kMlpHid + k], lane_value(h1, k), c);
  const float h2 = fmaxf(c, 0.0f);
  float s0 = w[kOffB3], s1 = w[kOffB3 + 1];
#pragma unroll 8
  for (int k = 0; k < kMlpHid; ++k) {
    const float hk = lane_value(h2, k);
    s0 = fmaf(w[kOffW3 + k], hk, s0);
    s1 = fmaf(w[kOffW3 + kMlpHid + k], hk, s1);
  }
  y0 = s0;
  y1 = s1;
}

}  // namespace rbfs
