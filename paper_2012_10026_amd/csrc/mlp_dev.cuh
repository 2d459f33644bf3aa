// Wave-level forward pass of the direction-switch MLP, used inside the
// persistent search kernel.  Every lane returns the same outputs; the sums
// run in a fixed order, so every workgroup computes bit-identical values and
// takes the same decision.
#pragma once
#include "common.cuh"
#include "switch.h"

namespace rbfs {

__device__ __forceinline__ void mlp_forward_wave(const float* __restrict__ w, const float* f,
                                                 float& y0, float& y1) {
  const int j = lane_id() & 31;
  float a = w[kOffB1 + j];
#pragma unroll
  for (int k = 0; k < kMlpIn; ++k) a = fmaf(w[kOffW1 + j * kMlpIn + k], f[k], a);
  const float h1 = fmaxf(a, 0.0f);
  float c = w[kOffB2 + j];
#pragma unroll 8
  for (int k = 0; k < kMlpHid; ++k) c = fmaf(w[kOffW2 + j * kMlpHid + k], __shfl(h1, k, kWave), c);
  const float h2 = fmaxf(c, 0.0f);
  float s0 = w[kOffB3], s1 = w[kOffB3 + 1];
#pragma unroll 8
  for (int k = 0; k < kMlpHid; ++k) {
    const float hk = __shfl(h2, k, kWave);
    s0 = fmaf(w[kOffW3 + k], hk, s0);
    s1 = fmaf(w[kOffW3 + kMlpHid + k], hk, s1);
  }
  y0 = s0;
  y1 = s1;
}

}  // namespace rbfs
