// Wave-level forward pass of the direction-switch MLP, used inside the
// persistent search kernel.  Every lane returns the same outputs; the sums
// run in a fixed order, so every workgroup computes bit-identical values and
// takes the same decision.
#pragma once
#include "common.h"
#include "switch.h"

namespace rbfs {

// A hidden layer's 32 outputs, one per lane j (lanes 32..63 repeat lanes
// 0..31), reach every lane through `hbuf` (32 floats of 16-byte aligned LDS
// owned by this wave): broadcast reads of four values at a time keep the next
// layer's multiply-add chain fed.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// w: a switch blob (layers 1 and 3 and the biases are read from it); w2: the
// second layer's rows, row j at w2 + j * kW2Stride (16-byte aligned).  The
// sums run over k in ascending order, so every layout gives the same bits.
template <int kW2Stride>
__device__ __forceinline__ void mlp_forward_wave(const float* __restrict__ w,
                                                 const float* __restrict__ w2, const float* f,
                                                 float& y0, float& y1, float* hbuf) {
  int j = lane_id() & 31;
  // computed here, not kept live from elsewhere in a calling kernel
  asm volatile("" : "+v"(j));
  const bool lo = lane_id() < 32;
  const float4* w1r = (const float4*)(w + kOffW1 + j * kMlpIn);
  const float4 wa = w1r[0], wb = w1r[1];
  float a = w[kOffB1 + j];
  a = fmaf(wa.x, f[0], a);
  a = fmaf(wa.y, f[1], a);
  a = fmaf(wa.z, f[2], a);
  a = fmaf(wa.w, f[3], a);
  a = fmaf(wb.x, f[4], a);
  a = fmaf(wb.y, f[5], a);
  a = fmaf(wb.z, f[6], a);
  a = fmaf(wb.w, f[7], a);
  if (lo) hbuf[j] = fmaxf(a, 0.0f);
  wave_lds_sync();
  const float4* w2r = (const float4*)(w2 + j * kW2Stride);
  const float4* h4 = (const float4*)hbuf;
  float c = w[kOffB2 + j];
  // two steps of 4 terms in flight: enough to cover the LDS latency without
  // the register demand of a full unroll inside a large kernel
#pragma unroll 2
  for (int q = 0; q < kMlpHid / 4; ++q) {
    const float4 x = w2r[q], h = h4[q];
    c = fmaf(x.x, h.x, c);
    c = fmaf(x.y, h.y, c);
    c = fmaf(x.z, h.z, c);
    c = fmaf(x.w, h.w, c);
  }
  wave_lds_sync();
  if (lo) hbuf[j] = fmaxf(c, 0.0f);
  wave_lds_sync();
  const float4* w30 = (const float4*)(w + kOffW3);
  const float4* w31 = (const float4*)(w + kOffW3 + kMlpHid);
  float s0 = w[kOffB3], s1 = w[kOffB3 + 1];
#pragma unroll 2
  for (int q = 0; q < kMlpHid / 4; ++q) {
    const float4 h = h4[q], u = w30[q], v = w31[q];
    s0 = fmaf(u.x, h.x, s0);
    s1 = fmaf(v.x, h.x, s1);
    s0 = fmaf(u.y, h.y, s0);
    s1 = fmaf(v.y, h.y, s1);
    s0 = fmaf(u.z, h.z, s0);
    s1 = fmaf(v.z, h.z, s1);
    s0 = fmaf(u.w, h.w, s0);
    s1 = fmaf(v.w, h.w, s1);
  }
  wave_lds_sync();
  y0 = s0;
  y1 = s1;
}

}  // namespace rbfs
