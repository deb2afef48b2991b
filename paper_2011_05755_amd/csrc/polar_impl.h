// Device helpers shared by the kernels that resample particles onto the
// polar grid: the image staged in LDS with a zero border, bilinear taps,
// twiddles and a wave-level barrier.
#pragma once

#include "mra_common.h"

namespace mra {

__device__ __forceinline__ float2 w256f(const float2* cs, int e) {
  float2 c = cs[e & 255];
  return make_float2(c.x, -c.y);  // exp(-2 pi i e / 256)
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void stage_image(float* img, const float* src, int L, int Lp, int pad) {
  for (int i = threadIdx.x; i < Lp * Lp; i += blockDim.x) {
    const int yy = i / Lp - pad, xx = i % Lp - pad;
    img[i] = (yy >= 0 && yy < L && xx >= 0 && xx < L) ? src[yy * L + xx] : 0.f;
  }
}

__device__ __forceinline__ float bilin(const float* img, int o, int Lp, float fx, float fy) {
  const float i00 = img[o], i10 = img[o + 1], i01 = img[o + Lp], i11 = img[o + Lp + 1];
  const float top = i00 + fx * (i10 - i00);
  const float bot = i01 + fx * (i11 - i01);
  return top + fy * (bot - top);
}

}  // namespace mra
