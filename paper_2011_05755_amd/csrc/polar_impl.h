// Device helpers shared by the kernels that resample particles onto the
// polar grid: the image staged in LDS with a zero border, bilinear taps,
// twiddles and a wave-level barrier.
#pragma once

#include "mra_common.h"

namespace mra {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// (cos, sin)(2 pi j / 256) as float-float pairs, cos = ch + cl and
// sin = sh + sl, staged in LDS: the resampling positions and, through
// (ch, sh), the ring FFT twiddles.
struct __attribute__((aligned(16))) CosSin {
  float ch, sh, cl, sl;
};

__device__ __forceinline__ void stage_cs(CosSin* t, const double2* cs64) {
  for (int j = threadIdx.x; j < kNphi; j += blockDim.x) {
    const double2 v = cs64[j];
    CosSin c;
    c.ch = (float)v.x;
    c.sh = (float)v.y;
    c.cl = (float)(v.x - (double)c.ch);
    c.sl = (float)(v.y - (double)c.sh);
    t[j] = c;
  }
}

// exp(-2 pi i e / 256) from the staged table
__device__ __forceinline__ float2 twid(const CosSin* t, int e) {
  const float2 v = *reinterpret_cast<const float2*>(t + e);
  return make_float2(v.x, -v.y);
}

// Batches of eight loads per thread are issued before any is stored, so the
// HBM latency is paid once per batch rather than once per element.
__device__ __forceinline__ void stage_image(float* img, const float* src, int L, int Lp, int pad) {
  constexpr int kB = 8;
  const int n = Lp * Lp;
  for (int i0 = threadIdx.x; i0 < n; i0 += kB * blockDim.x) {
    float v[kB];
#pragma unroll
    for (int b = 0; b < kB; ++b) {
      const int i = i0 + b * blockDim.x;
      const int yy = i / Lp - pad, xx = i % Lp - pad;
      v[b] = (i < n && yy >= 0 && yy < L && xx >= 0 && xx < L) ? src[yy * L + xx] : 0.f;
    }
#pragma unroll
    for (int b = 0; b < kB; ++b) {
      const int i = i0 + b * blockDim.x;
      if (i < n) img[i] = v[b];
    }
  }
}

// The same taps for a byte offset o4 of the top-left pixel and the row pitch
// Lp4 in bytes.
__device__ __forceinline__ float bilin4(const float* img, int o4, int Lp4, float fx, float fy) {
  const char* p = reinterpret_cast<const char*>(img) + o4;
  const float i00 = *reinterpret_cast<const float*>(p), i10 = *reinterpret_cast<const float*>(p + 4);
  const float i01 = *reinterpret_cast<const float*>(p + Lp4), i11 = *reinterpret_cast<const float*>(p + Lp4 + 4);
  const float top = i00 + fx * (i10 - i00);
  const float bot = i01 + fx * (i11 - i01);
  return top + fy * (bot - top);
}

// Offset (in pixels) of integer shift s = sy_index * S1 + sx_index, both
// indices counted from -T, for an image of pitch Lp: (sy - T) Lp + (sx - T).
// s / S1 is taken as (s * m) >> 16 with m = ceil(65536 / S1), which is exact
// for 0 <= s < 65536 / S1 (here s < 289 and S1 <= 17).
__device__ __forceinline__ int shift_offset(int s, int S1, int m, int T, int Lp) {
  const int q = __mul24(s, m) >> 16;
  return __mul24(q, Lp - S1) + s - T * (Lp + 1);
}

// Bilinear taps of the staged image at offset rr (cos, sin) of angle entry
// c from a shift's centre pixel.  Floor and fractions come from the
// float-float cos/sin: each fraction is within a few FP32 ulps of the one
// the FP64 position gives.  Where the position lies within rounding of a
// pixel boundary, floor(rr * ch) can be one off the exact floor; the
// fraction is then just outside [0, 1), the sample is the same up to
// rounding, and the taps reach one pixel further, which the zero border of
// the staged image allows for.  Integer shifts move the taps by whole
// pixels, so one position split serves every shift: the byte offset of the
// top-left tap from the shift's centre pixel, and the four weights.
__device__ __forceinline__ int polar_offset(float rr, const CosSin& c, int Lp4) {
  const float xf = floorf(rr * c.ch), yf = floorf(rr * c.sh);
  return __mul24((int)yf, Lp4) + 4 * (int)xf;
}
__device__ __forceinline__ void polar_weights(float rr, const CosSin& c, float& w00, float& w10, float& w01,
                                              float& w11) {
  const float xf = floorf(rr * c.ch), yf = floorf(rr * c.sh);
  const float fx = fmaf(rr, c.cl, fmaf(rr, c.ch, -xf));
  const float fy = fmaf(rr, c.sl, fmaf(rr, c.sh, -yf));
  const float gx = 1.f - fx, gy = 1.f - fy;
  w00 = gx * gy;
  w10 = fx * gy;
  w01 = gx * fy;
  w11 = fx * fy;
}
__device__ __forceinline__ float bilin4w(const float* img, int o4, int Lp4, float w00, float w10, float w01,
                                         float w11) {
  const char* p = reinterpret_cast<const char*>(img) + o4;
  const float i00 = *reinterpret_cast<const float*>(p), i10 = *reinterpret_cast<const float*>(p + 4);
  const float i01 = *reinterpret_cast<const float*>(p + Lp4), i11 = *reinterpret_cast<const float*>(p + Lp4 + 4);
  return fmaf(w11, i11, fmaf(w01, i01, fmaf(w10, i10, w00 * i00)));
}

__device__ __forceinline__ float bilin(const float* img, int o, int Lp, float fx, float fy) {
  const float i00 = img[o], i10 = img[o + 1], i01 = img[o + Lp], i11 = img[o + Lp + 1];
  const float top = i00 + fx * (i10 - i00);
  const float bot = i01 + fx * (i11 - i01);
  return top + fy * (bot - top);
}

}  // namespace mra
