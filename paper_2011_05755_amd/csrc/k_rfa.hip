// Alignment against a single reference (K = 1, the pass of reference-free
// alignment): resampling, ring FFTs, correlation, inverse FFT over angle and
// the arg-max fused in one kernel, one 4-wave workgroup per particle.
//
// With one reference the correlation is a ring-weighted sum of products per
// frequency slot, far too thin for the matrix cores, so the spectra never
// leave the chip.  The particle's shifts are processed in groups of eight
// rows.  For a group, wave w resamples and transforms rings w, w + 4, ...
// (lane (l, row) as in the resampling kernel) and keeps, per slot it owns,
// the four ring sums
//   U00 = sum (a-b)(c-d), U01 = sum (a-b)(c+d), U11 = sum (a+b)(c+d), U10 = sum (a+b)(c-d)
// of P = a + ib (particle) and c + id (the reference spectrum with w_r,
// 1/norm and the inverse-DFT scale folded in) in registers.  The four
// waves' partial sums are then added in a fixed order in LDS, the 256-point
// inverse DFT of each row gives the CC of the unmirrored (real part) and
// mirrored (imaginary part) particle at every angle, and the best and
// runner-up are kept per lane, then per workgroup.
#include <climits>

#include "mra_common.h"
#include "mra_fft.h"
#include "polar_impl.h"

namespace mra {

namespace {

// 4 waves per particle (the resampling kernel runs 8): the 64 accumulators
// per lane leave room for two waves per SIMD, and 35 rings split evenly
constexpr int kRfaWaves = 4;
constexpr int kRfaThreads = 64 * kRfaWaves;

size_t rfa_lds_bytes(int Lp) {
  return (size_t)((Lp * Lp + 3) & ~3) * sizeof(float) + (size_t)kRfaWaves * 64 * 9 * sizeof(float2) +
         (size_t)kNphi * sizeof(CosSin);
}

constexpr int kRowStride = 136;  // float4 per row of the summed spectra (128 slots, padded)

struct Best {
  float v;  // best CC
  int i;    // its candidate index (m S + s) 256 + angle
  float s;  // best CC over every other candidate
};

// Merge candidate (v, i) carrying runner-up s into b.  Larger CC wins, then
// the smaller index; the runner-up is the largest of everything else.
__device__ __forceinline__ void take(Best& b, float v, int i, float s) {
  if (v > b.v || (v == b.v && i < b.i)) {
    b.s = fmaxf(fmaxf(b.s, s), b.v);
    b.v = v;
    b.i = i;
  } else {
    b.s = fmaxf(fmaxf(b.s, s), v);
  }
}

// 64 accumulators per lane on top of the resampler's registers: at most
// 256 VGPRs, two waves per SIMD.
__global__ __launch_bounds__(kRfaThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_rfa(RfaArgs a) {
  extern __shared__ float smem[];
  float* img = smem;
  float2* scr = reinterpret_cast<float2*>(smem + ((a.Lp * a.Lp + 3) & ~3));
  CosSin* cs = reinterpret_cast<CosSin*>(scr + kRfaWaves * 64 * 9);
  float4* V = reinterpret_cast<float4*>(scr);     // summed spectra; aliases the scratch between groups
  const int n = blockIdx.x;
  stage_image(img, a.parts + (size_t)n * a.L * a.L, a.L, a.Lp, a.pad);
  stage_cs(cs, a.cs64);
  __syncthreads();

  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), ln = threadIdx.x & 63;
  const int l = ln >> 3, rl = ln & 7;
  float2* my = scr + w * 64 * 9;                  // per-wave transposition scratch
  const int base = (a.cx + a.pad) * a.Lp + (a.cx + a.pad);
  const int Lp4 = 4 * a.Lp, s1m = (65536 + a.S1 - 1) / a.S1;
  Best best{-INFINITY, INT_MAX, -INFINITY};
  const int ngrp = (a.S + 7) >> 3;

  for (int grp = 0; grp < ngrp; ++grp) {
    float acc[16][4];
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e][0] = acc[e][1] = acc[e][2] = acc[e][3] = 0.f;

    for (int ring = w; ring < a.R; ring += kRfaWaves) {
      // opaque lane indices: addresses are recomputed per ring instead of
      // being held in registers across the loop
      int lx = l, rx = rl;
      asm volatile("" : "+v"(lx), "+v"(rx));
      int k1a, k1b;
      fwd_cols(lx, k1a, k1b);
      const int s = grp * 8 + rx;
      const int sc = s < a.S ? s : a.S - 1;       // rows past the last shift repeat it (never chosen)
      const int o4 = 4 * (base + shift_offset(sc, a.S1, s1m, a.T, a.Lp));

      // 32 bilinear samples from the stencil table, read from the cache in
      // two batches of 16 (this kernel is bound by its vector ALU work, so
      // cached stencils beat positions computed in the loop)
      const Stencil* sp = a.stencil + ring * kNphi + 2 * lx;
      float v[32];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        Stencil st[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int i = 16 * h + j;
          st[j] = sp[16 * (i >> 1) + (i & 1)];
        }
#pragma unroll
        for (int j = 0; j < 16; ++j)
          v[16 * h + j] = bilin4(img, o4 + __mul24(st[j].dy, Lp4) + st[j].bx, Lp4, st[j].fx, st[j].fy);
        __builtin_amdgcn_sched_barrier(0);
      }

      float2 z[16];
#pragma unroll
      for (int n1 = 0; n1 < 16; ++n1) z[n1] = make_float2(v[2 * n1], v[2 * n1 + 1]);
      dft16<-1>(z);
#pragma unroll
      for (int k1 = 1; k1 < 16; ++k1) z[k1] = cmul(z[k1], twid(cs, 2 * ((lx * k1) & 127)));
      float2 Za[8], Zb[8];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int k1 = 0; k1 < 8; ++k1) my[(lx * 8 + rx) * 9 + k1] = z[8 * h + k1];
        wave_sync();
#pragma unroll
        for (int n2 = 0; n2 < 8; ++n2) {
          if (h == 0) Za[n2] = my[(n2 * 8 + rx) * 9 + k1a];
          else Zb[n2] = my[(n2 * 8 + rx) * 9 + k1b - 8];
        }
        wave_sync();
      }
      dft8<-1>(Za);
      dft8<-1>(Zb);

      const float2* G = a.G + ring * kSlots;
      int e = 0;
      fwd_emit(lx, Za, Zb, [&](int f) { return twid(cs, f & 255); }, [&](int slot, float re, float im) {
        const float al = re - im, be = re + im;
        const float2 g = G[slot];                 // (c - d, c + d)
        acc[e][0] += al * g.x;
        acc[e][1] += al * g.y;
        acc[e][2] += be * g.y;
        acc[e][3] += be * g.x;
        ++e;
      });
    }
    __syncthreads();  // every wave is done with its transposition scratch

    // fixed-order sum of the four waves' partial spectra: V[row][slot]
    int sl[16];
    emit_slots(l, sl);
    for (int ww = 0; ww < kRfaWaves; ++ww) {
      if (w == ww) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          float4* d = V + rl * kRowStride + sl[e];
          float4 x = make_float4(acc[e][0], acc[e][1], acc[e][2], acc[e][3]);
          if (ww > 0) {
            const float4 o = *d;
            x = make_float4(o.x + x.x, o.y + x.y, o.z + x.z, o.w + x.w);
          }
          *d = x;
        }
      }
      __syncthreads();
    }

    // inverse DFT over angle: wave w takes rows 2w, 2w + 1 with 16 lanes each
    const int row = 2 * w + ((ln >> 4) & 1);
    const int q = ln & 15;
    float2* P = reinterpret_cast<float2*>(V + row * kRowStride);
    float2 x[16];
    if (ln < 32) {
      // pass 1, column q: x[k1] = H[16 k1 + q] with H_e = U00 + i U01 of slot e
      // (e <= 127) and U11 + i U10 of slot 256 - e (e >= 128; slot 0 for 128)
#pragma unroll
      for (int k1 = 0; k1 < 16; ++k1) {
        const int e = 16 * k1 + q;
        const bool up = e >= 128;
        const float4 u = V[row * kRowStride + (up ? ((256 - e) & 127) : e)];
        x[k1] = up ? make_float2(u.z, u.w) : make_float2(u.x, u.y);
      }
      inv_pass1(q, x, [&](int e) { return twid(cs, e & 255); });
    }
    wave_sync();  // the wave's two rows are read before they are overwritten
    if (ln < 32) {
#pragma unroll
      for (int n1 = 0; n1 < 16; ++n1) P[17 * n1 + q] = x[n1];
    }
    wave_sync();
    if (ln < 32) {
#pragma unroll
      for (int k2 = 0; k2 < 16; ++k2) x[k2] = P[17 * q + k2];
      inv_pass2(x);  // x[n2] = CC at angle q + 16 n2
      const int s = grp * 8 + row;
      if (s < a.S) {
#pragma unroll
        for (int n2 = 0; n2 < 16; ++n2) {
          const int ang = q + 16 * n2;
          take(best, x[n2].x, s * kNphi + ang, -INFINITY);
          if (a.M == 2) take(best, x[n2].y, (a.S + s) * kNphi + ang, -INFINITY);
        }
      }
    }
    __syncthreads();  // the scratch is free for the next group
  }

  for (int o = 32; o > 0; o >>= 1) {
    const float ov = __shfl_xor(best.v, o), os = __shfl_xor(best.s, o);
    const int oi = __shfl_xor(best.i, o);
    take(best, ov, oi, os);
  }
  float* rv = reinterpret_cast<float*>(scr);
  int* ri = reinterpret_cast<int*>(scr) + 2 * kRfaWaves;
  if (ln == 0) {
    rv[w] = best.v;
    rv[kRfaWaves + w] = best.s;
    ri[w] = best.i;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    Best b{rv[0], ri[0], rv[kRfaWaves]};
    for (int ww = 1; ww < kRfaWaves; ++ww) take(b, rv[ww], ri[ww], rv[kRfaWaves + ww]);
    const int64_t gi = a.out_off + n;
    int idx = b.i;
    float cc = b.v;
    if (idx == INT_MAX) {  // every candidate was NaN
      idx = 0;
      cc = NAN;
    }
    const int ang = idx & 255, ms = idx >> 8;
    const int m = ms >= a.S ? 1 : 0;
    const int s = ms - m * a.S;
    a.ref[gi] = 0;
    a.mirror[gi] = m;
    a.shift_y[gi] = s / a.S1 - a.T;
    a.shift_x[gi] = s % a.S1 - a.T;
    a.psi[gi] = (kNphi - ang) & 255;
    a.cc[gi] = cc;
    if (a.cc2) a.cc2[gi] = b.s;
    if (a.flat) a.flat[gi] = idx;
  }
}

}  // namespace

hipError_t launch_rfa(const RfaArgs& a, hipStream_t st) {
  if (a.n_part <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rfa, dim3(a.n_part), dim3(kRfaThreads), rfa_lds_bytes(a.Lp), st, a);
  return hipGetLastError();
}

}  // namespace mra
