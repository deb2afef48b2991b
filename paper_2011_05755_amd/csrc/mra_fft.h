// Small fixed-size complex DFTs used by the ring transforms.
//
// The per-ring forward transform of the polar samples (Algorithm 1) and
// the inverse transform over angle of the correlation spectra (Sec. 3) are built
// from 4-, 8- and 16-point DFTs evaluated in registers.  SIGN = -1 is the
// forward kernel exp(-2 pi i k n / N), SIGN = +1 the inverse kernel
// exp(+2 pi i k n / N) (unnormalised).  Inputs and outputs are in natural
// order.  Everything here is plain float arithmetic usable on host and
// device, so the building blocks are unit-tested on the CPU.
#pragma once

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define MRA_HD __host__ __device__ __forceinline__
#else
#include <cmath>
struct float2 { float x, y; };
static inline float2 make_float2(float a, float b) { return float2{a, b}; }
#define MRA_HD inline
#endif

namespace mra {

MRA_HD float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
MRA_HD float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
MRA_HD float2 cmul(float2 a, float2 w) {
  return make_float2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}
MRA_HD float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
MRA_HD float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// a * (SIGN * i)
template <int SIGN>
MRA_HD float2 mul_i(float2 a) {
  return SIGN > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// 4-point DFT in place.
template <int SIGN>
MRA_HD void dft4(float2& x0, float2& x1, float2& x2, float2& x3) {
  float2 t0 = cadd(x0, x2), t1 = csub(x0, x2);
  float2 t2 = cadd(x1, x3), t3 = mul_i<SIGN>(csub(x1, x3));
  x0 = cadd(t0, t2);
  x2 = csub(t0, t2);
  x1 = cadd(t1, t3);
  x3 = csub(t1, t3);
}

// cos / sin of multiples of pi/8 (exact mathematical constants).
constexpr float kC1 = 0.92387953251128675613f;  // cos(pi/8)
constexpr float kS1 = 0.38268343236508977173f;  // sin(pi/8)
constexpr float kR2 = 0.70710678118654752440f;  // cos(pi/4)

// 8-point DFT in place: radix 4 over even/odd inputs, then one radix-2 pass.
template <int SIGN>
MRA_HD void dft8(float2 (&v)[8]) {
  dft4<SIGN>(v[0], v[2], v[4], v[6]);   // a[0][n1] in v[2 n1]
  dft4<SIGN>(v[1], v[3], v[5], v[7]);   // a[1][n1] in v[2 n1 + 1]
  v[3] = cmul(v[3], make_float2(kR2, SIGN * kR2));
  v[5] = mul_i<SIGN>(v[5]);
  v[7] = cmul(v[7], make_float2(-kR2, SIGN * kR2));
  float2 o[8];
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
    o[n1] = cadd(v[2 * n1], v[2 * n1 + 1]);
    o[n1 + 4] = csub(v[2 * n1], v[2 * n1 + 1]);
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = o[i];
}

// 16-point DFT in place: radix 4 x radix 4 with the 9 inner twiddles.
template <int SIGN>
MRA_HD void dft16(float2 (&v)[16]) {
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) dft4<SIGN>(v[k2], v[4 + k2], v[8 + k2], v[12 + k2]);
  // v[4 n1 + k2] now holds a[k2][n1]; multiply by w16^(SIGN k2 n1)
  v[5] = cmul(v[5], make_float2(kC1, SIGN * kS1));    // e = 1
  v[9] = cmul(v[9], make_float2(kR2, SIGN * kR2));    // e = 2
  v[13] = cmul(v[13], make_float2(kS1, SIGN * kC1));  // e = 3
  v[6] = cmul(v[6], make_float2(kR2, SIGN * kR2));    // e = 2
  v[10] = mul_i<SIGN>(v[10]);                         // e = 4
  v[14] = cmul(v[14], make_float2(-kR2, SIGN * kR2)); // e = 6
  v[7] = cmul(v[7], make_float2(kS1, SIGN * kC1));    // e = 3
  v[11] = cmul(v[11], make_float2(-kR2, SIGN * kR2)); // e = 6
  v[15] = cmul(v[15], make_float2(-kC1, -SIGN * kS1));// e = 9
  float2 o[16];
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
    float2 b0 = v[4 * n1], b1 = v[4 * n1 + 1], b2 = v[4 * n1 + 2], b3 = v[4 * n1 + 3];
    dft4<SIGN>(b0, b1, b2, b3);
    o[n1] = b0;
    o[n1 + 4] = b1;
    o[n1 + 8] = b2;
    o[n1 + 12] = b3;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = o[i];
}

// Real-input post-processing of a 256-point real FFT computed as a
// 128-point complex FFT Z of z[m] = p[2m] + i p[2m+1]:
//   E = (Z_f + conj Z_g)/2,  O = -i (Z_f - conj Z_g)/2,  g = 128 - f,
//   P_f = E + W^f O,  P_g = conj(E - W^f O),   W = exp(-2 pi i / 256).
// `w` is W^f.  Valid for 1 <= f <= 127 (f = 64 gives P_f = P_g = conj Z_64).
MRA_HD void real_split(float2 zf, float2 zg, float2 w, float2& pf, float2& pg) {
  float2 e = make_float2(0.5f * (zf.x + zg.x), 0.5f * (zf.y - zg.y));
  float2 o = make_float2(0.5f * (zf.y + zg.y), -0.5f * (zf.x - zg.x));
  float2 t = cmul(w, o);
  pf = cadd(e, t);
  pg = cconj(csub(e, t));
}

}  // namespace mra

namespace mra {

// ---------------------------------------------------------------------------
// Forward 256-point real ring FFT with eight cooperating lanes.
//
// z[m] = p[2m] + i p[2m+1] (m = 0..127) is transformed as a 16 x 8
// Cooley-Tukey FFT: lane l (0..7) holds z[8 n1 + l], n1 = 0..15, i.e. the
// samples p[16 n1 + 2 l] and p[16 n1 + 2 l + 1].
//   step 1: Y[l][k1] = DFT16 over n1, times W128^(l k1)
//   (transpose)
//   step 2: Z[k1 + 16 k2] = DFT8 over l of Y[l][k1]
// Lane l then owns the two columns k1 in fwd_cols(l), chosen so that every
// frequency f it holds has its partner 128 - f in the same lane, which makes
// the real-input split (real_split) lane-local.
// ---------------------------------------------------------------------------
MRA_HD void fwd_cols(int l, int& k1a, int& k1b) {
  k1a = l == 0 ? 0 : l;
  k1b = l == 0 ? 8 : 16 - l;
}

// Emit the ring spectrum held by lane l.  Za[k2] = Z[k1a + 16 k2],
// Zb[k2] = Z[k1b + 16 k2]; `w256(f)` returns exp(-2 pi i f / 256).
// emit(slot, a, b) is called once per frequency slot: slot f in 1..127
// receives (Re P_f, Im P_f); slot 0 receives (P_0, P_128), both real.
//
// Every lane runs the same eight steps (lane 0's special bins are patched
// in by selects, so a wave never splits); step k2 emits the slots f and
// 128 - f of one real split:
//   l != 0:  f = l + 16 k2            from (Za[k2], Zb[7 - k2])
//   l == 0:  k2 = 1..3: f = 16 k2     from (Za[k2], Za[8 - k2])
//            k2 = 4..7: f = 16 k2 - 56 from (Zb[k2 - 4], Zb[11 - k2])
//            k2 = 0: slot 0 = (P_0, P_128) = (Re + Im, Re - Im) of Z_0 and
//                    slot 64 = conj Z_64 (f = 64 pairs with itself)
template <class W, class E>
MRA_HD void fwd_emit(int l, const float2 (&Za)[8], const float2 (&Zb)[8], W w256, E emit) {
  const bool z = l == 0;
#pragma unroll
  for (int k2 = 0; k2 < 8; ++k2) {
    float2 x, y;
    int f;
    if (k2 == 0) {
      x = Za[0];
      y = Zb[7];
      f = l;
    } else if (k2 < 4) {
      x = Za[k2];
      y = z ? Za[8 - k2] : Zb[7 - k2];
      f = z ? 16 * k2 : l + 16 * k2;
    } else {
      x = z ? Zb[k2 - 4] : Za[k2];
      y = z ? Zb[11 - k2] : Zb[7 - k2];
      f = z ? 16 * k2 - 56 : l + 16 * k2;
    }
    float2 pf, pg;
    real_split(x, y, w256(f), pf, pg);
    int g = 128 - f;
    if (k2 == 0) {
      pf = z ? make_float2(Za[0].x + Za[0].y, Za[0].x - Za[0].y) : pf;
      pg = z ? make_float2(Za[4].x, -Za[4].y) : pg;
      g = z ? 64 : g;
    }
    emit(f, pf.x, pf.y);
    emit(g, pg.x, pg.y);
  }
}

// The slots fwd_emit hands lane l, in emission order (they depend on l only).
MRA_HD void emit_slots(int l, int (&sl)[16]) {
  const bool z = l == 0;
#pragma unroll
  for (int k2 = 0; k2 < 8; ++k2) {
    const int f = k2 == 0 ? l : (z ? (k2 < 4 ? 16 * k2 : 16 * k2 - 56) : l + 16 * k2);
    sl[2 * k2] = f;
    sl[2 * k2 + 1] = (k2 == 0 && z) ? 64 : 128 - f;
  }
}

// ---------------------------------------------------------------------------
// Inverse transform over angle of the correlation spectra of one
// (row, reference) pair, both mirrors at once.
//
// With P = a + i b the particle ring spectrum and c + i d the weighted,
// normalised reference spectrum at slot f, the matrix cores produce
//   U00 = sum_r (a-b)(c-d),  U01 = sum_r (a-b)(c+d),
//   U11 = sum_r (a+b)(c+d),  U10 = sum_r (a+b)(c-d).
// For 1 <= f <= 127 these are exactly
//   H_f       = G0_f + i G1_f       = U00 + i U01,
//   H_{256-f} = conj G0_f + i conj G1_f = U11 + i U10,
// where G0_f = sum_r w_r conj(P) Q (unmirrored) and G1_f = sum_r w_r P Q
// (mirrored image: its spectrum is conj P).  The inverse DFT of H then
// gives z[a] = c0[a] + i c1[a]: the CC of the unmirrored (real part) and the
// mirrored (imaginary part) particle at every angle a.  Slot 0 packs f = 0
// and f = 128 (a, b, c, d real), for which H_0 = g0 (1 + i) and
// H_128 = g128 (1 + i) with g0 = (U00+U01+U10+U11)/4, g128 = (U00-U01-U10+U11)/4.
//
// The 256-point inverse DFT runs as 16 x 16: pass 1 takes, for each k2, the
// DFT16 over k1 of V[16 k1 + k2] and multiplies output n1 by
// exp(+2 pi i n1 k2 / 256); pass 2 takes, for each n1, the DFT16 over k2 of
// the pass-1 values V[16 n1 + k2], giving z[n1 + 16 n2].
// ---------------------------------------------------------------------------
MRA_HD void slot0_fix(float2& h0, float2& h128) {
  // on entry h0 = (U00, U01), h128 = (U11, U10)
  const float u00 = h0.x, u01 = h0.y, u11 = h128.x, u10 = h128.y;
  const float g0 = 0.25f * ((u00 + u11) + (u01 + u10));
  const float g128 = 0.25f * ((u00 + u11) - (u01 + u10));
  h0 = make_float2(g0, g0);
  h128 = make_float2(g128, g128);
}

// Pass 1 for column k2 (x[k1] = V[16 k1 + k2]); `w256(e)` = exp(-2 pi i e / 256).
template <class W>
MRA_HD void inv_pass1(int k2, float2 (&x)[16], W w256) {
  if (k2 == 0) slot0_fix(x[0], x[8]);
  dft16<+1>(x);
  if (k2 != 0) {
#pragma unroll
    for (int n1 = 1; n1 < 16; ++n1) x[n1] = cmul(x[n1], cconj(w256(n1 * k2)));
  }
}

// Pass 2 for row n1 (x[k2] = V[16 n1 + k2]); afterwards x[n2] = z[n1 + 16 n2].
MRA_HD void inv_pass2(float2 (&x)[16]) { dft16<+1>(x); }

}  // namespace mra
