// Ring-weighted correlation of every particle row with every reference
// (Sec. 3: FFT(x)' x FFT(y) per ring, references on a second grid axis,
// inverse FFT of the CC table, arg-max by reduction as in Fig. 2), fused so
// that the CC table is never written to memory.
//
// A workgroup owns 8 particle rows (row = particle * S + shift) and loops
// over all references in tiles of 8.  For each frequency slot f the matrix
// cores compute the 16 x 16 block
//     U[(p,row), (q,ref)] = sum_r A_f[(p,row), r] * B_f[r, (q,ref)],
//     A rows: p = 0 -> a - b, p = 1 -> a + b  (particle spectrum a + ib)
//     B cols: q = 0 -> c - d, q = 1 -> c + d  (reference spectrum c + id,
//             weighted by w_r, divided by the ring norm and by 256)
// whose four entries per (row, ref) are the spectrum H of the complex signal
// c0 + i c1 (unmirrored CC + i * mirrored CC) at f and 256 - f (see
// mra_fft.h).  The 128 slots of all 64 (row, ref) pairs sit in LDS (128 KiB);
// then a 16 x 16 inverse FFT over angle (two passes through LDS) yields the
// CC at all 256 angles for both mirrors, and the running maximum with the
// smallest-flat-index tie rule is kept per row across reference tiles.
#include "mra_common.h"
#include "mra_fft.h"

namespace mra {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float2 w256c(const float2* cs, int e) {
  float2 c = cs[e & 255];
  return make_float2(c.x, -c.y);
}

// logical index j (0..255) of a pair's spectrum -> float2 index in LDS state
__device__ __forceinline__ int vidx(int j, int P) {
  const int slot = j < 128 ? j : ((256 - j) & 127);
  const int half = j < 128 ? 0 : 1;
  return (slot * 2 + half) * 64 + P;
}

__device__ __forceinline__ bool better(float v, int i, float bv, int bi) {
  return v > bv || (v == bv && i < bi);
}

template <int PREC, bool TABLE>
__global__ __launch_bounds__(kCorrThreads) void k_corr(CorrArgs a) {
  extern __shared__ float smem[];
  float* st = smem;                                       // [128][2][64][2]
  float2* stc = reinterpret_cast<float2*>(smem);
  float* cand_v = smem + kSlots * 2 * 64 * 2;             // [4][64]
  int* cand_i = reinterpret_cast<int*>(cand_v + 256);     // [4][64]
  float* rb_v = reinterpret_cast<float*>(cand_i + 256);   // [8]
  int* rb_i = reinterpret_cast<int*>(rb_v + 8);           // [8]

  const int tile = blockIdx.x;
  const int tid = threadIdx.x, w = tid >> 6, ln = tid & 63;
  if (tid < 8) {
    rb_v[tid] = -INFINITY;
    rb_i[tid] = 0x7fffffff;
  }

  float a_scale = 1.f, unscale = 1.f;
  if (PREC == kFP16) {
    // power-of-two scale so that |a +- b| <= 2 * 256 * max|pixel| maps below 2^14
    const float m = fmaxf(*a.maxabs * 512.f, 1e-30f);
    const int e = 14 - (int)ceilf(log2f(m));
    a_scale = ldexpf(1.f, e);
    unscale = 1.f / (a_scale * a.b_scale);
  }

  // output-lane mapping of the 16 x 16 MFMA block
  const int o_p = ln >> 5, o_q = (ln >> 3) & 1, o_ref = ln & 7, o_row0 = ((ln >> 4) & 1) * 4;

  for (int kt = 0; kt < a.n_ref_tiles; ++kt) {
    // ---------------- contraction on the matrix cores ----------------
    for (int i = 0; i < kSlots / 4; ++i) {
      const int slot = w + 4 * i;
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      const float* ap = a.A + ((size_t)(tile * kSlots + slot) * a.R4) * 64 + ln;
      if (PREC == kFP32) {
        const float* bp = a.B32 + ((size_t)(kt * kSlots + slot) * a.R4) * 64 + ln;
        for (int t = 0; t < a.R4; ++t)
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ap[t * 64], bp[t * 64], acc, 0, 0, 0);
      } else {
        const uint4* bp = reinterpret_cast<const uint4*>(a.B16) + ((size_t)(kt * kSlots + slot) * a.NS) * 64 + ln;
        for (int s = 0; s < a.NS; ++s) {
          float av[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int t = 8 * s + e;
            av[e] = t < a.R4 ? ap[t * 64] * a_scale : 0.f;
          }
          const uint4 braw = bp[s * 64];
          if (PREC == kBF16) {
            bf16x8 av16, bv16;
#pragma unroll
            for (int e = 0; e < 8; ++e) av16[e] = (__bf16)av[e];
            __builtin_memcpy(&bv16, &braw, 16);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av16, bv16, acc, 0, 0, 0);
          } else {
            f16x8 av16, bv16;
#pragma unroll
            for (int e = 0; e < 8; ++e) av16[e] = (_Float16)av[e];
            __builtin_memcpy(&bv16, &braw, 16);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(av16, bv16, acc, 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int i2 = 0; i2 < 4; ++i2) {
        const int P = (o_row0 + i2) * 8 + o_ref;
        st[((slot * 2 + o_p) * 64 + P) * 2 + (o_q ^ o_p)] = acc[i2];
      }
    }
    __syncthreads();

    // ---------------- inverse FFT over angle, pass 1 ----------------
    const int P = ln;
    for (int c = 0; c < 4; ++c) {
      const int k2 = w + 4 * c;
      float2 x[16];
#pragma unroll
      for (int k1 = 0; k1 < 16; ++k1) x[k1] = stc[vidx(16 * k1 + k2, P)];
      inv_pass1(k2, x, [&](int e) { return w256c(a.cs32, e); });
#pragma unroll
      for (int n1 = 0; n1 < 16; ++n1) stc[vidx(16 * n1 + k2, P)] = x[n1];
    }
    __syncthreads();

    // ---------------- pass 2 + arg-max ----------------
    const int row_l = P >> 3, ref_l = P & 7;
    const int row = tile * kRowTile + row_l;
    const int k = kt * kRefTile + ref_l;
    float bv = -INFINITY;
    int bi = 0x7fffffff;
    for (int c = 0; c < 4; ++c) {
      const int n1 = w + 4 * c;
      float2 x[16];
#pragma unroll
      for (int k2 = 0; k2 < 16; ++k2) x[k2] = stc[vidx(16 * n1 + k2, P)];
      inv_pass2(x);
      if (TABLE) {
        if (row < a.rows && k < a.K) {
          const int n = row / a.S, s = row - n * a.S;
          for (int m = 0; m < a.M; ++m) {
            float* o = a.table + ((((size_t)n * a.K + k) * a.M + m) * a.S + s) * kNphi;
#pragma unroll
            for (int n2 = 0; n2 < 16; ++n2) o[n1 + 16 * n2] = (m ? x[n2].y : x[n2].x) * unscale;
          }
        }
      } else {
#pragma unroll
        for (int n2 = 0; n2 < 16; ++n2) {
          const int ang = n1 + 16 * n2;
          if (better(x[n2].x, ang, bv, bi)) { bv = x[n2].x; bi = ang; }
          if (a.M == 2 && better(x[n2].y, 256 + ang, bv, bi)) { bv = x[n2].y; bi = 256 + ang; }
        }
      }
    }
    if (!TABLE) {
      cand_v[w * 64 + P] = bv;
      cand_i[w * 64 + P] = bi;
    }
    __syncthreads();
    if (!TABLE && tid < 8) {
      const int r = tile * kRowTile + tid;
      if (r < a.rows) {
        const int s = r % a.S;
        float best = rb_v[tid];
        int besti = rb_i[tid];
        for (int ref = 0; ref < kRefTile; ++ref) {
          const int kk = kt * kRefTile + ref;
          if (kk >= a.K) break;
          for (int ww = 0; ww < 4; ++ww) {
            const float v = cand_v[ww * 64 + tid * 8 + ref];
            const int li = cand_i[ww * 64 + tid * 8 + ref];
            if (li == 0x7fffffff) continue;
            const int m = li >> 8, ang = li & 255;
            const int iota = ((kk * a.M + m) * a.S + s) * kNphi + ang;
            if (better(v, iota, best, besti)) { best = v; besti = iota; }
          }
        }
        rb_v[tid] = best;
        rb_i[tid] = besti;
      }
    }
    __syncthreads();
  }
  if (!TABLE && tid < 8) {
    const int r = tile * kRowTile + tid;
    if (r < a.rows) {
      a.row_cc[r] = rb_v[tid] * unscale;
      a.row_idx[r] = rb_i[tid];
    }
  }
}

hipError_t launch_corr(int prec, bool table, const CorrArgs& a, hipStream_t st) {
  if (a.n_row_tiles <= 0) return hipSuccess;
  const size_t lds = (size_t)kSlots * 2 * 64 * 2 * sizeof(float) + 2 * 256 * sizeof(float) + 16 * sizeof(float);
  dim3 grid(a.n_row_tiles), block(kCorrThreads);
#define MRA_LAUNCH(P, T) hipLaunchKernelGGL((k_corr<P, T>), grid, block, lds, st, a)
  if (table) {
    if (prec == kFP32) MRA_LAUNCH(kFP32, true);
    else if (prec == kBF16) MRA_LAUNCH(kBF16, true);
    else MRA_LAUNCH(kFP16, true);
  } else {
    if (prec == kFP32) MRA_LAUNCH(kFP32, false);
    else if (prec == kBF16) MRA_LAUNCH(kBF16, false);
    else MRA_LAUNCH(kFP16, false);
  }
#undef MRA_LAUNCH
  return hipGetLastError();
}

// Per-particle merge of its S row results (arg-max over shifts with the
// same tie rule) and decoding of the flat index into alignment parameters.
__global__ __launch_bounds__(256) void k_merge(MergeArgs a) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= a.n_part) return;
  float best = -INFINITY;
  int bi = 0x7fffffff;
  for (int s = 0; s < a.S; ++s) {
    const float v = a.row_cc[(size_t)n * a.S + s];
    const int i = a.row_idx[(size_t)n * a.S + s];
    if (better(v, i, best, bi)) { best = v; bi = i; }
  }
  const int64_t o = a.out_off + n;
  if (bi == 0x7fffffff) {  // no ordered candidate (NaN input): report an invalid winner
    a.ref[o] = -1;
    a.mirror[o] = 0;
    a.shift_x[o] = 0;
    a.shift_y[o] = 0;
    a.psi[o] = 0;
    a.cc[o] = NAN;
    if (a.flat) a.flat[o] = -1;
    if (a.cc2) a.cc2[o] = NAN;
    return;
  }
  const int ang = bi & 255;
  int rest = bi >> 8;
  const int s = rest % a.S;
  rest /= a.S;
  const int m = rest % a.M, k = rest / a.M;
  a.ref[o] = k;
  a.mirror[o] = m;
  a.shift_x[o] = s % a.S1 - a.T;
  a.shift_y[o] = s / a.S1 - a.T;
  a.psi[o] = (kNphi - ang) & 255;
  a.cc[o] = best;
  if (a.flat) a.flat[o] = bi;
  if (a.cc2) a.cc2[o] = NAN;
}

hipError_t launch_merge(const MergeArgs& a, hipStream_t st) {
  if (a.n_part <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_merge, dim3((a.n_part + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace mra
