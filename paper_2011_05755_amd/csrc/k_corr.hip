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
//
// Eight waves: wave w owns slots w, w+8, ..., w+120 in the contraction.  The
// particle operand A of those 16 slots is read from HBM once per workgroup
// and kept in registers (FP32 for R4 <= 9; converted to 16 bits for the
// BF16 / FP16 forms) for all reference tiles; the reference operand B is
// streamed from L2 with a two-slot prefetch.
#include <type_traits>

#include "mra_common.h"
#include "mra_fft.h"

namespace mra {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kCorrWaves = kCorrThreads / 64;
constexpr int kSlotsPerWave = kSlots / kCorrWaves;
constexpr int kMaxResidentR4 = 9;

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

template <int PREC>
struct Op16;
template <>
struct Op16<kBF16> {
  typedef bf16x8 T;
  static __device__ __forceinline__ T cvt(const float (&v)[8]) {
    T r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = (__bf16)v[e];
    return r;
  }
  static __device__ __forceinline__ f32x4 mfma(T a, T b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Op16<kFP16> {
  typedef f16x8 T;
  static __device__ __forceinline__ T cvt(const float (&v)[8]) {
    T r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = (_Float16)v[e];
    return r;
  }
  static __device__ __forceinline__ f32x4 mfma(T a, T b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

// Particle operand of lane ln for slot `slot`: ring g*R4 + t of lane group
// g = ln/16 at element t*16 (A layout [tile][slot][ring][16]).  Rings >= R
// are padding that the polar kernel never writes: callers mask them.
__device__ __forceinline__ const float* a_lane(const CorrArgs& a, int R4, int tile, int slot, int ln) {
  return a.A + (size_t)(tile * kSlots + slot) * 64 * R4 + ((ln >> 4) * R4) * 16 + (ln & 15);
}
__device__ __forceinline__ bool ring_ok(const CorrArgs& a, int R4, int ln, int t) {
  return (ln >> 4) * R4 + t < a.R;
}

// store a 16x16 MFMA block of slot `slot` into the LDS spectrum state
__device__ __forceinline__ void store_block(float* st, int slot, int ln, f32x4 acc) {
  const int p = ln >> 5, q = (ln >> 3) & 1, ref = ln & 7, row0 = ((ln >> 4) & 1) * 4;
#pragma unroll
  for (int i2 = 0; i2 < 4; ++i2) {
    const int P = (row0 + i2) * 8 + ref;
    st[((slot * 2 + p) * 64 + P) * 2 + (q ^ p)] = acc[i2];
  }
}

// Contraction of one reference tile for the wave's 16 slots, FP32 operands.
// RT > 0: compile-time R4 (A resident in registers when RT <= 9);
// RT == 0: runtime R4, A streamed.
template <int RT>
struct Fp32Contract {
  static constexpr bool kResident = RT > 0 && RT <= kMaxResidentR4;
  static constexpr int kR = kResident ? RT : 1;
  float areg[kSlotsPerWave][kR];

  __device__ __forceinline__ void load_a(const CorrArgs& a, int tile, int w, int ln) {
    if (kResident) {
#pragma unroll
      for (int i = 0; i < kSlotsPerWave; ++i) {
        const float* ap = a_lane(a, RT, tile, w + kCorrWaves * i, ln);
#pragma unroll
        for (int t = 0; t < RT; ++t) areg[i][t] = ring_ok(a, RT, ln, t) ? __builtin_nontemporal_load(ap + t * 16) : 0.f;
      }
    }
  }

  __device__ __forceinline__ void run(const CorrArgs& a, float* st, int tile, int kt, int w, int ln) {
    const int R4 = RT > 0 ? RT : a.R4;
    if constexpr (RT > 0) {
      float b[4][RT];
      auto loadb = [&](int i, float (&dst)[RT]) {
        const float* bp = a.B32 + ((size_t)(kt * kSlots + w + kCorrWaves * i) * RT) * 64 + ln;
#pragma unroll
        for (int t = 0; t < RT; ++t) dst[t] = bp[t * 64];
      };
      float av[4][kResident ? 1 : RT];
      auto loada = [&](int i, float (&dst)[kResident ? 1 : RT]) {
        if constexpr (!kResident) {
          const float* ap = a_lane(a, RT, tile, w + kCorrWaves * i, ln);
#pragma unroll
          for (int t = 0; t < RT; ++t) dst[t] = ring_ok(a, RT, ln, t) ? ap[t * 16] : 0.f;
        }
      };
      loadb(0, b[0]);
      loada(0, av[0]);
      loadb(1, b[1]);
      loada(1, av[1]);
#pragma unroll
      for (int i = 0; i < kSlotsPerWave; i += 2) {
        // two independent accumulation chains keep the matrix pipe busy
        f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          const float x0 = kResident ? areg[i][kResident ? t : 0] : av[i % 4][kResident ? 0 : t];
          const float x1 = kResident ? areg[i + 1][kResident ? t : 0] : av[(i + 1) % 4][kResident ? 0 : t];
          acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(x0, b[i % 4][t], acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(x1, b[(i + 1) % 4][t], acc1, 0, 0, 0);
        }
        if (i + 2 < kSlotsPerWave) {
          loadb(i + 2, b[(i + 2) % 4]);
          loada(i + 2, av[(i + 2) % 4]);
        }
        if (i + 3 < kSlotsPerWave) {
          loadb(i + 3, b[(i + 3) % 4]);
          loada(i + 3, av[(i + 3) % 4]);
        }
        store_block(st, w + kCorrWaves * i, ln, acc0);
        store_block(st, w + kCorrWaves * (i + 1), ln, acc1);
      }
    } else {
      for (int i = 0; i < kSlotsPerWave; ++i) {
        const int slot = w + kCorrWaves * i;
        const float* ap = a_lane(a, R4, tile, slot, ln);
        const float* bp = a.B32 + ((size_t)(kt * kSlots + slot) * R4) * 64 + ln;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int t = 0; t < R4; ++t)
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ring_ok(a, R4, ln, t) ? ap[t * 16] : 0.f, bp[t * 64], acc, 0, 0, 0);
        store_block(st, slot, ln, acc);
      }
    }
  }
};

// Contraction with 16-bit operands.  RT > 0: compile-time R4; A is
// converted once (scaled for FP16) and kept packed in registers, two 16-bit
// values per dword, for all reference tiles.  RT == 0: runtime R4, A
// converted per use.  One MFMA step covers 8 rings per lane group.
template <int PREC, int RT>
struct Half16Contract {
  typedef typename Op16<PREC>::T V;
  static constexpr int kNS = RT > 0 ? (RT + 7) / 8 : 1;
  static constexpr int kW = RT > 0 ? (RT + 1) / 2 : 1;   // dwords holding real rings
  u32x4 areg[kSlotsPerWave][kNS];

  static __device__ __forceinline__ uint16_t bits(float x) {
    if constexpr (PREC == kBF16) return __builtin_bit_cast(uint16_t, (__bf16)x);
    else return __builtin_bit_cast(uint16_t, (_Float16)x);
  }

  __device__ __forceinline__ V conv(const CorrArgs& a, int tile, int slot, int s, int ln, float scale) {
    const float* ap = a_lane(a, a.R4, tile, slot, ln);
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int t = 8 * s + e;
      v[e] = (t < a.R4 && ring_ok(a, a.R4, ln, t)) ? ap[t * 16] * scale : 0.f;
    }
    return Op16<PREC>::cvt(v);
  }

  __device__ __forceinline__ void load_a(const CorrArgs& a, int tile, int w, int ln, float scale) {
    if constexpr (RT > 0) {
      // issue the loads of 4 slots before converting any of them, so the
      // memory latency is paid 4 times per workgroup instead of 16
      constexpr int kBatch = RT <= 9 ? 4 : 2;
#pragma unroll
      for (int i0 = 0; i0 < kSlotsPerWave; i0 += kBatch) {
        float v[kBatch][RT];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
          const float* ap = a_lane(a, RT, tile, w + kCorrWaves * (i0 + b), ln);
#pragma unroll
          for (int t = 0; t < RT; ++t) v[b][t] = __builtin_nontemporal_load(ap + t * 16);
        }
#pragma unroll
        for (int b = 0; b < kBatch; ++b)
#pragma unroll
          for (int d = 0; d < 4 * kNS; ++d) {
            const int t0 = 2 * d, t1 = 2 * d + 1;
            const float x0 = (t0 < RT && ring_ok(a, RT, ln, t0)) ? v[b][t0 < RT ? t0 : 0] * scale : 0.f;
            const float x1 = (t1 < RT && ring_ok(a, RT, ln, t1)) ? v[b][t1 < RT ? t1 : 0] * scale : 0.f;
            areg[i0 + b][d / 4][d % 4] = d < kW ? ((uint32_t)bits(x0) | ((uint32_t)bits(x1) << 16)) : 0u;
          }
      }
    }
  }

  __device__ __forceinline__ V operand(int i, int s) const { return __builtin_bit_cast(V, areg[i][s]); }

  __device__ __forceinline__ void run(const CorrArgs& a, float* st, int tile, int kt, int w, int ln, float scale) {
    const uint4* B = reinterpret_cast<const uint4*>(a.B16);
    if constexpr (RT > 0) {
      uint4 b[2][kNS];
      auto loadb = [&](int i, uint4 (&dst)[kNS]) {
        const uint4* bp = B + ((size_t)(kt * kSlots + w + kCorrWaves * i) * kNS) * 64 + ln;
#pragma unroll
        for (int s = 0; s < kNS; ++s) dst[s] = bp[s * 64];
      };
      loadb(0, b[0]);
#pragma unroll
      for (int i = 0; i < kSlotsPerWave; ++i) {
        if (i + 1 < kSlotsPerWave) loadb(i + 1, b[(i + 1) % 2]);
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < kNS; ++s) acc = Op16<PREC>::mfma(operand(i, s), __builtin_bit_cast(V, b[i % 2][s]), acc);
        store_block(st, w + kCorrWaves * i, ln, acc);
      }
    } else {
      for (int i = 0; i < kSlotsPerWave; ++i) {
        const int slot = w + kCorrWaves * i;
        const uint4* bp = B + ((size_t)(kt * kSlots + slot) * a.NS) * 64 + ln;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int s = 0; s < a.NS; ++s)
          acc = Op16<PREC>::mfma(conv(a, tile, slot, s, ln, scale), __builtin_bit_cast(V, bp[s * 64]), acc);
        store_block(st, slot, ln, acc);
      }
    }
  }
};

template <int PREC, int RT, bool TABLE>
__global__ __launch_bounds__(kCorrThreads) void k_corr(CorrArgs a) {
  extern __shared__ float smem[];
  float* st = smem;                                        // [128][2][64][2]
  float2* stc = reinterpret_cast<float2*>(smem);
  float* cand_v = smem + kSlots * 2 * 64 * 2;              // [8 waves][64 pairs]
  int* cand_i = reinterpret_cast<int*>(cand_v + kCorrThreads);
  float* rb_v = reinterpret_cast<float*>(cand_i + kCorrThreads);  // [8 rows]
  int* rb_i = reinterpret_cast<int*>(rb_v + 8);
  float2* tw = reinterpret_cast<float2*>(rb_i + 8);         // exp(-2 pi i e / 256)

  const int tile = blockIdx.x;
  const int tid = threadIdx.x, ln = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (tid < 8) {
    rb_v[tid] = -INFINITY;
    rb_i[tid] = 0x7fffffff;
  }
  if (tid < kNphi) tw[tid] = w256c(a.cs32, tid);

  float a_scale = 1.f, unscale = 1.f;
  if (PREC == kFP16) {
    // power-of-two scale so that |a +- b| <= 2 * 256 * max|pixel| maps below 2^14
    const float m = fmaxf(*a.maxabs * 512.f, 1e-30f);
    const int e = 14 - (int)ceilf(log2f(m));
    a_scale = ldexpf(1.f, e);
    unscale = 1.f / (a_scale * a.b_scale);
  }

  using Contract = typename std::conditional<PREC == kFP32, Fp32Contract<RT>, Half16Contract<PREC == kFP32 ? kBF16 : PREC, RT>>::type;
  Contract con;
  if constexpr (PREC == kFP32) con.load_a(a, tile, w, ln);
  else con.load_a(a, tile, w, ln, a_scale);

  for (int kt = 0; kt < a.n_ref_tiles; ++kt) {
    // ---------------- contraction on the matrix cores ----------------
    if constexpr (PREC == kFP32) con.run(a, st, tile, kt, w, ln);
    else con.run(a, st, tile, kt, w, ln, a_scale);
    __syncthreads();

    // ---------------- inverse FFT over angle, pass 1 ----------------
    const int P = ln;
#pragma unroll 1
    for (int c = 0; c < 16 / kCorrWaves; ++c) {
      const int k2 = w + kCorrWaves * c;
      float2 x[16];
#pragma unroll
      for (int k1 = 0; k1 < 16; ++k1) x[k1] = stc[vidx(16 * k1 + k2, P)];
      inv_pass1(k2, x, [&](int e) { return tw[e & 255]; });
#pragma unroll
      for (int n1 = 0; n1 < 16; ++n1) stc[vidx(16 * n1 + k2, P)] = x[n1];
    }
    __syncthreads();

    // ---------------- pass 2 + arg-max ----------------
    const int row_l = P >> 3, ref_l = P & 7;
    const int row = tile * kRowTile + row_l;
    const int k = kt * kRefTile + ref_l;
    // only values above the row's best of earlier reference tiles can win
    // (a tie with an earlier tile loses: its flat index is smaller)
    const float thr = rb_v[row_l];
    float bv = -INFINITY;
    int bi = 0x7fffffff;
#pragma unroll 1
    for (int c = 0; c < 16 / kCorrWaves; ++c) {
      const int n1 = w + kCorrWaves * c;
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
        float mx = -INFINITY;
#pragma unroll
        for (int n2 = 0; n2 < 16; ++n2) mx = fmaxf(mx, a.M == 2 ? fmaxf(x[n2].x, x[n2].y) : x[n2].x);
        if (mx > thr && mx >= bv) {
#pragma unroll
          for (int n2 = 0; n2 < 16; ++n2) {
            const int ang = n1 + 16 * n2;
            if (better(x[n2].x, ang, bv, bi)) { bv = x[n2].x; bi = ang; }
            if (a.M == 2 && better(x[n2].y, 256 + ang, bv, bi)) { bv = x[n2].y; bi = 256 + ang; }
          }
        }
      }
    }
    if (!TABLE) {
      cand_v[w * 64 + P] = bv;
      cand_i[w * 64 + P] = bi;
    }
    __syncthreads();
    if (!TABLE) {
      // wave r reduces row r: lane = (wave of origin, ref)
      const int r = w;
      const int ww = ln >> 3, ref = ln & 7;
      const int rr = tile * kRowTile + r;
      const int kk = kt * kRefTile + ref;
      float v = cand_v[ww * 64 + r * 8 + ref];
      const int li = cand_i[ww * 64 + r * 8 + ref];
      int iota = 0x7fffffff;
      if (li != 0x7fffffff && kk < a.K && rr < a.rows) {
        const int m = li >> 8, ang = li & 255;
        iota = ((kk * a.M + m) * a.S + rr % a.S) * kNphi + ang;
      } else {
        v = -INFINITY;
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const float v2 = __shfl_xor(v, o);
        const int i2 = __shfl_xor(iota, o);
        if (better(v2, i2, v, iota)) { v = v2; iota = i2; }
      }
      if (ln == 0 && iota != 0x7fffffff && better(v, iota, rb_v[r], rb_i[r])) {
        rb_v[r] = v;
        rb_i[r] = iota;
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

size_t corr_lds_bytes() {
  return (size_t)kSlots * 2 * 64 * 2 * sizeof(float) + 2 * kCorrThreads * sizeof(float) + 16 * sizeof(float) +
         kNphi * sizeof(float2);
}

template <int PREC, int RT, bool TABLE>
static void launch_one(const CorrArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((k_corr<PREC, RT, TABLE>), dim3(a.n_row_tiles), dim3(kCorrThreads), corr_lds_bytes(), st, a);
}

template <int PREC, bool TABLE>
static void dispatch_r4(const CorrArgs& a, hipStream_t st) {
  switch (a.R4) {
#define MRA_CASE(n) case n: launch_one<PREC, n, TABLE>(a, st); break;
    MRA_CASE(1) MRA_CASE(2) MRA_CASE(3) MRA_CASE(4) MRA_CASE(5) MRA_CASE(6) MRA_CASE(7) MRA_CASE(8)
    MRA_CASE(9) MRA_CASE(10) MRA_CASE(11) MRA_CASE(12) MRA_CASE(13) MRA_CASE(14) MRA_CASE(15) MRA_CASE(16)
#undef MRA_CASE
    default: launch_one<PREC, 0, TABLE>(a, st); break;
  }
}

hipError_t launch_corr(int prec, bool table, const CorrArgs& a, hipStream_t st) {
  if (a.n_row_tiles <= 0) return hipSuccess;
  if (table) {
    if (prec == kFP32) launch_one<kFP32, 0, true>(a, st);
    else if (prec == kBF16) launch_one<kBF16, 0, true>(a, st);
    else launch_one<kFP16, 0, true>(a, st);
  } else if (prec == kFP32) {
    dispatch_r4<kFP32, false>(a, st);
  } else if (prec == kBF16) {
    dispatch_r4<kBF16, false>(a, st);
  } else {
    dispatch_r4<kFP16, false>(a, st);
  }
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
