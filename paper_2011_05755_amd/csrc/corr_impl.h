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
// NW waves (8, or 4 in one FP32 variant): wave w owns slots w, w+NW, ... in
// the contraction.  In the resident variants the particle operand A of
// those slots is read from HBM once per row tile and kept in registers (FP32:
// R4 <= 9 with 8 waves, R4 <= 12 with 4 waves; packed 16-bit for the BF16 /
// FP16 forms) for all reference tiles; the streamed variants re-read it per
// reference tile.  The reference operand B is streamed from L2 with a slot
// prefetch.  Variants are tile configurations that an autotuner chooses
// between; they do not change any result.
#pragma once
#include <type_traits>

#include "mra_common.h"
#include "mra_fft.h"

namespace mra {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

constexpr int kMaxBatch = kMaxBatchPieces;

__device__ __forceinline__ float2 w256c(const float2* cs, int e) {
  float2 c = cs[e & 255];
  return make_float2(c.x, -c.y);
}

__device__ __forceinline__ bool better(float v, int i, float bv, int bi) {
  return v > bv || (v == bv && i < bi);
}

template <int PREC>
struct Op16;
template <>
struct Op16<kBF16> {
  typedef bf16x8 T;
  static __device__ __forceinline__ uint16_t bits(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
  static __device__ __forceinline__ f32x4 mfma(T a, T b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Op16<kFP16> {
  typedef f16x8 T;
  static __device__ __forceinline__ uint16_t bits(float x) { return __builtin_bit_cast(uint16_t, (_Float16)x); }
  static __device__ __forceinline__ f32x4 mfma(T a, T b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

// Order of the 16 x 16 matrix-core block.  Its rows are (row, p) and its
// columns (ref, q), interleaved: block row 2 row + p, block column 2 ref + q.
// The reference operand is packed in that column order; the particle
// operand is stored with position p * 8 + row, which block row j reads
// through a_block_pos(j).  Lane ln then holds column 2 ref + q = ln & 15 for the
// rows 2 (ln / 16) and 2 (ln / 16) + 1, both p: the four entries U_pq of a
// (row, ref) pair sit in two neighbouring lanes (q = 0, 1).
__device__ __forceinline__ int a_block_pos(int j) { return (j & 1) * 8 + (j >> 1); }
// The (row, ref) pair that lane ln gathers, as row * 8 + ref: row
// 2 (ln / 16) + q, ref (ln / 2) & 7, q = ln & 1.
__device__ __forceinline__ int lane_pair(int ln) { return (2 * (ln >> 4) + (ln & 1)) * 8 + ((ln >> 1) & 7); }

// Particle operand of lane ln for slot `slot`: ring g*R4 + t of lane group
// g = ln/16 at element t * ring_stride(LAYOUT) (kRingMajor or kSlotMajor,
// fixed per contraction form; the host has the resampler write the same
// one; kRingPerm is read two slots at a time with a_pair).  Rings >= R are
// padding that the polar kernel never writes: callers mask them.
// RX > 0: R4 == RX is known at compile time.
constexpr int ring_stride(int layout) { return layout == kSlotMajor ? 16 : kSlots * 16; }
template <int LAYOUT, int RX = 0>
__device__ __forceinline__ const float* a_lane(const CorrArgs& a, int tile, int slot, int ln) {
  static_assert(LAYOUT != kRingPerm, "the paired layout is read with a_pair");
  const int R4 = RX > 0 ? RX : a.R4;
  if constexpr (LAYOUT == kSlotMajor)
    return a.A + (size_t)(tile * kSlots + slot) * 64 * R4 + ((ln >> 4) * R4) * 16 + a_block_pos(ln & 15);
  return a.A + ((size_t)(tile * 4 + (ln >> 4)) * R4 * kSlots + slot) * 16 + a_block_pos(ln & 15);
}
// Element t of the lane's operand: ring (ln/16)*R4 + t.  The load is never
// conditional (a conditional load waits for its data before the next one is
// issued): its element index is clamped into the slot's block, and elements
// t >= R4 and padding rings >= R (which hold no data) are cleared by an AND
// with a mask that is opaque to the optimiser, which would otherwise turn
// the select back into a branch around the load.
template <int LAYOUT, int RX = 0>
__device__ __forceinline__ float a_elem(const CorrArgs& a, const float* ap, int ln, int t, bool nt) {
  const int R4 = RX > 0 ? RX : a.R4;
  const int tt = t < R4 ? t : R4 - 1;
  const float x = nt ? __builtin_nontemporal_load(ap + tt * ring_stride(LAYOUT)) : ap[tt * ring_stride(LAYOUT)];
  uint32_t keep = (t < R4 && (ln >> 4) * R4 + t < a.R) ? 0xffffffffu : 0u;
  asm("" : "+v"(keep));
  return __uint_as_float(__float_as_uint(x) & keep);
}

// Elements t of two slots at once in the permuted layout (kRingPerm): ap
// points at element 0 of the lane's pair block; masks as in a_elem.
typedef float f32x2 __attribute__((ext_vector_type(2)));
template <int RX = 0>
__device__ __forceinline__ f32x2 a_pair(const CorrArgs& a, const float* ap, int ln, int t) {
  const int R4 = RX > 0 ? RX : a.R4;
  const int tt = t < R4 ? t : R4 - 1;
  const f32x2 x = __builtin_nontemporal_load(reinterpret_cast<const f32x2*>(ap + tt * kSlots * 16));
  uint32_t keep = (t < R4 && (ln >> 4) * R4 + t < a.R) ? 0xffffffffu : 0u;
  asm("" : "+v"(keep));
  f32x2 r;
  r.x = __uint_as_float(__float_as_uint(x.x) & keep);
  r.y = __uint_as_float(__float_as_uint(x.y) & keep);
  return r;
}

// Frequency slots below kLowSlots enter the pruning bound with their exact
// magnitudes, the others through their summed energy.
constexpr int kLowSlots = 32;

// swap the values of neighbouring lanes (DPP quad_perm [1, 0, 3, 2]; every
// lane is enabled, so no old value is needed)
__device__ __forceinline__ float swap_adjacent(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xb1, 0xf, 0xf, false));
}

// Block of slot `slot` -> the lane's pair (lane_pair(ln) = P): the four
// entries U_pq gathered with one exchange between the two lanes of the
// pair, stored as the state halves (U00, U01) and (U11, U10), and added to
// the pair's pruning bound: a slot below kLowSlots (low) with the exact
// magnitudes of its two spectrum values per mirror, a slot above through
// its energy, the sum of the squares.
__device__ __forceinline__ void pair_block(float2* stc, int slot, int ln, int P, f32x4 acc, bool low, float& b0,
                                           float& b1, float& en) {
  const bool q = ln & 1;
  // lane q = 0 holds (row 2g: U00, U10; row 2g + 1: U00, U10), lane q = 1
  // the same rows' U01, U11; each sends the entries of the other's row
  const float r0 = swap_adjacent(q ? acc[0] : acc[2]), r1 = swap_adjacent(q ? acc[1] : acc[3]);
  const float u00 = q ? r0 : acc[0], u01 = q ? acc[2] : r0;
  const float u10 = q ? r1 : acc[1], u11 = q ? acc[3] : r1;
  stc[(slot * 2) * 64 + P] = make_float2(u00, u01);
  stc[(slot * 2 + 1) * 64 + P] = make_float2(u11, u10);
  const float s1 = u00 + u11, d1 = u00 - u11, s2 = u01 + u10, d2 = u01 - u10;
  if (low) {
    if (slot == 0) {  // |g_0| + |g_128|, the same for both mirrors
      const float g = 0.25f * (fabsf(s1 + s2) + fabsf(s1 - s2));
      b0 += g;
      b1 += g;
    } else {          // 2|G_0,f| = |(s1, d2)|, 2|G_1,f| = |(s2, d1)|
      b0 += sqrtf(s1 * s1 + d2 * d2);
      b1 += sqrtf(s2 * s2 + d1 * d1);
    }
  } else {
    en = fmaf(u00, u00, fmaf(u01, u01, fmaf(u10, u10, fmaf(u11, u11, en))));
  }
}

// Contraction of one reference tile with FP32 operands for the wave's
// 128/NW slots (slot = w + NW*i).  EXACT: R4 == MAXR, else R4 <= MAXR at
// run time (mixed ring counts in one batched launch).  RES: the
// particle operand of all the wave's slots is loaded once per row tile and
// kept in registers for every reference tile; otherwise it is streamed with
// the reference operand.  Operands of the next two slots are prefetched.
template <int NW, int MAXR, bool RES, bool EXACT>
struct Fp32Contract {
  static constexpr int SPW = kSlots / NW;
  static constexpr int RX = EXACT ? MAXR : 0;
  static constexpr int LAYOUT = (NW == 8 && RES) ? kRingPerm : kSlotMajor;
  float areg[RES ? SPW : 1][RES ? MAXR : 1];
  float bound0, bound1, energy;  // the lane's pair's pruning bound terms (pair_block)

  // the lane's reference operand of slot `slot` in reference tile kt
  __device__ __forceinline__ void load_b(const CorrArgs& a, int kt, int slot, int ln, float (&dst)[MAXR]) const {
    const int R4 = EXACT ? MAXR : a.R4;
    const float* bp = a.B32 + ((size_t)(kt * kSlots + slot) * R4) * 64 + ln;
#pragma unroll
    for (int t = 0; t < MAXR; ++t) dst[t] = bp[(t < R4 ? t : R4 - 1) * 64];  // unconditional
  }
  // PRE (8 waves, resident operand, ring count exact): the reference
  // operand of the wave's first slot of reference tile kt is loaded before
  // the inverse FFT of the previous tile, so its latency passes under it
  // (one slot: the registers of two would spill in these forms)
  static constexpr bool PRE = RES && NW == 8 && EXACT;
  float bpre[PRE ? MAXR : 1];
  __device__ __forceinline__ void prefetch(const CorrArgs& a, int kt, int w, int ln) {
    if constexpr (PRE) load_b(a, kt, w, ln, bpre);
  }

  __device__ __forceinline__ void load_a(const CorrArgs& a, int tile, int w, int ln) {
    if constexpr (RES) {
      if constexpr (LAYOUT == kRingPerm) {
        // the wave's slots w + 8 i sit at positions 16 w + i, in pairs
        // (i even, i + 1) interleaved by element: one base address, constant
        // offsets, one 8-byte load for two slots
        const int R4 = RX > 0 ? RX : a.R4;
        const float* a0 = a.A + ((size_t)(tile * 4 + (ln >> 4)) * R4 * kSlots + 16 * w) * 16 + 2 * a_block_pos(ln & 15);
#pragma unroll
        for (int i2 = 0; i2 < SPW / 2; ++i2) {
#pragma unroll
          for (int t = 0; t < MAXR; ++t) {
            const f32x2 v = a_pair<RX>(a, a0 + 32 * i2, ln, t);
            areg[2 * i2][t] = v.x;
            areg[2 * i2 + 1][t] = v.y;
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < SPW; ++i) {
          const float* ap = a_lane<LAYOUT, RX>(a, tile, w + NW * i, ln);
#pragma unroll
          for (int t = 0; t < MAXR; ++t) areg[i][t] = a_elem<LAYOUT, RX>(a, ap, ln, t, true);
        }
      }
    }
  }

  __device__ __forceinline__ void run(const CorrArgs& a, float2* stc, int tile, int kt, int w, int ln) {
    const int R4 = EXACT ? MAXR : a.R4;
    const int P = lane_pair(ln);
    bound0 = bound1 = energy = 0.f;
    auto loadb = [&](int i, float (&dst)[MAXR]) { load_b(a, kt, w + NW * i, ln, dst); };
    if constexpr (RES) {
      // slots in pairs: two independent accumulation chains keep the matrix
      // pipe busy; the reference operand of the next pair is in flight
      float b[4][MAXR];
      if constexpr (PRE) {
#pragma unroll
        for (int t = 0; t < MAXR; ++t) b[0][t] = bpre[t];
      } else {
        loadb(0, b[0]);
      }
      loadb(1, b[1]);
#pragma unroll
      for (int i = 0; i < SPW; i += 2) {
        f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < MAXR; ++t) {
          if (t < R4) {
            acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(areg[i][t], b[i % 4][t], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(areg[i + 1][t], b[(i + 1) % 4][t], acc1, 0, 0, 0);
          }
        }
        if (i + 2 < SPW) loadb(i + 2, b[(i + 2) % 4]);
        if (i + 3 < SPW) loadb(i + 3, b[(i + 3) % 4]);
        pair_block(stc, w + NW * i, ln, P, acc0, i < kLowSlots / NW, bound0, bound1, energy);
        pair_block(stc, w + NW * (i + 1), ln, P, acc1, i + 1 < kLowSlots / NW, bound0, bound1, energy);
      }
    } else {
      // both operands streamed, one slot ahead (explicit double buffer so
      // that the slot loop need not be unrolled)
      float b0[MAXR], a0[MAXR], b1[MAXR], a1[MAXR];
      auto loada = [&](int i, float (&dst)[MAXR]) {
        const float* ap = a_lane<LAYOUT, RX>(a, tile, w + NW * i, ln);
#pragma unroll
        for (int t = 0; t < MAXR; ++t) dst[t] = a_elem<LAYOUT, RX>(a, ap, ln, t, false);
      };
      auto chain = [&](const float (&x)[MAXR], const float (&y)[MAXR], int slot) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < MAXR; ++t)
          if (t < R4) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x[t], y[t], acc, 0, 0, 0);
        pair_block(stc, slot, ln, P, acc, slot < kLowSlots, bound0, bound1, energy);
      };
      loadb(0, b0);
      loada(0, a0);
#pragma unroll 1
      for (int i = 0; i < SPW; i += 2) {
        loadb(i + 1, b1);
        loada(i + 1, a1);
        chain(a0, b0, w + NW * i);
        if (i + 2 < SPW) {
          loadb(i + 2, b0);
          loada(i + 2, a0);
        }
        chain(a1, b1, w + NW * (i + 1));
      }
    }
  }
};

// Contraction with 16-bit operands; NS = ceil(MAXR / 8) <= 2 steps of 8
// rings per lane group, R4 <= MAXR (EXACT: every work item's R4 lies in the
// bucket MAXR - 3 .. MAXR, or 1 .. 8 for MAXR = 8: ceil(R4 / 8) == NS, and at
// MAXR = 16 the reference operand's last step is 8 wide).  With MAXR = 12 the second step holds at most 4 rings
// per lane group (NARROW): the resident particle operand keeps 2 dwords of it
// per slot instead of 4.  The particle operand
// arrives rounded to the contraction's type (FP16 already scaled per
// particle) in the 16-bit ring-major layout.  RES: it is read once per row
// tile and kept packed in registers, two values per dword; otherwise it is
// re-read per reference tile, one slot ahead.  The reference operand's last
// step is stored as wide as its rings need (b16_tail_width) and read with
// dword loads of that width.
template <int PREC, int NW, int MAXR, bool EXACT, bool RES>
struct Half16Contract {
  static constexpr int SPW = kSlots / NW;
  static constexpr int NS = (MAXR + 7) / 8;
  static_assert(NS <= 2, "at most two steps of 8 rings per lane group");
  static constexpr bool NARROW = NS == 2 && MAXR - 8 <= 4;
  static constexpr int NF = NARROW ? 1 : NS;  // steps held 8 wide
  typedef typename Op16<PREC>::T V;
  // one slot's operand of the lane: the steps held 8 wide, then (NARROW) the
  // last step's 4 elements
  struct Frag {
    u32x4 f[NF];
    u32x2 t;
  };
  Frag areg[RES ? SPW : 1];
  float bound0, bound1, energy;  // the lane's pair's pruning bound terms (pair_block)
  Frag bpre;                     // RES: reference operand of the wave's first slot, loaded ahead

  // Element t (ring (ln/16) R4 + t) of the lane's row for each t < MAXR is
  // read unconditionally: the index is clamped into the row tile's rings,
  // and elements t >= R4 and padding rings >= R are cleared by an AND with a
  // mask the optimiser cannot see through.
  __device__ __forceinline__ uint32_t keep_mask(const CorrArgs& a, int t, int ln) const {
    uint32_t keep = (t < a.R4 && (ln >> 4) * a.R4 + t < a.R) ? ~0u : 0u;
    asm("" : "+v"(keep));
    return keep;
  }
  __device__ __forceinline__ const uint16_t* ring_block(const CorrArgs& a, int tile, int t, int ln) const {
    const int tt = t < a.R4 ? t : a.R4 - 1;
    return reinterpret_cast<const uint16_t*>(a.A) + ((size_t)(tile * 4 + (ln >> 4)) * a.R4 + tt) * kSlots * 16;
  }
  // Two 16-bit values as the contraction's dword: x's and y's element j of
  // their 8 (v_perm byte selection)
  static __device__ __forceinline__ uint32_t pick2(uint32_t x, uint32_t y, int odd) {
    return __builtin_amdgcn_perm(y, x, odd ? 0x07060302u : 0x05040100u);
  }

  // The lane's operand of slot `slot` (streamed variant): one 2-byte load
  // per element.
  __device__ __forceinline__ void fetch(const CorrArgs& a, int tile, int slot, int ln, Frag& dst, bool nt) {
    const int idx = a16_index(slot_pos(slot), a_block_pos(ln & 15));
    uint32_t v[8 * NS];
#pragma unroll
    for (int t = 0; t < 8 * NS; ++t) {
      if (t < MAXR) {
        const uint16_t* bp = ring_block(a, tile, t, ln) + idx;
        const uint32_t x = nt ? (uint32_t)__builtin_nontemporal_load(bp) : (uint32_t)*bp;
        v[t] = x & keep_mask(a, t, ln);
      } else {
        v[t] = 0u;
      }
    }
#pragma unroll
    for (int d = 0; d < 4 * NF; ++d) dst.f[d / 4][d % 4] = v[2 * d] | (v[2 * d + 1] << 16);
    if constexpr (NARROW) {
      dst.t[0] = v[8] | (v[9] << 16);
      dst.t[1] = v[10] | (v[11] << 16);
    }
  }

  // RES: the operand of all the wave's slots w + 8 i.  Per element t, two
  // 16-byte loads (the interleaved runs 2 w and 2 w + 1) give slots i < 8
  // and i >= 8; the dwords are then regrouped per slot.
  __device__ __forceinline__ void load_a(const CorrArgs& a, int tile, int w, int ln) {
    if constexpr (RES) {
      static_assert(NW == 8, "the interleaved runs hold 8 slots of each of 8 waves");
      const int k = a_block_pos(ln & 15);
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        u32x4 u[8 * NS];
#pragma unroll
        for (int t = 0; t < 8 * NS; ++t) {
          if (t < MAXR) {
            const u32x4* bp = reinterpret_cast<const u32x4*>(ring_block(a, tile, t, ln) + a16_index(16 * w + 8 * hh, k));
            u[t] = __builtin_nontemporal_load(bp) & keep_mask(a, t, ln);
          } else {
            u[t] = u32x4{0u, 0u, 0u, 0u};
          }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          Frag& f = areg[8 * hh + j];
#pragma unroll
          for (int d = 0; d < 4 * NF; ++d) f.f[d / 4][d % 4] = pick2(u[2 * d][j >> 1], u[2 * d + 1][j >> 1], j & 1);
          if constexpr (NARROW) {
            f.t[0] = pick2(u[8][j >> 1], u[9][j >> 1], j & 1);
            f.t[1] = pick2(u[10][j >> 1], u[11][j >> 1], j & 1);
          }
        }
      }
    }
  }

  // the lane's reference operand of slot `slot` in reference tile kt.  Last-step
  // dword j of the lane is read at index min(j, h - 1): a dword j >= h
  // repeats stored values, which meet the particle operand's elements t >=
  // R4, all zero, so it adds exact zeros (every stored value is finite).
  // With ns == 1 the last-step address is step 0's, read and unused.
  __device__ __forceinline__ void load_b(const CorrArgs& a, int kt, int slot, int ln, Frag& dst) const {
    const int ns = EXACT ? NS : a.NS;
    const int bt = a.BT;                          // last step: bt elements per lane
    const int se = (ns - 1) * 512 + 64 * bt;      // elements per slot block
    const int h = bt / 2;                         // dwords per lane in the last step
    const uint16_t* bp = a.B16 + (size_t)(kt * kSlots + slot) * se;
    dst.f[0] = *reinterpret_cast<const u32x4*>(bp + ln * 8);  // step 0 is always 8 wide
    if constexpr (NS == 2) {
      const uint32_t* tp = reinterpret_cast<const uint32_t*>(bp + (ns - 1) * 512 + ln * bt);
      if constexpr (NARROW) {
#pragma unroll
        for (int j = 0; j < 2; ++j) dst.t[j] = tp[j < h ? j : h - 1];
      } else if constexpr (EXACT) {
        dst.f[1] = *reinterpret_cast<const u32x4*>(tp);  // 8 wide: one 16-byte load
      } else {
        // (four 4-byte loads cost the address path four times one 16-byte
        // load: batched launches keep the ring buckets apart to avoid this)
#pragma unroll
        for (int j = 0; j < 4; ++j) dst.f[1][j] = tp[j < h ? j : h - 1];
      }
    }
  }
  // RES: start loading the first slot of reference tile kt, which the next
  // run() uses (its latency then passes during the inverse FFT)
  __device__ __forceinline__ void prefetch(const CorrArgs& a, int kt, int w, int ln) {
    if constexpr (RES) load_b(a, kt, w, ln, bpre);
  }

  __device__ __forceinline__ void run(const CorrArgs& a, float2* stc, int tile, int kt, int w, int ln) {
    const int ns = EXACT ? NS : a.NS;
    const int P = lane_pair(ln);
    bound0 = bound1 = energy = 0.f;
    auto loadb = [&](int i, Frag& dst) { load_b(a, kt, w + NW * i, ln, dst); };
    auto chain = [&](const Frag& x, const Frag& y, int slot, bool low) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < NF; ++s)
        if (s < ns) acc = Op16<PREC>::mfma(__builtin_bit_cast(V, x.f[s]), __builtin_bit_cast(V, y.f[s]), acc);
      if constexpr (NARROW) {
        // the last step is a K = 32 product with elements 4..7 zero: a K = 16
        // product accumulated straight onto the K = 32 one's result gave
        // wrong sums on gfx950 when the two issued back to back
        const u32x4 xa = {x.t[0], x.t[1], 0u, 0u}, yb = {y.t[0], y.t[1], 0u, 0u};
        if (ns == NS) acc = Op16<PREC>::mfma(__builtin_bit_cast(V, xa), __builtin_bit_cast(V, yb), acc);
      }
      pair_block(stc, slot, ln, P, acc, low, bound0, bound1, energy);
    };
    if constexpr (RES) {
      Frag b[2];
      b[0] = bpre;
#pragma unroll
      for (int i = 0; i < SPW; ++i) {
        if (i + 1 < SPW) loadb(i + 1, b[(i + 1) % 2]);
        chain(areg[RES ? i : 0], b[i % 2], w + NW * i, i < kLowSlots / NW);
        // keep each slot's store next to its products (a schedule that
        // defers them all holds 16 blocks of results and runs slower)
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
      // explicit double buffer so that the slot loop need not be unrolled
      Frag b0, b1, x0, x1;
      loadb(0, b0);
      fetch(a, tile, w, ln, x0, false);
#pragma unroll 1
      for (int i = 0; i < SPW; i += 2) {
        loadb(i + 1, b1);
        fetch(a, tile, w + NW * (i + 1), ln, x1, false);
        chain(x0, b0, w + NW * i, i < kLowSlots / NW);
        if (i + 2 < SPW) {
          loadb(i + 2, b0);
          fetch(a, tile, w + NW * (i + 2), ln, x0, false);
        }
        chain(x1, b1, w + NW * (i + 1), i + 1 < kLowSlots / NW);
      }
    }
  }
};

template <int NW>
struct CorrSmem {
  float* st;                // [128][2][64][2] spectra of the 64 (row, ref) pairs
  float2* stc;
  unsigned long long* key;  // [8] best candidate of each row so far (ordered key, 0 = none)
  float4* pp;               // [2][NW][64] per (reference-tile parity, wave, pair): low-slot bound of
                            // both mirrors, high-slot energy, unused
  int* list;                // [NW][64] each wave's list of the pairs that need the inverse FFT
  float* thr;               // [8] each row's best before this reference tile's inverse FFT
  float* pt;                // [8] best over the rows of the row's particle (this tile and carried)
  int* ppart;               // [8] particle of each row slot (-1 past the chunk)
  float* carry_v;           // best of the particle that the run's next tile may continue
  int* carry_p;             // that particle (-1: none)
  float2* tw;               // exp(-2 pi i e / 256)
  __device__ __forceinline__ CorrSmem(float* smem) {
    st = smem;
    stc = reinterpret_cast<float2*>(smem);
    key = reinterpret_cast<unsigned long long*>(smem + kSlots * 2 * 64 * 2);
    pp = reinterpret_cast<float4*>(key + 8);
    list = reinterpret_cast<int*>(pp + 2 * NW * 64);
    thr = reinterpret_cast<float*>(list + NW * 64);
    pt = thr + 8;
    ppart = reinterpret_cast<int*>(pt + 8);
    carry_v = reinterpret_cast<float*>(ppart + 8);
    carry_p = reinterpret_cast<int*>(carry_v + 2);
    tw = reinterpret_cast<float2*>(carry_p + 2);
  }
  static constexpr size_t bytes() {
    return (size_t)kSlots * 2 * 64 * 2 * sizeof(float) + 8 * sizeof(unsigned long long) +
           2 * NW * 64 * sizeof(float4) + NW * 64 * sizeof(int) +
           8 * sizeof(float) * 2 + 8 * sizeof(int) + 2 * sizeof(float) + 2 * sizeof(int) + kNphi * sizeof(float2);
  }
};

__device__ __forceinline__ void lds_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A candidate (CC value v, flat index iota < 2^31 - 1) as one 64-bit key whose
// unsigned order is the arg-max order: larger v first, then smaller iota.  0
// is below every candidate.
__device__ __forceinline__ unsigned long long cand_key(float v, int iota) {
  const uint32_t u = __float_as_uint(v == 0.f ? 0.f : v);  // -0 ties with +0, as in the float order
  const uint32_t o = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return ((unsigned long long)o << 32) | (unsigned long long)(0x7fffffffu - (uint32_t)iota);
}
__device__ __forceinline__ float key_value(unsigned long long k) {
  if (k == 0ull) return -INFINITY;
  const uint32_t o = (uint32_t)(k >> 32);
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}
__device__ __forceinline__ int key_index(unsigned long long k) {
  return k == 0ull ? 0x7fffffff : (int)(0x7fffffffu - (uint32_t)k);
}

// The pruning threshold a particle's best so far imposes on its rows: the
// best itself, or (re-ranked 16-bit forms) margin * |best| below it, so that
// every row within that margin of the particle's best keeps its exact best.
__device__ __forceinline__ float part_thr(float best, float margin) {
  return (margin > 0.f && best > -INFINITY) ? best - margin * fabsf(best) : best;
}

// Power-of-two FP16 scale of chunk row r: |a +- b| <= 2 * 256 * max|pixel|
// of the row's particle is mapped below 2^14.
__device__ __forceinline__ float fp16_scale(const CorrArgs& a, int r) {
  return r >= a.rows ? 1.f : fp16_operand_scale(a.maxabs[r / a.S]);
}

// What a tile computes: the per-row arg-max, the full CC table (debug), or
// the arg-max with one candidate per particle left out (the runner-up pass).
constexpr int kArgmax = 0, kTable = 1, kRunnerUp = 2;

// One 8-row tile against every reference tile (see the file comment).
//
// Exact pruning (a.prune, not in table mode): after the contraction of a
// reference tile, every (row, ref) pair gets an upper bound of its CC over
// all angles, per mirror m,
//   c_m[a] <= |g_0| + |g_128| + sum_{f=1}^{127} 2 |G_m,f|,
// with the terms of slots below kLowSlots taken exactly from the spectra and
// the rest bounded by Cauchy-Schwarz through the pairs' high-slot energy
// (sum of 2|G_m,f| <= sqrt(2 * 96 * sum of the squared MFMA entries)).  A pair
// whose bound, inflated by 2^-12 against rounding, is below the threshold of
// its row cannot matter, so its inverse FFT and arg-max are skipped.  The
// threshold is the larger of the row's own best over earlier reference tiles
// (a tie with it loses on the flat index) and the best over every row of the
// same particle seen so far, in this tile and in the earlier tiles of the
// workgroup's run (part_thr: minus a.margin of it for the re-ranked 16-bit
// forms).  A row's reported best is exact whenever it reaches that particle
// threshold, so the particle's winner (and, with a margin, every row the
// re-ranking considers) is the same with and without pruning.  Most pairs of
// a particle's later tiles fall below it, and a reference tile with no live
// pair skips the inverse FFT and its barriers altogether.
template <int PREC, int NW, class Contract, int MODE, bool SPLIT>
__device__ __forceinline__ void corr_tile(const CorrArgs& a, int tile, const CorrSmem<NW>& sm, Contract& con) {
  constexpr int CPW = 16 / NW;  // inverse-FFT columns (pass 1) and rows (pass 2) per wave
  // the lane index is opaque in every tile, so that nothing derived from it
  // is hoisted out of the run's tile loop and kept live across it
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int ln = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (tid < 8) {
    const int row = tile * kRowTile + tid;
    const int part = row < a.rows ? row / a.S : -1;
    sm.key[tid] = 0ull;
    sm.ppart[tid] = part;
    sm.pt[tid] = (part >= 0 && part == *sm.carry_p) ? *sm.carry_v : -INFINITY;
  }
  // (FP16: each particle's operand rows come scaled by a power of two of its
  // own, exact, so results do not depend on how particles are grouped)
  con.load_a(a, tile, w, ln);
  int* list = sm.list + w * 64;
  // Pruning (not in table mode, and not with 4 waves, whose registers are
  // full with the resident operand) stops for the rest of the row tile when a
  // reference tile after the second still leaves more than 56 of its 64 pairs
  // live: the bound then costs more than it saves (references that are
  // themselves noisy images).
  bool prune = MODE != kTable && NW == 8 && a.prune;

  for (int kt = 0; kt < a.n_ref_tiles; ++kt) {
    const int par = kt & 1;  // energy and bound partials alternate, so a wave may write the next
                             // tile's while another still reads this one's
    // ---------------- contraction on the matrix cores ----------------
    con.run(a, sm.stc, tile, kt, w, ln);
    // the next reference tile's first operand (tile 0 again after the last:
    // the run's next row tile starts there)
    con.prefetch(a, kt + 1 < a.n_ref_tiles ? kt + 1 : 0, w, ln);
    // the wave's share of each pair's bound (its slots' terms, gathered in
    // the contraction by the pair's lanes)
    if (prune) sm.pp[(par * NW + w) * 64 + lane_pair(ln)] = make_float4(con.bound0, con.bound1, con.energy, 0.f);
    __syncthreads();
    // each row's best before this tile's candidates arrive: candidates of this
    // tile are recorded only above it (equal values of earlier tiles have
    // smaller flat indices)
    if (MODE != kTable && tid < 8) sm.thr[tid] = key_value(sm.key[tid]);

    // ---------------- which pairs need the inverse FFT ----------------
    uint64_t live = ~0ull;
    if (prune) {
      // (the lane index made opaque again, so that the addresses below are
      // computed here rather than kept live across the contraction)
      int P = ln;
      asm volatile("" : "+v"(P));
      float B0 = 0.f, B1 = 0.f, E = 0.f;
#pragma unroll
      for (int w2 = 0; w2 < NW; ++w2) {
        const float4 b = sm.pp[(par * NW + w2) * 64 + P];
        B0 += b.x;
        B1 += b.y;
        E += b.z;
      }
      const float bound = (a.M == 2 ? fmaxf(B0, B1) : B0) + sqrtf(2.f * (kSlots - kLowSlots) * E);
      const int row_l = P >> 3, ref_l = P & 7;
      const float thr = fmaxf(key_value(sm.key[row_l]), part_thr(sm.pt[row_l], a.margin));
      const bool keep = tile * kRowTile + row_l < a.rows && kt * kRefTile + ref_l < a.K &&
                        !(bound * (1.f + 1.f / 4096.f) < thr);
      live = __ballot(keep);
    }
    const int n_live = __popcll(live);
    if (prune && kt >= 2 && n_live > 56) prune = false;  // wave-uniform
    if (n_live == 0) continue;  // workgroup-uniform: every wave read the same partials
    {
      const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(live >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)live, 0));
      if ((live >> ln) & 1) list[rank] = ln;
      lds_wave_sync();
    }
    // The inverse FFT of the live pairs.  With CPWX columns (pass 1) and
    // rows (pass 2) per wave, the working waves' columns / rows are
    // CPWX * w + c, c = 0 .. CPWX-1: lane group c (LPCX lanes) takes column /
    // row c for the live pairs list[n0 + ln % LPCX].  The first waves hold
    // rows below 8 and the others rows from 8 on, so that every wave's
    // pass-2 addresses share one shape (a lane base plus constant offsets).
    // At most 16 live pairs (most reference tiles) fit 4 columns of 16
    // lanes per wave: then waves 0..3 (one per SIMD) do the passes and the
    // others wait at the barriers, so each SIMD issues one wave's
    // instructions instead of two.
    auto passes = [&](auto cpw_c) {
      constexpr int CPWX = decltype(cpw_c)::value, LPCX = 64 / CPWX;
      const bool work = CPWX * w < 16;  // wave-uniform

      // ---------------- inverse FFT over angle, pass 1 ----------------
      // H_j (j = 16 k1 + k2) of pair P: half 0 of slot j (j < 128) or half 1
      // of slot 256 - j (j >= 128; slot 0 for j = 128)
      if (work) {
#pragma unroll 1
        for (int n0 = 0; n0 < n_live; n0 += LPCX) {
          // lane-derived values are recomputed here rather than kept live
          // across the reference loop, where the registers hold the operand
          int lnx = ln;
          asm volatile("" : "+v"(lnx));
          const int lane_n = lnx % LPCX, k2 = CPWX * w + lnx / LPCX;
          const bool act = n0 + lane_n < n_live;
          const int P = list[act ? n0 + lane_n : 0];
          const int lo = k2 * 128 + P, hi = P - k2 * 128;
          const int mid = k2 == 0 ? 64 + P : hi + 257 * 64;
          auto at = [&](int k1) { return k1 < 8 ? lo + k1 * 2048 : (k1 == 8 ? mid : hi + (513 - 32 * k1) * 64); };
          float2 x[16];
#pragma unroll
          for (int k1 = 0; k1 < 16; ++k1) x[k1] = sm.stc[at(k1)];
          inv_pass1(k2, x, [&](int e) { return sm.tw[e & 255]; });
          if (act) {
#pragma unroll
            for (int n1 = 0; n1 < 16; ++n1) sm.stc[at(n1)] = x[n1];
          }
        }
      }
      __syncthreads();

      // ---------------- pass 2 + arg-max ----------------
      // Rows below 8 read upwards from slot 16 n1, the others downwards from
      // slot 256 - 16 n1.  SPLIT: one loop per direction (each wave runs one),
      // so that either keeps its 16 reads at constant offsets from one address
      // (in one loop the compiler merges the two read sets into 31 per-element
      // addresses); the 4-wave kernels, whose registers are full, keep one loop.
      auto pass2 = [&](auto dir_c) {
        constexpr int dir = decltype(dir_c)::value;  // 1 up, 2 down, 0 either (chosen per wave)
#pragma unroll 1
        for (int n0 = 0; n0 < n_live; n0 += LPCX) {
          int lnx = ln;
          asm volatile("" : "+v"(lnx));
          const int lane_n = lnx % LPCX, c = lnx / LPCX, n1 = CPWX * w + c;
          const bool act = n0 + lane_n < n_live;
          const int P = list[act ? n0 + lane_n : 0];
          const int row_l = P >> 3, ref_l = P & 7;
          const int row = tile * kRowTile + row_l;
          const int k = kt * kRefTile + ref_l;
          float2 x[16];
          const bool low = dir == 1 || (dir == 0 && CPWX * w < 8);
          if (low) {
            const int base = n1 * 2048 + P;
#pragma unroll
            for (int k2 = 0; k2 < 16; ++k2) x[k2] = sm.stc[base + k2 * 128];
          } else if constexpr (dir == 2) {
            const int base = (513 - 32 * n1) * 64 + P;  // k2 = 0; k2 steps go down by 128
            int top = base - 15 * 128;                  // k2 = 15, the lowest address
            asm volatile("" : "+v"(top));               // the base of the reads (not re-associated)
            x[0] = sm.stc[n1 == 8 ? 64 + P : base];
#pragma unroll
            for (int k2 = 1; k2 < 16; ++k2) x[k2] = sm.stc[top + (15 - k2) * 128];
          } else {
            const int base = (513 - 32 * n1) * 64 + P;
            x[0] = sm.stc[n1 == 8 ? 64 + P : base];
#pragma unroll
            for (int k2 = 1; k2 < 16; ++k2) x[k2] = sm.stc[base - k2 * 128];
          }
          inv_pass2(x);
          if constexpr (MODE == kTable) {
            if (act && row < a.rows && k < a.K) {
              const int n = row / a.S, s = row - n * a.S;
              const float unscale = PREC == kFP16 ? 1.f / (fp16_scale(a, row) * a.b_scale) : 1.f;
              for (int m = 0; m < a.M; ++m) {
                float* o = a.table + ((((size_t)n * a.K + k) * a.M + m) * a.S + s) * kNphi;
#pragma unroll
                for (int n2 = 0; n2 < 16; ++n2) o[n1 + 16 * n2] = (m ? x[n2].y : x[n2].x) * unscale;
              }
            }
          } else {
            // only values above the row's best of earlier reference tiles can
            // win (a tie with an earlier tile loses: its flat index is smaller)
            const float thr = sm.thr[row_l];
            const bool valid = act && row < a.rows && k < a.K;
            // the candidate left out of this pass (key m * 256 + angle of this
            // lane's (row, ref)), or -1
            int ex = -1;
            if (MODE == kRunnerUp && valid) {
              const int n = row / a.S, s = row - n * a.S;
              const int e = a.excl[n];
              if (e >= 0) {
                const int rest = e >> 8, se = rest % a.S, km = rest / a.S;
                if (se == s && km / a.M == k) ex = (km % a.M) * 256 + (e & 255);
              }
            }
            float bv = -INFINITY;
            int bi = 0x7fffffff;
            float mx = -INFINITY;
#pragma unroll
            for (int n2 = 0; n2 < 16; ++n2) mx = fmaxf(mx, a.M == 2 ? fmaxf(x[n2].x, x[n2].y) : x[n2].x);
            if (MODE == kArgmax && mx > thr) {
              // the lane's best is mx; its key is the smallest among the
              // candidates equal to it (keys grow with n2, mirror 1 after 0)
              bv = mx;
              if (a.M == 2) {
#pragma unroll
                for (int n2 = 15; n2 >= 0; --n2) bi = x[n2].y == mx ? 256 + n1 + 16 * n2 : bi;
              }
#pragma unroll
              for (int n2 = 15; n2 >= 0; --n2) bi = x[n2].x == mx ? n1 + 16 * n2 : bi;
            } else if (MODE == kRunnerUp && mx > thr) {
#pragma unroll
              for (int n2 = 0; n2 < 16; ++n2) {
                const int ang = n1 + 16 * n2;
                if (ang != ex && better(x[n2].x, ang, bv, bi)) { bv = x[n2].x; bi = ang; }
                if (a.M == 2 && 256 + ang != ex && better(x[n2].y, 256 + ang, bv, bi)) {
                  bv = x[n2].y;
                  bi = 256 + ang;
                }
              }
            }
            if (valid && bi != 0x7fffffff && bv > thr) {
              const int iota = ((k * a.M + (bi >> 8)) * a.S + row % a.S) * kNphi + (bi & 255);
              atomicMax(&sm.key[row_l], cand_key(bv, iota));
            }
          }
        }
      };
      if (work) {
        if constexpr (SPLIT) {
          if (CPWX * w < 8) pass2(std::integral_constant<int, 1>{});  // wave-uniform
          else pass2(std::integral_constant<int, 2>{});
        } else {
          pass2(std::integral_constant<int, 0>{});
        }
      }
    };
    if constexpr (NW == 8) {
      if (n_live <= 16) passes(std::integral_constant<int, 4>{});  // workgroup-uniform
      else passes(std::integral_constant<int, 2>{});
    } else {
      passes(std::integral_constant<int, CPW>{});
    }
    __syncthreads();
    // the particle bests of the rows, for the next reference tile's bound
    if (MODE != kTable && tid < 8) {
      float b = sm.pt[tid];
      const int part = sm.ppart[tid];
#pragma unroll
      for (int r = 0; r < kRowTile; ++r)
        if (sm.ppart[r] == part) b = fmaxf(b, key_value(sm.key[r]));
      sm.pt[tid] = b;
    }
  }
  __syncthreads();
  if (MODE != kTable && tid < 8) {
    const int r = tile * kRowTile + tid;
    if (r < a.rows) {
      const unsigned long long kk = sm.key[tid];
      const float unscale = PREC == kFP16 ? 1.f / (fp16_scale(a, r) * a.b_scale) : 1.f;
      a.row_cc[r] = key_value(kk) * unscale;
      a.row_idx[r] = key_index(kk);
    }
    // the particle of the last row continues into the run's next tile
    float b = sm.pt[tid];
    const int part = sm.ppart[tid];
#pragma unroll
    for (int r2 = 0; r2 < kRowTile; ++r2)
      if (sm.ppart[r2] == part) b = fmaxf(b, key_value(sm.key[r2]));
    if (tid == 7) {
      *sm.carry_p = part;
      *sm.carry_v = b;
    }
  }
}

template <int PREC, int NW, int MAXR, bool RES, bool EXACT>
struct ContractFor {
  typedef typename std::conditional<PREC == kFP32, Fp32Contract<NW, MAXR, RES, EXACT>,
                                    Half16Contract<PREC == kFP32 ? kBF16 : PREC, NW, MAXR, EXACT, RES>>::type type;
};

// Row tiles of run `run` (a.tiles_per_run consecutive tiles), in order, so
// that a particle's best carries from one of its tiles to the next.
template <int PREC, int NW, class Contract, int MODE, bool SPLIT>
__device__ __forceinline__ void corr_run(const CorrArgs& a, int run, const CorrSmem<NW>& sm, Contract& con) {
  const int t0 = run * a.tiles_per_run;
  const int t1 = min(t0 + a.tiles_per_run, a.n_row_tiles);
  if (threadIdx.x == 0) *sm.carry_p = -1;
  lds_wave_sync();
  con.prefetch(a, 0, __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), threadIdx.x & 63);
  for (int t = t0; t < t1; ++t) corr_tile<PREC, NW, Contract, MODE, SPLIT>(a, t, sm, con);
}

template <int PREC, int NW, int MAXR, bool RES, bool EXACT, int MODE>
__global__ __launch_bounds__(NW * 64) void k_corr(CorrArgs a) {
  extern __shared__ float smem[];
  CorrSmem<NW> sm(smem);
  if (threadIdx.x < kNphi) sm.tw[threadIdx.x] = w256c(a.cs32, threadIdx.x);
  typename ContractFor<PREC, NW, MAXR, RES, EXACT>::type con;
  corr_run<PREC, NW, decltype(con), MODE, NW == 8>(a, blockIdx.x, sm, con);
}

// Batched form over the runs of several stacks' row tiles: workgroup g takes
// run g of the concatenated run list (run_start[p] is piece p's first).
template <int PREC, int NW, int MAXR, bool RES, bool EXACT>
__global__ __launch_bounds__(NW * 64) void k_corr_batch(CorrBatch b) {
  extern __shared__ float smem[];
  CorrSmem<NW> sm(smem);
  if (threadIdx.x < kNphi) sm.tw[threadIdx.x] = w256c(b.piece[0].cs32, threadIdx.x);
  typename ContractFor<PREC, NW, MAXR, RES, EXACT>::type con;
  const int item = blockIdx.x;
  if (item >= b.run_start[b.n]) return;
  int p = 0;
  while (p + 1 < b.n && b.run_start[p + 1] <= item) ++p;
  corr_run<PREC, NW, decltype(con), kArgmax, NW == 8>(b.piece[p], item - b.run_start[p], sm, con);
}

template <int P_, int NW_, int MR_, bool RES_, bool EXACT_>
struct Cfg {
  static constexpr int P = P_, NW = NW_, MR = MR_;
  static constexpr bool RES = RES_, EXACT = EXACT_;
};

template <class C, int MODE>
inline void launch_mode(const CorrArgs& a, hipStream_t st) {
  const int runs = (a.n_row_tiles + a.tiles_per_run - 1) / a.tiles_per_run;
  hipLaunchKernelGGL((k_corr<C::P, C::NW, C::MR, C::RES, C::EXACT, MODE>), dim3(runs), dim3(C::NW * 64),
                     CorrSmem<C::NW>::bytes(), st, a);
}

template <class C>
inline void launch_one(const CorrArgs& a, bool table, hipStream_t st) {
  if (table) launch_mode<C, kTable>(a, st);
  else launch_mode<C, kArgmax>(a, st);
}

template <class C>
inline void launch_one(const CorrBatch& b, int grid, hipStream_t st) {
  (void)grid;
  hipLaunchKernelGGL((k_corr_batch<C::P, C::NW, C::MR, C::RES, C::EXACT>), dim3(b.run_start[b.n]),
                     dim3(C::NW * 64), CorrSmem<C::NW>::bytes(), st, b);
}

// Per-precision instantiation sets (one translation unit each).  `b` null:
// one launch over a's row tiles (table: write the CC table); else the
// persistent launch over b's pieces with `grid` workgroups.
void corr_dispatch_fp32(int variant, int r4min, int r4max, const CorrArgs* a, bool table, const CorrBatch* b,
                        int grid, hipStream_t st);
void corr_dispatch_bf16(int variant, int r4min, int r4max, const CorrArgs* a, bool table, const CorrBatch* b,
                        int grid, hipStream_t st);
void corr_dispatch_fp16(int variant, int r4min, int r4max, const CorrArgs* a, bool table, const CorrBatch* b,
                        int grid, hipStream_t st);

// The runner-up pass (one instantiation per precision: the generic
// streamed-operand configuration, any R4 <= 16).
void corr_runner_up_fp32(const CorrArgs& a, hipStream_t st);
void corr_runner_up_bf16(const CorrArgs& a, hipStream_t st);
void corr_runner_up_fp16(const CorrArgs& a, hipStream_t st);

template <class C>
inline void corr_go(const CorrArgs* a, bool table, const CorrBatch* b, int grid, hipStream_t st) {
  if (b) launch_one<C>(*b, grid, st);
  else launch_one<C>(*a, table, st);
}

// 16-bit forms: operand ring bucket MAXR in {8, 12, 16} (R4 <= 8, 9..12,
// 13..16); exact where every work item lies in the bucket (then the step
// count is fixed, and at 16 the last step is 8 wide), else the run-time form.
template <int PREC, bool RES>
inline void corr_dispatch_16(int r4min, int r4max, const CorrArgs* a, bool table, const CorrBatch* b, int grid,
                             hipStream_t st) {
  if (r4max <= 8) return corr_go<Cfg<PREC, 8, 8, RES, true>>(a, table, b, grid, st);
  if (r4max <= 12) {
    if (r4min > 8) return corr_go<Cfg<PREC, 8, 12, RES, true>>(a, table, b, grid, st);
    return corr_go<Cfg<PREC, 8, 12, RES, false>>(a, table, b, grid, st);
  }
  if (r4min > 12) return corr_go<Cfg<PREC, 8, 16, RES, true>>(a, table, b, grid, st);
  return corr_go<Cfg<PREC, 8, 16, RES, false>>(a, table, b, grid, st);
}

}  // namespace mra
