// Shift + polar resampling and per-ring FFT of particle images (Algorithm 1:
// each shifted particle resampled to polar coordinates and transformed per
// ring), the FP32 re-score of a winning candidate, and the per-particle max |pixel|.
//
// One 8-wave workgroup per particle (about 68 KB of LDS at L = 76, so two
// workgroups share a CU: 16 waves, against 12 with three 4-wave groups, which
// ran 10 % slower).  The image is staged once in LDS with a zero
// border (coalesced HBM read), beside a float-float cos/sin table; the
// (ring, 8-row group) items of the particle are split between the waves.
// In an item, lane (l, row) needs the 32 samples p[16 n1 + 2l + e] of shift
// `row`; integer shifts move the bilinear taps by whole pixels, so each of
// the 8 lanes of group l computes the positions and weights of 4 of those
// angles (from the table: the item loop issues no memory loads) and samples
// them at all 8 shifts, and a transpose through LDS regroups the samples by
// shift.
// The 256-point real FFT runs as a 16 x 8 complex FFT across the eight
// lanes l of a shift, with a transpose through a per-wave LDS scratch, and
// the spectra are staged there again so that an item's 128 slots of one
// ring are written as one contiguous 8 KB run of the operand (the kernel is
// bound by its HBM writes, and runs of 64-byte pieces scattered over the
// tile write far slower).
#include "mra_common.h"
#include "mra_fft.h"
#include "polar_impl.h"

namespace mra {

// Workgroup -> item: consecutive items on the same XCD (workgroups are dealt
// to the 8 XCDs round-robin), so row tiles shared by neighbouring particles
// are completed in one L2.  The grid is a multiple of 8.
__device__ __forceinline__ int xcd_item() {
  const int per_xcd = gridDim.x / 8;
  return (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
}

// lane J's value of each group of 8 consecutive lanes, to all 8
// (ds_swizzle bit-mask mode: source lane = (lane & 0x18) | J within 32)
template <int J>
__device__ __forceinline__ int group_bcast(int v) {
  return __builtin_amdgcn_ds_swizzle(v, 0x18 | (J << 5));
}

// Operand element type written in mode 0: FP32 (kRingPerm or kSlotMajor,
// chosen at run time), or BF16 / FP16 in kRingPerm16.
enum PolarOut { kOutF32 = 0, kOutBF16 = 1, kOutFP16 = 2 };

// Two values in the contraction's 16-bit type, each rounded to nearest
// (even) once, packed with x in the low half.
template <int OUT>
__device__ __forceinline__ uint32_t pack16(float x, float y) {
  typedef float f32x2v __attribute__((ext_vector_type(2)));
  const f32x2v v = {x, y};
  if constexpr (OUT == kOutBF16) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
  } else {
    typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, f16x2));
  }
}

template <int MODE, int OUT>
__device__ __forceinline__ void polar_particle(const PolarArgs& a, int n, float* smem) {
  float* img = smem;
  float2* scr = reinterpret_cast<float2*>(smem + ((a.Lp * a.Lp + 3) & ~3));
  CosSin* cs = reinterpret_cast<CosSin*>(scr + kPolarWaves * 64 * 9);
  stage_image(img, a.parts + (size_t)n * a.L * a.L, a.L, a.Lp, a.pad);
  stage_cs(cs, a.cs64);
  __syncthreads();

  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), ln = threadIdx.x & 63;
  const int l = ln >> 3, rl = ln & 7;
  float2* my = scr + w * 64 * 9;                // per-wave scratch: 64 lanes x 9 float2
  float* stage = reinterpret_cast<float*>(my);  // [64 slots][16] in each staging round
  const int base = (a.cx + a.pad) * a.Lp + (a.cx + a.pad);
  const int Lp4 = 4 * a.Lp, s1m = (65536 + a.S1 - 1) / a.S1;
  // lane rl handles row (q0 + grp) * 8 + rl: groups are aligned to the
  // correlation kernel's 8-row tiles
  const int row0 = n * a.S;
  const int q0 = row0 >> 3;
  const int ngrp = ((row0 + a.S - 1) >> 3) - q0 + 1;

  // (ring, row group) items in contiguous blocks per wave (balanced)
  const int n_items = a.R * ngrp;
  const int per_wave = (n_items + kPolarWaves - 1) / kPolarWaves;
  const int it0 = w * per_wave, it1 = min(n_items, it0 + per_wave);
  for (int item = it0; item < it1; ++item) {
    const int ring = item / ngrp, grp = item - ring * ngrp;
    // FP32 operand: the shift and lane indices are made opaque here, so that
    // the addresses derived from them are recomputed in every item instead
    // of being hoisted out of the loop and kept in registers (kept, with
    // those of the lane group's index lx, they take the kernel past 128
    // registers and two workgroups per CU); the 16-bit instances keep them
    // all (about 20 % fewer vector instructions).
    const int lx = l;
    int rx = rl, lnx = ln;
    if constexpr (OUT == kOutF32) {
      asm volatile("" : "+v"(rx), "+v"(lnx));
      // (their ranges restated, so that products with them take the 24-bit multiplier)
      rx &= 7;
      lnx &= 63;
    }
    int k1a, k1b;
    fwd_cols(lx, k1a, k1b);
    const int row = (q0 + grp) * 8 + rx;
    const int s = row - row0;
    const bool valid = s >= 0 && s < a.S;
    const int sc = s < 0 ? 0 : (s < a.S ? s : a.S - 1);
    const int o4 = 4 * (base + shift_offset(sc, a.S1, s1m, a.T, a.Lp));

    // 32 bilinear samples v[i] = p[16 n1 + 2 l + e] (i = 2 n1 + e) of this
    // lane's shift, the positions taken from the staged cos/sin (no memory
    // loads in the loop).  Positions and weights do not depend on the shift:
    // lane rx of group l takes them for the angles i = rx (mod 8) and
    // samples those at all 8 shifts of the item; a transpose through the
    // wave's scratch, in two halves of 16 angles, hands each lane its own
    // shift's samples.
    const float rr = (float)(a.r_min + ring);
    const CosSin* cp = cs + 2 * lx;
    // byte offsets of the item's 8 shifts (lane j of the group computed shift j's)
    const int o4s[8] = {group_bcast<0>(o4), group_bcast<1>(o4), group_bcast<2>(o4), group_bcast<3>(o4),
                        group_bcast<4>(o4), group_bcast<5>(o4), group_bcast<6>(o4), group_bcast<7>(o4)};
    float* tr = reinterpret_cast<float*>(my);  // [64 (l, shift)][17]: row pitch 17 spreads the banks
    float v[32];
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
      float smp[2][8];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int i = 16 * hf + 8 * b + rx;
        const CosSin c = cp[16 * (i >> 1) + (i & 1)];
        const int off = polar_offset(rr, c, Lp4);
        float w00, w10, w01, w11;
        polar_weights(rr, c, w00, w10, w01, w11);
#pragma unroll
        for (int j = 0; j < 8; ++j) smp[b][j] = bilin4w(img, o4s[j] + off, Lp4, w00, w10, w01, w11);
      }
      wave_sync();  // the scratch's earlier readers are done
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int j = 0; j < 8; ++j) tr[(lx * 8 + j) * 17 + 8 * b + rx] = smp[b][j];
      wave_sync();
#pragma unroll
      for (int q = 0; q < 16; ++q) v[16 * hf + q] = tr[(lx * 8 + rx) * 17 + q];
    }
    wave_sync();  // before the FFT's transposes reuse the scratch

    if (MODE == 1) {
      if (valid) {
        float* o = a.out + (((size_t)n * a.S + s) * a.R + ring) * kNphi;
#pragma unroll
        for (int i = 0; i < 32; ++i) o[16 * (i >> 1) + 2 * lx + (i & 1)] = v[i];
      }
      continue;
    }

    float2 z[16];
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) z[n1] = make_float2(v[2 * n1], v[2 * n1 + 1]);
    dft16<-1>(z);
#pragma unroll
    for (int k1 = 1; k1 < 16; ++k1) z[k1] = cmul(z[k1], twid(cs, 2 * ((lx * k1) & 127)));
    // transpose through the scratch in two halves: lane l's first column
    // k1a lies in 0..7, its second k1b in 8..15.  Entries are ordered
    // (l, shift) with the shift fastest, which spreads a wave's accesses
    // over the banks better than (shift, l).
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

    if (MODE == 0) {
      // Every real split yields one slot below 64 and one above (128 - f, or
      // lane 0's 0 and 64): keep both, then stage [slot][p*8 + row] for the
      // 64 low slots and then the 64 high ones, and write the 64-byte
      // (ring, slot) segments of the tile with 16-byte stores, each store
      // instruction covering whole 128-byte lines.  The four
      // 16-byte chunks of a slot are XOR-swizzled by slot & 3, so the eight
      // lanes l that write at once hit distinct banks.
      int lo_s[8], hi_s[8];
      float lo_a[8], lo_b[8], hi_a[8], hi_b[8];
      int e = 0, s0 = 0;
      float a0 = 0.f, b0 = 0.f;
      fwd_emit(lx, Za, Zb, [&](int f) { return twid(cs, f & 255); },
               [&](int slot, float re, float im) {
                 const int k = e >> 1;
                 if ((e++ & 1) == 0) {
                   s0 = slot; a0 = re - im; b0 = re + im;
                 } else {
                   const bool first_low = s0 < slot;
                   lo_s[k] = first_low ? s0 : slot;
                   hi_s[k] = first_low ? slot : s0;
                   lo_a[k] = first_low ? a0 : re - im;
                   lo_b[k] = first_low ? b0 : re + im;
                   hi_a[k] = first_low ? re - im : a0;
                   hi_b[k] = first_low ? re + im : b0;
                 }
               });
      const int tile = q0 + grp;
      const int first = row0 - tile * 8;            // rows of this tile before the particle
      const int last = row0 + a.S - tile * 8;       // first row after the particle
      // otherwise the lane's segment of slot s = 64 h + 16 it + j (j = lane /
      // 4), slot stride ss: a per-lane part computed once per item and a
      // uniform offset
      const bool slot_major = a.a_layout == kSlotMajor, perm = a.a_layout == kRingPerm;
      // 16-bit operand: each value rounded once, as the contraction's matrix
      // cores take it (FP16 scaled by the particle's power of two)
      constexpr bool half = OUT != kOutF32;
      const float hscale = OUT == kOutFP16 ? fp16_operand_scale(a.maxabs[n]) : 1.f;
      const int ss = slot_major ? a.R4 * 64 : 16;
      float* dst = a.out + (slot_major ? (size_t)tile * kSlots * a.R4 * 64 + ring * 16
                                       : ((size_t)tile * 4 * a.R4 + ring) * kSlots * 16);
      const int part = lnx & 3;                       // rows (part & 1) * 4 .. +3 of p = part >> 1
      const int r0 = (part & 1) * 4;
      const bool full = r0 >= first && r0 + 4 <= last;
      const int j = lnx >> 2;
      float* const lane_dst = dst + (size_t)__mul24(j, ss) + part * 4;
      // kRingPerm: lane (pp = lane / 8, c = lane % 8) writes elements 2c, 2c+1
      // (rows rp, rp + 1) of the position pair 16 it + 4 h + lp, whose slots
      // are 64 h + sp and 64 h + sp + 8, interleaved by element
      const int pp = lnx >> 3, c = lnx & 7;
      const int lp = 8 * (pp >> 2) + (pp & 3), sp = (pp >> 2) + 16 * (pp & 3);
      const int rp = 2 * (c & 3);
      const bool full_p = rp >= first && rp + 2 <= last;
      float* const pair_dst = dst + 32 * lp + 4 * c;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int sl = h ? hi_s[k] - 64 : lo_s[k];
          const int sw = (sl & 3) << 2;
          stage[sl * 16 + (rx ^ sw)] = h ? hi_a[k] : lo_a[k];
          stage[sl * 16 + ((8 + rx) ^ sw)] = h ? hi_b[k] : lo_b[k];
        }
        wave_sync();
        if constexpr (half) {
          // kRingPerm16: the staged slots 64 h + sl are positions 16 (sl % 8)
          // + 8 h + sl / 8, i.e. the runs G = 2 w + h (w = sl % 8); lane
          // (w, k) of chunk c = lane + 64 q writes element k of the 8
          // positions of run G as one 16-byte store (one row, so a chunk is
          // written whole or not at all)
          uint16_t* blk = reinterpret_cast<uint16_t*>(a.out) + (size_t)(tile * 4 * a.R4 + ring) * kSlots * 16;
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int cix = lnx + 64 * q, w = cix >> 4, k = cix & 15, row = k & 7;
            uint32_t u[4];
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
              const int sl0 = w + 16 * jj, sl1 = sl0 + 8;  // positions 2 jj, 2 jj + 1 of the run
              float v0 = stage[sl0 * 16 + (k ^ ((sl0 & 3) << 2))];
              float v1 = stage[sl1 * 16 + (k ^ ((sl1 & 3) << 2))];
              if constexpr (OUT == kOutFP16) {
                v0 *= hscale;
                v1 *= hscale;
              }
              u[jj] = pack16<OUT>(v0, v1);
            }
            if (row >= first && row < last)
              *reinterpret_cast<uint4*>(blk + a16_index(16 * w + 8 * h, k)) = make_uint4(u[0], u[1], u[2], u[3]);
          }
          wave_sync();
        } else {
#pragma unroll
          for (int it = 0; it < 4; ++it) {
            if (perm) {
              const int s0 = 2 * it + sp, s1 = s0 + 8, sw = (s0 & 3) << 2;  // s1 & 3 == s0 & 3
              const float2 v0 = *reinterpret_cast<const float2*>(stage + s0 * 16 + ((2 * c) ^ sw));
              const float2 v1 = *reinterpret_cast<const float2*>(stage + s1 * 16 + ((2 * c) ^ sw));
              float* o = pair_dst + 32 * (16 * it + 4 * h);
              if (full_p) {
                *reinterpret_cast<float4*>(o) = make_float4(v0.x, v1.x, v0.y, v1.y);
              } else {
                if (rp >= first && rp < last) { o[0] = v0.x; o[1] = v1.x; }
                if (rp + 1 >= first && rp + 1 < last) { o[2] = v0.y; o[3] = v1.y; }
              }
              continue;
            }
            const int sl = it * 16 + (lnx >> 2);
            const float4 val = *reinterpret_cast<const float4*>(stage + sl * 16 + ((part ^ (sl & 3)) << 2));
            float* o = lane_dst + (size_t)(64 * h + 16 * it) * ss;
            if (full) {
              *reinterpret_cast<float4*>(o) = val;
            } else {
              if (r0 + 0 >= first && r0 + 0 < last) o[0] = val.x;
              if (r0 + 1 >= first && r0 + 1 < last) o[1] = val.y;
              if (r0 + 2 >= first && r0 + 2 < last) o[2] = val.z;
              if (r0 + 3 >= first && r0 + 3 < last) o[3] = val.w;
            }
          }
          wave_sync();
        }
      }
    } else {  // MODE 2: plain spectra
      float* o = a.out + (((size_t)n * a.S + (valid ? s : 0)) * a.R + ring) * 129 * 2;
      fwd_emit(lx, Za, Zb, [&](int f) { return twid(cs, f & 255); },
               [&](int slot, float re, float im) {
                 if (!valid) return;
                 if (slot == 0) {
                   o[0] = re; o[1] = 0.f;
                   o[256] = im; o[257] = 0.f;
                 } else {
                   o[2 * slot] = re;
                   o[2 * slot + 1] = im;
                 }
               });
    }
  }
}

template <int MODE, int OUT>
__global__ __launch_bounds__(kPolarThreads) void k_polar_fft(PolarArgs a) {
  extern __shared__ float smem[];
  const int n = xcd_item();
  if (n >= a.n_part) return;
  polar_particle<MODE, OUT>(a, n, smem);
}

// every piece of a batch writes the same operand type
template <int OUT>
__global__ __launch_bounds__(kPolarThreads) void k_polar_batch(PolarBatch b) {
  extern __shared__ float smem[];
  const int item = xcd_item();
  if (item >= b.start[b.n]) return;
  int p = 0;
  while (p + 1 < b.n && b.start[p + 1] <= item) ++p;
  polar_particle<0, OUT>(b.piece[p], item - b.start[p], smem);
}

static int polar_out(const PolarArgs& a) {
  return a.a_layout != kRingPerm16 ? kOutF32 : (a.prec == kFP16 ? kOutFP16 : kOutBF16);
}

size_t polar_lds_bytes(int Lp) {
  return (size_t)((Lp * Lp + 3) & ~3) * sizeof(float) + (size_t)kPolarWaves * 64 * 9 * sizeof(float2) +
         (size_t)kNphi * sizeof(CosSin);
}

hipError_t launch_polar_batch(const PolarBatch& b, hipStream_t st) {
  if (b.n <= 0 || b.start[b.n] <= 0) return hipSuccess;
  int lp = 0;
  const int out = polar_out(b.piece[0]);
  for (int i = 0; i < b.n; ++i) {
    lp = b.piece[i].Lp > lp ? b.piece[i].Lp : lp;
    if (polar_out(b.piece[i]) != out) return hipErrorInvalidValue;
  }
  const dim3 grid((b.start[b.n] + 7) / 8 * 8), block(kPolarThreads);
  const size_t lds = polar_lds_bytes(lp);
  switch (out) {
    case kOutF32: hipLaunchKernelGGL(k_polar_batch<kOutF32>, grid, block, lds, st, b); break;
    case kOutBF16: hipLaunchKernelGGL(k_polar_batch<kOutBF16>, grid, block, lds, st, b); break;
    default: hipLaunchKernelGGL(k_polar_batch<kOutFP16>, grid, block, lds, st, b); break;
  }
  return hipGetLastError();
}

hipError_t launch_polar(int mode, const PolarArgs& a, hipStream_t st) {
  if (a.n_part <= 0) return hipSuccess;
  const size_t lds = polar_lds_bytes(a.Lp);
  dim3 grid((a.n_part + 7) / 8 * 8), block(kPolarThreads);
  switch (mode) {
    case 0:
      switch (polar_out(a)) {
        case kOutF32: hipLaunchKernelGGL((k_polar_fft<0, kOutF32>), grid, block, lds, st, a); break;
        case kOutBF16: hipLaunchKernelGGL((k_polar_fft<0, kOutBF16>), grid, block, lds, st, a); break;
        default: hipLaunchKernelGGL((k_polar_fft<0, kOutFP16>), grid, block, lds, st, a); break;
      }
      break;
    case 1: hipLaunchKernelGGL((k_polar_fft<1, kOutF32>), grid, block, lds, st, a); break;
    default: hipLaunchKernelGGL((k_polar_fft<2, kOutF32>), grid, block, lds, st, a); break;
  }
  return hipGetLastError();
}

// FP32 re-score of each particle's winner: the direct double sum
// sum_r w_r sum_j p_{s,m}[r][j] * qhat_k[r][(j + a) mod 256] with a = -psi.
// The mirrored samples are the unmirrored stencil read at angle -j (the
// stencil table is built symmetric in j <-> 256 - j).  With a.rows >= 2 the
// candidates are the winners of the particle's a.rows best rows of the 16-bit
// pass and their neighbours one angle step either side; the best FP32 value
// wins (ties: the smallest flat index) and replaces the parameters.  Rows
// whose 16-bit best lies more than a.margin of the particle's 16-bit
// best below it are left out (they cannot win at 16-bit accuracy).
constexpr int kMaxRescoreRows = 8;
constexpr int kMaxRows = 289;  // shifts per particle at the largest search range (+-8)
constexpr int kRescoreRed = 24;  // reduction slots: 4 waves x 3 lags x up to 2 candidates

// FP32 CC of (ref k, shift soff, mirror m) at the lags lag0 + d, d < ND, for
// the image staged in img; red holds 4 ND doubles.  Reduction in a fixed
// order (per-thread FP32 ring sum, then FP64 across the block), the same for
// every d.
template <int ND>
__device__ __forceinline__ void rescore_lags(const RescoreArgs& a, const float* img, double* red, int k, int m,
                                             int soff, int lag0, double (&out)[ND]) {
  const int base = (a.cx + a.pad) * a.Lp + (a.cx + a.pad);
  const int j = threadIdx.x;
  const int jj = m ? ((kNphi - j) & 255) : j;
  const float* q = a.qhat + (size_t)k * a.R * kNphi;
  float acc[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) acc[d] = 0.f;
  // unrolled so that the stencil and spectrum loads of several rings are in
  // flight at once (the loop is bound by their latency, not by arithmetic)
#pragma unroll 8
  for (int r = 0; r < a.R; ++r) {
    const Stencil st = a.stencil[r * kNphi + jj];
    const float p = bilin(img, base + st.dy * a.Lp + (st.bx >> 2) + soff, a.Lp, st.fx, st.fy);
    const float w = (float)(a.r_min + r);
#pragma unroll
    for (int d = 0; d < ND; ++d) acc[d] += w * (p * q[r * kNphi + ((j + lag0 + d) & 255)]);
  }
  // FP64 sum over the 256 threads in a fixed order: a butterfly within each
  // wave (every lane ends with the wave's sum), then the four waves' sums in
  // wave order
  double v[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    v[d] = (double)acc[d];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[d] += __shfl_xor(v[d], o);
  }
  if ((j & 63) == 0) {
#pragma unroll
    for (int d = 0; d < ND; ++d) red[d * 4 + (j >> 6)] = v[d];
  }
  __syncthreads();
#pragma unroll
  for (int d = 0; d < ND; ++d) out[d] = ((red[d * 4] + red[d * 4 + 1]) + red[d * 4 + 2]) + red[d * 4 + 3];
  __syncthreads();
}

// The same FP32 CC for NC candidates (ref k[c], mirror m[c], shift soff[c])
// at the lags lag0[c] + d, d < 3, evaluated together: each ring's stencil is
// loaded once per mirror that occurs (MIXED: both occur) and serves every
// candidate of that mirror, and the NC * 3 sums share one reduction (red
// holds 12 NC doubles).  Every sum takes the arithmetic of rescore_lags<3> in
// the same order, so the values are bit-identical to evaluating the
// candidates one at a time.  The unroll keeps either form within 80
// registers, six workgroups per CU (the four-candidate form needs 117, and
// its occupancy costs more than the shared loads save).
template <int NC, bool MIXED>
__device__ __forceinline__ void rescore_group(const RescoreArgs& a, const float* img, double* red, const int* k,
                                              const int* m, const int* soff, const int* lag0, double (&out)[NC][3]) {
  const int base = (a.cx + a.pad) * a.Lp + (a.cx + a.pad);
  const int j = threadIdx.x;
  const int jm = (kNphi - j) & 255;
  // unmixed: every candidate's mirror is m[0]
  const Stencil* st0 = a.stencil + (MIXED ? j : (m[0] ? jm : j));
  const Stencil* st1 = a.stencil + jm;
  float acc[NC][3];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int d = 0; d < 3; ++d) acc[c][d] = 0.f;
  static_assert(NC * 12 <= kRescoreRed, "reduction slots");
  constexpr int kUnroll = NC == 1 ? 8 : 2;
#pragma unroll kUnroll
  for (int r = 0; r < a.R; ++r) {
    const Stencil s0 = st0[r * kNphi];
    Stencil s1 = s0;
    if constexpr (MIXED) s1 = st1[r * kNphi];
    const float w = (float)(a.r_min + r);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const Stencil st = (MIXED && m[c]) ? s1 : s0;
      const float p = bilin(img, base + st.dy * a.Lp + (st.bx >> 2) + soff[c], a.Lp, st.fx, st.fy);
      const float* q = a.qhat + ((size_t)k[c] * a.R + r) * kNphi;
#pragma unroll
      for (int d = 0; d < 3; ++d) acc[c][d] += w * (p * q[(j + lag0[c] + d) & 255]);
    }
  }
  // the reduction of rescore_lags, for every sum
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double v = (double)acc[c][d];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
      if ((j & 63) == 0) red[(c * 3 + d) * 4 + (j >> 6)] = v;
    }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double* r4 = red + (c * 3 + d) * 4;
      out[c][d] = ((r4[0] + r4[1]) + r4[2]) + r4[3];
    }
  __syncthreads();
}

// Candidates cand[0 .. NC - 1] (flat indices, NC <= 2):
// their FP32 values at the three lags around each one's angle, folded into
// (best, best_i) in list order (ties: the smallest flat index).
template <int NC>
__device__ __forceinline__ void rescore_fold(const RescoreArgs& a, const float* img, double* red, const int* cand,
                                             float& best, int& best_i) {
  int k[NC], m[NC], soff[NC], lag0[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int idx = __builtin_amdgcn_readfirstlane(cand[c]);  // the same in every lane
    const int ang = idx & 255;
    int rest = idx >> 8;
    const int s = rest % a.S;
    rest /= a.S;
    m[c] = rest % a.M;
    k[c] = rest / a.M;
    soff[c] = (s / a.S1 - a.T) * a.Lp + (s % a.S1 - a.T);
    lag0[c] = (ang + 255) & 255;
  }
  bool mixed = false;  // workgroup-uniform
#pragma unroll
  for (int c = 1; c < NC; ++c) mixed |= m[c] != m[0];
  double v[NC][3];
  if (mixed)
    rescore_group<NC, true>(a, img, red, k, m, soff, lag0, v);
  else
    rescore_group<NC, false>(a, img, red, k, m, soff, lag0, v);
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int i2 = (__builtin_amdgcn_readfirstlane(cand[c]) & ~255) | ((lag0[c] + d) & 255);
      const float f = (float)v[c][d];
      if (f > best || (f == best && i2 < best_i)) {
        best = f;
        best_i = i2;
      }
    }
}

__device__ __forceinline__ void rescore_particle(const RescoreArgs& a, int n, float* smem) {
  float* img = smem;
  double* red = reinterpret_cast<double*>(smem + ((a.Lp * a.Lp + 1) & ~1));
  int* cand = reinterpret_cast<int*>(red + kRescoreRed);  // candidate rows' flat indices
  const int64_t gi = a.out_off + n;
  stage_image(img, a.parts + (size_t)n * a.L * a.L, a.L, a.Lp, a.pad);
  if (a.rows <= 1) {
    __syncthreads();
    const int k = a.ref[gi], m = a.mirror[gi] ? 1 : 0;
    const int sx = a.shift_x[gi], sy = a.shift_y[gi];
    if (k < 0 || k >= a.K || sx < -a.T || sx > a.T || sy < -a.T || sy > a.T) {
      if (threadIdx.x == 0) a.cc[gi] = NAN;
      return;  // uniform over the block
    }
    double v[1];
    rescore_lags<1>(a, img, red, k, m, sy * a.Lp + sx, (kNphi - a.psi[gi]) & 255, v);
    if (threadIdx.x == 0) a.cc[gi] = (float)v[0];
    return;
  }
  // the a.rows best rows of the 16-bit pass, by wave 0: lane l holds rows
  // l + 64 i, and each round takes the largest (value, then smallest flat
  // index) of the rows not yet taken across the wave.  Rows without a
  // candidate (index 2^31 - 1) and NaN values never count.
  if (threadIdx.x < 64) {
    constexpr int kPer = (kMaxRows + 63) / 64;
    const int l = threadIdx.x;
    float lv[kPer];
    int li[kPer];
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int s = l + 64 * e;
      lv[e] = s < a.S ? a.row_cc[(size_t)n * a.S + s] : -INFINITY;
      li[e] = s < a.S ? a.row_idx[(size_t)n * a.S + s] : 0x7fffffff;
      if (lv[e] != lv[e]) li[e] = 0x7fffffff;
    }
    const int nr = a.rows < kMaxRescoreRows ? a.rows : kMaxRescoreRows;
    float top = -INFINITY;
    for (int t = 0; t < kMaxRescoreRows; ++t) {
      float bv = -INFINITY;
      int bi = 0x7fffffff;
      if (t < nr) {  // uniform
#pragma unroll
        for (int e = 0; e < kPer; ++e)
          if (li[e] != 0x7fffffff && (lv[e] > bv || (lv[e] == bv && li[e] < bi))) {
            bv = lv[e];
            bi = li[e];
          }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          const float ov = __shfl_xor(bv, o);
          const int oi = __shfl_xor(bi, o);
          if (ov > bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
          }
        }
#pragma unroll
        for (int e = 0; e < kPer; ++e)
          if (li[e] == bi) li[e] = 0x7fffffff;  // taken (flat indices are distinct)
      }
      if (t == 0) top = bv;
      // only rows within the re-ranking margin of the particle's best are
      // candidates; pruning keeps their bests exact
      const float lim = top > -INFINITY ? top - a.margin * fabsf(top) : top;
      if (l == 0) cand[t] = (t < nr && bv >= lim) ? bi : 0x7fffffff;
    }
  }
  __syncthreads();
  int nc = 0;  // the candidates form a prefix of the list (values descend)
  while (nc < kMaxRescoreRows && __builtin_amdgcn_readfirstlane(cand[nc]) != 0x7fffffff) ++nc;
  float best = -INFINITY;
  int best_i = 0x7fffffff;
  for (int t0 = 0; t0 < nc; t0 += 2) {  // workgroup-uniform
    if (nc - t0 == 1)
      rescore_fold<1>(a, img, red, cand + t0, best, best_i);
    else
      rescore_fold<2>(a, img, red, cand + t0, best, best_i);
  }
  if (threadIdx.x != 0) return;
  if (best_i == 0x7fffffff) {  // the 16-bit pass found no candidate: keep its (invalid) result
    a.cc[gi] = NAN;
    return;
  }
  const int ang = best_i & 255;
  int rest = best_i >> 8;
  const int s = rest % a.S;
  rest /= a.S;
  const int m = rest % a.M, k = rest / a.M;
  a.ref_w[gi] = k;
  a.mirror_w[gi] = m;
  a.shift_x_w[gi] = s % a.S1 - a.T;
  a.shift_y_w[gi] = s / a.S1 - a.T;
  a.psi_w[gi] = (kNphi - ang) & 255;
  a.cc[gi] = best;
  if (a.flat_w) a.flat_w[gi] = best_i;
  if (a.win) a.win[n] = best_i;
}

static size_t rescore_lds_bytes(int Lp) {
  return (size_t)((Lp * Lp + 1) & ~1) * sizeof(float) + kRescoreRed * sizeof(double) +
         kMaxRescoreRows * sizeof(int);
}

__global__ __launch_bounds__(256) void k_rescore(RescoreArgs a) {
  extern __shared__ float smem[];
  rescore_particle(a, blockIdx.x, smem);
}

__global__ __launch_bounds__(256) void k_rescore_batch(RescoreBatch b) {
  extern __shared__ float smem[];
  const int item = blockIdx.x;
  int p = 0;
  while (p + 1 < b.n && b.start[p + 1] <= item) ++p;
  rescore_particle(b.piece[p], item - b.start[p], smem);
}

hipError_t launch_rescore(const RescoreArgs& a, hipStream_t st) {
  if (a.n_part <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rescore, dim3(a.n_part), dim3(256), rescore_lds_bytes(a.Lp), st, a);
  return hipGetLastError();
}

hipError_t launch_rescore_batch(const RescoreBatch& b, hipStream_t st) {
  if (b.n <= 0 || b.start[b.n] <= 0) return hipSuccess;
  int lp = 0;
  for (int i = 0; i < b.n; ++i) lp = b.piece[i].Lp > lp ? b.piece[i].Lp : lp;
  hipLaunchKernelGGL(k_rescore_batch, dim3(b.start[b.n]), dim3(256), rescore_lds_bytes(lp), st, b);
  return hipGetLastError();
}

// Sub-step angle of each particle's final winner: the FP32 CC at lags
// a - 1, a, a + 1 (a = -psi) and the vertex of the parabola through them.
__global__ __launch_bounds__(256) void k_refine(RescoreArgs a) {
  extern __shared__ float smem[];
  float* img = smem;
  double* red = reinterpret_cast<double*>(smem + ((a.Lp * a.Lp + 1) & ~1));
  const int n = blockIdx.x;
  const int64_t gi = a.out_off + n;
  stage_image(img, a.parts + (size_t)n * a.L * a.L, a.L, a.Lp, a.pad);
  __syncthreads();
  const int k = a.ref[gi], m = a.mirror[gi] ? 1 : 0;
  const int sx = a.shift_x[gi], sy = a.shift_y[gi], psi = a.psi[gi];
  if (k < 0 || k >= a.K || sx < -a.T || sx > a.T || sy < -a.T || sy > a.T) {
    if (threadIdx.x == 0) a.psi_frac[gi] = NAN;
    return;  // uniform over the block
  }
  const int ang = (kNphi - psi) & 255;
  double v[3];
  rescore_lags<3>(a, img, red, k, m, sy * a.Lp + sx, (ang + 255) & 255, v);
  if (threadIdx.x == 0) {
    const double den = v[0] - 2.0 * v[1] + v[2];
    double d = den < 0.0 ? 0.5 * (v[0] - v[2]) / den : 0.0;
    d = d < -0.5 ? -0.5 : (d > 0.5 ? 0.5 : d);
    double f = (double)psi - d;
    if (f < 0.0) f += kNphi;
    if (f >= kNphi) f -= kNphi;
    a.psi_frac[gi] = (float)f;
  }
}

hipError_t launch_refine(const RescoreArgs& a, hipStream_t st) {
  if (a.n_part <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_refine, dim3(a.n_part), dim3(256), rescore_lds_bytes(a.Lp), st, a);
  return hipGetLastError();
}

// max |pixel| of each particle image (the FP16 operand scale): one
// workgroup per particle, out[n] for n < n_part.
__global__ __launch_bounds__(256) void k_part_maxabs(const float* x, int LL, float* out) {
  __shared__ float red[4];
  const float* img = x + (size_t)blockIdx.x * LL;
  float m = 0.f;
  for (int i = threadIdx.x; i < LL; i += 256) m = fmaxf(m, fabsf(img[i]));
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

hipError_t launch_part_maxabs(const float* x, int n_part, int L, float* out, hipStream_t st) {
  if (n_part <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_part_maxabs, dim3(n_part), dim3(256), 0, st, x, L * L, out);
  return hipGetLastError();
}

}  // namespace mra
