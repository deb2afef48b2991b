// Reference preparation (Algorithm 1: each reference resampled to polar
// coordinates and transformed per ring), done once per reference set in FP64:
//   q_k[r][j]  bilinear polar samples at zero shift,
//   nu_k       weighted ring norm sqrt(sum_r w_r sum_j q^2),
//   Q_k[r][f]  per-ring DFT (direct sum), times w_r / (nu_k * 256),
// then packed into the operand layouts of the correlation kernel:
//   FP32  [ref tile][slot][t < R4][64], lane = g*16 + 2*(ref%8) + q, ring = g*R4 + t
//   16-bit [ref tile][slot][s < NS - 1][64][8] (the same lanes), ring = g*R4 + 8 s + e,
//          then the last step [64][BT] (BT = 2, 4 or 8: as wide as its rings need)
// with q = 0 -> c - d and q = 1 -> c + d for c + id = Q_f (slot f = 1..127)
// and c = Q_0, d = Q_128 in slot 0; with one reference also
//   single [ring][slot] (c - d, c + d) for the fused single-reference kernel.
#include "mra_common.h"

namespace mra {

__global__ void k_ref_polar(RefArgs a) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)a.K * a.R * kNphi) return;
  const int j = i % kNphi;
  const int ring = (i / kNphi) % a.R;
  const int k = i / ((int64_t)kNphi * a.R);
  const int c = a.L / 2;
  const double r = a.r_min + ring;
  const double x = c + r * a.cs64[j].x, y = c + r * a.cs64[j].y;
  const double x0 = floor(x), y0 = floor(y);
  const double fx = x - x0, fy = y - y0;
  const int ix = (int)x0, iy = (int)y0;
  const float* img = a.refs + (size_t)k * a.L * a.L;
  auto pix = [&](int xx, int yy) -> double {
    return (xx >= 0 && xx < a.L && yy >= 0 && yy < a.L) ? (double)img[yy * a.L + xx] : 0.0;
  };
  a.q64[i] = (1 - fx) * (1 - fy) * pix(ix, iy) + fx * (1 - fy) * pix(ix + 1, iy) +
             (1 - fx) * fy * pix(ix, iy + 1) + fx * fy * pix(ix + 1, iy + 1);
}

__global__ __launch_bounds__(256) void k_ref_norm(RefArgs a) {
  __shared__ double red[256];
  const int k = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < a.R * kNphi; i += 256) {
    const double q = a.q64[(size_t)k * a.R * kNphi + i];
    acc += (double)(a.r_min + i / kNphi) * q * q;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double nu = sqrt(red[0]);
    a.norm[k] = nu;
    a.inv[k] = a.normalize ? (nu > 0.0 ? 1.0 / nu : 0.0) : 1.0;
  }
}

__global__ void k_ref_spectra(RefArgs a) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)a.K * 129 * a.R) return;
  const int ring = i % a.R;
  const int f = (i / a.R) % 129;
  const int k = i / ((int64_t)a.R * 129);
  const double* q = a.q64 + ((size_t)k * a.R + ring) * kNphi;
  double re = 0.0, im = 0.0;
  for (int j = 0; j < kNphi; ++j) {
    const double2 w = a.cs64[(f * j) & 255];
    re += q[j] * w.x;
    im -= q[j] * w.y;
  }
  const double s = (double)(a.r_min + ring) * a.inv[k] / kNphi;
  a.Qs[i] = make_double2(re * s, im * s);
}

__global__ void k_ref_qhat(RefArgs a) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)a.K * a.R * kNphi) return;
  const int k = i / ((int64_t)a.R * kNphi);
  a.qhat32[i] = (float)(a.q64[i] * a.inv[k]);
}

__device__ __forceinline__ double packed_value(const RefArgs& a, int kt, int slot, int lane, int t) {
  // lane = 16 g + 2 ref + q: ring group g, column (ref, q) of the contraction's block
  const int g = lane >> 4, n = lane & 15;
  const int q = n & 1, ref = kt * kRefTile + (n >> 1);
  const int ring = g * a.R4 + t;
  if (t >= a.R4 || ring >= a.R || ref >= a.K) return 0.0;
  const double2* Q = a.Qs + (size_t)ref * 129 * a.R;
  double c, d;
  if (slot == 0) {
    c = Q[0 * a.R + ring].x;
    d = Q[128 * a.R + ring].x;
  } else {
    c = Q[slot * a.R + ring].x;
    d = Q[slot * a.R + ring].y;
  }
  return q ? c + d : c - d;
}

__global__ void k_ref_bmax(RefArgs a) {
  const int64_t total = (int64_t)a.n_ref_tiles * kSlots * a.R4 * 64;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  float m = 0.f;
  if (i < total) {
    const int lane = i % 64, t = (i / 64) % a.R4;
    const int slot = (i / (64 * (int64_t)a.R4)) % kSlots, kt = i / (64 * (int64_t)a.R4 * kSlots);
    m = (float)fabs(packed_value(a, kt, slot, lane, t));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) atomicMax(reinterpret_cast<unsigned int*>(a.bmax), __float_as_uint(m));
}

__global__ void k_ref_pack32(RefArgs a) {
  const int64_t total = (int64_t)a.n_ref_tiles * kSlots * a.R4 * 64;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int lane = i % 64, t = (i / 64) % a.R4;
  const int slot = (i / (64 * (int64_t)a.R4)) % kSlots, kt = i / (64 * (int64_t)a.R4 * kSlots);
  a.B32[i] = (float)packed_value(a, kt, slot, lane, t);
}

__global__ void k_ref_pack16(RefArgs a) {
  const int se = b16_slot_elems(a.R4), bt = b16_tail_width(a.R4);
  const int64_t total = (int64_t)a.n_ref_tiles * kSlots * se;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int off = i % se;
  const int slot = (i / se) % kSlots, kt = i / ((int64_t)se * kSlots);
  const int full = (a.NS - 1) * 512;  // elements of the steps stored 8 wide
  int lane, t;
  if (off < full) {
    lane = (off / 8) % 64;
    t = 8 * (off / 512) + off % 8;
  } else {
    lane = (off - full) / bt;
    t = 8 * (a.NS - 1) + (off - full) % bt;
  }
  const double v = packed_value(a, kt, slot, lane, t) * a.b_scale;
  if (a.prec == kBF16) {
    __bf16 h = (__bf16)(float)v;
    a.B16[i] = __builtin_bit_cast(uint16_t, h);
  } else {
    _Float16 h = (_Float16)(float)v;
    a.B16[i] = __builtin_bit_cast(uint16_t, h);
  }
}

// K = 1: the single reference's weighted spectrum per (ring, slot) as
// (c - d, c + d), read by the fused single-reference kernel.
__global__ void k_ref_pack_single(RefArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.R * kSlots) return;
  const int ring = i / kSlots, slot = i % kSlots;
  double c, d;
  if (slot == 0) {
    c = a.Qs[0 * a.R + ring].x;
    d = a.Qs[128 * a.R + ring].x;
  } else {
    c = a.Qs[slot * a.R + ring].x;
    d = a.Qs[slot * a.R + ring].y;
  }
  a.G1[i] = make_float2((float)(c - d), (float)(c + d));
}

static inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

hipError_t launch_ref_stage1(const RefArgs& a, hipStream_t st) {
  const int64_t nq = (int64_t)a.K * a.R * kNphi;
  hipLaunchKernelGGL(k_ref_polar, dim3(blocks_for(nq, 256)), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_ref_norm, dim3(a.K), dim3(256), 0, st, a);
  const int64_t ns = (int64_t)a.K * 129 * a.R;
  hipLaunchKernelGGL(k_ref_spectra, dim3(blocks_for(ns, 256)), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_ref_qhat, dim3(blocks_for(nq, 256)), dim3(256), 0, st, a);
  const int64_t nb = (int64_t)a.n_ref_tiles * kSlots * a.R4 * 64;
  hipLaunchKernelGGL(k_ref_bmax, dim3(blocks_for(nb, 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_ref_stage2(const RefArgs& a, hipStream_t st) {
  if (a.G1) hipLaunchKernelGGL(k_ref_pack_single, dim3(blocks_for((int64_t)a.R * kSlots, 256)), dim3(256), 0, st, a);
  if (a.prec == kFP32) {
    const int64_t n = (int64_t)a.n_ref_tiles * kSlots * a.R4 * 64;
    hipLaunchKernelGGL(k_ref_pack32, dim3(blocks_for(n, 256)), dim3(256), 0, st, a);
  } else {
    const int64_t n = (int64_t)a.n_ref_tiles * kSlots * b16_slot_elems(a.R4);
    hipLaunchKernelGGL(k_ref_pack16, dim3(blocks_for(n, 256)), dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

}  // namespace mra
