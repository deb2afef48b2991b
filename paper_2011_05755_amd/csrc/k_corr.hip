// Host side of the correlation kernel (variant selection and launch) and
// the per-particle merge of row results.  The kernel itself is in
// corr_impl.h, instantiated per precision in k_corr_{fp32,bf16,fp16}.hip.
#include "corr_impl.h"

namespace mra {

// Variant ids (chosen by the caller; see corr_variant_ok):
//   FP32:   0 = 8 waves, A resident, R4 <= 9; 1 = 4 waves, A resident, R4 <= 12;
//           2 = 8 waves, A streamed, R4 <= 16
//   16-bit: 0 = A converted once per row tile and resident, 1 = A re-read
//           and converted per reference tile (8 waves, R4 <= 16)
bool corr_variant_ok(int prec, int variant, int R4) {
  if (R4 < 1 || R4 > 16) return false;
  if (prec == kFP32) return (variant == 0 && R4 <= 9) || (variant == 1 && R4 <= 12) || variant == 2;
  return variant == 0 || variant == 1;
}

int corr_default_variant(int prec, int R4) {
  if (prec == kFP32) return R4 <= 9 ? 0 : 2;
  return 0;
}

static void dispatch(int prec, int variant, int r4min, int r4max, const CorrArgs* a, bool table,
                     const CorrBatch* b, int grid, hipStream_t st) {
  if (prec == kFP32) corr_dispatch_fp32(variant, r4min, r4max, a, table, b, grid, st);
  else if (prec == kBF16) corr_dispatch_bf16(variant, r4min, r4max, a, table, b, grid, st);
  else corr_dispatch_fp16(variant, r4min, r4max, a, table, b, grid, st);
}

hipError_t launch_corr(int prec, int variant, bool table, const CorrArgs& a, hipStream_t st) {
  if (a.n_row_tiles <= 0) return hipSuccess;
  if (table) variant = prec == kFP32 ? 2 : 0;  // any R4 (the host writes the operand for this form)
  if (!corr_variant_ok(prec, variant, a.R4)) return hipErrorInvalidValue;
  dispatch(prec, variant, a.R4, a.R4, &a, table, nullptr, 0, st);
  return hipGetLastError();
}

hipError_t launch_corr_runner_up(int prec, const CorrArgs& a, hipStream_t st) {
  if (a.n_row_tiles <= 0) return hipSuccess;
  if (a.R4 < 1 || a.R4 > 16 || !a.excl) return hipErrorInvalidValue;
  if (prec == kFP32) corr_runner_up_fp32(a, st);
  else if (prec == kBF16) corr_runner_up_bf16(a, st);
  else corr_runner_up_fp16(a, st);
  return hipGetLastError();
}

hipError_t launch_corr_batch(int prec, int variant, const CorrBatch& b, int grid, hipStream_t st) {
  if (b.n <= 0 || grid <= 0) return hipSuccess;
  int r4min = 1 << 30, r4max = 0;
  for (int i = 0; i < b.n; ++i) {
    r4max = b.piece[i].R4 > r4max ? b.piece[i].R4 : r4max;
    r4min = b.piece[i].R4 < r4min ? b.piece[i].R4 : r4min;
  }
  if (!corr_variant_ok(prec, variant, r4max)) return hipErrorInvalidValue;
  dispatch(prec, variant, r4min, r4max, nullptr, false, &b, grid, st);
  return hipGetLastError();
}

// Per-particle merge of its S row results (arg-max over shifts with the
// same tie rule) and decoding of the flat index into alignment parameters.
__device__ __forceinline__ void merge_particle(const MergeArgs& a, int n) {
  float best = -INFINITY;
  int bi = 0x7fffffff;
  for (int s = 0; s < a.S; ++s) {
    const float v = a.row_cc[(size_t)n * a.S + s];
    const int i = a.row_idx[(size_t)n * a.S + s];
    if (better(v, i, best, bi)) { best = v; bi = i; }
  }
  const int64_t o = a.out_off + n;
  if (a.runner_up) {  // second pass: the best over every candidate but the winner
    a.cc2[o] = bi == 0x7fffffff ? NAN : best;
    return;
  }
  if (a.win) a.win[n] = bi == 0x7fffffff ? -1 : bi;
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

__global__ __launch_bounds__(256) void k_merge(MergeArgs a) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n < a.n_part) merge_particle(a, n);
}

__global__ __launch_bounds__(256) void k_merge_batch(MergeBatch b) {
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= b.start[b.n]) return;
  int p = 0;
  while (p + 1 < b.n && b.start[p + 1] <= item) ++p;
  merge_particle(b.piece[p], item - b.start[p]);
}

hipError_t launch_merge(const MergeArgs& a, hipStream_t st) {
  if (a.n_part <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_merge, dim3((a.n_part + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_merge_batch(const MergeBatch& b, hipStream_t st) {
  if (b.n <= 0 || b.start[b.n] <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_merge_batch, dim3((b.start[b.n] + 255) / 256), dim3(256), 0, st, b);
  return hipGetLastError();
}

}  // namespace mra
