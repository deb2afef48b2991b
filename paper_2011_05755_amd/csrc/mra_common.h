// Shared constants, launch-argument structs and launcher declarations of
// the MRA kernels (gfx950).  Host code includes this to launch; kernels
// include it for the argument layouts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mra {

constexpr int kNphi = 256;          // angles per ring (the paper's workloads)
constexpr int kSlots = 128;         // frequency slots: f = 1..127, slot 0 = (f 0, f 128)

constexpr int kRowTile = 8;         // particle rows (shift, particle) per correlation tile
constexpr int kRefTile = 8;         // references per correlation tile
constexpr int kPolarWaves = 8;      // resampling workgroup: 8 waves, 8 shifts x 8 FFT lanes each
constexpr int kPolarThreads = 64 * kPolarWaves;
constexpr int kMaxBatchPieces = 12; // stack pieces per batched launch (kernel-argument table)
constexpr int kAvgChunk = 32;       // particles per partial class sum
constexpr int kAvgThreads = 256;
constexpr int kMaxRunTiles = 48;    // consecutive row tiles per correlation workgroup (a run), at most

enum Prec { kFP32 = 0, kBF16 = 1, kFP16 = 2 };

// Re-ranked 16-bit forms: the rows whose 16-bit best lies within this
// fraction of the particle's best are the re-ranking candidates (and keep
// their exact best under pruning): one unit roundoff of the contraction's
// operand type, 2^-8 for BF16 and 2^-11 for FP16.
__host__ __device__ constexpr float rerank_margin(int prec) {
  return prec == kBF16 ? 1.f / 256.f : (prec == kFP16 ? 1.f / 2048.f : 0.f);
}

// Layouts of the particle operand A (per row tile of 8 rows, 16 floats per
// (ring, slot): p*8 + row%8):
//   kRingMajor  [ring < 4*R4][slot][16]: one (ring, row group) item of the
//               resampler writes one contiguous 8 KB run
//   kRingPerm   the same with slot s at position slot_pos(s), so that the
//               slots s = w + 8 i of correlation wave w are contiguous, and
//               positions 2m, 2m+1 interleaved element by element in one
//               128-byte block (float 2k + (pos & 1) holds element k), so
//               that one 8-byte load per lane reads both (FP32, 8 waves,
//               operand resident)
//   kSlotMajor  [slot][ring < 4*R4][16]: each slot's rings contiguous (FP32
//               4-wave and streamed contractions, which re-read the operand)
//   kRingPerm16  the 16-bit forms: elements rounded once by the resampler in
//               the contraction's type (BF16, or FP16 scaled by a power of two
//               per particle), [ring < 4*R4][128 positions][16] per row tile
//               with slot s at position slot_pos(s) (wave w's slots w + 8 i at
//               16 w + i) and each run of 8 positions interleaved by element:
//               element k of position 8 G + j at a16_index(8 G + j, k), so that
//               one 16-byte load gives a lane element k of 8 of its wave's slots
enum ALayout { kRingMajor = 0, kRingPerm = 1, kSlotMajor = 2, kRingPerm16 = 3 };
__host__ __device__ constexpr int slot_pos(int s) { return (s & 7) * 16 + (s >> 3); }
// 16-bit index of element k of position pos within one (row tile, ring) block
__host__ __device__ constexpr int a16_index(int pos, int k) { return (pos >> 3) * 128 + k * 8 + (pos & 7); }
// The layout a correlation launch reads (and the resampler must write).
__host__ __device__ constexpr int a_layout_for(int prec, int variant) {
  return prec != kFP32 ? kRingPerm16 : (variant == 0 ? kRingPerm : kSlotMajor);
}
// bytes per operand element of a layout
__host__ __device__ constexpr int a_elem_bytes(int layout) { return layout == kRingPerm16 ? 2 : 4; }

// 16-bit reference operand of one (reference tile, slot): NS = ceil(R4 / 8)
// steps of 8 rings per lane group; with NS >= 2 the last step is stored only
// as wide as the rings it holds (2, 4 or 8 elements per lane): the
// contraction reads that many, and the elements it pads with meet zeros of
// the particle operand.
__host__ __device__ constexpr int b16_tail_width(int R4) {
  return R4 <= 8 ? 8 : (R4 - 8 * ((R4 - 1) / 8) <= 2 ? 2 : (R4 - 8 * ((R4 - 1) / 8) <= 4 ? 4 : 8));
}
// 16-bit elements per (reference tile, slot) block
__host__ __device__ constexpr int b16_slot_elems(int R4) { return (((R4 + 7) / 8 - 1) * 8 + b16_tail_width(R4)) * 64; }

// Power-of-two FP16 scale of a particle's operand: |a +- b| <= 2 * 256 *
// max|pixel| is mapped below 2^14.
__device__ __forceinline__ float fp16_operand_scale(float maxabs) {
  const float m = fmaxf(maxabs * 512.f, 1e-30f);
  return ldexpf(1.f, 14 - (int)ceilf(log2f(m)));
}

// Entry of the particle sampling stencil for ring r and angle j (FP64
// positions, used by the FP32 re-score and the single-reference kernel): the floor (dx, dy) of
// r*(cos, sin)(theta_j), stored as bx = 4 dx (the byte offset of the column
// in a float row) and dy, and the bilinear fractions.
struct __attribute__((aligned(16))) Stencil {
  int bx, dy;
  float fx, fy;
};

// Resample + ring-FFT kernel.  out layout depends on the mode:
//  mode 0: correlation operand A in layout a_layout (ALayout),
//          inner index p*8 + row%8 (p = 0: a-b, p = 1: a+b); rings >= R are
//          never written (the correlation kernel masks them)
//  mode 1: polar samples [n][S][R][256]
//  mode 2: ring spectra  [n][S][R][129][2]
struct PolarArgs {
  const float* parts;  // first particle of the chunk, [n][L][L]
  int n_part;
  int L, R, R4, T, S1, S;
  int Lp, pad, cx;     // LDS image side (with zero border), border width, centre
  int r_min;           // radius of ring 0
  int a_layout;        // mode 0: ALayout of the operand
  int prec;            // kRingPerm16: kBF16 or kFP16
  const float* maxabs; // kFP16: max |pixel| of each particle of the chunk (operand scale)
  const double2* cs64; // (cos, sin)(2 pi j / 256)
  float* out;          // (mode 0, kRingPerm16: 16-bit elements)
};

// Fused contraction + inverse FFT over angle + arg-max.
struct CorrArgs {
  const float* A;        // [row tiles][...] in layout a_layout (ALayout; 16-bit elements for kRingPerm16)
  int a_layout;
  int n_row_tiles;
  int rows;              // valid rows in the chunk (n * S)
  const float* B32;      // [ref tiles][128][R4][64]
  const uint16_t* B16;   // [ref tiles][128][b16_slot_elems(R4)]: NS - 1 steps [64][8], then [64][BT]
  int R, R4, NS, n_ref_tiles, K, S, M;
  int BT;                // b16_tail_width(R4)
  const float* maxabs;   // FP16: max |pixel| of each particle of the chunk (A scale), else null
  float b_scale;         // FP16: power-of-two scale folded into B16
  const float2* cs32;
  float* row_cc;         // [rows] best CC of the row
  int* row_idx;          // [rows] flat index of the row's best
  float* table;          // debug: [n][K][M][S][256], else null
  const int* excl;       // per particle of the chunk: flat index left out of the arg-max, or null
  int prune;             // 1: skip the inverse FFT of pairs whose CC bound is below the row's threshold
  int tiles_per_run;     // consecutive row tiles per workgroup (>= 1)
  float margin;          // particle threshold: best - margin * |best| (0: the best itself)
};

// Batched correlation: pieces of several stacks in one launch, one
// workgroup per run of row tiles.  run_start[i] is the first run of piece i;
// run_start[n] the total.
struct CorrBatch {
  int n;
  int run_start[kMaxBatchPieces + 1];
  CorrArgs piece[kMaxBatchPieces];
};

struct MergeArgs {
  const float* row_cc;
  const int* row_idx;
  int n_part, S, S1, T, M;
  int64_t out_off;
  int32_t *ref, *shift_x, *shift_y, *psi, *mirror, *flat;
  float *cc, *cc2;
  int32_t* win;          // chunk-local copy of each winner's flat index, or null
  int runner_up;         // 1: rows hold the best without the winner; write only cc2
};

struct RescoreArgs {
  const float* parts;
  int n_part;
  int64_t out_off;
  int L, R, r_min, Lp, pad, cx, K, T;
  const Stencil* stencil;
  const float* qhat;     // [K][R][256]
  const int32_t *ref, *shift_x, *shift_y, *psi, *mirror;
  float* cc;
  // Re-ranking (rows >= 2): the winners of the particle's `rows` best rows of
  // the 16-bit pass and their neighbours within +-1 angle are re-scored in
  // FP32 and the best of them becomes the result.  rows <= 1: the winner only.
  int rows, S1, S, M;
  float margin;          // rows within this fraction of the particle's 16-bit best are candidates
  const float* row_cc;   // [n_part][S] of the 16-bit pass
  const int* row_idx;
  int32_t *ref_w, *shift_x_w, *shift_y_w, *psi_w, *mirror_w, *flat_w;  // re-ranked outputs
  int32_t* win;          // chunk-local winner copy for the runner-up pass, or null
  float* psi_frac;       // refinement launch: sub-step angle of the final winner
};

// Batched forms of the per-particle kernels: item i of the launch is
// particle i - start[p] of piece p with start[p] <= i < start[p + 1].
struct PolarBatch {
  int n;
  int start[kMaxBatchPieces + 1];
  PolarArgs piece[kMaxBatchPieces];
};
struct MergeBatch {
  int n;
  int start[kMaxBatchPieces + 1];
  MergeArgs piece[kMaxBatchPieces];
};
struct RescoreBatch {
  int n;
  int start[kMaxBatchPieces + 1];
  RescoreArgs piece[kMaxBatchPieces];
};

// Alignment against one reference (K = 1): resampling, ring FFTs,
// correlation, inverse FFT and arg-max fused per particle.
struct RfaArgs {
  const float* parts;    // first particle of the call, [n][L][L]
  int n_part;
  int64_t out_off;
  int L, R, T, S1, S, M, Lp, pad, cx, r_min;
  const Stencil* stencil;  // [R][256]
  const double2* cs64;
  const float2* G;       // [R][128]: (c - d, c + d) of the reference's weighted spectrum per slot
  int32_t *ref, *shift_x, *shift_y, *psi, *mirror, *flat;
  float *cc, *cc2;
};

// ---- launchers (one .hip file each) ----
hipError_t launch_polar(int mode, const PolarArgs& a, hipStream_t st);
size_t polar_lds_bytes(int Lp);
hipError_t launch_corr(int prec, int variant, bool table, const CorrArgs& a, hipStream_t st);
hipError_t launch_corr_runner_up(int prec, const CorrArgs& a, hipStream_t st);
hipError_t launch_corr_batch(int prec, int variant, const CorrBatch& b, int grid, hipStream_t st);
// row tiles per correlation run for a launch of `tiles` tiles on n_cu CUs:
// long runs carry each particle's best across its tiles (fewer tiles start
// without a threshold), enough runs keep every CU busy to the launch's end.
// Runs of up to 8 tiles as long as every CU gets 3 runs; longer ones (up to
// kMaxRunTiles) while every CU still gets 20, which measured best on the
// 100k workload at 32 and 128 GiB workspaces.
inline int corr_tiles_per_run(int tiles, int n_cu) {
  const int cu = n_cu > 0 ? n_cu : 1;
  const int a = tiles / (3 * cu), b = tiles / (20 * cu);
  const int g = b > (a < 8 ? a : 8) ? b : (a < 8 ? a : 8);
  return g < 1 ? 1 : (g > kMaxRunTiles ? kMaxRunTiles : g);
}
bool corr_variant_ok(int prec, int variant, int R4);
int corr_default_variant(int prec, int R4);
hipError_t launch_merge(const MergeArgs& a, hipStream_t st);
hipError_t launch_rescore(const RescoreArgs& a, hipStream_t st);
hipError_t launch_polar_batch(const PolarBatch& b, hipStream_t st);
hipError_t launch_merge_batch(const MergeBatch& b, hipStream_t st);
hipError_t launch_rescore_batch(const RescoreBatch& b, hipStream_t st);
hipError_t launch_refine(const RescoreArgs& a, hipStream_t st);  // psi_frac from the final parameters
hipError_t launch_part_maxabs(const float* x, int n_part, int L, float* out, hipStream_t st);
hipError_t launch_rfa(const RfaArgs& a, hipStream_t st);
// zero `bytes` (a multiple of 16) at p (16-byte aligned) with a kernel
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st);
// count[0] += #{i : cls[i] != prev[i]}; then prev = cls
hipError_t launch_count_changed(const int32_t* cls, int32_t* prev, int n, int* count, hipStream_t st);

// reference preparation
struct RefArgs {
  const float* refs;
  int K, L, r_min, R, R4, NS, n_ref_tiles, normalize, prec;
  const double2* cs64;
  double* q64;       // [K][R][256]
  double* inv;       // [K]  1/norm (or 1)
  double* norm;      // [K]
  double2* Qs;       // [K][129][R]  w_r Q / (norm 256)
  float* qhat32;     // [K][R][256]
  float* B32;
  uint16_t* B16;
  float2* G1;        // K = 1: [R][128] (c - d, c + d) per slot, else null
  float* bmax;       // device scalar: max |B| (for the FP16 scale)
  float b_scale;
};
hipError_t launch_ref_stage1(const RefArgs& a, hipStream_t st);  // polar, norm, spectra, qhat, bmax
hipError_t launch_ref_stage2(const RefArgs& a, hipStream_t st);  // pack B32 / B16

// class averages
struct AvgArgs {
  const float* parts;
  int64_t N;
  int K, L, cx;
  const int32_t *ref, *shift_x, *shift_y, *psi, *mirror;
  const double2* cs64;
  int n_blk;            // ceil(N / 1024)
  int* blk_cnt;         // [n_blk][K]
  int* blk_off;         // [n_blk][K]
  int* cls_start;       // [K + 1]
  int* chunk_start;     // [K + 1]
  int* order;           // [N]
  int max_chunks;
  float* partial;       // [max_chunks][L*L]
  float* averages;      // [K][L][L] in/out
  int32_t* counts;      // [K]
};
hipError_t launch_averages(const AvgArgs& a, hipStream_t st);

}  // namespace mra
