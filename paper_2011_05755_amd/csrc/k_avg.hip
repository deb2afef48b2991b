// Class-average update (Algorithm 1: each image is transformed by its
// alignment parameters and the aligned images of a class give its new
// reference Y').  Each particle is warped back into its reference frame,
//   aligned(u) = Bil(X; c + s + Mir^m Rot(psi 2 pi / 256)(u - c)),
// and summed per class.  The sum runs in a fixed order so the result does
// not depend on scheduling:
//   1. per block of 1024 particles, per-class counts;
//   2. one workgroup scans them into stable class offsets and splits every
//      class into chunks of at most kAvgChunk particles;
//   3. particles are scattered into class order (stable; one workgroup per
//      block of 1024 particles);
//   4. one workgroup per chunk stages each image in LDS (coalesced read),
//      warps it and accumulates the chunk (at most kAvgChunk particles) in
//      FP32 registers;
//   5. per class and pixel the chunk sums are added in chunk order and
//      divided by the count; classes without members keep their image.
#include "mra_common.h"

namespace mra {

constexpr int kAvgBlk = 1024;

__global__ __launch_bounds__(256) void k_avg_hist(AvgArgs a) {
  extern __shared__ int hist[];
  for (int k = threadIdx.x; k < a.K; k += 256) hist[k] = 0;
  __syncthreads();
  const int64_t n0 = (int64_t)blockIdx.x * kAvgBlk;
  for (int i = threadIdx.x; i < kAvgBlk; i += 256) {
    const int64_t n = n0 + i;
    if (n < a.N) {
      const int k = a.ref[n];
      if (k >= 0 && k < a.K) atomicAdd(&hist[k], 1);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < a.K; k += 256) a.blk_cnt[(size_t)blockIdx.x * a.K + k] = hist[k];
}

// Per class: the total over blocks, then (one thread, K steps) the class and
// chunk starts, then each block's offset = class start + earlier blocks'
// counts.  The per-block loops carry no load-to-load dependence, so the
// loads of several blocks are in flight at once.
__global__ __launch_bounds__(256) void k_avg_scan(AvgArgs a) {
  for (int k = threadIdx.x; k < a.K; k += 256) {
    int run = 0;
#pragma unroll 8
    for (int b = 0; b < a.n_blk; ++b) run += a.blk_cnt[(size_t)b * a.K + k];
    a.counts[k] = run;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int cs = 0, ch = 0;
    for (int k = 0; k < a.K; ++k) {
      const int n = a.counts[k];
      a.cls_start[k] = cs;
      a.chunk_start[k] = ch;
      cs += n;
      ch += (n + kAvgChunk - 1) / kAvgChunk;
    }
    a.cls_start[a.K] = cs;
    a.chunk_start[a.K] = ch;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < a.K; k += 256) {
    int run = a.cls_start[k];
#pragma unroll 8
    for (int b = 0; b < a.n_blk; ++b) {
      const int c = a.blk_cnt[(size_t)b * a.K + k];
      a.blk_off[(size_t)b * a.K + k] = run;
      run += c;
    }
  }
}

// One workgroup of 16 waves per block of kAvgBlk particles (K up to
// kScatterMaxK): each wave ranks its 64 particles within their classes
// (ballot, rank by mbcnt) and counts them per class in LDS; per class, the
// waves' counts are turned into offsets in wave order after the block's own
// offset; then every particle goes to offset + rank, so each class's list
// stays in ascending particle order.
constexpr int kScatterMaxK = 2048;  // 16 x K ints of LDS
__global__ __launch_bounds__(1024) void k_avg_scatter16(AvgArgs a) {
  extern __shared__ int cnt[];  // [16][K]
  const int b = blockIdx.x, w = threadIdx.x >> 6, ln = threadIdx.x & 63;
  for (int i = threadIdx.x; i < 16 * a.K; i += 1024) cnt[i] = 0;
  __syncthreads();
  const int64_t n = (int64_t)b * kAvgBlk + threadIdx.x;
  int k = -1;
  if (n < a.N) {
    const int kk = a.ref[n];
    if (kk >= 0 && kk < a.K) k = kk;
  }
  int rank = 0;
  uint64_t todo = __ballot(k >= 0);
  while (todo) {
    const int leader = __ffsll((unsigned long long)todo) - 1;
    const int kk = __shfl(k, leader);
    const uint64_t same = __ballot(k == kk);
    if (k == kk) rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(same >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)same, 0));
    if (ln == leader) cnt[w * a.K + kk] = __popcll(same);
    todo &= ~same;
  }
  __syncthreads();
  for (int kk = threadIdx.x; kk < a.K; kk += 1024) {
    int run = a.blk_off[(size_t)b * a.K + kk];
    for (int w2 = 0; w2 < 16; ++w2) {
      const int c = cnt[w2 * a.K + kk];
      cnt[w2 * a.K + kk] = run;
      run += c;
    }
  }
  __syncthreads();
  if (k >= 0) a.order[cnt[w * a.K + k] + rank] = (int)n;
}

// Larger K: one wave per block of kAvgBlk particles, 64 at a time in particle order:
// the lanes of one class take consecutive places (ballot, rank by mbcnt)
// and the class's next place, kept in LDS, advances by their count, so each
// class's list stays in ascending particle order.
__global__ __launch_bounds__(64) void k_avg_scatter(AvgArgs a) {
  extern __shared__ int off[];
  const int b = blockIdx.x;
  for (int k = threadIdx.x; k < a.K; k += 64) off[k] = a.blk_off[(size_t)b * a.K + k];
  __syncthreads();
  const int64_t n0 = (int64_t)b * kAvgBlk;
  for (int j = 0; j < kAvgBlk; j += 64) {
    const int64_t n = n0 + j + threadIdx.x;
    int k = -1;
    if (n < a.N) {
      const int kk = a.ref[n];
      if (kk >= 0 && kk < a.K) k = kk;
    }
    uint64_t todo = __ballot(k >= 0);
    while (todo) {
      const int leader = __ffsll((unsigned long long)todo) - 1;
      const int kk = __shfl(k, leader);
      const uint64_t same = __ballot(k == kk);
      const int base = off[kk];
      if (k == kk) {
        const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(same >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)same, 0));
        a.order[base + rank] = (int)n;
      }
      __builtin_amdgcn_wave_barrier();
      if ((int)threadIdx.x == leader) off[kk] = base + __popcll(same);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      todo &= ~same;
    }
  }
}

template <int PPT>
__global__ __launch_bounds__(kAvgThreads) void k_avg_accum(AvgArgs a) {
  extern __shared__ float img[];
  const int c = blockIdx.x;
  if (c >= a.chunk_start[a.K]) return;
  int lo = 0, hi = a.K - 1;  // largest k with chunk_start[k] <= c (classes may be empty)
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.chunk_start[mid] <= c) lo = mid; else hi = mid - 1;
  }
  const int k = lo;
  const int start = a.cls_start[k] + (c - a.chunk_start[k]) * kAvgChunk;
  int end = start + kAvgChunk;
  if (end > a.cls_start[k + 1]) end = a.cls_start[k + 1];
  const int L = a.L, L2 = L * L;
  // the image sits in LDS with a zero border, one pixel before and two after
  // each row and column: positions clamped to [-1, L] then need no bounds
  // tests (a clamped position lands on border taps, as zero as the pixels
  // outside the box, and inside the box nothing changes).  One more cell
  // past the image takes the staging writes of a thread's slots beyond the
  // L x L pixels, so that no pixel loop branches.
  const int Lb = L + 3;
  const int spare = Lb * Lb;
  for (int i = threadIdx.x; i <= spare; i += kAvgThreads) img[i] = 0.f;
  // each thread's pixels u = tid + i * kAvgThreads; the next particle's
  // pixels are loaded into registers while the current one is warped
  // (slots past the image re-read the last pixel: their value goes to the
  // spare cell, and the loads stay unconditional)
  float nxt[PPT];
  auto fetch = [&](int pi) {
    const float* src = a.parts + (size_t)__builtin_amdgcn_readfirstlane(a.order[pi]) * L2;
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      // (the offset is opaque so that the 64-bit addresses are formed per
      // load, not kept in registers across the particle loop)
      uint32_t u = threadIdx.x + i * kAvgThreads;
      u = u < (uint32_t)L2 ? u : L2 - 1;
      asm volatile("" : "+v"(u));
      nxt[i] = __builtin_nontemporal_load(src + u);
    }
  };
  // Per pixel slot: (row << 16) | column (pixel (0, 0) for slots past the
  // image), and the LDS index of its staging cell (the spare one past the
  // image).  The packed coordinates are unpacked per particle (made opaque
  // below) rather than held as floats across the particle loop.
  uint32_t rc[PPT];
  int cell[PPT];
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int u = threadIdx.x + i * kAvgThreads;
    const int row = u < L2 ? u / L : 0, col = u < L2 ? u % L : 0;
    rc[i] = ((uint32_t)row << 16) | (uint32_t)col;
    cell[i] = u < L2 ? (row + 1) * Lb + col + 1 : spare;
  }
  const float Lf = (float)L, Lbf = (float)Lb;
  const float* img1 = img + Lb + 1;  // pixel (0, 0)
  // each chunk (at most kAvgChunk particles) is summed in FP32; the chunk
  // sums are added in FP64 by k_avg_final
  float acc[PPT];
#pragma unroll
  for (int i = 0; i < PPT; ++i) acc[i] = 0.f;
  if (start < end) fetch(start);
  for (int pi = start; pi < end; ++pi) {
    const int n = __builtin_amdgcn_readfirstlane(a.order[pi]);
    __syncthreads();  // the previous particle's warp has finished reading img
#pragma unroll
    for (int i = 0; i < PPT; ++i) img[cell[i]] = nxt[i];
    __syncthreads();
    if (pi + 1 < end) fetch(pi + 1);
    // sample position c + s + Mir^m Rot(psi)(u - c), in FP32 (positions are
    // below 2^8, so the bilinear fractions carry ~1e-5 px of rounding):
    //   X = ox + cs vx - sn vy,  Y = oy + m (sn vx + cs vy),  (vx, vy) = (col, row) - c
    // with the centre folded into the offsets
    const double2 cs64 = a.cs64[a.psi[n] & 255];
    const float cs = (float)cs64.x, sn = (float)cs64.y;
    const float msign = a.mirror[n] ? -1.f : 1.f;
    const float cxf = (float)a.cx;
    const float msn = msign * sn, mcs = msign * cs;
    const float ox = (float)(a.cx + a.shift_x[n]) - (cs - sn) * cxf;
    const float oy = (float)(a.cx + a.shift_y[n]) - (msn + mcs) * cxf;
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      uint32_t r = rc[i];
      asm volatile("" : "+v"(r));
      const float col = (float)(r & 0xffffu), row = (float)(r >> 16);
      const float X = __builtin_amdgcn_fmed3f(fmaf(cs, col, fmaf(-sn, row, ox)), -1.f, Lf);
      const float Y = __builtin_amdgcn_fmed3f(fmaf(msn, col, fmaf(mcs, row, oy)), -1.f, Lf);
      const float x0 = floorf(X), y0 = floorf(Y);
      const float fx = X - x0, fy = Y - y0;
      const int o = (int)fmaf(y0, Lbf, x0);  // exact: |y0 Lb + x0| < 2^24
      const float i00 = img1[o], i10 = img1[o + 1], i01 = img1[o + Lb], i11 = img1[o + Lb + 1];
      const float top = i00 + fx * (i10 - i00);
      const float bot = i01 + fx * (i11 - i01);
      acc[i] += top + fy * (bot - top);
    }
  }
  float* out = a.partial + (size_t)c * L2;
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int u = threadIdx.x + i * kAvgThreads;
    if (u < L2) out[u] = (float)acc[i];
  }
}

__global__ void k_avg_final(AvgArgs a) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int L2 = a.L * a.L;
  if (i >= (int64_t)a.K * L2) return;
  const int k = i / L2, u = i % L2;
  const int cnt = a.counts[k];
  if (cnt == 0) return;
  double s = 0.0;
  for (int c = a.chunk_start[k]; c < a.chunk_start[k + 1]; ++c) s += a.partial[(size_t)c * L2 + u];
  a.averages[i] = (float)(s / cnt);
}

hipError_t launch_averages(const AvgArgs& a, hipStream_t st) {
  if (a.N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_avg_hist, dim3(a.n_blk), dim3(256), (size_t)a.K * sizeof(int), st, a);
  hipLaunchKernelGGL(k_avg_scan, dim3(1), dim3(256), 0, st, a);
  if (a.K <= kScatterMaxK)
    hipLaunchKernelGGL(k_avg_scatter16, dim3(a.n_blk), dim3(1024), (size_t)16 * a.K * sizeof(int), st, a);
  else
    hipLaunchKernelGGL(k_avg_scatter, dim3(a.n_blk), dim3(64), (size_t)a.K * sizeof(int), st, a);
  const int L2 = a.L * a.L;
  const size_t lds = ((size_t)(a.L + 3) * (a.L + 3) + 1) * sizeof(float);
  const int ppt = (L2 + kAvgThreads - 1) / kAvgThreads;
  dim3 g(a.max_chunks), b(kAvgThreads);
  if (ppt <= 16) hipLaunchKernelGGL(k_avg_accum<16>, g, b, lds, st, a);
  else if (ppt <= 24) hipLaunchKernelGGL(k_avg_accum<24>, g, b, lds, st, a);
  else if (ppt <= 32) hipLaunchKernelGGL(k_avg_accum<32>, g, b, lds, st, a);
  else if (ppt <= 48) hipLaunchKernelGGL(k_avg_accum<48>, g, b, lds, st, a);
  else if (ppt <= 64) hipLaunchKernelGGL(k_avg_accum<64>, g, b, lds, st, a);
  else hipLaunchKernelGGL(k_avg_accum<100>, g, b, lds, st, a);
  const int64_t nf = (int64_t)a.K * L2;
  hipLaunchKernelGGL(k_avg_final, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace mra
