// Convergence test of the iterative MRA loop (the outer repeat of
// Algorithm 1): count the particles whose class differs from the previous
// pass and remember the new classes for the next one.  Also a plain zero
// fill, used in place of a memset node where the alignment path clears
// memory (so that a caller can capture that path in a HIP graph).
#include <algorithm>

#include "mra_common.h"

namespace mra {

namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void k_count_changed(const int32_t* __restrict__ cls,
                                                            int32_t* __restrict__ prev, int n,
                                                            int* __restrict__ count) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  bool changed = false;
  if (i < n) {
    const int32_t k = cls[i];
    changed = k != prev[i];
    prev[i] = k;
  }
  const unsigned long long m = __ballot(changed);
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(count, __popcll(m));
}

// Zero n 16-byte words (grid-stride).
__global__ __launch_bounds__(kThreads) void k_fill_zero(uint4* __restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

}  // namespace

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  if (((uintptr_t)p & 15) || (bytes & 15)) return hipErrorInvalidValue;
  const size_t n = bytes / 16;
  const size_t blocks = std::min<size_t>((n + kThreads - 1) / kThreads, 2048);
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(kThreads), 0, st, (uint4*)p, n);
  return hipGetLastError();
}

hipError_t launch_count_changed(const int32_t* cls, int32_t* prev, int n, int* count, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_count_changed, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, st, cls, prev, n,
                     count);
  return hipGetLastError();
}

}  // namespace mra
