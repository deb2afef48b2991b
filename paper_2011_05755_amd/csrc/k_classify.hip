// Convergence test of the iterative MRA loop (the outer repeat of
// Algorithm 1): count the particles whose class differs from the previous
// pass and remember the new classes for the next one.
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

}  // namespace

hipError_t launch_count_changed(const int32_t* cls, int32_t* prev, int n, int* count, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_count_changed, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, st, cls, prev, n,
                     count);
  return hipGetLastError();
}

}  // namespace mra
