// BF16 instantiations of the correlation kernel.
#include "corr_impl.h"

namespace mra {

// variant 0: particle operand converted once per row tile and resident;
// 1: re-read and converted per reference tile.
void corr_dispatch_bf16(int variant, int r4min, int r4max, const CorrArgs* a, bool table, const CorrBatch* b,
                        int grid, hipStream_t st) {
  if (variant == 0) corr_dispatch_16<kBF16, true>(r4min, r4max, a, table, b, grid, st);
  else corr_dispatch_16<kBF16, false>(r4min, r4max, a, table, b, grid, st);
}

void corr_runner_up_bf16(const CorrArgs& a, hipStream_t st) {
  launch_mode<Cfg<kBF16, 8, 16, true, false>, kRunnerUp>(a, st);  // operand resident, R4 <= 16
}

}  // namespace mra
