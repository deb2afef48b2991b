// FP32 instantiations of the correlation kernel.
#include "corr_impl.h"

namespace mra {

// variant 0: 8 waves, particle operand resident (R4 exact where every work
// item shares it); 1: 4 waves, resident, R4 <= 12; 2: 8 waves, streamed.
void corr_dispatch_fp32(int variant, int r4min, int r4max, const CorrArgs* a, bool table, const CorrBatch* b,
                        int grid, hipStream_t st) {
  auto go = [&](auto c) { corr_go<decltype(c)>(a, table, b, grid, st); };
  if (variant == 0) {
    if (r4min != r4max) return go(Cfg<kFP32, 8, 9, true, false>{});
    switch (r4max) {
      case 1: return go(Cfg<kFP32, 8, 1, true, true>{});
      case 2: return go(Cfg<kFP32, 8, 2, true, true>{});
      case 3: return go(Cfg<kFP32, 8, 3, true, true>{});
      case 4: return go(Cfg<kFP32, 8, 4, true, true>{});
      case 5: return go(Cfg<kFP32, 8, 5, true, true>{});
      case 6: return go(Cfg<kFP32, 8, 6, true, true>{});
      case 7: return go(Cfg<kFP32, 8, 7, true, true>{});
      case 8: return go(Cfg<kFP32, 8, 8, true, true>{});
      default: return go(Cfg<kFP32, 8, 9, true, true>{});
    }
  }
  if (variant == 1) return go(Cfg<kFP32, 4, 12, true, false>{});
  return go(Cfg<kFP32, 8, 16, false, false>{});
}

// runner-up pass over the operand the first pass read: resident when that was
// the 8-wave resident form's layout (R4 <= 9), else streamed (slot-major)
void corr_runner_up_fp32(const CorrArgs& a, hipStream_t st) {
  if (a.a_layout == kRingPerm) launch_mode<Cfg<kFP32, 8, 9, true, false>, kRunnerUp>(a, st);
  else launch_mode<Cfg<kFP32, 8, 16, false, false>, kRunnerUp>(a, st);
}

}  // namespace mra
