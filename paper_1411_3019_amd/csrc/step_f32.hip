// step_f32.hip -- step-kernel instances of the FP32 force class, variants 0
// and 1 of kStepVariants (the others are in step_f32_hi.hip).
#include "launch.hpp"

namespace mdk {

void launch_step_f32(const StepLaunch& L, int variant, bool all, bool stream) {
  switch (variant) {
    case 0:
      MDK_LAUNCH4(k_step_f32, kStepVariants[0].waves, kStepVariants[0].halo, L, all, stream);
      break;
    case 1:
      MDK_LAUNCH4(k_step_f32, kStepVariants[1].waves, kStepVariants[1].halo, L, all, stream);
      break;
    default:
      launch_step_f32_hi(L, variant, all, stream);
      break;
  }
}

}  // namespace mdk
