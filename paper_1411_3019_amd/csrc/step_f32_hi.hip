// step_f32_hi.hip -- step-kernel instances of the FP32 force class, variants 2
// and 3 of kStepVariants.
#include "launch.hpp"

namespace mdk {

void launch_step_f32_hi(const StepLaunch& L, int variant, bool all, bool stream) {
  if (variant == 3)
    MDK_LAUNCH4(k_step_f32, kStepVariants[3].waves, kStepVariants[3].halo, L, all, stream);
  else
    MDK_LAUNCH4(k_step_f32, kStepVariants[2].waves, kStepVariants[2].halo, L, all, stream);
}

}  // namespace mdk
