// step_model.hip -- step-kernel instances of bead-model jobs (both force classes).
#include "launch.hpp"

namespace mdk {

void launch_step_model(const StepLaunch& L, bool f64, bool all, bool stream) {
  if (f64)
    MDK_LAUNCH4(k_step_model, 5, kHaloLdsDefault, L, all, stream);
  else
    MDK_LAUNCH4(k_step_model_f32, 5, kHaloLdsDefault, L, all, stream);
}

}  // namespace mdk
