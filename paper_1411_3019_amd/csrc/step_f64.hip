// step_f64.hip -- step-kernel instances of the FP64 force class.
#include "launch.hpp"

namespace mdk {

void launch_step_f64(const StepLaunch& L, bool all, bool stream) {
  MDK_LAUNCH4(k_step_f64, 5, kHaloLdsDefault, L, all, stream);
}

}  // namespace mdk
