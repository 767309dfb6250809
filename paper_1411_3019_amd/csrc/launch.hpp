// launch.hpp -- host-side launchers of the step kernels.  Each force class's
// instances are compiled in a translation unit of their own (step_*.hip), so
// the library builds in parallel; the engine calls these launchers.
#pragma once

#include "step.hpp"

namespace mdk {

// FP32-class step-kernel instances the autotuner chooses among: occupancy
// target (wavefronts per SIMD) and halo entries staged in LDS.
struct StepVariant {
  int waves, halo;
};
constexpr StepVariant kStepVariants[] = {{6, kHaloLdsDefault}, {7, 512}, {7, 384}, {5, 1024}};
constexpr int kNumStepVariants = (int)(sizeof(kStepVariants) / sizeof(kStepVariants[0]));

// Arguments of one step launch: the grid, the stream, the buffers, the tile
// list of the class (job per tile, first slot per tile, tile count on the
// device) and the step offset t within the chunk.
struct StepLaunch {
  dim3 grid;
  hipStream_t stream;
  const DevBufs* B;
  const int* tile_job;
  const int64_t* tile_first;
  const int* ntiles;
  int t;
};

// all: kernels built with every surface kind (jobs on the height field or the
// bridge); stream: streaming stores of the new state.
void launch_step_f64(const StepLaunch& L, bool all, bool stream);
void launch_step_model(const StepLaunch& L, bool f64, bool all, bool stream);
void launch_step_f32(const StepLaunch& L, int variant, bool all, bool stream);
void launch_step_f32_hi(const StepLaunch& L, int variant, bool all, bool stream);  // variants 2..

// The four instances (surface set x store policy) of one kernel template.
#define MDK_LAUNCH4(KERNEL, WAVES, HALO, L, ALL, STREAM)                                                        \
  do {                                                                                                          \
    const dim3 blk_(kTile);                                                                                     \
    if (ALL) {                                                                                                  \
      if (STREAM)                                                                                               \
        hipLaunchKernelGGL((KERNEL<true, true, WAVES, HALO>), (L).grid, blk_, 0, (L).stream, *(L).B,            \
                           (L).B->jobs, (L).B->models, (L).tile_job, (L).tile_first, (L).ntiles, (L).t);       \
      else                                                                                                      \
        hipLaunchKernelGGL((KERNEL<true, false, WAVES, HALO>), (L).grid, blk_, 0, (L).stream, *(L).B,           \
                           (L).B->jobs, (L).B->models, (L).tile_job, (L).tile_first, (L).ntiles, (L).t);       \
    } else {                                                                                                    \
      if (STREAM)                                                                                               \
        hipLaunchKernelGGL((KERNEL<false, true, WAVES, HALO>), (L).grid, blk_, 0, (L).stream, *(L).B,           \
                           (L).B->jobs, (L).B->models, (L).tile_job, (L).tile_first, (L).ntiles, (L).t);       \
      else                                                                                                      \
        hipLaunchKernelGGL((KERNEL<false, false, WAVES, HALO>), (L).grid, blk_, 0, (L).stream, *(L).B,          \
                           (L).B->jobs, (L).B->models, (L).tile_job, (L).tile_first, (L).ntiles, (L).t);       \
    }                                                                                                           \
  } while (0)

}  // namespace mdk
