// Launchers of the optimiser kernels (optim.hip).
#pragma once

#include <cmath>

#include "sgs_common.h"

namespace sgs {

constexpr int kAdamGroups = 8;
constexpr int kAdamPoseThreads = 64;  // the pose step: one block, one thread per view
static_assert(GS_MAX_VIEWS <= kAdamPoseThreads, "every view's pose in the one block");

hipError_t launch_adam(const gs_adam_group* groups, int n_groups, float b1, float b2, float eps, int step,
                       hipStream_t s);
// step_dev non-null: the step count is read from and written back to device
// memory (step is then unused).
hipError_t launch_pose_step(gs_view* views_dev, int n_views, const float* grad, float* m, float* v, float lr_rho,
                            float lr_phi, float b1, float b2, float eps, int step, int32_t* step_dev,
                            hipStream_t s);

}  // namespace sgs
