// Launchers of the map-growth and scale-regularisation kernels (growth.hip).
#pragma once

#include "sgs_common.h"

namespace sgs {

size_t expand_workspace_bytes(int64_t P);
hipError_t launch_expand(const uint8_t* masks, const float* rgb_t, const float* depth_t, const float* feat_init,
                         int n_feat, int64_t P, const gs_view* views_dev, int n_views, int64_t* n_dev,
                         int64_t capacity, int64_t* candidates, const gs_gaussian_grads& g, void* ws, hipStream_t s);
size_t dsr_workspace_bytes(int64_t n);
hipError_t launch_dsr(const float* log_scale, int64_t n, float w_big, float w_small, float* grad_ls, double* out,
                      void* ws, hipStream_t s);

}  // namespace sgs
