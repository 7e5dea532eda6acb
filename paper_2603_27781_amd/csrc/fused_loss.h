// The image-space loss of gs_loss_grad (GS^3LAM Sec. 3.3.4 / 3.4: L1 colour,
// L1 depth, cross-entropy of softmax(W^T F)) evaluated in the epilogue of
// the forward compositing kernel, where each pixel's rendered values are
// still in registers (gs_render_fwd_loss).
#pragma once

#include "sgs_common.h"

namespace sgs {

// Kernel-side arguments of the fused loss (by value).
struct FusedLoss {
    const float* rgb_t;     // [3][P]
    const float* depth_t;   // [P]
    const int32_t* labels;  // [P]
    const float* Wt;        // the decoder transposed, [K][F] (a kernel argument of its own, __restrict__)
    int K;                  // classes (0: no semantic term)
    float w0, w1, w2;       // term weights
    float* grad_out;        // [5 + F][P]
    double* partials;       // [3][total_tiles]: the terms summed over each tile
};

// The fused path keeps the class logits in registers next to the rendered
// channels: at most this many feature channels and classes (with 20 the
// kernel fits 96 registers, five wavefronts per SIMD, without spills; with
// 32 it spilled).
constexpr int kFusedMaxFeat = 16, kFusedMaxClasses = 20;

size_t fused_loss_workspace_bytes(int total_tiles);
hipError_t launch_render_fwd_loss(const float* rec, const float* app, int n, int n_feat, const int32_t* inst,
                                  const int32_t* inst_gid, const int32_t* ranges, const gs_view* views_dev,
                                  int n_views, int total_tiles, int64_t total_pixels, const RasterConst& c,
                                  int lds_batch, int persistent, float* out, float* T_final, int32_t* last,
                                  int32_t* queue, const float* rgb_t, const float* depth_t, const int32_t* labels,
                                  const float* decoder, int n_classes, const float* weights, float* grad_out,
                                  double* loss, void* ws, hipStream_t s);

// Pieces of the plain loss path the fused one shares (loss.hip): the
// decoder transpose, and the fixed-order sum of three term-major partial
// arrays [3][n] into loss[4] = (colour, depth, semantic, total).
hipError_t launch_transpose_decoder(const float* W, int F, int K, float* Wt, hipStream_t s);
hipError_t launch_loss_sums(const double* partials, int n, double* stage, double* loss, hipStream_t s);

}  // namespace sgs
