// Pieces shared by the image-space loss kernels (the plain losses and the
// SLAM losses with masks and SSIM).
#pragma once

#include "sgs_common.h"

namespace sgs {

// Copies the decoder W [F][K] (row-major) transposed into Wt [K][F], so that
// a class row is contiguous for the per-pixel kernels.
__global__ void k_transpose_decoder(const float* __restrict__ W, int F, int K, float* __restrict__ Wt);

// Fixed-order sums of per-block partials, first stage over many workgroups:
// block b sums elements [b * kSumChunk, (b + 1) * kSumChunk) of each of the
// `terms` term-major arrays src[term][n] into dst[term][gridDim.x] (the
// partials are written from every XCD, so one workgroup reading them all
// would pay many long round trips).
constexpr int kSumThreads = 256, kSumPer = 16, kSumChunk = kSumThreads * kSumPer;
__global__ void k_sum_stage(const double* __restrict__ src, int n, int terms, double* __restrict__ dst);
inline int sum_stage_blocks(int64_t n) { return (int)((n + kSumChunk - 1) / kSumChunk); }

// Cross-entropy of softmax(W^T f + b) (b optional) against `lab` for one pixel (the fixed
// linear decoder standing in for F_cnn, Sec. 3.2.2, Eq. 8) and its gradient
// gf = dCE/df = sum_k W[.][k] softmax_k - W[.][lab].  With at most KC
// classes the logits stay in registers; KC = 0 recomputes them in the second
// pass.  A class row of Wt is wavefront-uniform, so its values are scalar
// loads feeding the FMAs directly.
template <int F, int KC>
__device__ __forceinline__ float semantic_ce(const float (&fv)[F > 0 ? F : 1], const float* __restrict__ Wt, int K,
                                             int lab, float (&gf)[F > 0 ? F : 1],
                                             const float* __restrict__ bias = nullptr) {
    float m = -INFINITY, zl = 0.0f, se = 0.0f;
    float ga[F > 0 ? F : 1];
#pragma unroll
    for (int f = 0; f < F; ++f) ga[f] = 0.0f;
    if constexpr (KC > 0) {
        float z[KC];
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            if (k < K) {
                const float* wr = Wt + k * F;
                float acc = bias != nullptr ? bias[k] : 0.0f;
#pragma unroll
                for (int f = 0; f < F; ++f) acc = fmaf(wr[f], fv[f], acc);
                z[k] = acc;
                m = fmaxf(m, acc);
                zl = k == lab ? acc : zl;
            }
        }
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            if (k < K) {
                const float* wr = Wt + k * F;
                const float e = __expf(z[k] - m);
                se += e;
#pragma unroll
                for (int f = 0; f < F; ++f) ga[f] = fmaf(wr[f], e, ga[f]);
            }
        }
    } else {
        for (int k = 0; k < K; ++k) {
            const float* wr = Wt + k * F;
            float acc = bias != nullptr ? bias[k] : 0.0f;
#pragma unroll
            for (int f = 0; f < F; ++f) acc = fmaf(wr[f], fv[f], acc);
            m = fmaxf(m, acc);
            zl = k == lab ? acc : zl;
        }
        for (int k = 0; k < K; ++k) {
            const float* wr = Wt + k * F;
            float acc = bias != nullptr ? bias[k] : 0.0f;
#pragma unroll
            for (int f = 0; f < F; ++f) acc = fmaf(wr[f], fv[f], acc);
            const float e = __expf(acc - m);
            se += e;
#pragma unroll
            for (int f = 0; f < F; ++f) ga[f] = fmaf(wr[f], e, ga[f]);
        }
    }
    const float inv = 1.0f / se;
    const bool lab_ok = lab >= 0 && lab < K;
#pragma unroll
    for (int f = 0; f < F; ++f) gf[f] = ga[f] * inv - (lab_ok ? Wt[lab * F + f] : 0.0f);
    return (m + __logf(se)) - zl;
}

}  // namespace sgs
