// Optimiser steps of the SLAM loop (Supp. C.1 learning rates):
//   - Adam over up to kAdamGroups parameter planes in one launch
//     (blockIdx.y = group), each with its own learning rate;
//   - tracking's pose step: Adam on each view's twist gradient, then the
//     left update T <- Exp(dxi) T of the view's world-to-camera [R|t],
//     written in place into the device view records the kernels read, so a
//     tracking iteration needs no host round trip.
#include "optim.h"

namespace sgs {

namespace {

struct AdamGroups {
    float* p[kAdamGroups];
    const float* g[kAdamGroups];
    float* m[kAdamGroups];
    float* v[kAdamGroups];
    int64_t n[kAdamGroups];
    float lr[kAdamGroups];
};

__global__ void __launch_bounds__(256) k_adam(AdamGroups G, float b1, float b2, float eps, float c1, float c2) {
    const int gi = blockIdx.y;
    const int64_t n = G.n[gi];
    float* __restrict__ p = G.p[gi];
    const float* __restrict__ g = G.g[gi];
    float* __restrict__ m = G.m[gi];
    float* __restrict__ v = G.v[gi];
    const float lr = G.lr[gi];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gv = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gv;
        const float vi = b2 * v[i] + (1.0f - b2) * gv * gv;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// 3x4 [R|t] = Exp(xi), xi = (rho, phi) (series for small |phi|)
__device__ void se3_exp(const float* xi, float* E) {
    const float r0 = xi[0], r1 = xi[1], r2 = xi[2], p0 = xi[3], p1 = xi[4], p2 = xi[5];
    const float th2 = p0 * p0 + p1 * p1 + p2 * p2, th = sqrtf(th2);
    float A, B, C;
    if (th < 1e-2f) {
        A = 1.0f - th2 / 6.0f;
        B = 0.5f - th2 / 24.0f;
        C = 1.0f / 6.0f - th2 / 120.0f;
    } else {
        A = sinf(th) / th;
        B = (1.0f - cosf(th)) / th2;
        C = (th - sinf(th)) / (th2 * th);
    }
    const float K[9] = {0.0f, -p2, p1, p2, 0.0f, -p0, -p1, p0, 0.0f};
    float K2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            K2[3 * i + j] = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
    const float rho[3] = {r0, r1, r2};
    for (int i = 0; i < 3; ++i) {
        float tv = 0.0f;
        for (int j = 0; j < 3; ++j) {
            const float I = i == j ? 1.0f : 0.0f;
            E[4 * i + j] = I + A * K[3 * i + j] + B * K2[3 * i + j];
            tv += (I + B * K[3 * i + j] + C * K2[3 * i + j]) * rho[j];
        }
        E[4 * i + 3] = tv;
    }
}

// step_dev (may be null): the Adam step count in device memory; the kernel
// takes t = *step_dev + 1, stores it back and forms the bias corrections
// from it (in double, as the host does), in place of c1 and c2.  One block.
__global__ void k_pose_step(gs_view* __restrict__ views, int n_views, const float* __restrict__ grad,
                            float* __restrict__ m, float* __restrict__ v, float lr_rho, float lr_phi, float b1,
                            float b2, float eps, float c1, float c2, int32_t* __restrict__ step_dev) {
    __shared__ float s_c[2];
    if (step_dev != nullptr) {
        if (threadIdx.x == 0) {
            const int t = *step_dev + 1;
            *step_dev = t;
            s_c[0] = (float)(1.0 - pow((double)b1, (double)t));
            s_c[1] = (float)(1.0 - pow((double)b2, (double)t));
        }
        __syncthreads();
        c1 = s_c[0];
        c2 = s_c[1];
    }
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= n_views) return;
    float dxi[6];
    for (int k = 0; k < 6; ++k) {
        const int i = 6 * w + k;
        const float gv = grad[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gv;
        const float vi = b2 * v[i] + (1.0f - b2) * gv * gv;
        m[i] = mi;
        v[i] = vi;
        dxi[k] = -(k < 3 ? lr_rho : lr_phi) * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
    float E[12], T[12];
    se3_exp(dxi, E);
    for (int k = 0; k < 12; ++k) T[k] = views[w].Rt[k];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 4; ++j) {
            float s = j == 3 ? E[4 * i + 3] : 0.0f;
            for (int k = 0; k < 3; ++k) s += E[4 * i + k] * T[4 * k + j];
            views[w].Rt[4 * i + j] = s;
        }
}

}  // namespace

hipError_t launch_adam(const gs_adam_group* groups, int n_groups, float b1, float b2, float eps, int step,
                       hipStream_t s) {
    AdamGroups G{};
    int64_t nmax = 0;
    for (int k = 0; k < n_groups; ++k) {
        G.p[k] = groups[k].param;
        G.g[k] = groups[k].grad;
        G.m[k] = groups[k].m;
        G.v[k] = groups[k].v;
        G.n[k] = groups[k].n;
        G.lr[k] = groups[k].lr;
        nmax = groups[k].n > nmax ? groups[k].n : nmax;
    }
    const float c1 = (float)(1.0 - std::pow((double)b1, (double)step));
    const float c2 = (float)(1.0 - std::pow((double)b2, (double)step));
    const int64_t want = (nmax + 255) / 256;
    const unsigned gx = (unsigned)(want < 4096 ? (want > 0 ? want : 1) : 4096);
    hipLaunchKernelGGL(k_adam, dim3(gx, (unsigned)n_groups), dim3(256), 0, s, G, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_pose_step(gs_view* views_dev, int n_views, const float* grad, float* m, float* v, float lr_rho,
                            float lr_phi, float b1, float b2, float eps, int step, int32_t* step_dev, hipStream_t s) {
    const float c1 = step_dev ? 1.0f : (float)(1.0 - std::pow((double)b1, (double)step));
    const float c2 = step_dev ? 1.0f : (float)(1.0 - std::pow((double)b2, (double)step));
    hipLaunchKernelGGL(k_pose_step, dim3(1), dim3(kAdamPoseThreads), 0, s, views_dev, n_views, grad, m, v, lr_rho,
                       lr_phi, b1, b2, eps, c1, c2, step_dev);
    return hipGetLastError();
}

}  // namespace sgs
