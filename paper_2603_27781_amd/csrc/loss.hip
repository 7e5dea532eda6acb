// Image-space losses and their gradient with respect to the rendered images,
// GS^3LAM Sec. 3.3.4 (mapping) and Sec. 3.4 (tracking):
//   L1 colour, L1 depth and a semantic cross-entropy on softmax(W^T F),
// each averaged over the pixels of its view, weighted by (w0, w1, w2).
// W is the fixed linear decoder standing in for F_cnn (Sec. 3.2.2, Eq. 8).
//
// One thread per pixel: the F feature channels stay in registers.  The
// decoder is first copied transposed (one row of F floats per class) into
// the workspace, so that in the pixel kernel a class row is one
// wavefront-uniform scalar load whose values feed the FMAs directly.  With
// at most KC classes the logits z_k = sum_f W[f][k] F_f are kept in
// registers: one pass computes them and their maximum, a second forms the
// softmax weights and dCE/dF_f = sum_k W[f][k] softmax_k - W[f][label].
// More classes recompute z in the second pass.  The loss value is reduced
// per block into a partial-sum array and then summed in a fixed order by
// one block (no same-address atomics, deterministic).
#include "fused_loss.h"
#include "loss_common.h"

namespace sgs {

constexpr int kLossThreads = 256;
constexpr int kLossKC = 64;  // most classes whose logits are kept in registers (32 or 64 variants)

__global__ void k_transpose_decoder(const float* __restrict__ W, int F, int K, float* __restrict__ Wt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= F * K) return;
    const int f = i / K, k = i - f * K;
    Wt[k * F + f] = W[i];
}

__global__ void __launch_bounds__(kSumThreads) k_sum_stage(const double* __restrict__ src, int n, int terms,
                                                           double* __restrict__ dst) {
    __shared__ double s[kSumThreads / kWave];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    for (int k = 0; k < terms; ++k) {
        double x[kSumPer];
#pragma unroll
        for (int u = 0; u < kSumPer; ++u) {
            const int i = blockIdx.x * kSumChunk + u * kSumThreads + tid;
            x[u] = src[(size_t)k * n + (i < n ? i : n - 1)];
            x[u] = i < n ? x[u] : 0.0;
        }
        double a = 0.0;
#pragma unroll
        for (int u = 0; u < kSumPer; ++u) a += x[u];
        for (int d = kWave / 2; d > 0; d >>= 1) a += __shfl_xor(a, d, kWave);
        if (lane == 0) s[wave] = a;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int w = 0; w < kSumThreads / kWave; ++w) t += s[w];
            dst[(size_t)k * gridDim.x + blockIdx.x] = t;
        }
        __syncthreads();
    }
}

template <int F, int KC>
__global__ void __launch_bounds__(kLossThreads) k_loss(const float* __restrict__ out, int64_t P,
                                                       const float* __restrict__ rgb_t,
                                                       const float* __restrict__ depth_t,
                                                       const int32_t* __restrict__ labels,
                                                       const float* __restrict__ Wt, int K, float w0, float w1,
                                                       float w2, const gs_view* __restrict__ views, int n_views,
                                                       float* __restrict__ grad_out, double* __restrict__ partials) {
    __shared__ double s_red[3][kLossThreads / kWave];
    const int tid = threadIdx.x;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + tid;
    double lc = 0.0, ld = 0.0, ls = 0.0;
    if (p < P) {
        int v = 0;
        while (v + 1 < n_views && views[v + 1].pixel_offset <= p) ++v;
        const float Pv = (float)((int64_t)views[v].width * views[v].height);
        const float gc = w0 / (3.0f * Pv), gd = w1 / Pv, gs = w2 / Pv;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float r = out[ch * P + p] - rgb_t[ch * P + p];
            lc += (double)fabsf(r);
            grad_out[ch * P + p] = r > 0.0f ? gc : (r < 0.0f ? -gc : 0.0f);
        }
        const float rd = out[3 * P + p] - depth_t[p];
        ld += (double)fabsf(rd);
        grad_out[3 * P + p] = rd > 0.0f ? gd : (rd < 0.0f ? -gd : 0.0f);
        grad_out[4 * P + p] = 0.0f;
        if (F > 0) {
            float fv[F > 0 ? F : 1];
#pragma unroll
            for (int f = 0; f < F; ++f) fv[f] = out[(5 + f) * P + p];
            float gf[F > 0 ? F : 1];
#pragma unroll
            for (int f = 0; f < F; ++f) gf[f] = 0.0f;
            if (K > 0 && w2 != 0.0f) ls += (double)semantic_ce<F, KC>(fv, Wt, K, labels[p], gf);
#pragma unroll
            for (int f = 0; f < F; ++f) grad_out[(5 + f) * P + p] = gs * gf[f];
        }
        lc *= (double)w0 / (3.0 * (double)Pv);
        ld *= (double)w1 / (double)Pv;
        ls *= (double)w2 / (double)Pv;
    }
    // block reduction of the three terms into this block's partial sums
    const int lane = tid & (kWave - 1), wave = tid / kWave;
    for (int d = kWave / 2; d > 0; d >>= 1) {
        lc += __shfl_xor(lc, d, kWave);
        ld += __shfl_xor(ld, d, kWave);
        ls += __shfl_xor(ls, d, kWave);
    }
    if (lane == 0) {
        s_red[0][wave] = lc;
        s_red[1][wave] = ld;
        s_red[2][wave] = ls;
    }
    __syncthreads();
    if (tid < 3) {
        double a = 0;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) a += s_red[tid][w];
        partials[(size_t)tid * gridDim.x + blockIdx.x] = a;  // term-major
    }
}

// Last stage of the fixed-order sum: stage holds the first-stage sums,
// term-major [3][nst]; loss = (colour, depth, semantic, total).  One block,
// wavefront shuffles, every sum in a fixed order.
__global__ void __launch_bounds__(kSumThreads) k_loss_final(const double* __restrict__ stage, int nst,
                                                            double* __restrict__ loss) {
    __shared__ double s[3][kSumThreads / kWave];
    const int t = threadIdx.x, lane = t & (kWave - 1), wave = t / kWave;
    double a[3] = {0.0, 0.0, 0.0};
    for (int i = t; i < nst; i += kSumThreads)
#pragma unroll
        for (int k = 0; k < 3; ++k) a[k] += stage[(size_t)k * nst + i];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        for (int d = kWave / 2; d > 0; d >>= 1) a[k] += __shfl_xor(a[k], d, kWave);
        if (lane == 0) s[k][wave] = a[k];
    }
    __syncthreads();
    if (t == 0) {
        double r[3];
        for (int k = 0; k < 3; ++k) {
            r[k] = 0.0;
            for (int w = 0; w < kSumThreads / kWave; ++w) r[k] += s[k][w];
            loss[k] = r[k];
        }
        loss[3] = (r[0] + r[1]) + r[2];
    }
}

hipError_t launch_transpose_decoder(const float* W, int F, int K, float* Wt, hipStream_t s) {
    if (F * K > 0) hipLaunchKernelGGL(k_transpose_decoder, dim3((unsigned)ceil_div(F * K, 256)), dim3(256), 0, s, W, F, K, Wt);
    return hipGetLastError();
}

hipError_t launch_loss_sums(const double* partials, int n, double* stage, double* loss, hipStream_t s) {
    const int nst = sum_stage_blocks(n);
    hipLaunchKernelGGL(k_sum_stage, dim3((unsigned)nst), dim3(kSumThreads), 0, s, partials, n, 3, stage);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(kSumThreads), 0, s, stage, nst, loss);
    return hipGetLastError();
}

// workspace: per-block partials (3 doubles each), their first-stage sums,
// then the transposed decoder
static size_t loss_partials_bytes(int64_t P) {
    const int64_t nblk = (P + kLossThreads - 1) / kLossThreads;
    return ((size_t)nblk * 3 * sizeof(double) + 255) / 256 * 256 +
           ((size_t)sum_stage_blocks(nblk) * 3 * sizeof(double) + 255) / 256 * 256;
}
size_t loss_workspace_bytes(int64_t P) {
    return loss_partials_bytes(P) + (size_t)32 * GS_MAX_CLASSES * sizeof(float);  // F <= 32
}

template <int F>
hipError_t launch_loss_t(const float* out, const float* rgb_t, const float* depth_t, const int32_t* labels,
                         const float* decoder, int K, const float* w, const gs_view* views, int n_views, int64_t P,
                         float* grad_out, double* loss, void* ws, hipStream_t s) {
    if (P == 0) return hipSuccess;
    const int nblk = (int)((P + kLossThreads - 1) / kLossThreads);
    double* partials = static_cast<double*>(ws);
    float* Wt = reinterpret_cast<float*>(static_cast<char*>(ws) + loss_partials_bytes(P));
    const bool sem = F > 0 && K > 0 && w[2] != 0.0f;
    if (sem)
        hipLaunchKernelGGL(k_transpose_decoder, dim3((unsigned)ceil_div(F * K, 256)), dim3(256), 0, s, decoder, F, K,
                           Wt);
    if (sem && K > kLossKC)
        hipLaunchKernelGGL((k_loss<F, 0>), dim3((unsigned)nblk), dim3(kLossThreads), 0, s, out, P, rgb_t, depth_t,
                           labels, Wt, K, w[0], w[1], w[2], views, n_views, grad_out, partials);
    else if (sem && K > 32)
        hipLaunchKernelGGL((k_loss<F, kLossKC>), dim3((unsigned)nblk), dim3(kLossThreads), 0, s, out, P, rgb_t,
                           depth_t, labels, Wt, K, w[0], w[1], w[2], views, n_views, grad_out, partials);
    else
        hipLaunchKernelGGL((k_loss<F, 32>), dim3((unsigned)nblk), dim3(kLossThreads), 0, s, out, P, rgb_t, depth_t,
                           labels, Wt, K, w[0], w[1], w[2], views, n_views, grad_out, partials);
    double* stage = partials + ((size_t)nblk * 3 * sizeof(double) + 255) / 256 * 256 / sizeof(double);
    const int nst = sum_stage_blocks(nblk);
    hipLaunchKernelGGL(k_sum_stage, dim3((unsigned)nst), dim3(kSumThreads), 0, s, partials, nblk, 3, stage);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(kSumThreads), 0, s, stage, nst, loss);
    return hipGetLastError();
}

hipError_t launch_loss(const float* out, int n_feat, const float* rgb_t, const float* depth_t, const int32_t* labels,
                       const float* decoder, int n_classes, const float* weights, const gs_view* views_dev,
                       int n_views, int64_t total_pixels, float* grad_out, double* loss, void* ws, hipStream_t s) {
    switch (n_feat) {
        case 0:
            return launch_loss_t<0>(out, rgb_t, depth_t, labels, decoder, n_classes, weights, views_dev, n_views,
                                    total_pixels, grad_out, loss, ws, s);
        case 8:
            return launch_loss_t<8>(out, rgb_t, depth_t, labels, decoder, n_classes, weights, views_dev, n_views,
                                    total_pixels, grad_out, loss, ws, s);
        case 32:
            return launch_loss_t<32>(out, rgb_t, depth_t, labels, decoder, n_classes, weights, views_dev, n_views,
                                     total_pixels, grad_out, loss, ws, s);
        default:
            return launch_loss_t<16>(out, rgb_t, depth_t, labels, decoder, n_classes, weights, views_dev, n_views,
                                     total_pixels, grad_out, loss, ws, s);
    }
}

}  // namespace sgs
