// Image-space losses and their gradient with respect to the rendered images,
// GS^3LAM Sec. 3.3.4 (mapping) and Sec. 3.4 (tracking):
//   L1 colour, L1 depth and a semantic cross-entropy on softmax(W^T F),
// each averaged over the pixels of its view, weighted by (w0, w1, w2).
// W is the fixed linear decoder standing in for F_cnn (Sec. 3.2.2, Eq. 8).
//
// One thread per pixel: the F feature channels stay in registers, the
// decoder sits in LDS (broadcast reads), and the softmax is evaluated with
// a running maximum (one pass for the log-sum-exp, one for the gradient) so
// no per-class array is needed.  The loss value is reduced per block into a
// partial-sum array and then summed in a fixed order by one block (no
// same-address atomics, deterministic).
#include "sgs_common.h"

namespace sgs {

template <int F>
__global__ void __launch_bounds__(256) k_loss(const float* __restrict__ out, int64_t P,
                                              const float* __restrict__ rgb_t, const float* __restrict__ depth_t,
                                              const int32_t* __restrict__ labels, const float* __restrict__ decoder,
                                              int K, float w0, float w1, float w2,
                                              const gs_view* __restrict__ views, int n_views,
                                              float* __restrict__ grad_out, double* __restrict__ partials) {
    __shared__ float sW[(F > 0 ? F : 1) * GS_MAX_CLASSES];
    __shared__ double s_red[3][256 / kWave];
    const int tid = threadIdx.x;
    if (F > 0) {
        for (int k = tid; k < F * K; k += blockDim.x) sW[k] = decoder[k];
    }
    __syncthreads();
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
            if (K > 0 && w2 != 0.0f) {
                const int lab = labels[p];
                // pass 1: running log-sum-exp of z_k = sum_f W[f][k] F_f
                float m = -INFINITY, se = 0.0f, zl = 0.0f;
                for (int k = 0; k < K; ++k) {
                    float z = 0.0f;
#pragma unroll
                    for (int f = 0; f < F; ++f) z = fmaf(sW[f * K + k], fv[f], z);
                    if (k == lab) zl = z;
                    if (z > m) {
                        se = se * __expf(m - z) + 1.0f;
                        m = z;
                    } else {
                        se += __expf(z - m);
                    }
                }
                const float inv = 1.0f / se;
                ls += (double)((m + __logf(se)) - zl);
                // pass 2: dCE/dF_f = sum_k W[f][k] (softmax_k - [k == label])
                for (int k = 0; k < K; ++k) {
                    float z = 0.0f;
#pragma unroll
                    for (int f = 0; f < F; ++f) z = fmaf(sW[f * K + k], fv[f], z);
                    const float e = __expf(z - m) * inv - (k == lab ? 1.0f : 0.0f);
#pragma unroll
                    for (int f = 0; f < F; ++f) gf[f] = fmaf(sW[f * K + k], e, gf[f]);
                }
            }
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
        partials[3 * (size_t)blockIdx.x + tid] = a;
    }
}

// Fixed-order sum of the per-block partials: loss = (colour, depth, semantic, total).
__global__ void __launch_bounds__(256) k_loss_final(const double* __restrict__ partials, int nblk,
                                                    double* __restrict__ loss) {
    __shared__ double s[3][256];
    double acc[3] = {0, 0, 0};
    for (int b = threadIdx.x; b < nblk; b += blockDim.x)
        for (int k = 0; k < 3; ++k) acc[k] += partials[3 * (size_t)b + k];
    for (int k = 0; k < 3; ++k) s[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int d = blockDim.x / 2; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d)
            for (int k = 0; k < 3; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        loss[0] = s[0][0];
        loss[1] = s[1][0];
        loss[2] = s[2][0];
        loss[3] = s[0][0] + s[1][0] + s[2][0];
    }
}

size_t loss_workspace_bytes(int64_t P) { return (size_t)((P + 255) / 256) * 3 * sizeof(double) + 16; }

template <int F>
hipError_t launch_loss_t(const float* out, const float* rgb_t, const float* depth_t, const int32_t* labels,
                         const float* decoder, int K, const float* w, const gs_view* views, int n_views, int64_t P,
                         float* grad_out, double* loss, void* ws, hipStream_t s) {
    if (P == 0) return hipSuccess;
    const int nblk = (int)((P + 255) / 256);
    double* partials = static_cast<double*>(ws);
    hipLaunchKernelGGL(k_loss<F>, dim3((unsigned)nblk), dim3(256), 0, s, out, P, rgb_t, depth_t, labels, decoder, K,
                       w[0], w[1], w[2], views, n_views, grad_out, partials);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, partials, nblk, loss);
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
