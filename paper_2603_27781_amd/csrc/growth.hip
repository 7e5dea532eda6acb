// Map growth and scale regularisation of GS^3LAM (Sec. 3.3.1-3.3.2):
//
//   adaptive expansion: every pixel with M_unobs (mask bit 1, from the SLAM
//   loss) and an observed depth D* > 0 adds one Gaussian at the unprojection
//   of its centre at D*, with the pixel's observed colour, caller-drawn
//   random features, opacity 0.5, scale D*/fx and the identity rotation.
//   New Gaussians are appended in pixel order (views back to back, rows,
//   columns) after the current count, which lives on the device: a count
//   kernel per block of pixels, one block that scans the counts and updates
//   the device-side Gaussian count, then a write kernel that ranks its
//   block's candidates with a block scan.  No host round trip.
//
//   depth-adaptive scale regularisation (Eq. 12): over the 3n per-axis
//   scales s = exp(log s) (the decision-path exponential, bit-identical to
//   any implementation of the same operation sequence), their mean and
//   population standard deviation, the sets s > mu + 2 sigma and
//   s < mu - 2 sigma, L_big = mean of s over the first, L_small = mean of
//   -log s over the second, and the gradient with respect to log s with the
//   sets held.  Every sum is per block in double, then in a fixed order.
#include "growth.h"
#include "decision_exp.h"

namespace sgs {

namespace {

constexpr int kGrowThreads = 256;
constexpr int kExpandItems = 4;  // pixels per thread
constexpr int kExpandChunk = kGrowThreads * kExpandItems;

__device__ __forceinline__ bool expand_candidate(const uint8_t* masks, const float* depth_t, int64_t p) {
    return ((masks[p] >> 1) & 1) && depth_t[p] > 0.0f;
}

__global__ void __launch_bounds__(kGrowThreads) k_expand_count(const uint8_t* __restrict__ masks,
                                                               const float* __restrict__ depth_t, int64_t P,
                                                               uint32_t* __restrict__ block_counts) {
    __shared__ uint32_t s_tmp[kGrowThreads / kWave];
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kExpandItems; ++k) {
        const int64_t p = (int64_t)blockIdx.x * kExpandChunk + k * kGrowThreads + threadIdx.x;
        if (p < P && expand_candidate(masks, depth_t, p)) ++c;
    }
    uint32_t total;
    block_exclusive<kGrowThreads>(c, s_tmp, &total);
    if (threadIdx.x == 0) block_counts[blockIdx.x] = total;
}

// One block: exclusive scan of the block counts in place, the number of
// candidates, and the Gaussian count n <- min(n + candidates, capacity)
// (n_before keeps the old count for the write kernel).
__global__ void __launch_bounds__(1024) k_expand_scan(uint32_t* __restrict__ block_counts, int nblk,
                                                      int64_t* __restrict__ n_dev, int64_t capacity,
                                                      int64_t* __restrict__ n_before,
                                                      int64_t* __restrict__ candidates) {
    __shared__ uint32_t s_tmp[1024 / kWave];
    const int per = (nblk + 1023) / 1024;
    const int b0 = threadIdx.x * per, b1 = min(b0 + per, nblk);
    uint32_t sum = 0;
    for (int b = b0; b < b1; ++b) sum += block_counts[b];
    uint32_t total;
    uint32_t run = block_exclusive<1024>(sum, s_tmp, &total);
    for (int b = b0; b < b1; ++b) {
        const uint32_t v = block_counts[b];
        block_counts[b] = run;
        run += v;
    }
    if (threadIdx.x == 0) {
        const int64_t n = *n_dev;
        *n_before = n;
        if (candidates != nullptr) *candidates = (int64_t)total;
        const int64_t m = n + (int64_t)total;
        *n_dev = m < capacity ? m : capacity;
    }
}

template <int F>
__global__ void __launch_bounds__(kGrowThreads) k_expand_write(const uint8_t* __restrict__ masks,
                                                               const float* __restrict__ rgb_t,
                                                               const float* __restrict__ depth_t,
                                                               const float* __restrict__ feat_init, int64_t P,
                                                               const gs_view* __restrict__ views, int n_views,
                                                               const uint32_t* __restrict__ block_offsets,
                                                               const int64_t* __restrict__ n_before, int64_t capacity,
                                                               gs_gaussian_grads g) {
    __shared__ uint32_t s_tmp[kGrowThreads / kWave];
    bool cand[kExpandItems];
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kExpandItems; ++k) {
        const int64_t p = (int64_t)blockIdx.x * kExpandChunk + k * kGrowThreads + threadIdx.x;
        cand[k] = p < P && expand_candidate(masks, depth_t, p);
        c += cand[k] ? 1u : 0u;
    }
    // the block's candidates in pixel order: item k of thread t is pixel
    // k * 256 + t of the chunk, so rank item-major: first all k = 0, ...
    uint32_t rank0[kExpandItems];
    uint32_t base = 0;
#pragma unroll
    for (int k = 0; k < kExpandItems; ++k) {
        uint32_t tot;
        rank0[k] = base + block_exclusive<kGrowThreads>(cand[k] ? 1u : 0u, s_tmp, &tot);
        base += tot;
    }
    const int64_t first = *n_before + (int64_t)block_offsets[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kExpandItems; ++k) {
        if (!cand[k]) continue;
        const int64_t i = first + rank0[k];
        if (i >= capacity) continue;
        const int64_t p = (int64_t)blockIdx.x * kExpandChunk + k * kGrowThreads + threadIdx.x;
        int v = 0;
        while (v + 1 < n_views && views[v + 1].pixel_offset <= p) ++v;
        const gs_view& vw = views[v];
        const int64_t q = p - vw.pixel_offset;
        const int y = (int)(q / vw.width), x = (int)(q - (int64_t)y * vw.width);
        const float d = depth_t[p];
        const float xc0 = ((float)x + 0.5f - vw.cx) / vw.fx * d, xc1 = ((float)y + 0.5f - vw.cy) / vw.fy * d;
        const float r0 = xc0 - vw.Rt[3], r1 = xc1 - vw.Rt[7], r2 = d - vw.Rt[11];
        // mu = R^T (x_c - t)
        g.mu[i] = vw.Rt[0] * r0 + vw.Rt[4] * r1 + vw.Rt[8] * r2;
        g.mu[capacity + i] = vw.Rt[1] * r0 + vw.Rt[5] * r1 + vw.Rt[9] * r2;
        g.mu[2 * capacity + i] = vw.Rt[2] * r0 + vw.Rt[6] * r1 + vw.Rt[10] * r2;
        const float lsv = logf(d / vw.fx);
        g.log_scale[i] = lsv;
        g.log_scale[capacity + i] = lsv;
        g.log_scale[2 * capacity + i] = lsv;
        g.quat[i] = 1.0f;
        g.quat[capacity + i] = 0.0f;
        g.quat[2 * capacity + i] = 0.0f;
        g.quat[3 * capacity + i] = 0.0f;
        g.opacity_logit[i] = 0.0f;  // opacity 0.5
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) g.color[ch * capacity + i] = rgb_t[ch * P + p];
#pragma unroll
        for (int f = 0; f < F; ++f) g.feat[f * capacity + i] = feat_init[f * P + p];
    }
}

// ---------------------------------------------------------------------------
// DSR
// ---------------------------------------------------------------------------
constexpr int kDsrItems = 16;
constexpr int kDsrChunk = kGrowThreads * kDsrItems;

// stats[0..7] (double): sum s, sum (s - mu)^2, sum over the big set of s,
// its count, sum over the small set of -log s, its count, mu, sigma.
__device__ __forceinline__ double block_sum_d(double v, double* s_red) {
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    if (lane == 0) s_red[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < kGrowThreads / kWave; ++w) t += s_red[w];
    __syncthreads();
    return t;
}

// PASS 0: partial sums of s; PASS 1: of (s - mu)^2; PASS 2: the two sets
__global__ void __launch_bounds__(kGrowThreads) k_dsr_partial(const float* __restrict__ ls, int64_t m, int pass,
                                                              const double* __restrict__ stats,
                                                              double* __restrict__ partials) {
    __shared__ double s_red[kGrowThreads / kWave];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    const double mu = pass > 0 ? stats[6] : 0.0, sd = pass > 1 ? stats[7] : 0.0;
    const double big = mu + 2.0 * sd, small = mu - 2.0 * sd;
    float x[kDsrItems];
#pragma unroll
    for (int k = 0; k < kDsrItems; ++k) {
        const int64_t j = (int64_t)blockIdx.x * kDsrChunk + k * kGrowThreads + threadIdx.x;
        x[k] = ls[j < m ? j : m - 1];
    }
#pragma unroll
    for (int k = 0; k < kDsrItems; ++k) {
        const int64_t j = (int64_t)blockIdx.x * kDsrChunk + k * kGrowThreads + threadIdx.x;
        if (j >= m) continue;
        const double s = (double)dec_exp(x[k]);
        if (pass == 0) {
            a0 += s;
        } else if (pass == 1) {
            a0 += (s - mu) * (s - mu);
        } else {
            if (s > big) {
                a0 += s;
                a1 += 1.0;
            }
            if (s < small) {
                a2 += -log(s);
                a3 += 1.0;
            }
        }
    }
    const int nb = gridDim.x;
    const double t0 = block_sum_d(a0, s_red);
    if (pass < 2) {
        if (threadIdx.x == 0) partials[blockIdx.x] = t0;
        return;
    }
    const double t1 = block_sum_d(a1, s_red), t2 = block_sum_d(a2, s_red), t3 = block_sum_d(a3, s_red);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = t0;
        partials[nb + blockIdx.x] = t1;
        partials[2 * nb + blockIdx.x] = t2;
        partials[3 * nb + blockIdx.x] = t3;
    }
}

// One block: the pass's sums in a fixed order, into stats (and, after the
// last pass, the outputs).
__global__ void __launch_bounds__(kGrowThreads) k_dsr_reduce(const double* __restrict__ partials, int nb, int pass,
                                                             int64_t m, float w_big, float w_small,
                                                             double* __restrict__ stats, double* __restrict__ out) {
    __shared__ double s_red[kGrowThreads / kWave];
    const int terms = pass < 2 ? 1 : 4;
    double r[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < terms; ++k) {
        double a = 0.0;
        for (int b = threadIdx.x; b < nb; b += kGrowThreads) a += partials[k * nb + b];
        r[k] = block_sum_d(a, s_red);
    }
    if (threadIdx.x != 0) return;
    if (pass == 0) {
        stats[0] = r[0];
        stats[6] = m > 0 ? r[0] / (double)m : 0.0;
    } else if (pass == 1) {
        stats[1] = r[0];
        stats[7] = m > 0 ? sqrt(r[0] / (double)m) : 0.0;
    } else {
        for (int k = 0; k < 4; ++k) stats[2 + k] = r[k];
        const double Lb = r[1] > 0.0 ? r[0] / r[1] : 0.0, Ls = r[3] > 0.0 ? r[2] / r[3] : 0.0;
        out[0] = Lb;
        out[1] = Ls;
        out[2] = (double)w_big * Lb + (double)w_small * Ls;
        out[3] = stats[6];
        out[4] = stats[7];
        out[5] = r[1];
        out[6] = r[3];
    }
}

// grad_ls[j] += w_big s / n_big (big set), -w_small / n_small (small set)
__global__ void __launch_bounds__(kGrowThreads) k_dsr_grad(const float* __restrict__ ls, int64_t m,
                                                           const double* __restrict__ stats, float w_big,
                                                           float w_small, float* __restrict__ grad) {
    const int64_t j = (int64_t)blockIdx.x * kGrowThreads + threadIdx.x;
    if (j >= m) return;
    const double mu = stats[6], sd = stats[7], nb = stats[3], ns = stats[5];
    const double s = (double)dec_exp(ls[j]);
    double g = 0.0;
    if (s > mu + 2.0 * sd) g += (double)w_big * s / nb;
    if (s < mu - 2.0 * sd) g += -(double)w_small / ns;
    if (g != 0.0) grad[j] += (float)g;
}

}  // namespace

size_t expand_workspace_bytes(int64_t P) {
    const int64_t nblk = (P + kExpandChunk - 1) / kExpandChunk;
    return ((size_t)nblk * 4 + 255) / 256 * 256 + 256;  // block offsets, then the old count
}

hipError_t launch_expand(const uint8_t* masks, const float* rgb_t, const float* depth_t, const float* feat_init,
                         int n_feat, int64_t P, const gs_view* views_dev, int n_views, int64_t* n_dev,
                         int64_t capacity, int64_t* candidates, const gs_gaussian_grads& g, void* ws, hipStream_t s) {
    const int nblk = (int)((P + kExpandChunk - 1) / kExpandChunk);
    uint32_t* counts = static_cast<uint32_t*>(ws);
    int64_t* n_before = reinterpret_cast<int64_t*>(static_cast<char*>(ws) + ((size_t)nblk * 4 + 255) / 256 * 256);
    hipLaunchKernelGGL(k_expand_count, dim3(nblk), dim3(kGrowThreads), 0, s, masks, depth_t, P, counts);
    hipLaunchKernelGGL(k_expand_scan, dim3(1), dim3(1024), 0, s, counts, nblk, n_dev, capacity, n_before, candidates);
    switch (n_feat) {
        case 0:
            hipLaunchKernelGGL(k_expand_write<0>, dim3(nblk), dim3(kGrowThreads), 0, s, masks, rgb_t, depth_t, feat_init,
                               P, views_dev, n_views, counts, n_before, capacity, g);
            break;
        case 8:
            hipLaunchKernelGGL(k_expand_write<8>, dim3(nblk), dim3(kGrowThreads), 0, s, masks, rgb_t, depth_t, feat_init,
                               P, views_dev, n_views, counts, n_before, capacity, g);
            break;
        case 32:
            hipLaunchKernelGGL(k_expand_write<32>, dim3(nblk), dim3(kGrowThreads), 0, s, masks, rgb_t, depth_t,
                               feat_init, P, views_dev, n_views, counts, n_before, capacity, g);
            break;
        default:
            hipLaunchKernelGGL(k_expand_write<16>, dim3(nblk), dim3(kGrowThreads), 0, s, masks, rgb_t, depth_t,
                               feat_init, P, views_dev, n_views, counts, n_before, capacity, g);
            break;
    }
    return hipGetLastError();
}

size_t dsr_workspace_bytes(int64_t n) {
    const int64_t m = 3 * n, nb = (m + kDsrChunk - 1) / kDsrChunk;
    return ((size_t)nb * 4 * 8 + 255) / 256 * 256 + 256;  // partials, then stats[8]
}

hipError_t launch_dsr(const float* log_scale, int64_t n, float w_big, float w_small, float* grad_ls, double* out,
                      void* ws, hipStream_t s) {
    const int64_t m = 3 * n;
    const int nb = (int)((m + kDsrChunk - 1) / kDsrChunk);
    double* partials = static_cast<double*>(ws);
    double* stats = reinterpret_cast<double*>(static_cast<char*>(ws) + ((size_t)nb * 4 * 8 + 255) / 256 * 256);
    for (int pass = 0; pass < 3; ++pass) {
        hipLaunchKernelGGL(k_dsr_partial, dim3(nb), dim3(kGrowThreads), 0, s, log_scale, m, pass, stats, partials);
        hipLaunchKernelGGL(k_dsr_reduce, dim3(1), dim3(kGrowThreads), 0, s, partials, nb, pass, m, w_big, w_small,
                           stats, out);
    }
    if (grad_ls != nullptr)
        hipLaunchKernelGGL(k_dsr_grad, dim3((unsigned)((m + kGrowThreads - 1) / kGrowThreads)), dim3(kGrowThreads), 0,
                           s, log_scale, m, stats, w_big, w_small, grad_ls);
    return hipGetLastError();
}

}  // namespace sgs
