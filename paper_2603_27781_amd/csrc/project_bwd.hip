// Backward of the projection (GS^3LAM Sec. 3.2, Eq. 2-3) and the pose
// gradient of Supp. B.1 as a 6-DoF twist.
//
// Forward recomputed in FP32 per (view, Gaussian):
//   p = R_CW mu + t,  M = R(q) diag(exp(log_s)),  T = J R_CW,  U = T M,
//   Sigma2D = U U^T + b I,  conic = Sigma2D^-1,  mean2d = (fx x/z + cx, fy y/z + cy)
// Backward, given dL/d(mean2d, conic, depth) accumulated by the render
// backward:
//   D = dL/dSigma2D = -Q dQ Q            (Q = conic, dQ symmetric)
//   dU = 2 D U,  dT = dU M^T,  dM = T^T dU,  dJ = dT R_CW^T
//   dp from mean2d, from J(p) and from depth (= z)
//   dmu = R_CW^T dp;  dR(q) = dM diag(s);  dlog_s = s * colsum(dM o R)
//   dq = (I - q^ q^T) dq^ / |q|
// Pose (left perturbation Exp(xi) T_CW):
//   G = dL/dSigma_c = J^T D J,  Sigma_c = (R_CW M)(R_CW M)^T,
//   dL/drho = sum dp,  dL/dphi = sum p x dp + 2 (Sigma_c G - G Sigma_c)_(12, 20, 01).
#include "sgs_common.h"

// This file is value path only (no decision feeds an integer): the compiler
// may fuse multiplies and adds here, unlike the rest of the library.
#pragma clang fp contract(fast)

namespace sgs {

struct Fwd {
    float p[3];
    float iz;  // 1 / p_z
    float xn, yn;
    float j00, j02, j11, j12;
    float T[6];   // J R_CW, 2x3
    float U[6];   // T M, 2x3
    float a, b, c;  // Sigma2D entries
};

struct Gauss {
    float q[4];     // unit quaternion
    float qn;       // |q|
    float s[3];
    float R[9];     // rotation of q
    float M[9];     // R diag(s)
};

__device__ __forceinline__ void load_gauss(const GaussPtrs& g, int i, Gauss& G) {
    const int n = g.n;
    const float q0 = g.quat[i], q1 = g.quat[(size_t)n + i], q2 = g.quat[2 * (size_t)n + i],
                q3 = g.quat[3 * (size_t)n + i];
    G.qn = sqrtf(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
    const float inv = 1.0f / G.qn;
    const float w = q0 * inv, x = q1 * inv, y = q2 * inv, z = q3 * inv;
    G.q[0] = w; G.q[1] = x; G.q[2] = y; G.q[3] = z;
    G.R[0] = 1.f - 2.f * (y * y + z * z); G.R[1] = 2.f * (x * y - w * z); G.R[2] = 2.f * (x * z + w * y);
    G.R[3] = 2.f * (x * y + w * z); G.R[4] = 1.f - 2.f * (x * x + z * z); G.R[5] = 2.f * (y * z - w * x);
    G.R[6] = 2.f * (x * z - w * y); G.R[7] = 2.f * (y * z + w * x); G.R[8] = 1.f - 2.f * (x * x + y * y);
    for (int k = 0; k < 3; ++k) G.s[k] = __expf(g.log_scale[(size_t)k * n + i]);
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) G.M[3 * r + k] = G.R[3 * r + k] * G.s[k];
}

// Rt: row-major [R|t] of the view; fx, fy its focal lengths.  Divisions go
// through one hardware reciprocal (about 1 ulp): nothing here is compared.
__device__ __forceinline__ void forward(const Gauss& G, const float* mu, const float* Rt, float fx, float fy,
                                        float blur, Fwd& f) {
    for (int k = 0; k < 3; ++k) f.p[k] = Rt[4 * k] * mu[0] + Rt[4 * k + 1] * mu[1] + Rt[4 * k + 2] * mu[2] + Rt[4 * k + 3];
    f.iz = __builtin_amdgcn_rcpf(f.p[2]);
    f.xn = f.p[0] * f.iz;
    f.yn = f.p[1] * f.iz;
    f.j00 = fx * f.iz;
    f.j11 = fy * f.iz;
    f.j02 = -f.j00 * f.xn;
    f.j12 = -f.j11 * f.yn;
    for (int k = 0; k < 3; ++k) {
        f.T[k] = f.j00 * Rt[k] + f.j02 * Rt[8 + k];
        f.T[3 + k] = f.j11 * Rt[4 + k] + f.j12 * Rt[8 + k];
    }
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k)
            f.U[3 * r + k] = f.T[3 * r] * G.M[k] + f.T[3 * r + 1] * G.M[3 + k] + f.T[3 * r + 2] * G.M[6 + k];
    f.a = f.U[0] * f.U[0] + f.U[1] * f.U[1] + f.U[2] * f.U[2] + blur;
    f.b = f.U[0] * f.U[3] + f.U[1] * f.U[4] + f.U[2] * f.U[5];
    f.c = f.U[3] * f.U[3] + f.U[4] * f.U[4] + f.U[5] * f.U[5] + blur;
}

// Backward of one view: accumulates dM (3x3), returns dp (3) and D (Sigma2D gradient).
__device__ __forceinline__ void backward_view(const Gauss& G, const Fwd& f, const float* Rt, float fx, float fy,
                                              const float4 g0, const float4 g1, float* dM, float* dp, float* D) {
    // conic Q from Sigma2D
    const float idet = __builtin_amdgcn_rcpf(f.a * f.c - f.b * f.b);
    const float A = f.c * idet, Bq = -f.b * idet, C = f.a * idet;
    const float dA = g0.z, dBh = 0.5f * g0.w, dC = g1.x;  // symmetric dQ: off-diagonals carry dB/2
    // D = -Q dQ Q
    D[0] = -(A * A * dA + 2.f * A * Bq * dBh + Bq * Bq * dC);
    D[1] = -(A * Bq * dA + (A * C + Bq * Bq) * dBh + Bq * C * dC);
    D[2] = -(Bq * Bq * dA + 2.f * Bq * C * dBh + C * C * dC);
    // dU = 2 D U
    float dU[6];
    for (int k = 0; k < 3; ++k) {
        dU[k] = 2.f * (D[0] * f.U[k] + D[1] * f.U[3 + k]);
        dU[3 + k] = 2.f * (D[1] * f.U[k] + D[2] * f.U[3 + k]);
    }
    // dT = dU M^T (2x3), dM += T^T dU (3x3)
    float dT[6];
    for (int r = 0; r < 2; ++r)
        for (int l = 0; l < 3; ++l)
            dT[3 * r + l] = dU[3 * r] * G.M[3 * l] + dU[3 * r + 1] * G.M[3 * l + 1] + dU[3 * r + 2] * G.M[3 * l + 2];
    for (int l = 0; l < 3; ++l)
        for (int k = 0; k < 3; ++k) dM[3 * l + k] += f.T[l] * dU[k] + f.T[3 + l] * dU[3 + k];
    // dJ = dT R_CW^T for the four non-zero entries of J
    const float dJ00 = dT[0] * Rt[0] + dT[1] * Rt[1] + dT[2] * Rt[2];
    const float dJ02 = dT[0] * Rt[8] + dT[1] * Rt[9] + dT[2] * Rt[10];
    const float dJ11 = dT[3] * Rt[4] + dT[4] * Rt[5] + dT[5] * Rt[6];
    const float dJ12 = dT[3] * Rt[8] + dT[4] * Rt[9] + dT[5] * Rt[10];
    const float iz = f.iz, iz2 = iz * iz;
    // mean2d = (fx x/z + cx, fy y/z + cy); depth = z
    float gx = g0.x * fx * iz;
    float gy = g0.y * fy * iz;
    float gz = -(g0.x * fx * f.p[0] + g0.y * fy * f.p[1]) * iz2 + g1.y;
    // J00 = fx/z, J02 = -fx x/z^2, J11 = fy/z, J12 = -fy y/z^2
    gz += -dJ00 * fx * iz2 - dJ11 * fy * iz2;
    gx += -dJ02 * fx * iz2;
    gy += -dJ12 * fy * iz2;
    gz += 2.f * (dJ02 * fx * f.p[0] + dJ12 * fy * f.p[1]) * iz2 * iz;
    dp[0] = gx;
    dp[1] = gy;
    dp[2] = gz;
}

__device__ __forceinline__ bool nonzero(const float4 a, const float4 b) {
    return a.x != 0.f || a.y != 0.f || a.z != 0.f || a.w != 0.f || b.x != 0.f || b.y != 0.f;
}

// Parameter gradients, one thread per Gaussian (no atomics: the views'
// contributions are summed in registers, in view order).  A Gaussian touches
// few of the views, so each lane walks only its own touched views (a bit
// mask, lowest view first): a wavefront runs as many rounds as its busiest
// lane has views, not one round per view, and each lane reads the camera of
// its current view from LDS.  Every plane the thread reads is loaded up
// front in one batch; the feature count is a template parameter so those
// loads are unrolled.
constexpr int kPbThreads = 256;
constexpr int kPbViewFloats = 16;  // Rt (12), fx, fy, 2 unused

// Zero mean, log-scale and quaternion gradients of Gaussian i (the write
// mode, for a Gaussian whose views contribute nothing to them).
__device__ __forceinline__ void write_zero_geometry(const GradPtrs& out, int n, int i) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        out.mu[(size_t)k * n + i] = 0.0f;
        out.log_scale[(size_t)k * n + i] = 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) out.quat[(size_t)k * n + i] = 0.0f;
}

// ACC: add to the gradient planes; otherwise write them, zeros included for
// Gaussians no view touches (the caller need not clear them first).  Written
// as 0 + value, so both give the same bits from cleared planes.
template <int F, bool ACC>
__global__ void __launch_bounds__(kPbThreads) k_project_bwd(GaussPtrs g, const gs_view* __restrict__ views,
                                                            int n_views, float blur,
                                                            const int32_t* __restrict__ touched,
                                                            const float4* __restrict__ grad_geo,
                                                            const float4* __restrict__ grad_app, GradPtrs out) {
    constexpr int GA4 = (4 + F) / 4;  // float4 per appearance-gradient row
    __shared__ float4 s_vw4[GS_MAX_VIEWS * kPbViewFloats / 4];
    float* s_vw = reinterpret_cast<float*>(s_vw4);
    for (int v = threadIdx.x; v < n_views; v += kPbThreads) {
        const gs_view& vw = views[v];
        float* d = s_vw + v * kPbViewFloats;
#pragma unroll
        for (int k = 0; k < 12; ++k) d[k] = vw.Rt[k];
        d[12] = vw.fx;
        d[13] = vw.fy;
    }
    __syncthreads();
    const int n = g.n;
    const int i = blockIdx.x * kPbThreads + threadIdx.x;
    if (i >= n) return;

    // views whose pair this Gaussian touches
    uint64_t mask = 0;
#pragma unroll 8
    for (int v = 0; v < n_views; ++v) mask |= (uint64_t)(touched[(size_t)v * n + i] > 0) << v;

    // appearance: opacity through the sigmoid, colour and feature as they are
    float4 ga[GA4];
#pragma unroll
    for (int q = 0; q < GA4; ++q) ga[q] = grad_app[(size_t)i * GA4 + q];
    const float lg = g.logit[i];
    float oc[3], of[F > 0 ? F : 1];
    const float ol = ACC ? out.logit[i] : 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) oc[k] = ACC ? out.color[(size_t)k * n + i] : 0.0f;
#pragma unroll
    for (int f = 0; f < F; ++f) of[f] = ACC ? out.feat[(size_t)f * n + i] : 0.0f;
    const float* gaf = reinterpret_cast<const float*>(ga);
    const float o = 1.0f / (1.0f + __expf(-lg));
    out.logit[i] = ol + gaf[0] * o * (1.0f - o);
#pragma unroll
    for (int k = 0; k < 3; ++k) out.color[(size_t)k * n + i] = oc[k] + gaf[1 + k];
#pragma unroll
    for (int f = 0; f < F; ++f) out.feat[(size_t)f * n + i] = of[f] + gaf[4 + f];
    if (mask == 0) {
        if constexpr (!ACC) write_zero_geometry(out, n, i);
        return;
    }

    Gauss G;
    load_gauss(g, i, G);
    const float mu[3] = {g.mu[i], g.mu[(size_t)n + i], g.mu[2 * (size_t)n + i]};
    float dM[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    float dmu[3] = {0, 0, 0};
    bool any = false;
    while (mask != 0) {
        const int v = __builtin_ctzll(mask);
        mask &= mask - 1;
        const size_t o2 = (size_t)v * n + i;
        const float4 g0 = grad_geo[2 * o2], g1 = grad_geo[2 * o2 + 1];
        if (!nonzero(g0, g1)) continue;
        any = true;
        const float* Rt = s_vw + v * kPbViewFloats;
        const float fx = Rt[12], fy = Rt[13];
        Fwd f;
        forward(G, mu, Rt, fx, fy, blur, f);
        float dp[3], D[3];
        backward_view(G, f, Rt, fx, fy, g0, g1, dM, dp, D);
        for (int k = 0; k < 3; ++k) dmu[k] += Rt[k] * dp[0] + Rt[4 + k] * dp[1] + Rt[8 + k] * dp[2];
    }
    if (!any) {
        if constexpr (!ACC) write_zero_geometry(out, n, i);
        return;
    }
    for (int k = 0; k < 3; ++k) out.mu[(size_t)k * n + i] = (ACC ? out.mu[(size_t)k * n + i] : 0.0f) + dmu[k];
    // M = R diag(s)
    float dR[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) dR[3 * r + k] = dM[3 * r + k] * G.s[k];
    for (int k = 0; k < 3; ++k) {
        const float ds = dM[k] * G.R[k] + dM[3 + k] * G.R[3 + k] + dM[6 + k] * G.R[6 + k];
        out.log_scale[(size_t)k * n + i] = (ACC ? out.log_scale[(size_t)k * n + i] : 0.0f) + ds * G.s[k];
    }
    // rotation of the unit quaternion (w, x, y, z): dR_ab / dq
    const float w = G.q[0], x = G.q[1], y = G.q[2], z = G.q[3];
    float dq[4];
    dq[0] = 2.f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dq[1] = 2.f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.f * x * dR[4] - w * dR[5] + z * dR[6] + w * dR[7] -
                   2.f * x * dR[8]);
    dq[2] = 2.f * (-2.f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] + z * dR[7] -
                   2.f * y * dR[8]);
    dq[3] = 2.f * (-2.f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.f * z * dR[4] + y * dR[5] + x * dR[6] +
                   y * dR[7]);
    const float dot = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
    const float iq = 1.0f / G.qn;
    for (int k = 0; k < 4; ++k)
        out.quat[(size_t)k * n + i] = (ACC ? out.quat[(size_t)k * n + i] : 0.0f) + (dq[k] - G.q[k] * dot) * iq;
}

// Twist contributions per (view, Gaussian), reduced per block in FP64.  A
// block takes kPoseChunk consecutive Gaussians of one view.  Few pairs are
// visible (under a tenth at the mapping workloads), so the block first lists
// the pairs with a nonzero 2D gradient in LDS, in index order (thread t
// screens Gaussians t, t + 256, ..., each round coalesced, ranked with
// ballots and per-wavefront counts), and then its threads take the listed
// pairs, entry e by thread e mod 256: every lane of the projection backward
// works on a visible pair instead of one in ten.  Each thread sums its
// entries in list order and the block sums the threads in a fixed order.
constexpr int kPoseThreads = 256;
constexpr int kPoseGPT = 8;  // Gaussians screened per thread
constexpr int kPoseChunk = kPoseThreads * kPoseGPT;
__global__ void __launch_bounds__(kPoseThreads) k_pose_partial(GaussPtrs g, const gs_view* __restrict__ views,
                                                               float blur, const int32_t* __restrict__ touched,
                                                               const float4* __restrict__ grad_geo,
                                                               double* __restrict__ partials, int nblk) {
    __shared__ int s_list[kPoseChunk];
    __shared__ uint32_t s_tmp[kPoseThreads / kWave];
    __shared__ double s_red[6][kPoseThreads / kWave];
    const int n = g.n;
    const int v = blockIdx.y;
    const int tid = threadIdx.x;
    const int base = blockIdx.x * kPoseChunk;
    uint32_t count = 0;
    for (int k = 0; k < kPoseGPT; ++k) {
        const int i = base + k * kPoseThreads + tid;
        bool keep = false;
        if (i < n && touched[(size_t)v * n + i] > 0) {
            const size_t o = (size_t)v * n + i;
            keep = nonzero(grad_geo[2 * o], grad_geo[2 * o + 1]);
        }
        uint32_t tot;
        const uint32_t rank = block_exclusive<kPoseThreads>(keep ? 1u : 0u, s_tmp, &tot);
        if (keep) s_list[count + rank] = i;
        count += tot;
    }
    __syncthreads();
    double tw[6] = {0, 0, 0, 0, 0, 0};
    const gs_view& vw = views[v];
    for (uint32_t e = tid; e < count; e += kPoseThreads) {
        const int i = s_list[e];
        const size_t o = (size_t)v * n + i;
        const float4 g0 = grad_geo[2 * o], g1 = grad_geo[2 * o + 1];
        Gauss G;
        load_gauss(g, i, G);
        const float mu[3] = {g.mu[i], g.mu[(size_t)n + i], g.mu[2 * (size_t)n + i]};
        Fwd f;
        forward(G, mu, vw.Rt, vw.fx, vw.fy, blur, f);
        float dM[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        float dp[3], D[3];
        backward_view(G, f, vw.Rt, vw.fx, vw.fy, g0, g1, dM, dp, D);
        // G_c = J^T D J with J = [[j00, 0, j02], [0, j11, j12]]
        const float J0[3] = {f.j00, 0.f, f.j02}, J1[3] = {0.f, f.j11, f.j12};
        float Gc[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                Gc[3 * a + b] = J0[a] * (D[0] * J0[b] + D[1] * J1[b]) + J1[a] * (D[1] * J0[b] + D[2] * J1[b]);
        // Sigma_c = W W^T, W = R_CW M
        const float* Rt = vw.Rt;
        float Wm[9];
        for (int r = 0; r < 3; ++r)
            for (int k = 0; k < 3; ++k)
                Wm[3 * r + k] = Rt[4 * r] * G.M[k] + Rt[4 * r + 1] * G.M[3 + k] + Rt[4 * r + 2] * G.M[6 + k];
        float Sc[9];
        for (int r = 0; r < 3; ++r)
            for (int k = 0; k < 3; ++k)
                Sc[3 * r + k] = Wm[3 * r] * Wm[3 * k] + Wm[3 * r + 1] * Wm[3 * k + 1] + Wm[3 * r + 2] * Wm[3 * k + 2];
        // antisymmetric part A = Sc G - G Sc, entries (1,2), (2,0), (0,1)
        auto SG = [&](int r, int k) { return Sc[3 * r] * Gc[k] + Sc[3 * r + 1] * Gc[3 + k] + Sc[3 * r + 2] * Gc[6 + k]; };
        auto GS = [&](int r, int k) { return Gc[3 * r] * Sc[k] + Gc[3 * r + 1] * Sc[3 + k] + Gc[3 * r + 2] * Sc[6 + k]; };
        const float* p = f.p;
        tw[0] += dp[0];
        tw[1] += dp[1];
        tw[2] += dp[2];
        tw[3] += (double)(p[1] * dp[2] - p[2] * dp[1]) + 2.0 * (double)(SG(1, 2) - GS(1, 2));
        tw[4] += (double)(p[2] * dp[0] - p[0] * dp[2]) + 2.0 * (double)(SG(2, 0) - GS(2, 0));
        tw[5] += (double)(p[0] * dp[1] - p[1] * dp[0]) + 2.0 * (double)(SG(0, 1) - GS(0, 1));
    }
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    for (int k = 0; k < 6; ++k) {
        double x = tw[k];
        for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
        if (lane == 0) s_red[k][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double acc = 0.0;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) acc += s_red[threadIdx.x][w];
        partials[((size_t)v * nblk + blockIdx.x) * 6 + threadIdx.x] = acc;
    }
}

// Per view: fixed-order sum of the block partials (deterministic).
__global__ void __launch_bounds__(256) k_pose_final(const double* __restrict__ partials, int nblk,
                                                    float* __restrict__ twist) {
    __shared__ double s[6][256];
    const int v = blockIdx.x;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblk; b += blockDim.x)
        for (int k = 0; k < 6; ++k) acc[k] += partials[((size_t)v * nblk + b) * 6 + k];
    for (int k = 0; k < 6; ++k) s[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int d = blockDim.x / 2; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d)
            for (int k = 0; k < 6; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x < 6) twist[6 * v + threadIdx.x] = (float)s[threadIdx.x][0];
}

hipError_t launch_project_bwd(const GaussPtrs& g, const gs_view* views_dev, int n_views, const RasterConst& c,
                              const int32_t* touched, const float* grad_geo, const float* grad_app,
                              const GradPtrs& out, bool accumulate, hipStream_t s) {
    if (g.n == 0) return hipSuccess;
    auto kern = accumulate ? k_project_bwd<16, true> : k_project_bwd<16, false>;
    switch (g.n_feat) {
        case 0: kern = accumulate ? k_project_bwd<0, true> : k_project_bwd<0, false>; break;
        case 8: kern = accumulate ? k_project_bwd<8, true> : k_project_bwd<8, false>; break;
        case 32: kern = accumulate ? k_project_bwd<32, true> : k_project_bwd<32, false>; break;
        case 16: break;
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)ceil_div(g.n, kPbThreads)), dim3(kPbThreads), 0, s, g, views_dev, n_views,
                       c.blur, touched, reinterpret_cast<const float4*>(grad_geo),
                       reinterpret_cast<const float4*>(grad_app), out);
    return hipGetLastError();
}

size_t pose_workspace_bytes(int n, int n_views) {
    const size_t nblk = (size_t)ceil_div(n > 0 ? n : 1, kPoseChunk);
    return nblk * (size_t)n_views * 6 * sizeof(double);
}

hipError_t launch_pose_grad(const GaussPtrs& g, const gs_view* views_dev, int n_views, const RasterConst& c,
                            const int32_t* touched, const float* grad_geo, void* ws, float* twist, hipStream_t s) {
    const int nblk = ceil_div(g.n > 0 ? g.n : 1, kPoseChunk);
    double* partials = static_cast<double*>(ws);
    hipLaunchKernelGGL(k_pose_partial, dim3((unsigned)nblk, (unsigned)n_views), dim3(kPoseThreads), 0, s, g, views_dev,
                       c.blur, touched, reinterpret_cast<const float4*>(grad_geo), partials, nblk);
    hipLaunchKernelGGL(k_pose_final, dim3((unsigned)n_views), dim3(256), 0, s, partials, nblk, twist);
    return hipGetLastError();
}

}  // namespace sgs
