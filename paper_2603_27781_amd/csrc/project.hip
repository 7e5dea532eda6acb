// Projection of every (view, Gaussian) pair: GS^3LAM Sec. 3.2, Eq. (2)-(3).
//
// One thread per Gaussian (grid ceil(n/256)): the Gaussian planes are read
// once as coalesced structure-of-arrays loads, and the thread projects the
// Gaussian into every view.
//
// Everything that decides an integer downstream -- culling, the projected
// mean, the conic, the depth key and the tile rectangle -- is evaluated in
// binary32 with one rounding per operation in a fixed order: this library is
// built with -ffp-contract=off, divisions and square roots are correctly
// rounded, and exp on this path is an explicit Cody-Waite reduction with a
// degree-6 Taylor polynomial (dec_exp) rather than the hardware
// approximation.  That makes the binning reproducible bit for bit by any
// IEEE binary32 implementation of the same sequence of operations.
#include "sgs_common.h"

namespace sgs {

// exp(x) = 2^n e^r, n = rint(x log2 e), r = x - n ln2 (ln2 split in a 16-bit
// head and a tail so n*head is exact); e^r by Taylor to degree 6 (Horner).
__device__ __forceinline__ float dec_exp(float x) {
    if (x != x) return x;
    x = x < -80.0f ? -80.0f : x;
    x = x > 80.0f ? 80.0f : x;
    const float n = rintf(x * 0x1.715476p+0f);
    float r = x - n * 0x1.62e4p-1f;
    r = r - n * 0x1.7f7d1cp-20f;
    float p = 0x1.6c16c2p-10f;  // 1/720
    p = 0x1.111112p-7f + r * p;   // 1/120
    p = 0x1.555556p-5f + r * p;   // 1/24
    p = 0x1.555556p-3f + r * p;   // 1/6
    p = 0.5f + r * p;
    p = 1.0f + r * p;
    p = 1.0f + r * p;
    return ldexpf(p, (int)n);
}

// One thread per Gaussian: the view-independent part (opacity cull, unit
// quaternion, rotation, scales, M = R S) is evaluated once, then every view
// is projected in turn; each view's outputs are written as coalesced rows.
__global__ void __launch_bounds__(256) k_project(GaussPtrs g, const gs_view* __restrict__ views, int n_views,
                                                 RasterConst c, float4* __restrict__ rec,
                                                 uint2* __restrict__ rect, int32_t* __restrict__ touched,
                                                 float* __restrict__ app, int app_stride) {
    const int n = g.n;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;

    if (app != nullptr) {
        // appearance record (c, f, 0...) gathered per instance by the render
        // kernels, written as float4 (app_stride is a multiple of 4)
        float4* a4 = reinterpret_cast<float4*>(app + (size_t)i * app_stride);
        const int F = g.n_feat;
        auto val = [&](int k) -> float {
            if (k < 3) return g.color[(size_t)k * n + i];
            if (k < 3 + F) return g.feat[(size_t)(k - 3) * n + i];
            return 0.0f;
        };
        for (int q = 0; q < app_stride / 4; ++q)
            a4[q] = make_float4(val(4 * q), val(4 * q + 1), val(4 * q + 2), val(4 * q + 3));
    }

    const float logit = g.logit[i];
    const float m0 = g.mu[i], m1 = g.mu[(size_t)n + i], m2 = g.mu[2 * (size_t)n + i];
    const float q0 = g.quat[i], q1 = g.quat[(size_t)n + i], q2 = g.quat[2 * (size_t)n + i],
                q3 = g.quat[3 * (size_t)n + i];
    const float n2 = ((q0 * q0 + q1 * q1) + q2 * q2) + q3 * q3;
    const bool alive = (logit > c.logit_min) && (n2 > 0.0f) && (n2 < INFINITY);
    // rotation of the unit quaternion and M = R S (Eq. 2)
    float M00 = 0.f, M01 = 0.f, M02 = 0.f, M10 = 0.f, M11 = 0.f, M12 = 0.f, M20 = 0.f, M21 = 0.f, M22 = 0.f;
    float op = 0.f;
    if (alive) {
        const float nrm = sqrtf(n2);
        const float w = q0 / nrm, x = q1 / nrm, y = q2 / nrm, z = q3 / nrm;
        const float r00 = 1.0f - 2.0f * (y * y + z * z);
        const float r01 = 2.0f * (x * y - w * z);
        const float r02 = 2.0f * (x * z + w * y);
        const float r10 = 2.0f * (x * y + w * z);
        const float r11 = 1.0f - 2.0f * (x * x + z * z);
        const float r12 = 2.0f * (y * z - w * x);
        const float r20 = 2.0f * (x * z - w * y);
        const float r21 = 2.0f * (y * z + w * x);
        const float r22 = 1.0f - 2.0f * (x * x + y * y);
        const float s0 = dec_exp(g.log_scale[i]);
        const float s1 = dec_exp(g.log_scale[(size_t)n + i]);
        const float s2 = dec_exp(g.log_scale[2 * (size_t)n + i]);
        M00 = r00 * s0; M01 = r01 * s1; M02 = r02 * s2;
        M10 = r10 * s0; M11 = r11 * s1; M12 = r12 * s2;
        M20 = r20 * s0; M21 = r21 * s1; M22 = r22 * s2;
        // value path: activated opacity (hardware exp is fine here)
        op = 1.0f / (1.0f + __expf(-logit));
    }

    for (int v = 0; v < n_views; ++v) {
        const gs_view& vw = views[v];
        const size_t o = (size_t)v * n + i;
        int32_t cnt = 0;
        const float* R = vw.Rt;  // row-major [R|t]: R[0..2] t at [3], [7], [11]
        const float p0 = ((R[0] * m0 + R[1] * m1) + R[2] * m2) + R[3];
        const float p1 = ((R[4] * m0 + R[5] * m1) + R[6] * m2) + R[7];
        const float p2 = ((R[8] * m0 + R[9] * m1) + R[10] * m2) + R[11];
        bool vis = alive && (p2 > c.z_near);
        const float xn = p0 / p2, yn = p1 / p2;
        const float limx = (c.guard * (0.5f * (float)vw.width)) / vw.fx;
        const float limy = (c.guard * (0.5f * (float)vw.height)) / vw.fy;
        vis = vis && (fabsf(xn) <= limx) && (fabsf(yn) <= limy);
        if (vis) {
            const float mx = vw.fx * xn + vw.cx;
            const float my = vw.fy * yn + vw.cy;
            // EWA (Eq. 3): J = d(pi)/dp, T = J R_CW, U = T M, Sigma2D = U U^T + b I
            const float j00 = vw.fx / p2, j11 = vw.fy / p2;
            const float j02 = -(j00 * xn), j12 = -(j11 * yn);
            const float T00 = j00 * R[0] + j02 * R[8];
            const float T01 = j00 * R[1] + j02 * R[9];
            const float T02 = j00 * R[2] + j02 * R[10];
            const float T10 = j11 * R[4] + j12 * R[8];
            const float T11 = j11 * R[5] + j12 * R[9];
            const float T12 = j11 * R[6] + j12 * R[10];
            const float U00 = (T00 * M00 + T01 * M10) + T02 * M20;
            const float U01 = (T00 * M01 + T01 * M11) + T02 * M21;
            const float U02 = (T00 * M02 + T01 * M12) + T02 * M22;
            const float U10 = (T10 * M00 + T11 * M10) + T12 * M20;
            const float U11 = (T10 * M01 + T11 * M11) + T12 * M21;
            const float U12 = (T10 * M02 + T11 * M12) + T12 * M22;
            const float a = ((U00 * U00 + U01 * U01) + U02 * U02) + c.blur;
            const float b = (U00 * U10 + U01 * U11) + U02 * U12;
            const float cc = ((U10 * U10 + U11 * U11) + U12 * U12) + c.blur;
            const float det = a * cc - b * b;
            vis = (det > 0.0f) && (det < INFINITY);
            if (vis) {
                const float rx = sqrtf(c.kbox * a) * 0x1.004p+0f;
                const float ry = sqrtf(c.kbox * cc) * 0x1.004p+0f;
                // tile rectangle (inclusive); tile is a power of two so the scale is exact
                const float inv = 1.0f / (float)c.tile;
                const int tx = ceil_div(vw.width, c.tile), ty = ceil_div(vw.height, c.tile);
                float fx0 = floorf((mx - rx) * inv), fx1 = floorf((mx + rx) * inv);
                float fy0 = floorf((my - ry) * inv), fy1 = floorf((my + ry) * inv);
                vis = (fx1 >= 0.0f) && (fx0 <= (float)(tx - 1)) && (fy1 >= 0.0f) && (fy0 <= (float)(ty - 1));
                if (vis) {
                    fx0 = fx0 < 0.0f ? 0.0f : fx0;
                    fy0 = fy0 < 0.0f ? 0.0f : fy0;
                    fx1 = fx1 > (float)(tx - 1) ? (float)(tx - 1) : fx1;
                    fy1 = fy1 > (float)(ty - 1) ? (float)(ty - 1) : fy1;
                    const int ix0 = (int)fx0, iy0 = (int)fy0, ix1 = (int)fx1, iy1 = (int)fy1;
                    cnt = (ix1 - ix0 + 1) * (iy1 - iy0 + 1);
                    // the record and rectangle of a pair are only read when it is visible
                    rec[2 * o] = make_float4(mx, my, cc / det, -b / det);
                    rec[2 * o + 1] = make_float4(a / det, op, p2, pack_radii(rx, ry));
                    rect[o] = make_uint2((uint32_t)ix0 | ((uint32_t)iy0 << 16),
                                         (uint32_t)ix1 | ((uint32_t)iy1 << 16));
                }
            }
        }
        touched[o] = cnt;
    }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t value, int64_t count) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = value;
}

hipError_t fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, value, count);
    return hipGetLastError();
}

hipError_t launch_project(const GaussPtrs& g, const gs_view* views_dev, int n_views, const RasterConst& c,
                          float* rec, uint32_t* rect, int32_t* touched, float* app, int app_stride_,
                          hipStream_t s) {
    if (g.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_project, dim3((unsigned)ceil_div(g.n, 256)), dim3(256), 0, s, g, views_dev, n_views, c,
                       reinterpret_cast<float4*>(rec), reinterpret_cast<uint2*>(rect), touched, app, app_stride_);
    return hipGetLastError();
}

}  // namespace sgs
