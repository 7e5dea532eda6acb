// Projection of every (view, Gaussian) pair: GS^3LAM Sec. 3.2, Eq. (2)-(3).
//
// One thread per Gaussian (grid ceil(n/256)): the Gaussian planes are read
// once as coalesced structure-of-arrays loads; the pairs that survive a
// cheap per-view screen are then projected by whole wavefronts at a time
// (see k_project).
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
#include "decision_exp.h"

namespace sgs {

// Per-view constants staged in LDS (20 floats, float4-aligned rows):
// [R|t] (12), fx, fy, cx, cy, the two guard limits, and the last tile
// column and row as floats.
constexpr int kViewFloats = 20;
constexpr int kProjThreads = 256;
constexpr int kProjWaves = kProjThreads / kWave;
constexpr int kProjRing = 128;  // queued (view, lane) entries per wavefront
constexpr int kProjG = 14;      // per-Gaussian values shared in LDS: M (9), opacity, mean (3), box k

// Camera-frame position p = R mu + t (one rounding per operation, fixed order).
__device__ __forceinline__ void cam_point(const float* R, float m0, float m1, float m2, float& p0, float& p1,
                                          float& p2) {
    p0 = ((R[0] * m0 + R[1] * m1) + R[2] * m2) + R[3];
    p1 = ((R[4] * m0 + R[5] * m1) + R[6] * m2) + R[7];
    p2 = ((R[8] * m0 + R[9] * m1) + R[10] * m2) + R[11];
}

// Guard limit of the frustum test, |x/z| <= guard (W/2) / fx.
__device__ __forceinline__ float guard_limit(float guard, int extent, float focal) {
    return (guard * (0.5f * (float)extent)) / focal;
}

// The exact projection of one (view, Gaussian) pair (Eq. 3) and its tile
// rectangle; writes the pair's record and rectangle when it is visible and
// returns its tile count (0 when culled).  The rectangle entry also carries
// the depth's bits, which the binning's emission reads from the same 16
// bytes (the record itself is a 32-byte gather it would fetch only for them).
__device__ __forceinline__ int32_t project_pair(const float* vw, const float* Mg, float op, float m0, float m1,
                                                float m2, float kbox, const RasterConst& c, size_t o,
                                                float4* __restrict__ rec, uint4* __restrict__ rect) {
    const float* R = vw;
    const float fx = vw[12], fy = vw[13], cx = vw[14], cy = vw[15], limx = vw[16], limy = vw[17];
    const float txm1 = vw[18], tym1 = vw[19];
    float p0, p1, p2;
    cam_point(R, m0, m1, m2, p0, p1, p2);
    if (!(p2 > c.z_near)) return 0;
    const float xn = p0 / p2, yn = p1 / p2;
    if (!((fabsf(xn) <= limx) && (fabsf(yn) <= limy))) return 0;
    const float M00 = Mg[0], M01 = Mg[1], M02 = Mg[2], M10 = Mg[3], M11 = Mg[4], M12 = Mg[5], M20 = Mg[6],
                M21 = Mg[7], M22 = Mg[8];
    const float mx = fx * xn + cx;
    const float my = fy * yn + cy;
    // EWA (Eq. 3): J = d(pi)/dp, T = J R_CW, U = T M, Sigma2D = U U^T + b I
    const float j00 = fx / p2, j11 = fy / p2;
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
    if (!((det > 0.0f) && (det < INFINITY))) return 0;
    const float rx = sqrtf(kbox * a) * 0x1.004p+0f;
    const float ry = sqrtf(kbox * cc) * 0x1.004p+0f;
    // tile rectangle (inclusive); tile is a power of two so the scale is exact
    const float inv = 1.0f / (float)c.tile;
    float fx0 = floorf((mx - rx) * inv), fx1 = floorf((mx + rx) * inv);
    float fy0 = floorf((my - ry) * inv), fy1 = floorf((my + ry) * inv);
    if (!((fx1 >= 0.0f) && (fx0 <= txm1) && (fy1 >= 0.0f) && (fy0 <= tym1))) return 0;
    fx0 = fx0 < 0.0f ? 0.0f : fx0;
    fy0 = fy0 < 0.0f ? 0.0f : fy0;
    fx1 = fx1 > txm1 ? txm1 : fx1;
    fy1 = fy1 > tym1 ? tym1 : fy1;
    const int ix0 = (int)fx0, iy0 = (int)fy0, ix1 = (int)fx1, iy1 = (int)fy1;
    // the record and rectangle of a pair are only read when it is visible
    rec[2 * o] = make_float4(mx, my, cc / det, -b / det);
    rec[2 * o + 1] = make_float4(a / det, op, p2, pack_radii(rx, ry));
    rect[o] = make_uint4((uint32_t)ix0 | ((uint32_t)iy0 << 16), (uint32_t)ix1 | ((uint32_t)iy1 << 16),
                         __float_as_uint(p2), 0u);
    return (ix1 - ix0 + 1) * (iy1 - iy0 + 1);
}

// One thread per Gaussian: the view-independent part (opacity cull, unit
// quaternion, rotation, scales, M = R S) is evaluated once and shared in LDS.
// Most (view, Gaussian) pairs fall outside the view, so the thread only
// screens each view with a conservative frustum test that needs no division;
// the pairs that pass are queued per wavefront as (view, lane) entries and
// projected exactly 64 at a time, every lane on a different pair, instead of
// every wavefront running the whole projection for every view.  The screen
// culls a pair only if |p_x| > limx p_z (1 + 2^-10) (or the same in y),
// which implies |fl(p_x / p_z)| > limx, so the exact test decides every
// pair as it would alone.
// The feature count is a template parameter so that the appearance copy is
// one batch of independent loads followed by the float4 stores.
template <int F>
__global__ void __launch_bounds__(kProjThreads) k_project(GaussPtrs g, const gs_view* __restrict__ views,
                                                          int n_views, RasterConst c, float4* __restrict__ rec,
                                                          uint4* __restrict__ rect, int32_t* __restrict__ touched,
                                                          float4* __restrict__ app) {
    constexpr int AS = ((3 + F) + 3) / 4 * 4;  // floats per appearance record
    __shared__ float4 s_vw4[GS_MAX_VIEWS * kViewFloats / 4];
    __shared__ float s_g[kProjG][kProjThreads];
    __shared__ int s_ring[kProjWaves][kProjRing];
    float* s_vw = reinterpret_cast<float*>(s_vw4);
    const int n = g.n;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int i = blockIdx.x * kProjThreads + tid;
    const bool valid = i < n;

    for (int v = tid; v < n_views; v += kProjThreads) {
        const gs_view& vw = views[v];
        float* d = s_vw + v * kViewFloats;
#pragma unroll
        for (int k = 0; k < 12; ++k) d[k] = vw.Rt[k];
        d[12] = vw.fx;
        d[13] = vw.fy;
        d[14] = vw.cx;
        d[15] = vw.cy;
        d[16] = guard_limit(c.guard, vw.width, vw.fx);
        d[17] = guard_limit(c.guard, vw.height, vw.fy);
        d[18] = (float)(ceil_div(vw.width, c.tile) - 1);
        d[19] = (float)(ceil_div(vw.height, c.tile) - 1);
    }

    // every plane is read up front with an in-range index (one batch of
    // independent loads per thread, no branches between them; the
    // appearance planes only when their records are wanted, a uniform test)
    const int ic = valid ? i : n - 1;
    float av[AS];
    if (app != nullptr) {
#pragma unroll
        for (int k = 0; k < AS; ++k)
            av[k] = k < 3 ? g.color[(size_t)k * n + ic] : (k < 3 + F ? g.feat[(size_t)(k - 3) * n + ic] : 0.0f);
    }
    const float logit = g.logit[ic];
    const float m0 = g.mu[ic], m1 = g.mu[(size_t)n + ic], m2 = g.mu[2 * (size_t)n + ic];
    const float q0 = g.quat[ic], q1 = g.quat[(size_t)n + ic], q2 = g.quat[2 * (size_t)n + ic],
                q3 = g.quat[3 * (size_t)n + ic];
    const float ls0 = g.log_scale[ic], ls1 = g.log_scale[(size_t)n + ic], ls2 = g.log_scale[2 * (size_t)n + ic];
    if (valid && app != nullptr) {
        // appearance record (c, f, 0...) gathered per instance by the render
        // kernels, written as float4
        float4* a4 = app + (size_t)i * (AS / 4);
#pragma unroll
        for (int q = 0; q < AS / 4; ++q) a4[q] = make_float4(av[4 * q], av[4 * q + 1], av[4 * q + 2], av[4 * q + 3]);
    }

    const float n2 = ((q0 * q0 + q1 * q1) + q2 * q2) + q3 * q3;
    // opacity-aware box: the decision-path k, <= 0 for o <= alpha_min
    const float kbox = valid ? dec_box_k(logit, c.alpha_min) : 0.0f;
    const bool alive = valid && (logit > c.logit_min) && (kbox > 0.0f) && (n2 > 0.0f) && (n2 < INFINITY);
    if (alive) {
        // rotation of the unit quaternion and M = R S (Eq. 2)
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
        const float s0 = dec_exp(ls0);
        const float s1 = dec_exp(ls1);
        const float s2 = dec_exp(ls2);
        s_g[0][tid] = r00 * s0;
        s_g[1][tid] = r01 * s1;
        s_g[2][tid] = r02 * s2;
        s_g[3][tid] = r10 * s0;
        s_g[4][tid] = r11 * s1;
        s_g[5][tid] = r12 * s2;
        s_g[6][tid] = r20 * s0;
        s_g[7][tid] = r21 * s1;
        s_g[8][tid] = r22 * s2;
        // value path: activated opacity (hardware exp is fine here)
        s_g[9][tid] = 1.0f / (1.0f + __expf(-logit));
        s_g[10][tid] = m0;
        s_g[11][tid] = m1;
        s_g[12][tid] = m2;
        s_g[13][tid] = kbox;
    }
    __syncthreads();

    int* ring = s_ring[wave];
    const int gbase = blockIdx.x * kProjThreads + wave * kWave;  // Gaussian of lane 0
    // projects the queued entries [head, head + cnt), one per lane
    auto drain = [&](int head, int cnt) {
        if (lane < cnt) {
            const int e = ring[(head + lane) & (kProjRing - 1)];
            const int gl = e & (kWave - 1), v = e >> 6;
            const int col = wave * kWave + gl;
            float Mg[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) Mg[k] = s_g[k][col];
            const size_t o = (size_t)v * n + gbase + gl;
            touched[o] = project_pair(s_vw + v * kViewFloats, Mg, s_g[9][col], s_g[10][col], s_g[11][col],
                                      s_g[12][col], s_g[13][col], c, o, rec, rect);
        }
    };
    int head = 0, tail = 0;
    for (int v = 0; v < n_views; ++v) {
        const float* vw = s_vw + v * kViewFloats;
        bool cand = false;
        if (alive) {
            float p0, p1, p2;
            cam_point(vw, m0, m1, m2, p0, p1, p2);
            const float tx = (vw[16] * p2) * 0x1.004p+0f, ty = (vw[17] * p2) * 0x1.004p+0f;
            const bool far = (fabsf(p0) > tx && tx > 0x1p-100f) || (fabsf(p1) > ty && ty > 0x1p-100f);
            cand = (p2 > c.z_near) && !far;
        }
        if (valid && !cand) touched[(size_t)v * n + i] = 0;
        const uint64_t m = __ballot(cand);
        if (cand) ring[(tail + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0))) &
                       (kProjRing - 1)] = lane | (v << 6);
        tail += __popcll(m);
        if (tail - head >= kWave) {
            __builtin_amdgcn_wave_barrier();
            drain(head, kWave);
            head += kWave;
        }
    }
    __builtin_amdgcn_wave_barrier();
    while (head < tail) {
        drain(head, min(kWave, tail - head));
        head += kWave;
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
    if (app != nullptr && app_stride_ != app_stride(g.n_feat)) return hipErrorInvalidValue;
    auto kern = k_project<16>;
    switch (g.n_feat) {
        case 0: kern = k_project<0>; break;
        case 8: kern = k_project<8>; break;
        case 32: kern = k_project<32>; break;
        case 16: break;
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(kern, dim3((unsigned)ceil_div(g.n, kProjThreads)), dim3(kProjThreads), 0, s, g, views_dev,
                       n_views, c, reinterpret_cast<float4*>(rec), reinterpret_cast<uint4*>(rect), touched,
                       reinterpret_cast<float4*>(app));
    return hipGetLastError();
}

}  // namespace sgs
