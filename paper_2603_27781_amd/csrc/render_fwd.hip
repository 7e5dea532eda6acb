// Forward compositing, GS^3LAM Sec. 3.2.1 Eq. (4)-(6), Sec. 3.2.2 Eq. (7),
// Sec. 3.3.1 Eq. (10):
//   out_ch(p) = sum_i x_i,ch alpha_i T_i,   T_i = prod_{j<i} (1 - alpha_j)
// for colour (3), depth (1) and the F semantic feature channels, with the
// cumulative opacity written as 1 - T_final (equal to sum_i alpha_i T_i).
//
// Launch shape: one workgroup of TS*TS threads per (view, tile); each
// wavefront owns an 8x8 block of pixels (compact, so that a small splat
// touches few wavefronts).  The tile's depth-sorted list is walked in
// batches of B instances that the whole workgroup stages into LDS (geometry
// as two float4, appearance as (3+F) floats padded to float4, slot-major);
// every wavefront then reads them as broadcasts.
// Per batch, each wavefront ballots which Gaussians' pixel boxes reach its
// 8x8 block (one bit per Gaussian) and visits only those, with the next
// one's geometry already in flight; a pixel stops when T would fall below
// T_min, a wavefront stops when all of its pixels stopped and the workgroup
// stops when every wavefront did.
//
// persistent = 1 launches ~one wave of workgroups that pull tile indices
// from a device counter (all views share one queue), so views of uneven
// size are balanced inside one launch.
//
// LK > 0 (gs_render_fwd_loss) adds the image-space loss of gs_loss_grad in
// the epilogue: each pixel's rendered channels are still in registers, so
// the loss gradient is written without reading the image back, with the
// same per-pixel arithmetic as k_loss (semantic_ce with up to LK classes in
// registers); each tile's three loss terms go to partials[term][tile] and
// are summed in a fixed order afterwards.
#include "fused_loss.h"
#include "loss_common.h"
#include "raster_common.h"

namespace sgs {

// A wavefront-uniform value copied into a vector register once (one
// v_mov), so that its uses as an LDS address and as a select operand take
// that register instead of a fresh copy each.
__device__ __forceinline__ int to_vgpr(int s) {
    int v;
    __asm__("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
    return v;
}

template <int TS, int F, int B, int LK>
__device__ __forceinline__ void fwd_tile(int t, const float4* __restrict__ rec, const float4* __restrict__ app, int n,
                                         const int32_t* __restrict__ inst, const int32_t* __restrict__ inst_gid,
                                         const int2* __restrict__ ranges,
                                         const gs_view* __restrict__ views, int n_views, int64_t P,
                                         const RasterConst& c, float* __restrict__ out, float* __restrict__ T_final,
                                         int32_t* __restrict__ last, float4* s_g0, float4* s_g1, float4* s_app,
                                         int total_tiles, const FusedLoss& L, const float* __restrict__ Wt,
                                         double* s_red) {
    constexpr int NT = TS * TS;
    constexpr int AV = AppRec<F>::vec;
    static_assert((3 + F) % 4 == 3, "the staged appearance record needs its padding slot for the depth");
    constexpr int NQ = B / 64;  // 64-bit candidate masks per batch
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    constexpr int WPR = TS / 8;
    const int sbx = (wave % WPR) * 8, sby = (wave / WPR) * 8;

    const int v = view_of_tile(views, n_views, t);
    const gs_view& vw = views[v];
    const int tiles_x = ceil_div(vw.width, TS);
    const int lt = t - vw.tile_offset;
    const int tx = lt % tiles_x, ty = lt / tiles_x;
    const int x = tx * TS + sbx + (lane & 7);
    const int y = ty * TS + sby + (lane >> 3);
    const bool inside = x < vw.width && y < vw.height;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    const float wx0 = (float)(tx * TS + sbx) + 0.5f, wy0 = (float)(ty * TS + sby) + 0.5f;
    const size_t vbase = (size_t)v * n;
    const int2 rg = ranges[t];

    float acc[4 + F];
#pragma unroll
    for (int k = 0; k < 4 + F; ++k) acc[k] = 0.0f;
    float T = 1.0f;
    int lastj = 0;
    // lanes whose pixel is finished (outside the view, or T would fall
    // below T_min), as a wavefront mask: the per-step bookkeeping is then
    // scalar work on ballots of the two comparisons the step makes anyway
    uint64_t done_m = __builtin_amdgcn_ballot_w64(!inside);
    const float log2_amin = __log2f(c.alpha_min);
    const float amin = c.alpha_min, amax = c.alpha_max, tmin = c.T_min;
    // with the fused loss, the pixel's targets are requested now and first
    // used after the compositing loop, so their latency is hidden by it
    float tgt[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    int tlab = -1;
    if constexpr (LK > 0) {
        if (inside) {
            const int64_t p = vw.pixel_offset + (int64_t)y * vw.width + x;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) tgt[ch] = L.rgb_t[ch * P + p];
            tgt[3] = L.depth_t[p];
            if (F > 0 && L.K > 0) tlab = L.labels[p];
        }
    }

    for (int b0 = rg.x; b0 < rg.y; b0 += B) {
        if (__syncthreads_and(done_m == ~0ull)) break;
        const int nb = min(B, rg.y - b0);
        for (int k = tid; k < nb; k += NT) {
            const int gid = inst_gid[inst[b0 + k]];
            float4 a0, a1;
            stage_geometry(rec, vbase + gid, a0, a1);
            s_g0[k] = a0;
            s_g1[k] = a1;
            // the appearance record slot-major (s_app[q][k]): a wavefront's
            // stores of one slot are contiguous; the record's last float is
            // padding (3 + F is 3 mod 4): depth goes there
#pragma unroll
            for (int q = 0; q < AV; ++q) s_app[q * B + k] = app[(size_t)gid * AV + q];
            reinterpret_cast<float*>(s_app + (AV - 1) * B + k)[3] = a1.z;
        }
        __syncthreads();
        if (done_m != ~0ull) {
            uint64_t cand[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int k = 64 * q + lane;
                bool ok = false;
                if (k < nb) {
                    const float4 a0 = s_g0[k], a1 = s_g1[k];
                    ok = !box_misses(a0, a1, wx0, wy0) && !ellipse_misses(a0, a1, wx0, wy0, log2_amin);
                }
                cand[q] = __builtin_amdgcn_ballot_w64(ok);
            }
            bool wdone = false;
            // byte offset, within the staged arrays (16 bytes per
            // Gaussian in each), of the pixel's last contributor in this
            // batch, or -1
            int lastoff = -1;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                uint64_t m = cand[q];
                if (m == 0 || wdone) continue;
                int j = 64 * q + __builtin_ctzll(m);
                float4 g0 = s_g0[j], g1 = s_g1[j];
                // the candidate's byte offset in a vector register: the
                // next candidate's, formed for its geometry prefetch, serves
                // as the current one's on the following step
                int joff = to_vgpr(16 * j);
                for (;;) {
                    m &= m - 1;
                    const int jn = m ? 64 * q + __builtin_ctzll(m) : -1;
                    float4 av[AV];
#pragma unroll
                    for (int qq = 0; qq < AV; ++qq)
                        av[qq] = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(s_app + qq * B) + joff);
                    float dx, dy, G, qx, qy;
                    bool unc;
                    const float a = pair_alpha(g0, g1, px, py, amax, dx, dy, G, unc, qx, qy);
                    // g0 and g1 are dead from here: the next candidate's
                    // geometry is loaded into them (no register copies at the
                    // end of the step), unconditionally with a clamped index
                    // (a conditional load becomes a pointer select that
                    // leaves LDS addressing)
                    const int jpoff = to_vgpr(16 * (jn >= 0 ? jn : j));
                    g0 = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(s_g0) + jpoff);
                    g1 = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(s_g1) + jpoff);
                    // issue those loads here, half a step ahead of their use
                    // (left alone, the scheduler sinks them to the end of the
                    // step, next to their use)
                    __builtin_amdgcn_sched_barrier(0);
                    const float Tn = fmaf(-a, T, T);  // T (1 - alpha), one rounding
                    const uint64_t ok = __builtin_amdgcn_ballot_w64(a >= amin) & ~done_m;
                    const uint64_t low = __builtin_amdgcn_ballot_w64(Tn < tmin);
                    const uint64_t use = ok & ~low;
                    // No branch on whether any lane contributes: the
                    // candidates reach the block, so nearly every step has a
                    // contributor, and lanes not contributing add exactly 0 * x.
                    {
                        const float w = mask_select(use, a * T, 0.0f);
                        const float* ap = reinterpret_cast<const float*>(av);
                        acc[0] = fmaf(w, ap[0], acc[0]);
                        acc[1] = fmaf(w, ap[1], acc[1]);
                        acc[2] = fmaf(w, ap[2], acc[2]);
                        acc[3] = fmaf(w, ap[AV * 4 - 1], acc[3]);
#pragma unroll
                        for (int f = 0; f < F; ++f) acc[4 + f] = fmaf(w, ap[3 + f], acc[4 + f]);
                        T = mask_select(use, Tn, T);
                        lastoff = mask_select(use, joff, lastoff);
                    }
                    done_m |= ok & low;
                    if (done_m == ~0ull) {
                        wdone = true;
                        break;
                    }
                    if (jn < 0) break;
                    j = jn;
                    joff = jpoff;
                }
            }
            if (lastoff >= 0) lastj = b0 - rg.x + 1 + (lastoff >> 4);
        }
    }
    if (inside) {
        const int64_t p = vw.pixel_offset + (int64_t)y * vw.width + x;
        out[p] = acc[0];
        out[P + p] = acc[1];
        out[2 * P + p] = acc[2];
        out[3 * P + p] = acc[3];
        out[4 * P + p] = 1.0f - T;
#pragma unroll
        for (int f = 0; f < F; ++f) out[(5 + f) * P + p] = acc[4 + f];
        T_final[p] = T;
        last[p] = lastj;
    }
    if constexpr (LK > 0) {
        // the loss terms of this pixel, each already divided by its count
        double lt[3] = {0.0, 0.0, 0.0};
        if (inside) {
            const int64_t p = vw.pixel_offset + (int64_t)y * vw.width + x;
            const float Pv = (float)((int64_t)vw.width * vw.height);
            const float gc = L.w0 / (3.0f * Pv), gd = L.w1 / Pv, gs = L.w2 / Pv;
            double lc = 0.0;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const float r = acc[ch] - tgt[ch];
                lc += (double)fabsf(r);
                L.grad_out[ch * P + p] = r > 0.0f ? gc : (r < 0.0f ? -gc : 0.0f);
            }
            const float rd = acc[3] - tgt[3];
            L.grad_out[3 * P + p] = rd > 0.0f ? gd : (rd < 0.0f ? -gd : 0.0f);
            L.grad_out[4 * P + p] = 0.0f;
            double ls = 0.0;
            if constexpr (F > 0) {
                float fv[F > 0 ? F : 1], gf[F > 0 ? F : 1];
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    fv[f] = acc[4 + f];
                    gf[f] = 0.0f;
                }
                if (L.K > 0 && L.w2 != 0.0f) ls = (double)semantic_ce<F, LK>(fv, Wt, L.K, tlab, gf);
#pragma unroll
                for (int f = 0; f < F; ++f) L.grad_out[(5 + f) * P + p] = gs * gf[f];
            }
            lt[0] = lc * ((double)L.w0 / (3.0 * (double)Pv));
            lt[1] = (double)fabsf(rd) * ((double)L.w1 / (double)Pv);
            lt[2] = ls * ((double)L.w2 / (double)Pv);
        }
        // the tile's sums, in a fixed order: wavefront butterflies, then the
        // wavefronts in order
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            for (int d = kWave / 2; d > 0; d >>= 1) lt[k] += __shfl_xor(lt[k], d, kWave);
        }
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 3; ++k) s_red[k * (NT / kWave) + wave] = lt[k];
        }
        __syncthreads();
        if (tid < 3) {
            double a = 0.0;
            for (int w = 0; w < NT / kWave; ++w) a += s_red[tid * (NT / kWave) + w];
            L.partials[(size_t)tid * total_tiles + t] = a;
        }
    }
}

// With the fused loss the epilogue's logits raise the register count a
// little above the compositing loop's; the cap keeps five wavefronts per
// SIMD for the loop (at tile 8 the LDS batch limits residency anyway).
template <int TS, int F, int B, int LK>
__global__ void __launch_bounds__(TS* TS)
    __attribute__((amdgpu_waves_per_eu(LK > 0 && TS >= 16 ? 5 : 1, 8))) k_render_fwd(const float4* __restrict__ rec, const float4* __restrict__ app,
                                                       int n, const int32_t* __restrict__ inst,
                                                       const int32_t* __restrict__ inst_gid,
                                                       const int2* __restrict__ ranges,
                                                       const gs_view* __restrict__ views, int n_views,
                                                       int total_tiles, int64_t P, RasterConst c,
                                                       float* __restrict__ out, float* __restrict__ T_final,
                                                       int32_t* __restrict__ last, int32_t* queue, int persistent,
                                                       FusedLoss L, const float* __restrict__ Wt) {
    constexpr int AV = AppRec<F>::vec;
    __shared__ float4 s_g0[B];
    __shared__ float4 s_g1[B];
    __shared__ float4 s_app[B * AV];
    __shared__ double s_red[LK > 0 ? 3 * (TS * TS / kWave) : 1];
    __shared__ int s_tile;
    if (!persistent) {
        const int t = tile_of_block<TS>(blockIdx.x, total_tiles);
        if (t < 0) return;
        fwd_tile<TS, F, B, LK>(t, rec, app, n, inst, inst_gid, ranges, views, n_views, P, c, out, T_final, last, s_g0,
                               s_g1, s_app, total_tiles, L, Wt, s_red);
        return;
    }
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_tile = atomicAdd(queue, 1);
        __syncthreads();
        const int t = s_tile;
        if (t >= total_tiles) break;
        fwd_tile<TS, F, B, LK>(t, rec, app, n, inst, inst_gid, ranges, views, n_views, P, c, out, T_final, last, s_g0,
                               s_g1, s_app, total_tiles, L, Wt, s_red);
    }
}

__global__ void k_reset_queue(int32_t* q) {
    if (threadIdx.x < 4) q[threadIdx.x] = 0;
}

template <int TS, int F, int B, int LK>
hipError_t launch_fwd_t(const float* rec, const float* app, int n, const int32_t* inst, const int32_t* inst_gid,
                        const int32_t* ranges, const gs_view* views, int n_views, int total_tiles, int64_t P,
                        const RasterConst& c, int persistent, float* out, float* T_final, int32_t* last,
                        int32_t* queue, const FusedLoss& L, hipStream_t s) {
    auto kern = k_render_fwd<TS, F, B, LK>;
    unsigned grid = total_tiles > 0 ? tile_grid<TS>(total_tiles) : 0u;
    if (persistent) {
        int dev = 0, cus = 0, per_cu = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, TS * TS, 0);
        if (per_cu < 1) per_cu = 1;
        if (cus < 1) cus = 1;  // a failed query still drains the queue, with fewer workgroups
        unsigned cap = (unsigned)(cus * per_cu);
        grid = cap < (unsigned)total_tiles ? cap : (unsigned)total_tiles;
        hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, s, queue);
    }
    if (grid == 0) return hipGetLastError();
    hipLaunchKernelGGL(kern, dim3(grid), dim3(TS * TS), 0, s, reinterpret_cast<const float4*>(rec),
                       reinterpret_cast<const float4*>(app), n, inst, inst_gid, reinterpret_cast<const int2*>(ranges),
                       views, n_views, total_tiles, P, c, out, T_final, last, queue, persistent, L, L.Wt);
    return hipGetLastError();
}

template <int TS, int F, int LK>
hipError_t launch_fwd_b(int B, const float* rec, const float* app, int n, const int32_t* inst, const int32_t* inst_gid,
                        const int32_t* ranges, const gs_view* views, int n_views, int total_tiles, int64_t P,
                        const RasterConst& c, int persistent, float* out, float* T_final, int32_t* last,
                        int32_t* queue, const FusedLoss& L, hipStream_t s) {
    switch (B) {
        case 64:
            return launch_fwd_t<TS, F, 64, LK>(rec, app, n, inst, inst_gid, ranges, views, n_views, total_tiles, P, c,
                                               persistent, out, T_final, last, queue, L, s);
        case 128:
            return launch_fwd_t<TS, F, 128, LK>(rec, app, n, inst, inst_gid, ranges, views, n_views, total_tiles, P, c,
                                                persistent, out, T_final, last, queue, L, s);
        default:
            return launch_fwd_t<TS, F, 256, LK>(rec, app, n, inst, inst_gid, ranges, views, n_views, total_tiles, P, c,
                                                persistent, out, T_final, last, queue, L, s);
    }
}

template <int F, int LK>
hipError_t launch_fwd_f(int TS, int B, const float* rec, const float* app, int n, const int32_t* inst,
                        const int32_t* inst_gid, const int32_t* ranges, const gs_view* views, int n_views,
                        int total_tiles, int64_t P, const RasterConst& c, int persistent, float* out, float* T_final,
                        int32_t* last, int32_t* queue, const FusedLoss& L, hipStream_t s) {
    switch (TS) {
        case 8:
            return launch_fwd_b<8, F, LK>(B, rec, app, n, inst, inst_gid, ranges, views, n_views, total_tiles, P, c,
                                          persistent, out, T_final, last, queue, L, s);
        case 32:
            return launch_fwd_b<32, F, LK>(B, rec, app, n, inst, inst_gid, ranges, views, n_views, total_tiles, P, c,
                                           persistent, out, T_final, last, queue, L, s);
        default:
            return launch_fwd_b<16, F, LK>(B, rec, app, n, inst, inst_gid, ranges, views, n_views, total_tiles, P, c,
                                           persistent, out, T_final, last, queue, L, s);
    }
}

hipError_t launch_render_fwd(const float* rec, const float* app, int n, int n_feat, const int32_t* inst,
                             const int32_t* inst_gid, const int32_t* ranges, const gs_view* views_dev, int n_views,
                             int total_tiles, int64_t total_pixels, const RasterConst& c, int lds_batch,
                             int persistent, float* out, float* T_final, int32_t* last, int32_t* queue,
                             hipStream_t s) {
    const int TS = c.tile;
    const FusedLoss none{};
    switch (n_feat) {
        case 0:
            return launch_fwd_f<0, 0>(TS, lds_batch, rec, app, n, inst, inst_gid, ranges, views_dev, n_views,
                                      total_tiles, total_pixels, c, persistent, out, T_final, last, queue, none, s);
        case 8:
            return launch_fwd_f<8, 0>(TS, lds_batch, rec, app, n, inst, inst_gid, ranges, views_dev, n_views,
                                      total_tiles, total_pixels, c, persistent, out, T_final, last, queue, none, s);
        case 32:
            return launch_fwd_f<32, 0>(TS, lds_batch, rec, app, n, inst, inst_gid, ranges, views_dev, n_views,
                                       total_tiles, total_pixels, c, persistent, out, T_final, last, queue, none, s);
        default:
            return launch_fwd_f<16, 0>(TS, lds_batch, rec, app, n, inst, inst_gid, ranges, views_dev, n_views,
                                       total_tiles, total_pixels, c, persistent, out, T_final, last, queue, none, s);
    }
}

// workspace of the fused path: per-tile partials [3][total_tiles], their
// first-stage sums, the transposed decoder (at most 16 x 32 floats)
static size_t fused_partials_bytes(int total_tiles) {
    return ((size_t)total_tiles * 3 * sizeof(double) + 255) / 256 * 256;
}
static size_t fused_stage_bytes(int total_tiles) {
    return ((size_t)sum_stage_blocks(total_tiles) * 3 * sizeof(double) + 255) / 256 * 256;
}
size_t fused_loss_workspace_bytes(int total_tiles) {
    return fused_partials_bytes(total_tiles) + fused_stage_bytes(total_tiles) +
           (size_t)kFusedMaxFeat * kFusedMaxClasses * sizeof(float);
}

hipError_t launch_render_fwd_loss(const float* rec, const float* app, int n, int n_feat, const int32_t* inst,
                                  const int32_t* inst_gid, const int32_t* ranges, const gs_view* views_dev,
                                  int n_views, int total_tiles, int64_t total_pixels, const RasterConst& c,
                                  int lds_batch, int persistent, float* out, float* T_final, int32_t* last,
                                  int32_t* queue, const float* rgb_t, const float* depth_t, const int32_t* labels,
                                  const float* decoder, int n_classes, const float* weights, float* grad_out,
                                  double* loss, void* ws, hipStream_t s) {
    if (n_feat > kFusedMaxFeat || n_classes > kFusedMaxClasses) return hipErrorInvalidValue;
    char* w = static_cast<char*>(ws);
    FusedLoss L;
    L.rgb_t = rgb_t;
    L.depth_t = depth_t;
    L.labels = labels;
    L.Wt = reinterpret_cast<float*>(w + fused_partials_bytes(total_tiles) + fused_stage_bytes(total_tiles));
    L.K = n_feat > 0 ? n_classes : 0;
    L.w0 = weights[0];
    L.w1 = weights[1];
    L.w2 = weights[2];
    L.grad_out = grad_out;
    L.partials = reinterpret_cast<double*>(w);
    double* stage = reinterpret_cast<double*>(w + fused_partials_bytes(total_tiles));
    hipError_t e = hipSuccess;
    if (L.K > 0 && L.w2 != 0.0f) {
        e = launch_transpose_decoder(decoder, n_feat, L.K, const_cast<float*>(L.Wt), s);
        if (e != hipSuccess) return e;
    }
    const int TS = c.tile;
    switch (n_feat) {
        case 0:
            e = launch_fwd_f<0, kFusedMaxClasses>(TS, lds_batch, rec, app, n, inst, inst_gid, ranges, views_dev,
                                                  n_views, total_tiles, total_pixels, c, persistent, out, T_final,
                                                  last, queue, L, s);
            break;
        case 8:
            e = launch_fwd_f<8, kFusedMaxClasses>(TS, lds_batch, rec, app, n, inst, inst_gid, ranges, views_dev,
                                                  n_views, total_tiles, total_pixels, c, persistent, out, T_final,
                                                  last, queue, L, s);
            break;
        case 16:
            e = launch_fwd_f<16, kFusedMaxClasses>(TS, lds_batch, rec, app, n, inst, inst_gid, ranges, views_dev,
                                                   n_views, total_tiles, total_pixels, c, persistent, out, T_final,
                                                   last, queue, L, s);
            break;
        default:
            return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    return launch_loss_sums(L.partials, total_tiles, stage, loss, s);
}

}  // namespace sgs
