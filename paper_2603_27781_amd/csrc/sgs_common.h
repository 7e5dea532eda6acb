// Internal definitions shared by the HIP translation units of libsgs.
// Every kernel here targets gfx950 (CDNA4, wave64) only.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "../../include/sgs.h"

namespace sgs {

constexpr int kWave = 64;

// Constants of the rasterizer derived on the host from gs_config.
struct RasterConst {
    float z_near, blur, guard, alpha_min, alpha_max, T_min;
    float logit_min;  // (float)ln(alpha_min / (1 - alpha_min)): opacity cull
    int32_t tile;
};

// Plain-pointer view of the Gaussian planes, passed by value to kernels.
struct GaussPtrs {
    const float* mu;
    const float* log_scale;
    const float* quat;
    const float* logit;
    const float* color;
    const float* feat;
    int32_t n, n_feat;
};

struct GradPtrs {
    float* mu;
    float* log_scale;
    float* quat;
    float* logit;
    float* color;
    float* feat;
};

__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Tile order of the one-workgroup-per-tile launches.  Workgroup b runs on
// XCD b mod 8, and each XCD has its own L2; neighbouring tiles share most of
// their Gaussians, so the tiles go to the XCDs in runs of about 32 k pixels
// of consecutive tiles (the runs dealt round-robin), and the tiles an XCD
// has in flight are neighbours whose shared Gaussian records come from its
// own L2 instead of each being fetched again by another XCD.
constexpr int kXcds = 8;
// Run length, in tiles, for tile side ts.
__host__ __device__ constexpr int tile_run(int ts) { return 32768 / (ts * ts) > 8 ? 32768 / (ts * ts) : 8; }
inline unsigned tile_grid(int total_tiles, int run) {
    const int runs = (total_tiles + run - 1) / run;
    return (unsigned)((runs + kXcds - 1) / kXcds * kXcds * run);
}
// The tile of workgroup b of a tile_grid launch, or -1 (no tile: exit).
__device__ __forceinline__ int tile_of_block(int b, int total_tiles, int run) {
    const int x = b & (kXcds - 1), r = b / kXcds;
    const int round = r / run;
    const int t = (round * kXcds + x) * run + (r - round * run);
    return t < total_tiles ? t : -1;
}
template <int TS>
inline unsigned tile_grid(int total_tiles) {
    return tile_grid(total_tiles, tile_run(TS));
}
template <int TS>
__device__ __forceinline__ int tile_of_block(int b, int total_tiles) {
    return tile_of_block(b, total_tiles, tile_run(TS));
}

// Index of the view owning global tile t (views sorted by tile_offset).
__device__ inline int view_of_tile(const gs_view* views, int n_views, int t) {
    int v = 0;
    while (v + 1 < n_views && views[v + 1].tile_offset <= t) ++v;
    return v;
}

// Pack two non-negative radii as binary16, rounded up (a conservative box).
__device__ inline float pack_radii(float rx, float ry) {
    __half hx = __float2half_ru(rx);
    __half hy = __float2half_ru(ry);
    uint32_t bits = (uint32_t)__half_as_ushort(hx) | ((uint32_t)__half_as_ushort(hy) << 16);
    return __uint_as_float(bits);
}

__device__ inline float2 unpack_radii(float packed) {
    uint32_t bits = __float_as_uint(packed);
    return make_float2(__half2float(__ushort_as_half((unsigned short)(bits & 0xffffu))),
                       __half2float(__ushort_as_half((unsigned short)(bits >> 16))));
}

// Inclusive scans over the wavefront with DPP (no LDS): row shifts by 1, 2,
// 4, 8 within rows of 16 lanes, then the row broadcasts of lanes 15 and 31
// carry the row totals across rows.  Lanes without a predecessor at a step
// take the identity (-1 for the max over non-negative values, 0 for the sum).
__device__ __forceinline__ int wave_max_scan(int x) {
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x111, 0xf, 0xf, false));  // row_shr:1
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x112, 0xf, 0xf, false));  // row_shr:2
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x114, 0xf, 0xf, false));  // row_shr:4
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x118, 0xf, 0xf, false));  // row_shr:8
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x142, 0xa, 0xf, false));  // row_bcast:15 into rows 1, 3
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x143, 0xc, 0xf, false));  // row_bcast:31 into rows 2, 3
    return x;
}
__device__ __forceinline__ int wave_add_scan(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);
    return x;
}

// Lanes of the wavefront holding the same 8-bit digit as this lane, among
// the valid lanes (8 ballots, one per digit bit).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

// Exclusive scan of the block's NT thread totals (wave scans, then the wave
// totals in LDS); *total receives the block total.
template <int NT>
__device__ uint32_t block_exclusive(uint32_t v, uint32_t* s_tmp, uint32_t* total) {
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    // wave inclusive scan (DPP; two's-complement adds are the unsigned ones)
    const uint32_t x = (uint32_t)wave_add_scan((int)v);
    if (lane == kWave - 1) s_tmp[wave] = x;
    __syncthreads();
    uint32_t wbase = 0, tot = 0;
    for (int w = 0; w < NT / kWave; ++w) {
        const uint32_t s = s_tmp[w];
        if (w < wave) wbase += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return wbase + x - v;
}

// Fill kernel (used instead of hipMemsetAsync so that calls stay correct
// when captured in a HIP graph and replayed).
__global__ void k_fill_u32(uint32_t* p, uint32_t value, int64_t count);

hipError_t fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s);

// ---------------------------------------------------------------------------
// launchers (each defined in the translation unit of its kernels)
// ---------------------------------------------------------------------------
hipError_t launch_project(const GaussPtrs& g, const gs_view* views_dev, int n_views, const RasterConst& c,
                          float* rec, uint32_t* rect, int32_t* touched, float* app, int app_stride,
                          hipStream_t s);

size_t binsort_workspace_bytes(int n, int n_views, int64_t capacity);
hipError_t launch_binsort(const uint32_t* rect, const int32_t* touched, int n,
                          const gs_view* views_dev, int n_views, int total_tiles, int tile, void* ws,
                          int64_t capacity, uint32_t* tile_keys, int32_t* inst, int32_t* inst_gid,
                          int32_t* pair_first, int32_t* ranges, int64_t* counts, hipStream_t s);

hipError_t launch_render_fwd(const float* rec, const float* app, int n, int n_feat, const int32_t* inst,
                             const int32_t* inst_gid,
                             const int32_t* ranges, const gs_view* views_dev, int n_views, int total_tiles,
                             int64_t total_pixels, const RasterConst& c, int lds_batch, int persistent,
                             float* out, float* T_final, int32_t* last, int32_t* queue, hipStream_t s);

size_t slam_loss_workspace_bytes(int64_t P, const gs_view* views_host, int n_views, int n_feat,
                                 const gs_decoder* dec, const gs_slam_loss_opts& o);
hipError_t launch_slam_loss(const float* out, int n_feat, const float* rgb_t, const float* depth_t,
                            const int32_t* labels, const gs_decoder* dec, const gs_slam_loss_opts& o,
                            const gs_view* views_host, const gs_view* views_dev, int n_views, int64_t P,
                            float* grad_out, double* loss, float* median, uint8_t* masks, void* ws, hipStream_t s);
size_t loss_workspace_bytes(int64_t P);
hipError_t launch_loss(const float* out, int n_feat, const float* rgb_t, const float* depth_t,
                       const int32_t* labels, const float* decoder, int n_classes, const float* weights,
                       const gs_view* views_dev, int n_views, int64_t total_pixels, float* grad_out,
                       double* loss, void* ws, hipStream_t s);

int bwd_record_floats(int n_feat, bool params);
hipError_t launch_render_bwd(const float* rec, const float* app, int n, int n_feat, const int32_t* inst,
                             const int32_t* inst_gid, const int32_t* ranges, const gs_view* views_dev, int n_views,
                             int total_tiles, int64_t total_pixels, const RasterConst& c, int lds_batch,
                             int persistent, const float* T_final, const int32_t* last, const float* grad_out,
                             bool params, float* records, int32_t* queue, hipStream_t s);
hipError_t launch_reduce_records(const float* records, const int32_t* pair_first, const int32_t* touched, int n,
                                 int n_feat, int n_views, int64_t capacity, bool params, float* grad_geo,
                                 float* grad_app, hipStream_t s);

// accumulate: add to the planes of out; otherwise write every plane of every
// Gaussian (zeros where no view contributes).
hipError_t launch_project_bwd(const GaussPtrs& g, const gs_view* views_dev, int n_views, const RasterConst& c,
                              const int32_t* touched, const float* grad_geo, const float* grad_app,
                              const GradPtrs& out, bool accumulate, hipStream_t s);

size_t pose_workspace_bytes(int n, int n_views);
hipError_t launch_pose_grad(const GaussPtrs& g, const gs_view* views_dev, int n_views, const RasterConst& c,
                            const int32_t* touched, const float* grad_geo, void* ws, float* twist, hipStream_t s);

// Feature counts compiled into the render kernels.
inline bool feat_supported(int f) { return f == 0 || f == 8 || f == 16 || f == 32; }
inline int app_stride(int f) { return ((3 + f) + 3) / 4 * 4; }

}  // namespace sgs
