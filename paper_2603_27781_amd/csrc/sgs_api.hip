// Host side of the C ABI declared in include/sgs.h: argument validation,
// derived constants, workspace carving and kernel launches.  Nothing here
// allocates device memory, synchronises or reads device memory.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "sgs_common.h"
#include "fused_loss.h"
#include "growth.h"
#include "optim.h"

using namespace sgs;

namespace {

thread_local char g_hip_err[256] = {0};

int hip_status(hipError_t e) {
    if (e == hipSuccess) return GS_OK;
    std::snprintf(g_hip_err, sizeof(g_hip_err), "%s", hipGetErrorString(e));
    return GS_EHIP;
}

bool pow2_tile(int t) { return t == 8 || t == 16 || t == 32; }

int check_config(const gs_config* c) {
    if (!c) return GS_EINVAL;
    if (!pow2_tile(c->tile)) return GS_EUNSUPPORTED;
    if (c->lds_batch != 64 && c->lds_batch != 128 && c->lds_batch != 256) return GS_EUNSUPPORTED;
    if (c->lds_batch_bwd != 0 && c->lds_batch_bwd != 64 && c->lds_batch_bwd != 128 && c->lds_batch_bwd != 256)
        return GS_EUNSUPPORTED;
    if (!(c->alpha_min > 0.0f && c->alpha_min < 1.0f)) return GS_EINVAL;
    if (!(c->alpha_max > c->alpha_min && c->alpha_max < 1.0f)) return GS_EINVAL;
    if (!(c->T_min > 0.0f && c->T_min < 1.0f)) return GS_EINVAL;
    if (!(c->z_near > 0.0f) || !(c->blur >= 0.0f) || !(c->guard > 0.0f)) return GS_EINVAL;
    if (c->persistent != 0 && c->persistent != 1) return GS_EINVAL;
    return GS_OK;
}

RasterConst make_const(const gs_config* c) {
    RasterConst k;
    k.z_near = c->z_near;
    k.blur = c->blur;
    k.guard = c->guard;
    k.alpha_min = c->alpha_min;
    k.alpha_max = c->alpha_max;
    k.T_min = c->T_min;
    const double am = (double)c->alpha_min;
    k.logit_min = (float)std::log(am / (1.0 - am));
    k.tile = c->tile;
    return k;
}

// Views must be laid out back to back (as gs_views_layout does).
int check_views(const gs_view* views, const gs_view* views_dev, int n_views, int tile, int64_t* total_pixels,
                int* total_tiles) {
    if (!views || !views_dev) return GS_EINVAL;
    if (n_views < 1 || n_views > GS_MAX_VIEWS) return GS_EINVAL;
    int64_t px = 0;
    int64_t tl = 0;
    for (int v = 0; v < n_views; ++v) {
        const gs_view& w = views[v];
        if (w.width <= 0 || w.height <= 0 || w.width > 65535 * 8 || w.height > 65535 * 8) return GS_EINVAL;
        if (!(w.fx > 0.0f) || !(w.fy > 0.0f)) return GS_EINVAL;
        if (w.pixel_offset != px) return GS_EINVAL;
        if (tile > 0 && w.tile_offset != tl) return GS_EINVAL;
        px += (int64_t)w.width * w.height;
        if (tile > 0) tl += (int64_t)ceil_div(w.width, tile) * ceil_div(w.height, tile);
    }
    if (tl >= (1ll << 31) || px >= (1ll << 31)) return GS_EINVAL;
    if (total_pixels) *total_pixels = px;
    if (total_tiles) *total_tiles = (int)tl;
    return GS_OK;
}

int check_gauss(const gs_gaussians* g, bool need_app) {
    if (!g) return GS_EINVAL;
    if (g->n < 1) return GS_EINVAL;
    if (!g->mu || !g->log_scale || !g->quat || !g->opacity_logit) return GS_EINVAL;
    if (!feat_supported(g->n_feat)) return GS_EUNSUPPORTED;
    if (need_app && (!g->color || (g->n_feat > 0 && !g->feat))) return GS_EINVAL;
    return GS_OK;
}

GaussPtrs gauss_ptrs(const gs_gaussians* g) {
    GaussPtrs p;
    p.mu = g->mu;
    p.log_scale = g->log_scale;
    p.quat = g->quat;
    p.logit = g->opacity_logit;
    p.color = g->color;
    p.feat = g->feat;
    p.n = g->n;
    p.n_feat = g->n_feat;
    return p;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Scratch of gs_pose_grad_noalloc (the per-block partial twist sums), a
// file-scope device array: every GPU the library runs on holds its own copy
// until the process ends.  Host code never uses the array's name as an
// address (on the host it is only a stand-in for the symbol): its device
// address is looked up once per device with hipGetSymbolAddress and kept in
// g_scratch_ptr.
constexpr size_t kScratchBytes = (size_t)GS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call made with that device current).
int scratch_ptr(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e);
    if (dev < 0 || dev >= kMaxDevices) return GS_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_status(e);
        if (!p) return GS_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GS_OK;
}

size_t grad2d_bytes(int n, int n_feat, int n_views) {
    return ((size_t)n_views * n * 8 + (size_t)n * (4 + n_feat)) * sizeof(float);
}

// The fields of up to GS_MAX_VIEWS host views that gs_views_check compares,
// passed by value to its kernel (2.3 KB of kernel arguments).
struct ViewFields {
    int32_t width[GS_MAX_VIEWS], height[GS_MAX_VIEWS], tile_offset[GS_MAX_VIEWS];
    int64_t pixel_offset[GS_MAX_VIEWS];
    float fx[GS_MAX_VIEWS], fy[GS_MAX_VIEWS], cx[GS_MAX_VIEWS], cy[GS_MAX_VIEWS];
};

__device__ __forceinline__ bool same_bits(float a, float b) { return __float_as_uint(a) == __float_as_uint(b); }

// One wavefront, one lane per view: the number of views whose device copy
// differs from the host fields, written by lane 0 whatever it is.
__global__ void __launch_bounds__(kWave) k_views_check(ViewFields h, const gs_view* __restrict__ d, int n,
                                                       int check_tiles, int32_t* __restrict__ mismatch) {
    const int v = threadIdx.x;
    bool bad = false;
    if (v < n) {
        const gs_view& w = d[v];
        bad = w.width != h.width[v] || w.height != h.height[v] || w.pixel_offset != h.pixel_offset[v] ||
              (check_tiles && w.tile_offset != h.tile_offset[v]) || !same_bits(w.fx, h.fx[v]) ||
              !same_bits(w.fy, h.fy[v]) || !same_bits(w.cx, h.cx[v]) || !same_bits(w.cy, h.cy[v]);
    }
    const uint64_t m = __ballot(bad);
    if (v == 0) *mismatch = (int32_t)__popcll(m);
}

}  // namespace

extern "C" {

int gs_default_config(gs_config* cfg) {
    if (!cfg) return GS_EINVAL;
    cfg->z_near = 0.2f;
    cfg->blur = 0.3f;
    cfg->guard = 1.3f;
    cfg->alpha_min = 1.0f / 255.0f;
    cfg->alpha_max = 0.99f;
    cfg->T_min = 1e-4f;
    cfg->tile = 16;
    cfg->lds_batch = 256;
    cfg->persistent = 0;
    cfg->lds_batch_bwd = 0;
    return GS_OK;
}

int gs_views_layout(gs_view* views, int32_t n_views, int32_t tile, int64_t* total_pixels, int32_t* total_tiles) {
    if (!views || n_views < 1 || n_views > GS_MAX_VIEWS || !pow2_tile(tile)) return GS_EINVAL;
    int64_t px = 0, tl = 0;
    for (int v = 0; v < n_views; ++v) {
        if (views[v].width <= 0 || views[v].height <= 0) return GS_EINVAL;
        views[v].pixel_offset = px;
        views[v].tile_offset = (int32_t)tl;
        views[v].reserved = 0;
        px += (int64_t)views[v].width * views[v].height;
        tl += (int64_t)ceil_div(views[v].width, tile) * ceil_div(views[v].height, tile);
    }
    if (tl >= (1ll << 31)) return GS_EINVAL;
    if (total_pixels) *total_pixels = px;
    if (total_tiles) *total_tiles = (int32_t)tl;
    return GS_OK;
}

int32_t gs_app_stride(int32_t n_feat) { return n_feat < 0 ? -1 : (int32_t)app_stride(n_feat); }

int gs_views_check(const gs_view* views, const gs_view* views_dev, int32_t n_views, int32_t tile,
                   int32_t* mismatch_dev, gs_stream stream) {
    if (!mismatch_dev || (tile != 0 && !pow2_tile(tile))) return GS_EINVAL;
    const int st = check_views(views, views_dev, n_views, tile, nullptr, nullptr);
    if (st) return st;
    static_assert(GS_MAX_VIEWS <= kWave, "one lane per view");
    ViewFields h;
    std::memset(&h, 0, sizeof(h));
    for (int v = 0; v < n_views; ++v) {
        h.width[v] = views[v].width;
        h.height[v] = views[v].height;
        h.tile_offset[v] = views[v].tile_offset;
        h.pixel_offset[v] = views[v].pixel_offset;
        h.fx[v] = views[v].fx;
        h.fy[v] = views[v].fy;
        h.cx[v] = views[v].cx;
        h.cy[v] = views[v].cy;
    }
    hipLaunchKernelGGL(k_views_check, dim3(1), dim3(kWave), 0, (hipStream_t)stream, h, views_dev, (int)n_views,
                       tile > 0 ? 1 : 0, mismatch_dev);
    return hip_status(hipGetLastError());
}

int gs_project(const gs_gaussians* g, const gs_view* views, const gs_view* views_dev, int32_t n_views,
               const gs_config* cfg, float* rec, uint32_t* rect, int32_t* tiles_touched, float* app,
               gs_stream stream) {
    int st = check_gauss(g, app != nullptr);
    if (st) return st;
    if ((st = check_config(cfg))) return st;
    if ((st = check_views(views, views_dev, n_views, cfg->tile, nullptr, nullptr))) return st;
    if (!rec || !rect || !tiles_touched) return GS_EINVAL;
    if (!aligned16(rec) || !aligned16(rect) || (app && !aligned16(app))) return GS_EINVAL;
    if ((int64_t)g->n * n_views >= (1ll << 31)) return GS_EINVAL;
    return hip_status(launch_project(gauss_ptrs(g), views_dev, n_views, make_const(cfg), rec, rect, tiles_touched,
                                     app, app_stride(g->n_feat), reinterpret_cast<hipStream_t>(stream)));
}

int gs_bin_sort_workspace(int32_t n, int32_t n_views, int64_t capacity, size_t* bytes) {
    if (!bytes || n < 1 || n_views < 1 || n_views > GS_MAX_VIEWS || capacity < 0) return GS_EINVAL;
    if ((int64_t)n * n_views >= (1ll << 31) || capacity >= (1ll << 31)) return GS_EINVAL;
    *bytes = binsort_workspace_bytes(n, n_views, capacity);
    return GS_OK;
}

int gs_bin_sort(const uint32_t* rect, const int32_t* tiles_touched, int32_t n,
                const gs_view* views, const gs_view* views_dev, int32_t n_views, const gs_config* cfg, void* ws,
                size_t ws_bytes, int64_t capacity, uint32_t* tile_keys, int32_t* inst, int32_t* inst_gid,
                int32_t* pair_first, int32_t* tile_ranges, int64_t* counts, gs_stream stream) {
    int st = check_config(cfg);
    if (st) return st;
    int total_tiles = 0;
    if ((st = check_views(views, views_dev, n_views, cfg->tile, nullptr, &total_tiles))) return st;
    if (!rect || !tiles_touched || !ws || !tile_ranges || !counts || !pair_first) return GS_EINVAL;
    if (capacity > 0 && (!tile_keys || !inst || !inst_gid)) return GS_EINVAL;
    if (n < 1 || capacity < 0 || capacity >= (1ll << 31) || (int64_t)n * n_views >= (1ll << 31)) return GS_EINVAL;
    if (ws_bytes < binsort_workspace_bytes(n, n_views, capacity)) return GS_ECAPACITY;
    if (!aligned16(rect) || (reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return GS_EINVAL;
    return hip_status(launch_binsort(rect, tiles_touched, n, views_dev, n_views, total_tiles, cfg->tile, ws,
                                     capacity, tile_keys, inst, inst_gid, pair_first, tile_ranges, counts,
                                     reinterpret_cast<hipStream_t>(stream)));
}

int gs_render_fwd(const float* rec, const float* app, int32_t n, int32_t n_feat, const int32_t* inst,
                  const int32_t* inst_gid, const int32_t* tile_ranges, const gs_view* views,
                  const gs_view* views_dev, int32_t n_views, const gs_config* cfg, float* out, float* T_final,
                  int32_t* last, int32_t* queue, gs_stream stream) {
    int st = check_config(cfg);
    if (st) return st;
    int64_t P = 0;
    int total_tiles = 0;
    if ((st = check_views(views, views_dev, n_views, cfg->tile, &P, &total_tiles))) return st;
    if (!feat_supported(n_feat)) return GS_EUNSUPPORTED;
    if (n < 1 || !rec || !app || !inst || !inst_gid || !tile_ranges || !out || !T_final || !last) return GS_EINVAL;
    if (cfg->persistent && !queue) return GS_EINVAL;
    if (!aligned16(rec) || !aligned16(app)) return GS_EINVAL;
    return hip_status(launch_render_fwd(rec, app, n, n_feat, inst, inst_gid, tile_ranges, views_dev, n_views,
                                        total_tiles, P, make_const(cfg), cfg->lds_batch, cfg->persistent, out,
                                        T_final, last, queue, reinterpret_cast<hipStream_t>(stream)));
}

int gs_render_fwd_loss_workspace(const gs_view* views, int32_t n_views, int32_t tile, size_t* bytes) {
    if (!bytes || !views || n_views < 1 || n_views > GS_MAX_VIEWS) return GS_EINVAL;
    if (tile != 8 && tile != 16 && tile != 32) return GS_EINVAL;
    int64_t tl = 0;
    for (int v = 0; v < n_views; ++v) {
        if (views[v].width <= 0 || views[v].height <= 0) return GS_EINVAL;
        tl += (int64_t)ceil_div(views[v].width, tile) * ceil_div(views[v].height, tile);
    }
    if (tl >= (1ll << 31)) return GS_EINVAL;
    *bytes = fused_loss_workspace_bytes((int)tl);
    return GS_OK;
}

int gs_render_fwd_loss(const float* rec, const float* app, int32_t n, int32_t n_feat, const int32_t* inst,
                       const int32_t* inst_gid, const int32_t* tile_ranges, const gs_view* views,
                       const gs_view* views_dev, int32_t n_views, const gs_config* cfg, float* out, float* T_final,
                       int32_t* last, int32_t* queue, const float* rgb_target, const float* depth_target,
                       const int32_t* labels, const float* decoder, int32_t n_classes, const float* weights,
                       float* grad_out, double* loss, void* ws, size_t ws_bytes, gs_stream stream) {
    int st = check_config(cfg);
    if (st) return st;
    int64_t P = 0;
    int total_tiles = 0;
    if ((st = check_views(views, views_dev, n_views, cfg->tile, &P, &total_tiles))) return st;
    if (!feat_supported(n_feat)) return GS_EUNSUPPORTED;
    if (n_feat > kFusedMaxFeat || n_classes > kFusedMaxClasses) return GS_EUNSUPPORTED;
    if (n < 1 || !rec || !app || !inst || !inst_gid || !tile_ranges || !out || !T_final || !last) return GS_EINVAL;
    if (cfg->persistent && !queue) return GS_EINVAL;
    if (!aligned16(rec) || !aligned16(app)) return GS_EINVAL;
    if (!rgb_target || !depth_target || !weights || !grad_out || !loss || !ws) return GS_EINVAL;
    if (n_classes < 0) return GS_EINVAL;
    if (n_classes > 0 && n_feat > 0 && (!labels || !decoder)) return GS_EINVAL;
    if (ws_bytes < fused_loss_workspace_bytes(total_tiles)) return GS_ECAPACITY;
    if ((reinterpret_cast<uintptr_t>(ws) & 15u) != 0) return GS_EINVAL;
    return hip_status(launch_render_fwd_loss(rec, app, n, n_feat, inst, inst_gid, tile_ranges, views_dev, n_views,
                                             total_tiles, P, make_const(cfg), cfg->lds_batch, cfg->persistent, out,
                                             T_final, last, queue, rgb_target, depth_target, labels, decoder,
                                             n_feat > 0 ? n_classes : 0, weights, grad_out, loss, ws,
                                             reinterpret_cast<hipStream_t>(stream)));
}

int gs_loss_grad_workspace(int64_t total_pixels, size_t* bytes) {
    if (!bytes || total_pixels < 1) return GS_EINVAL;
    *bytes = loss_workspace_bytes(total_pixels);
    return GS_OK;
}

int gs_loss_grad(const float* out, int32_t n_feat, const float* rgb_target, const float* depth_target,
                 const int32_t* labels, const float* decoder, int32_t n_classes, const float* weights,
                 const gs_view* views, const gs_view* views_dev, int32_t n_views, float* grad_out, double* loss,
                 void* ws, size_t ws_bytes, gs_stream stream) {
    if (!feat_supported(n_feat)) return GS_EUNSUPPORTED;
    int64_t P = 0;
    int st = check_views(views, views_dev, n_views, 0, &P, nullptr);
    if (st) return st;
    if (!out || !rgb_target || !depth_target || !weights || !grad_out || !loss || !ws) return GS_EINVAL;
    if (n_classes < 0 || n_classes > GS_MAX_CLASSES) return GS_EINVAL;
    if (n_classes > 0 && n_feat > 0 && (!labels || !decoder)) return GS_EINVAL;
    if (ws_bytes < loss_workspace_bytes(P)) return GS_ECAPACITY;
    if ((reinterpret_cast<uintptr_t>(ws) & 15u) != 0) return GS_EINVAL;
    return hip_status(launch_loss(out, n_feat, rgb_target, depth_target, labels, decoder, n_feat > 0 ? n_classes : 0,
                                  weights, views_dev, n_views, P, grad_out, loss, ws,
                                  reinterpret_cast<hipStream_t>(stream)));
}

int gs_default_slam_loss_opts(gs_slam_loss_opts* o) {
    if (!o) return GS_EINVAL;
    o->w_color = 0.5f;
    o->w_depth = 1.0f;
    o->w_sem = 0.01f;
    o->ssim_lambda = 0.2f;
    o->tau_obs = 0.99f;
    o->tau_unobs = 0.5f;
    o->obs_factor = 10.0f;
    o->unobs_factor = 50.0f;
    o->flags = 0;
    return GS_OK;
}

static int check_decoder(int32_t n_feat, const gs_decoder* dec, const int32_t* labels) {
    if (dec == nullptr) return GS_OK;
    if (dec->n_classes < 0) return GS_EINVAL;
    if (dec->n_classes > GS_SLAM_MAX_CLASSES) return GS_EUNSUPPORTED;
    if (dec->n_classes > 0 && n_feat > 0 && (!dec->weight || !labels)) return GS_EINVAL;
    return GS_OK;
}

int gs_slam_loss_workspace(const gs_view* views, int32_t n_views, int32_t n_feat, const gs_decoder* dec,
                           const gs_slam_loss_opts* opts, size_t* bytes) {
    if (!bytes || !opts) return GS_EINVAL;
    if (!feat_supported(n_feat)) return GS_EUNSUPPORTED;
    int64_t P = 0;
    int st = check_views(views, views, n_views, 0, &P, nullptr);
    if (st) return st;
    if (dec && (dec->n_classes < 0 || dec->n_classes > GS_SLAM_MAX_CLASSES))
        return dec->n_classes < 0 ? GS_EINVAL : GS_EUNSUPPORTED;
    *bytes = slam_loss_workspace_bytes(P, views, n_views, n_feat, dec, *opts);
    return GS_OK;
}

int gs_slam_loss(const float* out, int32_t n_feat, const float* rgb_target, const float* depth_target,
                 const int32_t* labels, const gs_decoder* dec, const gs_slam_loss_opts* opts, const gs_view* views,
                 const gs_view* views_dev, int32_t n_views, float* grad_out, double* loss, float* median,
                 uint8_t* masks, void* ws, size_t ws_bytes, gs_stream stream) {
    if (!feat_supported(n_feat)) return GS_EUNSUPPORTED;
    int64_t P = 0;
    int st = check_views(views, views_dev, n_views, 0, &P, nullptr);
    if (st) return st;
    if (!out || !rgb_target || !depth_target || !opts || !grad_out || !loss || !ws) return GS_EINVAL;
    if ((st = check_decoder(n_feat, dec, labels))) return st;
    if ((opts->flags & ~(uint32_t)(GS_LOSS_OBS_MASK | GS_LOSS_BCE)) != 0) return GS_EINVAL;
    if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return GS_EINVAL;
    if (ws_bytes < slam_loss_workspace_bytes(P, views, n_views, n_feat, dec, *opts)) return GS_ECAPACITY;
    gs_decoder d{};
    if (dec != nullptr && n_feat > 0) d = *dec;  // without features there is no semantic term
    return hip_status(launch_slam_loss(out, n_feat, rgb_target, depth_target, labels, dec != nullptr ? &d : nullptr,
                                       *opts, views, views_dev, n_views, P, grad_out, loss, median, masks, ws,
                                       reinterpret_cast<hipStream_t>(stream)));
}

int gs_expand_workspace(int64_t total_pixels, size_t* bytes) {
    if (!bytes || total_pixels < 1) return GS_EINVAL;
    *bytes = expand_workspace_bytes(total_pixels);
    return GS_OK;
}

int gs_expand(const uint8_t* masks, const float* rgb_target, const float* depth_target, const float* feat_init,
              int32_t n_feat, const gs_view* views, const gs_view* views_dev, int32_t n_views,
              const gs_gaussian_planes* dst, int64_t capacity, int64_t* n_dev, int64_t* candidates_dev, void* ws,
              size_t ws_bytes, gs_stream stream) {
    if (!feat_supported(n_feat)) return GS_EUNSUPPORTED;
    int64_t P = 0;
    int st = check_views(views, views_dev, n_views, 0, &P, nullptr);
    if (st) return st;
    if (!masks || !rgb_target || !depth_target || !dst || !n_dev || !ws || capacity < 1) return GS_EINVAL;
    if (!dst->mu || !dst->log_scale || !dst->quat || !dst->opacity_logit || !dst->color) return GS_EINVAL;
    if (n_feat > 0 && (!dst->feat || !feat_init)) return GS_EINVAL;
    if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return GS_EINVAL;
    if (ws_bytes < expand_workspace_bytes(P)) return GS_ECAPACITY;
    return hip_status(launch_expand(masks, rgb_target, depth_target, feat_init, n_feat, P, views_dev, n_views, n_dev,
                                    capacity, candidates_dev, *dst, ws, reinterpret_cast<hipStream_t>(stream)));
}

int gs_dsr_workspace(int64_t n, size_t* bytes) {
    if (!bytes || n < 1) return GS_EINVAL;
    *bytes = dsr_workspace_bytes(n);
    return GS_OK;
}

int gs_dsr(const float* log_scale, int64_t n, float w_big, float w_small, float* grad_log_scale, double* out,
           void* ws, size_t ws_bytes, gs_stream stream) {
    if (!log_scale || !out || !ws || n < 1 || n > (1ll << 40)) return GS_EINVAL;
    if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return GS_EINVAL;
    if (ws_bytes < dsr_workspace_bytes(n)) return GS_ECAPACITY;
    return hip_status(launch_dsr(log_scale, n, w_big, w_small, grad_log_scale, out, ws,
                                 reinterpret_cast<hipStream_t>(stream)));
}

int gs_adam_step(const gs_adam_group* groups, int32_t n_groups, float beta1, float beta2, float eps, int32_t step,
                 gs_stream stream) {
    if (!groups || n_groups < 1 || n_groups > kAdamGroups || step < 1) return GS_EINVAL;
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps >= 0.0f)) return GS_EINVAL;
    for (int k = 0; k < n_groups; ++k)
        if (!groups[k].param || !groups[k].grad || !groups[k].m || !groups[k].v || groups[k].n < 0) return GS_EINVAL;
    return hip_status(launch_adam(groups, n_groups, beta1, beta2, eps, step, reinterpret_cast<hipStream_t>(stream)));
}

int gs_pose_step(gs_view* views_dev, int32_t n_views, const float* twist_grad, float* m, float* v, float lr_rho,
                 float lr_phi, float beta1, float beta2, float eps, int32_t step, gs_stream stream) {
    if (!views_dev || !twist_grad || !m || !v || n_views < 1 || n_views > GS_MAX_VIEWS || step < 1) return GS_EINVAL;
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps >= 0.0f)) return GS_EINVAL;
    return hip_status(launch_pose_step(views_dev, n_views, twist_grad, m, v, lr_rho, lr_phi, beta1, beta2, eps, step,
                                       nullptr, reinterpret_cast<hipStream_t>(stream)));
}

int gs_pose_step_dev(gs_view* views_dev, int32_t n_views, const float* twist_grad, float* m, float* v, float lr_rho,
                     float lr_phi, float beta1, float beta2, float eps, int32_t* step_dev, gs_stream stream) {
    if (!views_dev || !twist_grad || !m || !v || !step_dev || n_views < 1 || n_views > GS_MAX_VIEWS) return GS_EINVAL;
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps >= 0.0f)) return GS_EINVAL;
    return hip_status(launch_pose_step(views_dev, n_views, twist_grad, m, v, lr_rho, lr_phi, beta1, beta2, eps, 0,
                                       step_dev, reinterpret_cast<hipStream_t>(stream)));
}

int gs_render_bwd_workspace(int32_t n, int32_t n_feat, int32_t n_views, int64_t capacity, uint32_t flags,
                            size_t* grad2d_bytes_out, size_t* ws_bytes) {
    if (!grad2d_bytes_out || !ws_bytes || n < 1 || n_views < 1 || n_views > GS_MAX_VIEWS || capacity < 0)
        return GS_EINVAL;
    if (!feat_supported(n_feat)) return GS_EUNSUPPORTED;
    *grad2d_bytes_out = grad2d_bytes(n, n_feat, n_views);
    *ws_bytes = (size_t)(capacity > 0 ? capacity : 1) * bwd_record_floats(n_feat, (flags & GS_GRAD_PARAMS) != 0) *
                sizeof(float);
    return GS_OK;
}

int gs_render_bwd_records(const gs_gaussians* g, const float* rec, const float* app, const int32_t* inst,
                          const int32_t* inst_gid, int64_t capacity, const int32_t* tile_ranges, const gs_view* views,
                          const gs_view* views_dev, int32_t n_views, const gs_config* cfg, const float* T_final,
                          const int32_t* last, const float* grad_out, uint32_t flags, void* ws, size_t ws_bytes,
                          int32_t* queue, gs_stream stream) {
    const bool params = (flags & GS_GRAD_PARAMS) != 0;
    if (!g) return GS_EINVAL;
    if (g->n < 1) return GS_EINVAL;
    if (!feat_supported(g->n_feat)) return GS_EUNSUPPORTED;
    int st = check_config(cfg);
    if (st) return st;
    int64_t P = 0;
    int total_tiles = 0;
    if ((st = check_views(views, views_dev, n_views, cfg->tile, &P, &total_tiles))) return st;
    if ((flags & ~(uint32_t)(GS_GRAD_PARAMS | GS_GRAD_POSE)) != 0 || flags == 0) return GS_EINVAL;
    if (!rec || !app || !inst || !inst_gid || !tile_ranges || !T_final || !last || !grad_out || !ws) return GS_EINVAL;
    if (capacity < 0 || capacity >= (1ll << 31)) return GS_EINVAL;
    if (cfg->persistent && !queue) return GS_EINVAL;
    const size_t rec_bytes = (size_t)(capacity > 0 ? capacity : 1) * bwd_record_floats(g->n_feat, params) * sizeof(float);
    if (ws_bytes < rec_bytes) return GS_ECAPACITY;
    if (!aligned16(rec) || !aligned16(app) || !aligned16(ws)) return GS_EINVAL;
    const int batch = cfg->lds_batch_bwd ? cfg->lds_batch_bwd : cfg->lds_batch;
    return hip_status(launch_render_bwd(rec, app, g->n, g->n_feat, inst, inst_gid, tile_ranges, views_dev, n_views,
                                        total_tiles, P, make_const(cfg), batch, cfg->persistent, T_final, last,
                                        grad_out, params, static_cast<float*>(ws), queue,
                                        reinterpret_cast<hipStream_t>(stream)));
}

int gs_reduce_records(const void* ws, size_t ws_bytes, const int32_t* pair_first, const int32_t* tiles_touched,
                      int32_t n, int32_t n_feat, int32_t n_views, int64_t capacity, uint32_t flags, float* grad2d,
                      size_t grad2d_bytes_, gs_stream stream) {
    const bool params = (flags & GS_GRAD_PARAMS) != 0;
    if (n < 1 || n_views < 1 || n_views > GS_MAX_VIEWS) return GS_EINVAL;
    if (!feat_supported(n_feat)) return GS_EUNSUPPORTED;
    if ((flags & ~(uint32_t)(GS_GRAD_PARAMS | GS_GRAD_POSE)) != 0 || flags == 0) return GS_EINVAL;
    if (!ws || !pair_first || !tiles_touched || !grad2d) return GS_EINVAL;
    if (capacity < 0 || capacity >= (1ll << 31)) return GS_EINVAL;
    if (grad2d_bytes_ < grad2d_bytes(n, n_feat, n_views)) return GS_ECAPACITY;
    const size_t rec_bytes = (size_t)(capacity > 0 ? capacity : 1) * bwd_record_floats(n_feat, params) * sizeof(float);
    if (ws_bytes < rec_bytes) return GS_ECAPACITY;
    if (!aligned16(grad2d) || !aligned16(ws)) return GS_EINVAL;
    float* geo = grad2d;
    float* appg = grad2d + (size_t)n_views * n * 8;
    return hip_status(launch_reduce_records(static_cast<const float*>(ws), pair_first, tiles_touched, n, n_feat,
                                            n_views, capacity, params, geo, appg,
                                            reinterpret_cast<hipStream_t>(stream)));
}

int gs_render_bwd(const gs_gaussians* g, const float* rec, const float* app, const int32_t* inst,
                  const int32_t* inst_gid, const int32_t* pair_first, const int32_t* tiles_touched, int64_t capacity,
                  const int32_t* tile_ranges, const gs_view* views, const gs_view* views_dev, int32_t n_views,
                  const gs_config* cfg, const float* T_final, const int32_t* last, const float* grad_out,
                  uint32_t flags, float* grad2d, size_t grad2d_bytes_, void* ws, size_t ws_bytes, int32_t* queue,
                  gs_stream stream) {
    if (!g) return GS_EINVAL;
    if (!pair_first || !tiles_touched || !grad2d) return GS_EINVAL;
    if (g->n >= 1 && feat_supported(g->n_feat) && grad2d_bytes_ < grad2d_bytes(g->n, g->n_feat, n_views))
        return GS_ECAPACITY;
    if (!aligned16(grad2d)) return GS_EINVAL;
    const int st = gs_render_bwd_records(g, rec, app, inst, inst_gid, capacity, tile_ranges, views, views_dev, n_views,
                                         cfg, T_final, last, grad_out, flags, ws, ws_bytes, queue, stream);
    if (st) return st;
    return gs_reduce_records(ws, ws_bytes, pair_first, tiles_touched, g->n, g->n_feat, n_views, capacity, flags,
                             grad2d, grad2d_bytes_, stream);
}

static int project_bwd(const gs_gaussians* g, const gs_view* views, const gs_view* views_dev, int32_t n_views,
                       const gs_config* cfg, const int32_t* tiles_touched, const float* grad2d, size_t grad2d_bytes_,
                       gs_gaussian_grads* grads, bool accumulate, gs_stream stream) {
    int st = check_gauss(g, false);
    if (st) return st;
    if ((st = check_config(cfg))) return st;
    if ((st = check_views(views, views_dev, n_views, cfg->tile, nullptr, nullptr))) return st;
    if (!tiles_touched || !grad2d || !grads || !grads->mu || !grads->log_scale || !grads->quat || !grads->opacity_logit ||
        !grads->color || (g->n_feat > 0 && !grads->feat))
        return GS_EINVAL;
    if (grad2d_bytes_ < grad2d_bytes(g->n, g->n_feat, n_views)) return GS_ECAPACITY;
    if (!aligned16(grad2d)) return GS_EINVAL;
    GradPtrs o;
    o.mu = grads->mu;
    o.log_scale = grads->log_scale;
    o.quat = grads->quat;
    o.logit = grads->opacity_logit;
    o.color = grads->color;
    o.feat = grads->feat;
    const float* geo = grad2d;
    const float* appg = grad2d + (size_t)n_views * g->n * 8;
    return hip_status(launch_project_bwd(gauss_ptrs(g), views_dev, n_views, make_const(cfg), tiles_touched, geo, appg,
                                         o, accumulate, reinterpret_cast<hipStream_t>(stream)));
}

int gs_project_bwd(const gs_gaussians* g, const gs_view* views, const gs_view* views_dev, int32_t n_views,
                   const gs_config* cfg, const int32_t* tiles_touched, const float* grad2d, size_t grad2d_bytes_,
                   gs_gaussian_grads* grads, gs_stream stream) {
    return project_bwd(g, views, views_dev, n_views, cfg, tiles_touched, grad2d, grad2d_bytes_, grads, true, stream);
}

int gs_project_bwd_write(const gs_gaussians* g, const gs_view* views, const gs_view* views_dev, int32_t n_views,
                         const gs_config* cfg, const int32_t* tiles_touched, const float* grad2d,
                         size_t grad2d_bytes_, gs_gaussian_grads* grads, gs_stream stream) {
    return project_bwd(g, views, views_dev, n_views, cfg, tiles_touched, grad2d, grad2d_bytes_, grads, false, stream);
}

int gs_pose_grad_workspace(int32_t n, int32_t n_views, size_t* bytes) {
    if (!bytes || n < 1 || n_views < 1 || n_views > GS_MAX_VIEWS) return GS_EINVAL;
    *bytes = pose_workspace_bytes(n, n_views);
    return GS_OK;
}

int gs_pose_grad(const gs_gaussians* g, const gs_view* views, const gs_view* views_dev, int32_t n_views,
                 const gs_config* cfg, const int32_t* tiles_touched, const float* grad2d, void* ws, size_t ws_bytes,
                 float* twist, gs_stream stream) {
    int st = check_gauss(g, false);
    if (st) return st;
    if ((st = check_config(cfg))) return st;
    if ((st = check_views(views, views_dev, n_views, cfg->tile, nullptr, nullptr))) return st;
    if (!tiles_touched || !grad2d || !ws || !twist) return GS_EINVAL;
    if (ws_bytes < pose_workspace_bytes(g->n, n_views)) return GS_ECAPACITY;
    if (!aligned16(grad2d) || (reinterpret_cast<uintptr_t>(ws) & 15u) != 0) return GS_EINVAL;
    return hip_status(launch_pose_grad(gauss_ptrs(g), views_dev, n_views, make_const(cfg), tiles_touched, grad2d, ws,
                                       twist, reinterpret_cast<hipStream_t>(stream)));
}

int gs_pose_grad_noalloc(const gs_gaussians* g, const gs_view* views, const gs_view* views_dev, int32_t n_views,
                         const gs_config* cfg, const int32_t* tiles_touched, const float* grad2d, float* twist,
                         gs_stream stream) {
    int st = check_gauss(g, false);
    if (st) return st;
    if ((st = check_config(cfg))) return st;
    if ((st = check_views(views, views_dev, n_views, cfg->tile, nullptr, nullptr))) return st;
    if (!tiles_touched || !grad2d || !twist) return GS_EINVAL;
    if (!aligned16(grad2d)) return GS_EINVAL;
    if (pose_workspace_bytes(g->n, n_views) > kScratchBytes) return GS_ECAPACITY;
    void* ws = nullptr;
    if ((st = scratch_ptr(&ws))) return st;
    // k_pose_partial writes every partial k_pose_final reads, so the scratch
    // needs no clearing between calls.
    return hip_status(launch_pose_grad(gauss_ptrs(g), views_dev, n_views, make_const(cfg), tiles_touched, grad2d, ws,
                                       twist, reinterpret_cast<hipStream_t>(stream)));
}

const char* gs_error_string(int status) {
    switch (status) {
        case GS_OK: return "ok";
        case GS_EINVAL: return "invalid argument";
        case GS_ECAPACITY: return "buffer too small";
        case GS_EHIP: return "HIP error";
        case GS_EUNSUPPORTED: return "unsupported configuration";
        default: return "unknown status";
    }
}

const char* gs_last_hip_error(void) { return g_hip_err; }

int32_t gs_version(void) { return 100; }

}  // extern "C"
