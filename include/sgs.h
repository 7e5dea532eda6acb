/*
 * sgs.h -- C ABI of the MI355X (gfx950) semantic Gaussian-splatting
 * rasterizer: forward rendering of colour, depth, cumulative opacity and an
 * F-channel semantic feature from 3D Gaussians under a camera pose, the
 * image-space loss gradient, and the backward pass to every Gaussian
 * parameter and to a 6-DoF pose twist.
 *
 * Paper: GS^3LAM, "Gaussian Semantic Splatting SLAM" (ACM MM 2024).
 *   Sec. 3.2, Eq. (1)-(2)   SG-Field and Sigma = R S S^T R^T
 *   Sec. 3.2.1, Eq. (3)-(6) EWA projection, alpha, colour and depth blending
 *   Sec. 3.2.2, Eq. (7)-(8) semantic feature blending and decoding
 *   Sec. 3.3.1, Eq. (10)    cumulative opacity
 *   Sec. 3.3.4, Eq. (15)-(18); Sec. 3.4, Eq. (21)  losses
 *   Supp. B.1               Jacobian of the loss with respect to the pose
 *
 * Conventions shared by every entry point:
 *   - Every array argument is a DEVICE pointer owned by the caller unless
 *     its comment says "host".  The library allocates no device memory; the
 *     caller sizes workspaces with the *_workspace queries.
 *   - Gaussians are float32 structure-of-arrays planes (index i in [0, n)).
 *   - Images are planar float32 [channel][P_total] where P_total is the sum of
 *     width*height over the views and view v occupies
 *     [pixel_offset, pixel_offset + width*height), row-major.  Channel order:
 *     0,1,2 = R,G,B; 3 = depth; 4 = cumulative opacity; 5.. = features.
 *   - Pixel (u, v) has centre (u + 1/2, v + 1/2); (cx, cy) is in the same
 *     continuous image coordinates.
 *   - All calls are asynchronous on `stream`, never synchronise, never read
 *     device memory on the host and never allocate, so every call can be
 *     captured in a HIP graph.  Arguments are validated on the host before
 *     anything is launched; on an error nothing is launched.
 *   - Return value: GS_OK, or a negative gs_status.  HIP launch errors are
 *     reported as GS_EHIP (the HIP error string via gs_last_hip_error()).
 */
#ifndef SGS_H
#define SGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* gs_stream; /* a hipStream_t; NULL = default stream */

enum gs_status {
    GS_OK = 0,
    GS_EINVAL = -1,        /* bad argument (null pointer, size, layout)          */
    GS_ECAPACITY = -2,     /* a caller-sized buffer is too small                  */
    GS_EHIP = -3,          /* a HIP call failed                                   */
    GS_EUNSUPPORTED = -4   /* valid but not compiled (feature count, tile size)   */
};

enum gs_flags {
    GS_GRAD_PARAMS = 1,    /* gradients to the Gaussian parameters (mapping)      */
    GS_GRAD_POSE = 2       /* per-view 2D gradients kept for the pose twist       */
};

enum {
    GS_MAX_VIEWS = 64,
    GS_MAX_CLASSES = 256
};

/* The SG-Field of Eq. (1): mean mu, covariance through rotation quat and
 * log-scales (Eq. 2), opacity o = sigmoid(opacity_logit), colour c and an
 * n_feat-dimensional semantic feature f.  n_feat must be one of the compiled
 * values 0, 8, 16, 32 (GS_EUNSUPPORTED otherwise). */
typedef struct {
    const float* mu;            /* [3][n]                                   */
    const float* log_scale;     /* [3][n]                                   */
    const float* quat;          /* [4][n] (w, x, y, z), normalised inside   */
    const float* opacity_logit; /* [n]                                      */
    const float* color;         /* [3][n]                                   */
    const float* feat;          /* [n_feat][n] (may be NULL if n_feat == 0) */
    int32_t n;
    int32_t n_feat;
} gs_gaussians;

/* Gradients, same planes as gs_gaussians; ACCUMULATED (+=), so per-view calls
 * and one batched call give the same totals. */
typedef struct {
    float* mu;
    float* log_scale;
    float* quat;
    float* opacity_logit;
    float* color;
    float* feat;
} gs_gaussian_grads;

/* A pinhole camera with world->camera transform T_CW = [R|t] (Sec. 3.2.1).
 * pixel_offset and tile_offset are filled by gs_views_layout. 88 bytes. */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float Rt[12];               /* row-major 3x4 [R|t], world -> camera      */
    int64_t pixel_offset;       /* first pixel of the view in [C][P_total]    */
    int32_t tile_offset;        /* first global tile id of the view           */
    int32_t reserved;
} gs_view;

/* Rasterizer constants.  The paper states none of them; the defaults from
 * gs_default_config are the readings used throughout:
 *   z_near 0.2       cull if camera depth <= z_near
 *   blur 0.3         px^2 added to both diagonal entries of Sigma2D
 *   guard 1.3        cull if |x/z| > guard * (W/2) / fx (or the same in y)
 *   alpha_min 1/255  a pair with alpha < alpha_min is skipped
 *   alpha_max 0.99   alpha is clamped to alpha_max
 *   T_min 1e-4       stop before a Gaussian that would take T below T_min
 *   tile             tile side in pixels: 8, 16 or 32
 *   lds_batch        Gaussians staged in LDS per batch (64, 128 or 256)
 *   persistent       0: one workgroup per tile; 1: persistent workgroups
 *                    that pull (view, tile) items from a queue
 *   lds_batch_bwd    Gaussians staged per batch by the render backward
 *                    (64, 128 or 256; 0 = the same as lds_batch)
 */
typedef struct {
    float z_near, blur, guard, alpha_min, alpha_max, T_min;
    int32_t tile;
    int32_t lds_batch;
    int32_t persistent;
    int32_t lds_batch_bwd;
} gs_config;

/* Fills *cfg with the defaults listed above (tile 16, lds_batch 256,
 * persistent 0, lds_batch_bwd 0). */
int gs_default_config(gs_config* cfg);

/* Host helper: fills pixel_offset / tile_offset of a HOST array of views for
 * the given tile size and returns the totals.  Every entry point takes the
 * views twice: `views` (host, for sizes and offsets) and `views_dev`
 * (device copy of the same array, read by the kernels), which must agree in
 * everything but the poses (gs_views_check compares them on the device). */
int gs_views_layout(gs_view* views, int32_t n_views, int32_t tile, int64_t* total_pixels,
                    int32_t* total_tiles);

/* gs_views_check -- for callers that keep the two copies of their views
 * themselves (the pinhole cameras of Sec. 3.2.1): counts, on the device,
 * the views whose device copy differs, bit for bit, from the host array in
 * a field the entry points take from the host array -- width, height,
 * pixel_offset and, when tile > 0, tile_offset, which size their grids and
 * buffer extents -- or in the intrinsics fx, fy, cx, cy, and writes the
 * count to *mismatch_dev (one device int32, written whatever the count, so
 * nothing needs clearing; graph-capturable).  The poses Rt are not
 * compared: the kernels read them from the device copy only, and a caller
 * may update them there between graph replays.  Asynchronous; read
 * *mismatch_dev after the stream completes.  GS_EINVAL for a null pointer,
 * n_views outside [1, GS_MAX_VIEWS], a tile other than 0, 8, 16 or 32, or a
 * host array not laid out by gs_views_layout (for this tile; tile 0 checks
 * the pixel offsets only); nothing is launched then. */
int gs_views_check(const gs_view* views, const gs_view* views_dev, int32_t n_views, int32_t tile,
                   int32_t* mismatch_dev, gs_stream stream);

/* Floats per Gaussian of the appearance record written by gs_project:
 * (c0, c1, c2, f0 .. f_{F-1}) padded to a multiple of 4. */
int32_t gs_app_stride(int32_t n_feat);

/* ---------------------------------------------------------------------------
 * gs_project -- Eq. (2)-(3) for every (view, Gaussian) pair, one thread each.
 *   rec[V][n][8]  = (mx, my, A, B, C, o, d, r) : projected mean, conic
 *                   (Sigma2D^-1, quadratic form A dx^2 + 2B dx dy + C dy^2),
 *                   opacity, camera depth, and r = the pixel box half-sizes
 *                   (rx, ry) as two binary16 rounded up.
 *   rect[V][n][4] = tile rectangle, (tx0 | ty0 << 16, tx1 | ty1 << 16), inclusive,
 *                   then the bits of the camera depth d (as in rec) and 0
 *                   (16-byte aligned; gs_bin_sort reads the depth here)
 *   tiles_touched[V][n] = number of tiles in rect, 0 if culled
 *                   (rec and rect are written only for pairs with
 *                   tiles_touched > 0; other entries are left as they were)
 *   app[n][gs_app_stride(F)] = colour and feature, gathered per Gaussian by
 *                   the render kernels (may be NULL to skip).
 * Culling, the mean, the conic, the depth and the rectangle are computed in
 * binary32 with one rounding per operation in a fixed order (no contraction),
 * so that the tile binning and the depth order are reproducible bit for bit.
 * --------------------------------------------------------------------------- */
int gs_project(const gs_gaussians* g, const gs_view* views, const gs_view* views_dev, int32_t n_views,
               const gs_config* cfg, float* rec, uint32_t* rect, int32_t* tiles_touched, float* app,
               gs_stream stream);

/* ---------------------------------------------------------------------------
 * gs_bin_sort -- tile binning and depth sort (Sec. 3.2.1: tile-based
 * rasterization of Gaussians sorted in depth order).  Every visible
 * (view, Gaussian) pair emits one instance per tile of its rectangle; the
 * instances are sorted by (global tile id, binary32 depth, Gaussian index):
 * a stable device radix sort of the instances by tile, then each tile's
 * list by depth (its Gaussian-index order kept among equal depths).
 * An instance is identified by its emission index e (pairs in (view, index)
 * order, each pair's tiles row by row), so the instances of one pair occupy the
 * contiguous range [pair_first[pair], pair_first[pair] + tiles_touched[pair]).
 *   rect, tiles_touched     from gs_project (the depth key is read from rect)
 *   tile_keys[capacity]     global tile id of each sorted instance
 *   inst[capacity]          emission index of each sorted instance
 *   inst_gid[capacity]      Gaussian index of each emission index
 *                           (so inst_gid[inst[k]] is the k-th sorted Gaussian)
 *   pair_first[V][n]        first emission index of each visible pair
 *   tile_ranges[T_total][2] [start, end) of every global tile in the sorted list
 *   counts[5] (int64)       [0] instances, [1] visible pairs,
 *                           [2] 1 if the instance count exceeded capacity
 *                           (the lists are then truncated: read counts after
 *                           the stream completes and call again with
 *                           capacity >= counts[0]),
 *                           [3] 1 if a wait of the device sort's single-pass
 *                           scan gave up (a block's predecessor never
 *                           published within the spin limit): the later
 *                           binning kernels then stand down, every tile list
 *                           is left empty and the call's results must be
 *                           discarded (call again),
 *                           [4] sticky: set whenever [2] or [3] is set, by
 *                           every call, and cleared only by the caller (write
 *                           0 to it), so that one check after many calls (a
 *                           tracking run, a batch of mapping iterations)
 *                           shows whether any of them was truncated.
 * ws / ws_bytes: workspace of at least gs_bin_sort_workspace(...) bytes,
 * 256-byte aligned.  Instance counts must stay below 2^31.
 * --------------------------------------------------------------------------- */
int gs_bin_sort_workspace(int32_t n, int32_t n_views, int64_t capacity, size_t* bytes);
int gs_bin_sort(const uint32_t* rect, const int32_t* tiles_touched, int32_t n,
                const gs_view* views, const gs_view* views_dev, int32_t n_views, const gs_config* cfg,
                void* ws, size_t ws_bytes, int64_t capacity, uint32_t* tile_keys, int32_t* inst,
                int32_t* inst_gid, int32_t* pair_first, int32_t* tile_ranges, int64_t* counts, gs_stream stream);

/* ---------------------------------------------------------------------------
 * gs_render_fwd -- front-to-back compositing, Eq. (4), (6), (7), (10):
 *   alpha_i = min(alpha_max, o_i exp(-q_i / 2)),  q_i = sigma^T conic sigma >= 0
 *   out_ch  = sum_i x_i,ch alpha_i T_i,  T_i = prod_{j<i} (1 - alpha_j)
 * over each pixel's tile list in (depth, index) order, skipping alpha <
 * alpha_min and stopping before T would drop below T_min.  Background 0.
 *   inst, inst_gid, tile_ranges from gs_bin_sort; rec, app from gs_project.
 *   out[5+F][P_total], T_final[P_total], last[P_total] (number of list
 *   entries of the pixel's tile up to and including its last contributor).
 *   queue: >= 4 int32 of device memory, used when cfg->persistent (may be
 *   NULL otherwise); it is reset inside the call.
 * --------------------------------------------------------------------------- */
int gs_render_fwd(const float* rec, const float* app, int32_t n, int32_t n_feat, const int32_t* inst,
                  const int32_t* inst_gid, const int32_t* tile_ranges, const gs_view* views,
                  const gs_view* views_dev, int32_t n_views, const gs_config* cfg, float* out, float* T_final,
                  int32_t* last, int32_t* queue, gs_stream stream);

/* ---------------------------------------------------------------------------
 * gs_loss_grad -- image-space losses of Sec. 3.3.4 / 3.4 and their gradient:
 *   per view v (P_v pixels), each term a mean over its pixels,
 *   L_v = w0 * mean|C - C*| (over 3 P_v) + w1 * mean|D - D*|
 *       + w2 * mean CE(softmax(W^T F), label)
 * W is a fixed decoder [n_feat][n_classes] (row-major; the configured linear
 * stand-in for the paper's F_cnn, Eq. 8); n_classes == 0 drops the CE term.
 * Writes grad_out[5+F][P_total] = dL/d out (opacity channel 0) and WRITES
 * loss[4] (double, device) = (colour term, depth term, semantic term,
 * total), each summed over the views; the per-block partial sums go to ws
 * (gs_loss_grad_workspace bytes) and are added in a fixed order, so the
 * value is deterministic.  labels in [0, n_classes) (int32).
 * rgb_target [3][P_total], depth_target [P_total]; weights is a HOST array
 * of 3 floats (w0, w1, w2).  Views as for the other entry points.
 * --------------------------------------------------------------------------- */
int gs_loss_grad_workspace(int64_t total_pixels, size_t* bytes);
int gs_loss_grad(const float* out, int32_t n_feat, const float* rgb_target, const float* depth_target,
                 const int32_t* labels, const float* decoder, int32_t n_classes, const float* weights,
                 const gs_view* views, const gs_view* views_dev, int32_t n_views, float* grad_out, double* loss,
                 void* ws, size_t ws_bytes, gs_stream stream);

/* ---------------------------------------------------------------------------
 * gs_render_fwd_loss -- gs_render_fwd and gs_loss_grad in one pass: the
 * forward compositing of Eq. (4), (6), (7), (10) with the image-space loss
 * of Sec. 3.3.4 / 3.4 evaluated in the same kernel while each pixel's
 * rendered channels are still in registers, so the image is not read back.
 * Arguments as for the two calls (out, T_final, last and grad_out are all
 * written; loss[4] as for gs_loss_grad); grad_out holds the same values
 * gs_loss_grad would write from this out, and loss the same terms up to
 * the order of their FP64 sums (per tile here, per block of pixels there).
 * ws: gs_render_fwd_loss_workspace bytes, 16-byte aligned (per-tile
 * partial sums and the transposed decoder).  Supports n_feat <= 16 and
 * n_classes <= 20 (the logits stay in registers); beyond that it returns
 * GS_EUNSUPPORTED and the caller makes the two separate calls.
 * --------------------------------------------------------------------------- */
int gs_render_fwd_loss_workspace(const gs_view* views, int32_t n_views, int32_t tile, size_t* bytes);
int gs_render_fwd_loss(const float* rec, const float* app, int32_t n, int32_t n_feat, const int32_t* inst,
                       const int32_t* inst_gid, const int32_t* tile_ranges, const gs_view* views,
                       const gs_view* views_dev, int32_t n_views, const gs_config* cfg, float* out, float* T_final,
                       int32_t* last, int32_t* queue, const float* rgb_target, const float* depth_target,
                       const int32_t* labels, const float* decoder, int32_t n_classes, const float* weights,
                       float* grad_out, double* loss, void* ws, size_t ws_bytes, gs_stream stream);

/* ---------------------------------------------------------------------------
 * gs_slam_loss -- the SLAM losses with their masks: the mapping colour term
 * of Sec. 3.3.4, Eq. (15) (L1 plus an SSIM term), the observed-region mask
 * of the tracking loss, Sec. 3.4, Eq. (21), and the unobserved-region mask
 * of Sec. 3.3.1, Eq. (11), with the median depth error both masks refer to;
 * the semantic term through a learnable decoder (Sec. 3.2.2, Eq. 8), as a
 * cross-entropy or as the binary cross-entropy of Eq. (16), with the
 * decoder's own gradients.
 *   median (per view): the lower median (rank floor((m-1)/2), from 0, of m)
 *     of the binary32 residuals r = |D - D*| over the view's pixels with
 *     D* > 0, ranked by bit pattern (the float order; a NaN ranks above
 *     +inf); 0 when no pixel has D* > 0.  Exact (a radix select).
 *   masks[p], binary32 tests:
 *     bit 0  M_obs   = (O > tau_obs) and (r < obs_factor * median)
 *     bit 1  M_unobs = (O < tau_unobs) or (D > D* and r > unobs_factor * median)
 *   loss, per view v (P_v pixels), with M(p) = M_obs(p) if flags has
 *   GS_LOSS_OBS_MASK, else 1:
 *     colour L1  (1 - lambda) w_color / (3 P_v) sum_p M(p) |C(p) - C*(p)|_1
 *     SSIM       lambda w_color / (3 P_v) sum_c sum_p M(p) (1 - SSIM_c(p))
 *     depth      w_depth / P_v sum_p M(p) |D(p) - D*(p)|
 *     semantic   w_sem / P_v sum_p M(p) S(p)
 *   SSIM_c(p) (Wang et al. 2004) of colour channel c: local means,
 *   variances and covariance of the rendered and the target image under an
 *   11x11 Gaussian window of standard deviation 1.5 px (weights summing to
 *   1), pixels outside the view taken as 0, C1 = 0.01^2, C2 = 0.03^2.
 *   S(p): the decoder is a 1x1 convolution, z = W^T F(p) + b, p = softmax(z),
 *   y = one-hot(label(p)); CE: S = -log p_label; BCE (GS_LOSS_BCE, Eq. 16):
 *   S = -sum_k [y_k log p_k + (1 - y_k) log(1 - p_k)], every log clamped at
 *   -100 (a clamped log contributes no gradient).
 *   The masks are constants of the loss (no gradient flows through them).
 * Arguments: out [5+F][P_total] (the render), rgb_target [3][P_total],
 * depth_target [P_total], labels [P_total] int32 in [0, n_classes); dec
 * (HOST struct, may be NULL: no semantic term); opts is a HOST struct.
 * WRITES grad_out [5+F][P_total] = dL/d out (opacity channel 0); loss[5]
 * (double) = (colour L1, SSIM, depth, semantic, total), each summed over
 * the views in a fixed order (deterministic); median[V] (float, may be
 * NULL); masks [P_total] (uint8, may be NULL); dec->grad_weight [F][K] and
 * dec->grad_bias [K] when not NULL (written, not accumulated; summed in a
 * fixed order).  ws: at least gs_slam_loss_workspace bytes for the same
 * views, n_feat, dec and opts, 256-byte aligned, contents need not be
 * initialised.  Views as for the other entry points.  Errors: GS_EINVAL
 * (null or misaligned pointer, bad view list, flags), GS_ECAPACITY (ws too
 * small), GS_EUNSUPPORTED (n_feat not compiled, or more than
 * GS_SLAM_MAX_CLASSES classes).
 * --------------------------------------------------------------------------- */
typedef struct {
    float w_color, w_depth, w_sem; /* lambda_c, lambda_d, lambda_s (Eq. 18, 21)        */
    float ssim_lambda;             /* lambda of Eq. (15); 0 = L1 colour only (Eq. 21)  */
    float tau_obs, tau_unobs;      /* opacity thresholds of Eq. (21) and Eq. (11)      */
    float obs_factor;              /* 10: M_obs residual bound, in medians (Eq. 21)    */
    float unobs_factor;            /* 50: M_unobs residual bound, in medians (Eq. 11)  */
    uint32_t flags;                /* GS_LOSS_OBS_MASK | GS_LOSS_BCE                   */
} gs_slam_loss_opts;

enum {
    GS_LOSS_OBS_MASK = 1,          /* weight every term by M_obs (tracking, Eq. 21)    */
    GS_LOSS_BCE = 2,               /* semantic term: BCE of Eq. (16), not CE            */
    GS_SLAM_MAX_CLASSES = 64
};

/* The semantic decoder (a 1x1 convolution F -> K) and its gradients. */
typedef struct {
    const float* weight;           /* W [n_feat][n_classes], row-major (device)        */
    const float* bias;             /* b [n_classes] (device), or NULL for none          */
    float* grad_weight;            /* WRITTEN dL/dW [n_feat][n_classes], or NULL        */
    float* grad_bias;              /* WRITTEN dL/db [n_classes], or NULL                */
    int32_t n_classes;             /* K in [0, GS_SLAM_MAX_CLASSES]; 0 = no term        */
    int32_t reserved;
} gs_decoder;

/* Fills *opts with w = (0.5, 1.0, 0.01), lambda 0.2, tau_obs 0.99,
 * tau_unobs 0.5, factors 10 and 50, CE, no mask (the mapping loss). */
int gs_default_slam_loss_opts(gs_slam_loss_opts* opts);
int gs_slam_loss_workspace(const gs_view* views, int32_t n_views, int32_t n_feat, const gs_decoder* dec,
                           const gs_slam_loss_opts* opts, size_t* bytes);
int gs_slam_loss(const float* out, int32_t n_feat, const float* rgb_target, const float* depth_target,
                 const int32_t* labels, const gs_decoder* dec, const gs_slam_loss_opts* opts, const gs_view* views,
                 const gs_view* views_dev, int32_t n_views, float* grad_out, double* loss, float* median,
                 uint8_t* masks, void* ws, size_t ws_bytes, gs_stream stream);

/* ---------------------------------------------------------------------------
 * gs_expand -- adaptive Gaussian expansion, Sec. 3.3.1 (which pixels: the
 * unobserved-region mask, Eq. 11) with the initialisation of Sec. 3.3.2.
 * Every pixel p with M_unobs (bit 1 of masks, as gs_slam_loss writes it)
 * and an observed depth D*(p) > 0 adds one Gaussian, appended in pixel order
 * (views back to back, rows, columns) at index n, n + 1, ... while below
 * `capacity`:
 *   mean     the pixel centre (u + 1/2, v + 1/2) unprojected at D*:
 *            x_c = ((u + 1/2 - cx)/fx D*, (v + 1/2 - cy)/fy D*, D*),
 *            mu = R^T (x_c - t) for the view's world-to-camera [R|t];
 *   colour   the observed colour rgb_target[.][p];
 *   feature  feat_init[.][p] (random values drawn by the caller, the paper's
 *            random semantic coefficients), n_feat rows;
 *   opacity  0.5 (logit 0); log-scale log(D* / fx) on all three axes;
 *   rotation the identity quaternion (1, 0, 0, 0).
 * dst: the parameter planes (device), each with `capacity` columns.
 * n_dev (device int64, in/out): the current Gaussian count on entry,
 * min(count + candidates, capacity) on exit.  candidates_dev (device int64,
 * may be NULL): the number of candidate pixels.  Nothing is read back on the
 * host, so the call can be captured in a graph.  ws: gs_expand_workspace
 * bytes, 256-byte aligned.  Errors: GS_EINVAL (null pointer, bad views),
 * GS_ECAPACITY (ws too small), GS_EUNSUPPORTED (n_feat).
 * --------------------------------------------------------------------------- */
typedef gs_gaussian_grads gs_gaussian_planes; /* writable parameter planes */

int gs_expand_workspace(int64_t total_pixels, size_t* bytes);
int gs_expand(const uint8_t* masks, const float* rgb_target, const float* depth_target, const float* feat_init,
              int32_t n_feat, const gs_view* views, const gs_view* views_dev, int32_t n_views,
              const gs_gaussian_planes* dst, int64_t capacity, int64_t* n_dev, int64_t* candidates_dev, void* ws,
              size_t ws_bytes, gs_stream stream);

/* ---------------------------------------------------------------------------
 * gs_dsr -- depth-adaptive scale regularisation, Sec. 3.3.2, Eq. (12), over
 * the 3n per-axis scales s = exp(log s) of log_scale [3][n] (device; the
 * exponential is the projection's decision-path one, so the samples are the
 * same bits as any implementation of that sequence):
 *   mu_s, sigma_s: their mean and population standard deviation;
 *   L_big   = mean of s over {s > mu_s + 2 sigma_s},
 *   L_small = mean of -log s over {s < mu_s - 2 sigma_s} (0 for empty sets);
 *   loss    = w_big L_big + w_small L_small (Supp. C.1: 0.01, 0.001).
 * grad_log_scale [3][n] (device, may be NULL) is ACCUMULATED (+=) with
 * d loss / d log s, the sets and their counts held: w_big s / n_big on the
 * big set, -w_small / n_small on the small set.  out[7] (device double) =
 * (L_big, L_small, loss, mu_s, sigma_s, n_big, n_small).  Every sum is in a
 * fixed order (deterministic).  ws: gs_dsr_workspace bytes, 256-byte
 * aligned.  Errors: GS_EINVAL (n < 1, null pointer), GS_ECAPACITY.
 * --------------------------------------------------------------------------- */
int gs_dsr_workspace(int64_t n, size_t* bytes);
int gs_dsr(const float* log_scale, int64_t n, float w_big, float w_small, float* grad_log_scale, double* out,
           void* ws, size_t ws_bytes, gs_stream stream);

/* ---------------------------------------------------------------------------
 * gs_adam_step -- one Adam step (Kingma and Ba 2015, bias-corrected at step
 * `step` >= 1) over up to 8 parameter groups in one launch, each with its
 * own learning rate (Supp. C.1 gives the per-attribute rates of mapping):
 *   m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2;
 *   p <- p - lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * groups is a HOST array; every pointer in it is device memory (param, m, v
 * updated in place; grad read).  Binary32 throughout.
 * gs_pose_step -- tracking's pose update (Sec. 3.4): Adam as above on each
 * view's twist gradient twist_grad [V][6] = dL/d(rho, phi) (learning rate
 * lr_rho for rho, lr_phi for phi; m, v [V][6] device state), then the left
 * update T <- Exp(dxi) T of the view's world-to-camera [R|t], written in
 * place into views_dev (the records the other kernels read), so an
 * iteration needs no host round trip.  Errors: GS_EINVAL.
 * --------------------------------------------------------------------------- */
typedef struct {
    float* param;
    const float* grad;
    float* m;
    float* v;
    int64_t n;
    float lr;
    int32_t reserved;
} gs_adam_group;

int gs_adam_step(const gs_adam_group* groups, int32_t n_groups, float beta1, float beta2, float eps, int32_t step,
                 gs_stream stream);
int gs_pose_step(gs_view* views_dev, int32_t n_views, const float* twist_grad, float* m, float* v, float lr_rho,
                 float lr_phi, float beta1, float beta2, float eps, int32_t step, gs_stream stream);
/* gs_pose_step_dev -- gs_pose_step with Adam's step count in device memory:
 * each call takes t = *step_dev + 1 (int32, device), stores t back and uses
 * it for the bias corrections, so an iteration captured in a HIP graph
 * replays with the right step.  The caller clears *step_dev at the start of a
 * tracking run (with a kernel, not a memset, if that is captured too).  The
 * same update as gs_pose_step at step t.  Errors: GS_EINVAL. */
int gs_pose_step_dev(gs_view* views_dev, int32_t n_views, const float* twist_grad, float* m, float* v, float lr_rho,
                     float lr_phi, float beta1, float beta2, float eps, int32_t* step_dev, gs_stream stream);

/* ---------------------------------------------------------------------------
 * gs_render_bwd -- backward of gs_render_fwd.  Re-traverses each pixel's list
 * from `last` down, rebuilding T_i = T_{i+1} / (1 - alpha_i), and forms
 *   dL/dalpha_i = T_i (g . x_i) - S_i / (1 - alpha_i),
 *   S_i = sum_{j>i} (g . x_j) alpha_j T_j,
 * with g the pixel's upstream gradient grad_out[5+F][P_total] and x_i the
 * Gaussian's channel values (colour, depth, 1, feature).  Per-Gaussian sums
 * are reduced across each wavefront, added across the tile's wavefronts in
 * LDS, written as one record per instance into ws (no global atomics), then
 * summed per (view, Gaussian) pair in a fixed order.  The order in which the
 * wavefronts of a tile add into LDS is not fixed, so results may differ
 * between runs in the last bits (float rounding), nothing more.  WRITES
 * grad2d:
 *   grad2d geo [V][n][8]  = dL/d(mx, my, A, B, C, d), 2 unused   (per view;
 *                           written only for visible pairs, tiles_touched > 0)
 *   grad2d app [n][4+F]   = dL/d(o, c0, c1, c2, f...)            (all views)
 * (geo first, app right after it).  flags: GS_GRAD_PARAMS fills geo and app;
 * GS_GRAD_POSE alone (tracking, Sec. 3.4: the field is frozen) fills geo
 * only and skips colour, feature and opacity (app is left untouched).
 * inst, inst_gid, pair_first, tile_ranges, capacity: as given to / written by
 * gs_bin_sort; tiles_touched from gs_project.
 * gs_render_bwd_workspace gives grad2d_bytes and ws_bytes (capacity records).
 *
 * gs_render_bwd is gs_render_bwd_records followed by gs_reduce_records on the
 * same stream; the two halves are exported so that each can be timed or
 * scheduled on its own:
 *   gs_render_bwd_records  writes the per-instance records into ws
 *                          (ws_bytes as above; grad2d is not touched);
 *   gs_reduce_records      sums them per (view, Gaussian) pair into grad2d
 *                          (the record layout depends on flags and n_feat,
 *                          which must match the records call).
 * Errors: GS_EINVAL for NULL or misaligned (16 B) buffers, bad flags or
 * sizes; GS_ECAPACITY when grad2d_bytes or ws_bytes is too small;
 * GS_EUNSUPPORTED for an unsupported n_feat or launch configuration.
 * --------------------------------------------------------------------------- */
int gs_render_bwd_workspace(int32_t n, int32_t n_feat, int32_t n_views, int64_t capacity, uint32_t flags,
                            size_t* grad2d_bytes, size_t* ws_bytes);
int gs_render_bwd(const gs_gaussians* g, const float* rec, const float* app, const int32_t* inst,
                  const int32_t* inst_gid, const int32_t* pair_first, const int32_t* tiles_touched,
                  int64_t capacity, const int32_t* tile_ranges, const gs_view* views, const gs_view* views_dev,
                  int32_t n_views, const gs_config* cfg, const float* T_final, const int32_t* last,
                  const float* grad_out, uint32_t flags, float* grad2d, size_t grad2d_bytes, void* ws,
                  size_t ws_bytes, int32_t* queue, gs_stream stream);
int gs_render_bwd_records(const gs_gaussians* g, const float* rec, const float* app, const int32_t* inst,
                          const int32_t* inst_gid, int64_t capacity, const int32_t* tile_ranges,
                          const gs_view* views, const gs_view* views_dev, int32_t n_views, const gs_config* cfg,
                          const float* T_final, const int32_t* last, const float* grad_out, uint32_t flags,
                          void* ws, size_t ws_bytes, int32_t* queue, gs_stream stream);
int gs_reduce_records(const void* ws, size_t ws_bytes, const int32_t* pair_first, const int32_t* tiles_touched,
                      int32_t n, int32_t n_feat, int32_t n_views, int64_t capacity, uint32_t flags, float* grad2d,
                      size_t grad2d_bytes, gs_stream stream);

/* ---------------------------------------------------------------------------
 * gs_project_bwd -- backward of gs_project (Eq. 2-3) for the mapping step:
 * from grad2d of gs_render_bwd (GS_GRAD_PARAMS) to every parameter plane,
 * one thread per Gaussian summing its views in registers (no atomics):
 *   conic = Sigma2D^-1, Sigma2D = (J R_CW M)(J R_CW M)^T + bI, M = R(q) diag(e^s),
 *   mean2d = pi(R_CW mu + t), depth = (R_CW mu + t)_z, o = sigmoid(logit).
 * Pairs with tiles_touched == 0 are skipped.  ADDS the gradients to *grads.
 * --------------------------------------------------------------------------- */
int gs_project_bwd(const gs_gaussians* g, const gs_view* views, const gs_view* views_dev, int32_t n_views,
                   const gs_config* cfg, const int32_t* tiles_touched, const float* grad2d, size_t grad2d_bytes,
                   gs_gaussian_grads* grads, gs_stream stream);

/* gs_project_bwd_write -- gs_project_bwd that WRITES *grads instead of adding
 * to them: every plane of every Gaussian is written, zeros where no view
 * contributes, so a caller whose step starts from cleared gradients (one
 * batched launch over all its views) need not clear them first, and the
 * planes are not read.  Same arguments, layout and errors as gs_project_bwd;
 * the values equal those of gs_project_bwd on cleared planes, bit for bit. */
int gs_project_bwd_write(const gs_gaussians* g, const gs_view* views, const gs_view* views_dev, int32_t n_views,
                         const gs_config* cfg, const int32_t* tiles_touched, const float* grad2d,
                         size_t grad2d_bytes, gs_gaussian_grads* grads, gs_stream stream);

/* ---------------------------------------------------------------------------
 * gs_pose_grad -- Supp. B.1 written as a twist of the left perturbation
 * T(xi) = Exp(xi) T_CW, xi = (rho, phi):
 *   dL/drho = sum_i g_i,   dL/dphi = sum_i [p_i x g_i + 2 vex(G_i S_i - S_i G_i)]
 * with p_i the camera-space mean, S_i its camera-space covariance,
 * g_i = dL/dp_i and G_i = dL/dS_i obtained from grad2d (of gs_render_bwd)
 * through the EWA projection (pairs with tiles_touched == 0 are skipped).
 * The view-dependent feature term the paper
 * drops is zero here because colour and feature are view-independent.
 *   twist[V][6] (rho, phi), written (not accumulated).
 *   ws: gs_pose_grad_workspace bytes (per-block partial sums; the final sum
 *   runs in a fixed order, so the result is deterministic).
 * --------------------------------------------------------------------------- */
int gs_pose_grad_workspace(int32_t n, int32_t n_views, size_t* bytes);
int gs_pose_grad(const gs_gaussians* g, const gs_view* views, const gs_view* views_dev, int32_t n_views,
                 const gs_config* cfg, const int32_t* tiles_touched, const float* grad2d, void* ws,
                 size_t ws_bytes, float* twist, gs_stream stream);

/* ---------------------------------------------------------------------------
 * gs_pose_grad_noalloc -- gs_pose_grad without a workspace argument, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight tracking loops, harnesses that forbid allocation).  It computes the
 * same twist with the same kernels, bit for bit; the per-block partial sums
 * go to a fixed scratch array of GS_NOALLOC_SCRATCH_BYTES in the library's
 * own device memory (one copy per GPU, held until the process ends; nothing
 * is allocated or freed by the call).  Every partial is written before it is
 * read, so the array needs no clearing, but all calls on one GPU share it:
 * calls that overlap in time on one GPU (two streams, two host threads)
 * race and must be ordered by the caller.  The first call on each device
 * looks the array's address up (hipGetSymbolAddress); make that first call
 * outside stream capture.  Errors: as gs_pose_grad, and GS_ECAPACITY when
 * gs_pose_grad_workspace(n, n_views) exceeds GS_NOALLOC_SCRATCH_BYTES
 * (beyond about 22M Gaussians at 16 views); nothing is launched then.
 * --------------------------------------------------------------------------- */
enum { GS_NOALLOC_SCRATCH_BYTES = 8 << 20 };
int gs_pose_grad_noalloc(const gs_gaussians* g, const gs_view* views, const gs_view* views_dev, int32_t n_views,
                         const gs_config* cfg, const int32_t* tiles_touched, const float* grad2d, float* twist,
                         gs_stream stream);

/* Static description of a status code. */
const char* gs_error_string(int status);
/* Text of the last HIP error seen by this thread (empty if none). */
const char* gs_last_hip_error(void);
/* Library version (major * 10000 + minor * 100 + patch). */
int32_t gs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SGS_H */
