/*
 * sgs_oracle.c -- plain, slow FP64 CPU oracle for the semantic Gaussian
 * splatting rasterizer.  TEST INFRASTRUCTURE ONLY: it is called by the tests,
 * by the smoke check and by the benchmark's CPU-baseline leg, never by the
 * product path.  It shares no code, header or table with the HIP library.
 *
 * What it computes (GS^3LAM, Sec. 3.2 and Supp. B.1):
 *   - Eq. (2)  Sigma = R S S^T R^T from a quaternion and log-scales,
 *   - Eq. (3)  Sigma2D = J R_CW Sigma R_CW^T J^T (EWA splatting) plus a
 *              low-pass dilation b*I, its inverse (the conic),
 *   - Eq. (5)  alpha = o * exp(-1/2 sigma^T Sigma2D^-1 sigma),
 *   - Eq. (4), (6), (7), (10): front-to-back compositing of colour, depth,
 *              semantic feature and cumulative opacity in depth order,
 *   - the image-space loss gradients of Sec. 3.3.4 / 3.4 (L1 colour, L1
 *     depth, cross-entropy through a fixed linear decoder),
 *   - the backward pass to every Gaussian parameter, and the pose gradient
 *     of Supp. B.1 written as a 6-DoF twist (rho, phi) of a left
 *     perturbation T(xi) = Exp(xi) T_CW.
 *
 * Two precisions on purpose:
 *   - Discrete decisions (culling, the tile rectangle a Gaussian touches,
 *     the depth sort key) are taken in IEEE binary32 with one rounding per
 *     operation, in the fixed operation order written below, because that is
 *     the precision of the GPU path; every float op here is a plain
 *     binary32 add/sub/mul/div/sqrt (compiled with -ffp-contract=off), and
 *     exp on that path is the explicit Cody-Waite + degree-6 Taylor
 *     evaluation dec_expf.
 *   - Every value (alpha, compositing, losses, gradients) is FP64, from the
 *     FP32 inputs upcast exactly (or from FP64 inputs for finite
 *     differences).
 *
 * Readings where the paper is silent (pixel centre u+1/2, near plane,
 * frustum cull, dilation b, alpha_min / alpha_max / T_min, tie-break by
 * Gaussian index, zero background, un-normalised depth) are listed in the
 * design notes and passed in through `cfg`.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* cfg layout (float[8]): z_near, blur, guard, alpha_min, alpha_max, T_min, (unused), logit_min
 * logit_min = (float)ln(alpha_min/(1-alpha_min))  opacity cull threshold
 * The box size is per Gaussian (box_k below).                                  */
enum { C_ZNEAR = 0, C_BLUR, C_GUARD, C_AMIN, C_AMAX, C_TMIN, C_UNUSED, C_LOGITMIN };

/* view layout: [W, H, fx, fy, cx, cy, R00..R22, t0, t1, t2] = 18 values */
#define VSTRIDE 18

int orc_version(void) { return 3; }

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads used by the parallel loops from now on (timing of the oracle). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------- */
/* FP32 decision path                                                         */
/* ------------------------------------------------------------------------- */
static float dec_expf(float x) {
    if (x != x) return x;
    if (x < -80.0f) x = -80.0f;
    if (x > 80.0f) x = 80.0f;
    float n = rintf(x * 0x1.715476p+0f);
    float r = x - n * 0x1.62e4p-1f;
    r = r - n * 0x1.7f7d1cp-20f;
    float p = 0x1.6c16c2p-10f;
    p = 0x1.111112p-7f + r * p;
    p = 0x1.555556p-5f + r * p;
    p = 0x1.555556p-3f + r * p;
    p = 0.5f + r * p;
    p = 1.0f + r * p;
    p = 1.0f + r * p;
    return ldexpf(p, (int)n);
}

/* Natural logarithm of a positive normal binary32 y on the decision path.
 * Reduction: y = m * 2^e with m in [sqrt(1/2), sqrt(2)) -- frexp gives m in
 * [1/2, 1), and m below sqrt(1/2) is doubled (e lowered by one).  With
 * f = m - 1 (exact in that range) and s = f / (2 + f), ln m = 2 atanh(s),
 * whose odd series 2s (1 + z/3 + z^2/5 + z^3/7 + z^4/9 + z^5/11), z = s^2,
 * is truncated after the z^5 term (|s| < 0.172, so the next term is below
 * 1e-9 relative).  ln y = e ln2_hi + (ln m + e ln2_lo), with ln 2 split in
 * a short head (e * head exact) and a tail. */
static float dec_logf(float y) {
    int e;
    float m = frexpf(y, &e);
    if (m < 0x1.6a09e6p-1f) {   /* binary32 sqrt(1/2) */
        m = m + m;
        e = e - 1;
    }
    float f = m - 1.0f;
    float s = f / (2.0f + f);
    float z = s * s;
    float series = 0x1.745d18p-4f;            /* 1/11 */
    series = 0x1.c71c72p-4f + z * series;     /* 1/9  */
    series = 0x1.24924ap-3f + z * series;     /* 1/7  */
    series = 0x1.99999ap-3f + z * series;     /* 1/5  */
    series = 0x1.555556p-2f + z * series;     /* 1/3  */
    float two_s = s + s;
    float ln_m = two_s + (two_s * z) * series;
    float fe = (float)e;
    return fe * 0x1.62e4p-1f + (ln_m + fe * 0x1.7f7d1cp-20f);
}

/* Squared box radius, in standard deviations, of a Gaussian with opacity
 * logit l (the box that decides which tiles a Gaussian is binned to, so
 * that tiled rendering equals per-pixel rendering): alpha = o exp(-q/2)
 * reaches alpha_min only where q <= 2 ln(o / alpha_min), o = sigmoid(l)
 * evaluated on the decision path;
 * 2^-8 is added so that the box also holds the pairs whose binary32 alpha
 * rounds up to alpha_min.  Returns 0 when o / alpha_min <= 1 (culled). */
static float box_k(float logit, float alpha_min) {
    float o = 1.0f / (1.0f + dec_expf(-logit));
    float y = o / alpha_min;
    if (!(y > 1.0f)) return 0.0f;
    return 2.0f * dec_logf(y) + 0x1p-8f;
}

/* One (view, Gaussian) pair on the binary32 decision path.
 * Returns 1 if visible, 0 if culled.  rec = (mx, my, A, B, C, d, rx, ry). */
static int decide_one(const float* mu, const float* ls, const float* q, float logit,
                      const float* vw, const float* cfg, float* rec) {
    const float fx = vw[2], fy = vw[3], cx = vw[4], cy = vw[5];
    const float* R = vw + 6;
    const float* t = vw + 15;
    if (!(logit > cfg[C_LOGITMIN])) return 0;
    const float k = box_k(logit, cfg[C_AMIN]);
    if (!(k > 0.0f)) return 0;
    float p0 = ((R[0] * mu[0] + R[1] * mu[1]) + R[2] * mu[2]) + t[0];
    float p1 = ((R[3] * mu[0] + R[4] * mu[1]) + R[5] * mu[2]) + t[1];
    float p2 = ((R[6] * mu[0] + R[7] * mu[1]) + R[8] * mu[2]) + t[2];
    if (!(p2 > cfg[C_ZNEAR])) return 0;
    float xn = p0 / p2, yn = p1 / p2;
    float limx = (cfg[C_GUARD] * (0.5f * vw[0])) / fx;
    float limy = (cfg[C_GUARD] * (0.5f * vw[1])) / fy;
    if (!(fabsf(xn) <= limx) || !(fabsf(yn) <= limy)) return 0;
    float mx = fx * xn + cx;
    float my = fy * yn + cy;
    /* unit quaternion and rotation (Eq. 2) */
    float n2 = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3];
    if (!(n2 > 0.0f) || !(n2 < INFINITY)) return 0;
    float nrm = sqrtf(n2);
    float w = q[0] / nrm, x = q[1] / nrm, y = q[2] / nrm, z = q[3] / nrm;
    float r[9];
    r[0] = 1.0f - 2.0f * (y * y + z * z);
    r[1] = 2.0f * (x * y - w * z);
    r[2] = 2.0f * (x * z + w * y);
    r[3] = 2.0f * (x * y + w * z);
    r[4] = 1.0f - 2.0f * (x * x + z * z);
    r[5] = 2.0f * (y * z - w * x);
    r[6] = 2.0f * (x * z - w * y);
    r[7] = 2.0f * (y * z + w * x);
    r[8] = 1.0f - 2.0f * (x * x + y * y);
    float s0 = dec_expf(ls[0]), s1 = dec_expf(ls[1]), s2 = dec_expf(ls[2]);
    float M[9] = {r[0] * s0, r[1] * s1, r[2] * s2,
                  r[3] * s0, r[4] * s1, r[5] * s2,
                  r[6] * s0, r[7] * s1, r[8] * s2};
    /* EWA Jacobian (Eq. 3), T = J R_CW, U = T M, Sigma2D = U U^T + b I */
    float j00 = fx / p2, j11 = fy / p2;
    float j02 = -(j00 * xn), j12 = -(j11 * yn);
    float T0[3], T1[3];
    for (int k = 0; k < 3; ++k) {
        T0[k] = j00 * R[k] + j02 * R[6 + k];
        T1[k] = j11 * R[3 + k] + j12 * R[6 + k];
    }
    float U0[3], U1[3];
    for (int k = 0; k < 3; ++k) {
        U0[k] = (T0[0] * M[k] + T0[1] * M[3 + k]) + T0[2] * M[6 + k];
        U1[k] = (T1[0] * M[k] + T1[1] * M[3 + k]) + T1[2] * M[6 + k];
    }
    float a = ((U0[0] * U0[0] + U0[1] * U0[1]) + U0[2] * U0[2]) + cfg[C_BLUR];
    float b = (U0[0] * U1[0] + U0[1] * U1[1]) + U0[2] * U1[2];
    float c = ((U1[0] * U1[0] + U1[1] * U1[1]) + U1[2] * U1[2]) + cfg[C_BLUR];
    float det = a * c - b * b;
    if (!(det > 0.0f) || !(det < INFINITY)) return 0;
    rec[0] = mx;
    rec[1] = my;
    rec[2] = c / det;
    rec[3] = -b / det;
    rec[4] = a / det;
    rec[5] = p2;
    rec[6] = sqrtf(k * a) * 0x1.004p+0f;
    rec[7] = sqrtf(k * c) * 0x1.004p+0f;
    return 1;
}

/* Tile rectangle (inclusive) touched by the box [m-r, m+r]; 0 if none. */
static int tile_rect(const float* rec, int W, int H, int tile, int* out) {
    const float inv = 1.0f / (float)tile; /* power of two: exact */
    int tx = (W + tile - 1) / tile, ty = (H + tile - 1) / tile;
    float fx0 = floorf((rec[0] - rec[6]) * inv), fx1 = floorf((rec[0] + rec[6]) * inv);
    float fy0 = floorf((rec[1] - rec[7]) * inv), fy1 = floorf((rec[1] + rec[7]) * inv);
    if (!(fx1 >= 0.0f) || !(fx0 <= (float)(tx - 1))) return 0;
    if (!(fy1 >= 0.0f) || !(fy0 <= (float)(ty - 1))) return 0;
    if (fx0 < 0.0f) fx0 = 0.0f;
    if (fy0 < 0.0f) fy0 = 0.0f;
    if (fx1 > (float)(tx - 1)) fx1 = (float)(tx - 1);
    if (fy1 > (float)(ty - 1)) fy1 = (float)(ty - 1);
    out[0] = (int)fx0; out[1] = (int)fy0; out[2] = (int)fx1; out[3] = (int)fy1;
    return 1;
}

/* Decision path for all (view, Gaussian) pairs.
 * rect[V][n][4] (tx0, ty0, tx1, ty1 inclusive, -1 if culled), touched[V][n],
 * dbits[V][n] (binary32 bits of the camera depth), rec32[V][n][8] optional. */
void orc_decide(int n, const float* mu, const float* ls, const float* quat, const float* logit,
                int V, const float* views, const float* cfg, int tile,
                int32_t* rect, int32_t* touched, uint32_t* dbits, float* rec32) {
    for (int v = 0; v < V; ++v) {
        const float* vw = views + (size_t)v * VSTRIDE;
        const int W = (int)vw[0], H = (int)vw[1];
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            float m[3] = {mu[i], mu[n + i], mu[2 * (size_t)n + i]};
            float l[3] = {ls[i], ls[n + i], ls[2 * (size_t)n + i]};
            float q[4] = {quat[i], quat[n + i], quat[2 * (size_t)n + i], quat[3 * (size_t)n + i]};
            float rec[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            int r4[4] = {-1, -1, -1, -1};
            size_t o = (size_t)v * n + i;
            int vis = decide_one(m, l, q, logit[i], vw, cfg, rec);
            if (vis) vis = tile_rect(rec, W, H, tile, r4);
            if (!vis) { r4[0] = r4[1] = r4[2] = r4[3] = -1; }
            memcpy(rect + 4 * o, r4, sizeof(r4));
            touched[o] = vis ? (r4[2] - r4[0] + 1) * (r4[3] - r4[1] + 1) : 0;
            uint32_t bits;
            memcpy(&bits, &rec[5], 4);
            dbits[o] = vis ? bits : 0u;
            if (rec32) memcpy(rec32 + 8 * o, rec, sizeof(rec));
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Binning: every (view, tile, Gaussian) instance sorted by                   */
/* (view*tiles + tile, depth bits, Gaussian index).                           */
/* ------------------------------------------------------------------------- */
typedef struct { uint32_t tile; uint32_t dbits; int32_t gid; } inst_t;

static int inst_cmp(const void* pa, const void* pb) {
    const inst_t* a = (const inst_t*)pa;
    const inst_t* b = (const inst_t*)pb;
    if (a->tile != b->tile) return a->tile < b->tile ? -1 : 1;
    if (a->dbits != b->dbits) return a->dbits < b->dbits ? -1 : 1;
    if (a->gid != b->gid) return a->gid < b->gid ? -1 : 1;
    return 0;
}

/* tile_base[v] = first global tile id of view v; returns total tiles. */
static int64_t tile_bases(int V, const float* views, int tile, int64_t* base) {
    int64_t acc = 0;
    for (int v = 0; v < V; ++v) {
        int W = (int)views[(size_t)v * VSTRIDE], H = (int)views[(size_t)v * VSTRIDE + 1];
        base[v] = acc;
        acc += (int64_t)((W + tile - 1) / tile) * ((H + tile - 1) / tile);
    }
    return acc;
}

int64_t orc_total_tiles(int V, const float* views, int tile) {
    int64_t* b = (int64_t*)malloc(sizeof(int64_t) * (V > 0 ? V : 1));
    int64_t t = tile_bases(V, views, tile, b);
    free(b);
    return t;
}

/* Returns the instance count; fills keys/gids only if it is <= cap. */
int64_t orc_bin(int n, int V, const float* views, int tile, const int32_t* rect,
                const int32_t* touched, const uint32_t* dbits, int64_t cap,
                uint32_t* keys, int32_t* gids, int32_t* ranges) {
    int64_t* base = (int64_t*)malloc(sizeof(int64_t) * (V > 0 ? V : 1));
    int64_t total_tiles = tile_bases(V, views, tile, base);
    int64_t count = 0;
    for (size_t o = 0; o < (size_t)V * n; ++o) count += touched[o];
    if (count > cap) { free(base); return count; }
    inst_t* arr = (inst_t*)malloc(sizeof(inst_t) * (count > 0 ? count : 1));
    int64_t k = 0;
    for (int v = 0; v < V; ++v) {
        int W = (int)views[(size_t)v * VSTRIDE];
        int tx = (W + tile - 1) / tile;
        for (int i = 0; i < n; ++i) {
            size_t o = (size_t)v * n + i;
            if (!touched[o]) continue;
            const int32_t* r = rect + 4 * o;
            for (int y = r[1]; y <= r[3]; ++y)
                for (int x = r[0]; x <= r[2]; ++x) {
                    arr[k].tile = (uint32_t)(base[v] + (int64_t)y * tx + x);
                    arr[k].dbits = dbits[o];
                    arr[k].gid = i;
                    ++k;
                }
        }
    }
    qsort(arr, (size_t)count, sizeof(inst_t), inst_cmp);
    for (int64_t t = 0; t < total_tiles; ++t) { ranges[2 * t] = 0; ranges[2 * t + 1] = 0; }
    for (int64_t j = 0; j < count; ++j) {
        keys[j] = arr[j].tile;
        gids[j] = arr[j].gid;
        if (j == 0 || arr[j - 1].tile != arr[j].tile) ranges[2 * (int64_t)arr[j].tile] = (int32_t)j;
        ranges[2 * (int64_t)arr[j].tile + 1] = (int32_t)(j + 1);
    }
    free(arr);
    free(base);
    return count;
}

/* ------------------------------------------------------------------------- */
/* FP64 value path                                                            */
/* ------------------------------------------------------------------------- */
typedef struct {
    double mx, my, A, B, C, o, d;     /* mean2d, conic, opacity, depth   */
} proj_t;

static void quat_rot(const double* q, double* qh, double* r, double* nrm_out) {
    double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
    qh[0] = w; qh[1] = x; qh[2] = y; qh[3] = z;
    *nrm_out = n;
    r[0] = 1 - 2 * (y * y + z * z); r[1] = 2 * (x * y - w * z);     r[2] = 2 * (x * z + w * y);
    r[3] = 2 * (x * y + w * z);     r[4] = 1 - 2 * (x * x + z * z); r[5] = 2 * (y * z - w * x);
    r[6] = 2 * (x * z - w * y);     r[7] = 2 * (y * z + w * x);     r[8] = 1 - 2 * (x * x + y * y);
}

static void mat3_mul(const double* a, const double* b, double* c) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += a[3 * i + k] * b[3 * k + j];
            c[3 * i + j] = s;
        }
}
static void mat3_T(const double* a, double* t) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) t[3 * i + j] = a[3 * j + i];
}

/* Full forward geometry of one (view, Gaussian) pair in FP64.
 * Outputs p (camera point), Sc (camera covariance, 3x3), S2 (2x2 before inverse). */
typedef struct {
    double p[3], Sc[9], S2[3], J[6], Rq[9], qh[4], qn, s[3], Sig[9], o;
} geom_t;

static void geom64(const double* mu, const double* ls, const double* q, double logit,
                   const double* vw, double blur, geom_t* g) {
    const double fx = vw[2], fy = vw[3];
    const double* R = vw + 6;
    const double* t = vw + 15;
    for (int k = 0; k < 3; ++k) g->p[k] = R[3 * k] * mu[0] + R[3 * k + 1] * mu[1] + R[3 * k + 2] * mu[2] + t[k];
    quat_rot(q, g->qh, g->Rq, &g->qn);
    for (int k = 0; k < 3; ++k) g->s[k] = exp(ls[k]);
    /* Sigma = R S S^T R^T (Eq. 2) */
    double RS[9], RSt[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) RS[3 * i + j] = g->Rq[3 * i + j] * g->s[j];
    mat3_T(RS, RSt);
    mat3_mul(RS, RSt, g->Sig);
    /* Sigma_c = R_CW Sigma R_CW^T */
    double Rt[9], tmp[9];
    mat3_T(R, Rt);
    mat3_mul(R, g->Sig, tmp);
    mat3_mul(tmp, Rt, g->Sc);
    /* J = d(pi)/dp, Sigma2D = J Sigma_c J^T + b I (Eq. 3) */
    const double z = g->p[2];
    g->J[0] = fx / z; g->J[1] = 0; g->J[2] = -fx * g->p[0] / (z * z);
    g->J[3] = 0; g->J[4] = fy / z; g->J[5] = -fy * g->p[1] / (z * z);
    double JS[6];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += g->J[3 * i + k] * g->Sc[3 * k + j];
            JS[3 * i + j] = s;
        }
    double S00 = 0, S01 = 0, S11 = 0;
    for (int k = 0; k < 3; ++k) {
        S00 += JS[k] * g->J[k];
        S01 += JS[k] * g->J[3 + k];
        S11 += JS[3 + k] * g->J[3 + k];
    }
    g->S2[0] = S00 + blur; g->S2[1] = S01; g->S2[2] = S11 + blur;
    g->o = 1.0 / (1.0 + exp(-logit));
}

static void proj_from_geom(const geom_t* g, const double* vw, proj_t* pr) {
    const double z = g->p[2];
    pr->mx = vw[2] * g->p[0] / z + vw[4];
    pr->my = vw[3] * g->p[1] / z + vw[5];
    double det = g->S2[0] * g->S2[2] - g->S2[1] * g->S2[1];
    pr->A = g->S2[2] / det;
    pr->B = -g->S2[1] / det;
    pr->C = g->S2[0] / det;
    pr->o = g->o;
    pr->d = z;
}

static void load_gauss(int n, int i, const double* mu, const double* ls, const double* quat,
                       double* m, double* l, double* q) {
    for (int k = 0; k < 3; ++k) { m[k] = mu[(size_t)k * n + i]; l[k] = ls[(size_t)k * n + i]; }
    for (int k = 0; k < 4; ++k) q[k] = quat[(size_t)k * n + i];
}

/* FP64 projection of every (view, Gaussian) pair: proj[V][n][7] =
 * (mx, my, A, B, C, o, d).  Evaluated for every pair (culled ones too). */
void orc_project64(int n, const double* mu, const double* ls, const double* quat, const double* logit,
                   int V, const double* views, const float* cfg, double* proj) {
    for (int v = 0; v < V; ++v) {
        const double* vw = views + (size_t)v * VSTRIDE;
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            double m[3], l[3], q[4];
            load_gauss(n, i, mu, ls, quat, m, l, q);
            geom_t g;
            geom64(m, l, q, logit[i], vw, (double)cfg[C_BLUR], &g);
            proj_t pr;
            proj_from_geom(&g, vw, &pr);
            double* o = proj + 7 * ((size_t)v * n + i);
            o[0] = pr.mx; o[1] = pr.my; o[2] = pr.A; o[3] = pr.B; o[4] = pr.C; o[5] = pr.o; o[6] = pr.d;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Forward compositing (Eq. 4-7, 9)                                           */
/* ------------------------------------------------------------------------- */
typedef struct {
    int V, n, F, tile;
    const double* views;
    const float* cfg;
    const int32_t* ranges;
    const int32_t* gids;
    const double* color;   /* [3][n] */
    const double* feat;    /* [F][n] */
    const proj_t* proj;    /* [V][n] */
    const proj_t* dproj;   /* [V][n] geometry the alpha_min / T_min decisions are taken on */
    int64_t* tile_base;
    int64_t* pix_base;
} scene_ctx;

/* alpha of one pair; returns raw o*G before the clamp via *raw, G via *gauss,
 * and whether q was clamped at 0 via *qclamp. */
static double pair_alpha(const proj_t* pr, double px, double py, double amax,
                         double* raw, double* gauss, double* dx_o, double* dy_o, int* qclamp) {
    double dx = px - pr->mx, dy = py - pr->my;
    double q = pr->A * dx * dx + 2.0 * pr->B * dx * dy + pr->C * dy * dy;
    *qclamp = 0;
    if (q < 0.0) { q = 0.0; *qclamp = 1; }
    double G = exp(-0.5 * q);
    double a = pr->o * G;
    *raw = a;
    *gauss = G;
    *dx_o = dx;
    *dy_o = dy;
    return a < amax ? a : amax;
}

static double feat_of(const scene_ctx* s, int ch, int gid) {
    /* channel value x_ch of Gaussian gid: 0..2 colour, 3 depth (per view, handled by caller),
     * 4 opacity (1), 5.. feature */
    if (ch < 3) return s->color[(size_t)ch * s->n + gid];
    if (ch == 4) return 1.0;
    return s->feat[(size_t)(ch - 5) * s->n + gid];
}

static void pixel_forward(const scene_ctx* s, int v, int u, int w_, double* out, double* Tfinal,
                          int32_t* last, int32_t* ncontrib, double* margin_a, double* margin_t) {
    const double* vw = s->views + (size_t)v * VSTRIDE;
    const int W = (int)vw[0];
    const int tx = (W + s->tile - 1) / s->tile;
    const int64_t t = s->tile_base[v] + (int64_t)(w_ / s->tile) * tx + (u / s->tile);
    const int32_t beg = s->ranges[2 * t], end = s->ranges[2 * t + 1];
    const double amin = s->cfg[C_AMIN], amax = s->cfg[C_AMAX], tmin = s->cfg[C_TMIN];
    const int NC = 5 + s->F;
    const double px = u + 0.5, py = w_ + 0.5;
    double T = 1.0, mga = INFINITY, mgt = INFINITY;
    int lst = 0, cnt = 0;
    for (int ch = 0; ch < NC; ++ch) out[ch] = 0.0;
    for (int32_t k = beg; k < end; ++k) {
        const int gid = s->gids[k];
        const proj_t* pr = s->proj + (size_t)v * s->n + gid;
        double raw, G, dx, dy;
        int qc;
        double a = pair_alpha(pr, px, py, amax, &raw, &G, &dx, &dy, &qc);
        double m1 = fabs(a - amin) / amin;
        if (m1 < mga) mga = m1;
        if (a < amin) continue;
        double Tn = T * (1.0 - a);
        double m2 = fabs(Tn - tmin) / tmin;
        if (m2 < mgt) mgt = m2;
        if (Tn < tmin) break;
        double wgt = a * T;
        for (int ch = 0; ch < NC; ++ch) {
            double x = (ch == 3) ? pr->d : feat_of(s, ch, gid);
            out[ch] += x * wgt;
        }
        T = Tn;
        lst = k - beg + 1;
        ++cnt;
    }
    *Tfinal = T;
    *last = lst;
    *ncontrib = cnt;
    *margin_a = mga;
    *margin_t = mgt;
}

static void setup_ctx(scene_ctx* s, int n, int F, const double* color, const double* feat, int V,
                      const double* views, const float* cfg, int tile, const int32_t* ranges,
                      const int32_t* gids, const proj_t* proj) {
    s->V = V; s->n = n; s->F = F; s->tile = tile; s->views = views; s->cfg = cfg;
    s->ranges = ranges; s->gids = gids; s->color = color; s->feat = feat; s->proj = proj; s->dproj = proj;
    s->tile_base = (int64_t*)malloc(sizeof(int64_t) * (V > 0 ? V : 1));
    s->pix_base = (int64_t*)malloc(sizeof(int64_t) * (V + 1));
    int64_t tb = 0, pb = 0;
    for (int v = 0; v < V; ++v) {
        int W = (int)views[(size_t)v * VSTRIDE], H = (int)views[(size_t)v * VSTRIDE + 1];
        s->tile_base[v] = tb;
        s->pix_base[v] = pb;
        tb += (int64_t)((W + tile - 1) / tile) * ((H + tile - 1) / tile);
        pb += (int64_t)W * H;
    }
    s->pix_base[V] = pb;
}

static void free_ctx(scene_ctx* s) {
    free(s->tile_base);
    free(s->pix_base);
}

/* Forward render of every pixel (or of the pixels with pix_mask[p] != 0).
 * proj[V][n][7] from orc_project64; out[5+F][P]: R, G, B, depth, opacity,
 * features; Tfinal[P], last[P], ncontrib[P], and the smallest relative
 * distance of any alpha to alpha_min (margin_a[P]) and of any T (1 - alpha)
 * to T_min (margin_t[P]) met at the pixel. */
void orc_render(int n, int F, const double* color, const double* feat, int V, const double* views,
                const float* cfg, int tile, const int32_t* ranges, const int32_t* gids,
                const double* proj, const uint8_t* pix_mask, double* out, double* Tfinal,
                int32_t* last, int32_t* ncontrib, double* margin_a, double* margin_t) {
    scene_ctx s;
    setup_ctx(&s, n, F, color, feat, V, views, cfg, tile, ranges, gids, (const proj_t*)proj);
    const int64_t P = s.pix_base[V];
    const int NC = 5 + F;
    for (int v = 0; v < V; ++v) {
        const int W = (int)views[(size_t)v * VSTRIDE], H = (int)views[(size_t)v * VSTRIDE + 1];
#pragma omp parallel for schedule(dynamic, 1)
        for (int y = 0; y < H; ++y) {
            double acc[5 + 256];
            for (int x = 0; x < W; ++x) {
                const int64_t p = s.pix_base[v] + (int64_t)y * W + x;
                if (pix_mask && !pix_mask[p]) continue;
                pixel_forward(&s, v, x, y, acc, &Tfinal[p], &last[p], &ncontrib[p], &margin_a[p], &margin_t[p]);
                for (int ch = 0; ch < NC; ++ch) out[(size_t)ch * P + p] = acc[ch];
            }
        }
    }
    free_ctx(&s);
}

/* ------------------------------------------------------------------------- */
/* Image-space losses (Sec. 3.3.4 / 3.4), per view, each a mean over pixels: */
/*   L = lc * mean|C - C*| (over 3P_v) + ld * mean|D - D*| + ls * mean CE     */
/* CE = -log softmax(W^T F)[label], W is F x K row-major.                     */
/* ------------------------------------------------------------------------- */
void orc_loss(int F, int K, int V, const int64_t* pix_count, const double* out, const double* rgb_t,
              const double* depth_t, const int32_t* labels, const double* Wd, const double* weights,
              double* grad_out, double* loss_terms) {
    int64_t P = 0;
    for (int v = 0; v < V; ++v) P += pix_count[v];
    const int NC = 5 + F;
    memset(grad_out, 0, sizeof(double) * (size_t)NC * P);
    double Lc = 0, Ld = 0, Ls = 0;
    int64_t base = 0;
    for (int v = 0; v < V; ++v) {
        const int64_t Pv = pix_count[v];
        const double gc = weights[0] / (3.0 * (double)Pv), gd = weights[1] / (double)Pv,
                     gs = weights[2] / (double)Pv;
        double lc = 0, ld = 0, lsum = 0;
        for (int64_t j = 0; j < Pv; ++j) {
            const int64_t p = base + j;
            for (int ch = 0; ch < 3; ++ch) {
                double r = out[(size_t)ch * P + p] - rgb_t[(size_t)ch * P + p];
                lc += fabs(r);
                grad_out[(size_t)ch * P + p] = r > 0 ? gc : (r < 0 ? -gc : 0.0);
            }
            double rd = out[3 * (size_t)P + p] - depth_t[p];
            ld += fabs(rd);
            grad_out[3 * (size_t)P + p] = rd > 0 ? gd : (rd < 0 ? -gd : 0.0);
            if (K > 0 && weights[2] != 0.0) {
                double z[1024], mx = -INFINITY;
                for (int k = 0; k < K; ++k) {
                    double acc = 0;
                    for (int f = 0; f < F; ++f) acc += Wd[(size_t)f * K + k] * out[(size_t)(5 + f) * P + p];
                    z[k] = acc;
                    if (acc > mx) mx = acc;
                }
                double se = 0;
                for (int k = 0; k < K; ++k) se += exp(z[k] - mx);
                const int lab = labels[p];
                lsum += (mx + log(se)) - z[lab];
                for (int f = 0; f < F; ++f) {
                    double g = 0;
                    for (int k = 0; k < K; ++k) {
                        double sm = exp(z[k] - mx) / se - (k == lab ? 1.0 : 0.0);
                        g += Wd[(size_t)f * K + k] * sm;
                    }
                    grad_out[(size_t)(5 + f) * P + p] = gs * g;
                }
            }
        }
        Lc += weights[0] * lc / (3.0 * (double)Pv);
        Ld += weights[1] * ld / (double)Pv;
        Ls += weights[2] * lsum / (double)Pv;
        base += Pv;
    }
    loss_terms[0] = Lc;
    loss_terms[1] = Ld;
    loss_terms[2] = Ls;
    loss_terms[3] = Lc + Ld + Ls;
}

/* ------------------------------------------------------------------------- */
/* Backward pass                                                              */
/* ------------------------------------------------------------------------- */
/* Per-instance accumulator layout (doubles): dmx, dmy, dA, dB, dC, dd, do, dc[3], df[F] */
#define IA (10)

/* Per-pixel backward over its tile list.  The forward is re-run storing the
 * transmittance before every included Gaussian (no division), then the
 * gradient is accumulated in reverse with per-channel suffix sums
 *   dL/dalpha_i = sum_ch g_ch (x_i,ch T_i - S_ch / (1 - alpha_i)),
 *   S_ch = sum_{j > i} x_j,ch alpha_j T_j.
 * Which Gaussians are included (alpha >= alpha_min) and where the pixel
 * stops (T (1 - alpha) < T_min) is decided on s->dproj; every value comes
 * from s->proj (the two are the same unless a caller asks for decisions on
 * another geometry). */
static void pixel_backward(const scene_ctx* s, int v, int u, int w_, const double* gpix,
                           double* inst_acc, int32_t beg, int32_t end) {
    const double amin = s->cfg[C_AMIN], amax = s->cfg[C_AMAX], tmin = s->cfg[C_TMIN];
    const int NC = 5 + s->F;
    const int IS = IA + s->F;
    const double px = u + 0.5, py = w_ + 0.5;
    int cap = 64, m = 0;
    int32_t* ks = (int32_t*)malloc(sizeof(int32_t) * cap);
    double* Ts = (double*)malloc(sizeof(double) * cap);
    double T = 1.0, Td = 1.0;
    for (int32_t k = beg; k < end; ++k) {
        const size_t o = (size_t)v * s->n + s->gids[k];
        double raw, G, dx, dy;
        int qc;
        double ad = pair_alpha(s->dproj + o, px, py, amax, &raw, &G, &dx, &dy, &qc);
        if (ad < amin) continue;
        double Tdn = Td * (1.0 - ad);
        if (Tdn < tmin) break;
        double a = pair_alpha(s->proj + o, px, py, amax, &raw, &G, &dx, &dy, &qc);
        if (m == cap) {
            cap *= 2;
            ks = (int32_t*)realloc(ks, sizeof(int32_t) * cap);
            Ts = (double*)realloc(Ts, sizeof(double) * cap);
        }
        ks[m] = k;
        Ts[m] = T;
        ++m;
        T = T * (1.0 - a);
        Td = Tdn;
    }
    double S[5 + 256];
    for (int ch = 0; ch < NC; ++ch) S[ch] = 0.0;
    for (int i = m - 1; i >= 0; --i) {
        const int32_t k = ks[i];
        const int gid = s->gids[k];
        const proj_t* pr = s->proj + (size_t)v * s->n + gid;
        double raw, G, dx, dy;
        int qc;
        double a = pair_alpha(pr, px, py, amax, &raw, &G, &dx, &dy, &qc);
        const double Ti = Ts[i], wgt = a * Ti;
        double* acc = inst_acc + (size_t)(k - beg) * IS;
        double dalpha = 0.0;
        for (int ch = 0; ch < NC; ++ch) {
            double x = (ch == 3) ? pr->d : feat_of(s, ch, gid);
            dalpha += gpix[ch] * (x * Ti - S[ch] / (1.0 - a));
        }
        for (int ch = 0; ch < NC; ++ch) {
            double x = (ch == 3) ? pr->d : feat_of(s, ch, gid);
            S[ch] += x * wgt;
        }
        /* parameters that enter linearly: colour, depth, feature */
        acc[7] += gpix[0] * wgt;
        acc[8] += gpix[1] * wgt;
        acc[9] += gpix[2] * wgt;
        acc[5] += gpix[3] * wgt;
        for (int f = 0; f < s->F; ++f) acc[IA + f] += gpix[5 + f] * wgt;
        /* alpha = min(amax, o G), G = exp(-q/2) */
        if (raw < amax) {
            acc[6] += dalpha * G;                       /* dL/do */
            if (!qc) {
                const double dq = dalpha * (-0.5 * a);  /* dL/dq */
                acc[0] += dq * (-2.0) * (pr->A * dx + pr->B * dy);
                acc[1] += dq * (-2.0) * (pr->B * dx + pr->C * dy);
                acc[2] += dq * dx * dx;
                acc[3] += dq * 2.0 * dx * dy;
                acc[4] += dq * dy * dy;
            }
        }
    }
    free(ks);
    free(Ts);
}

/* Backward of the projection for one (view, Gaussian) pair.
 * g2[6] = dL/d(mx, my, A, B, C, d) in this view.
 * Outputs: dmu[3], dls[3], dq[4] (accumulated), gcam[3] = dL/dp,
 * Gcam[9] = dL/dSigma_c (symmetric, full). */
static void project_backward(const geom_t* g, const double* vw, const double* g2,
                             double* dmu, double* dls, double* dq, double* gcam, double* Gcam) {
    const double fx = vw[2], fy = vw[3];
    const double* R = vw + 6;
    const double x = g->p[0], y = g->p[1], z = g->p[2];
    /* conic Q = Sigma2D^-1; dL/dSigma2D = -Q dQ Q with symmetric dQ */
    double det = g->S2[0] * g->S2[2] - g->S2[1] * g->S2[1];
    double Q[4] = {g->S2[2] / det, -g->S2[1] / det, -g->S2[1] / det, g->S2[0] / det};
    double dQ[4] = {g2[2], 0.5 * g2[3], 0.5 * g2[3], g2[4]};
    double t1[4], dS[4];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) t1[2 * i + j] = dQ[2 * i] * Q[j] + dQ[2 * i + 1] * Q[2 + j];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) dS[2 * i + j] = -(Q[2 * i] * t1[j] + Q[2 * i + 1] * t1[2 + j]);
    /* Sigma2D = J Sc J^T + bI:  dL/dSc = J^T dS J,  dL/dJ = 2 dS J Sc */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) acc += g->J[3 * a + i] * dS[2 * a + b] * g->J[3 * b + j];
            Gcam[3 * i + j] = acc;
        }
    double JSc[6], dJ[6];
    for (int a = 0; a < 2; ++a)
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += g->J[3 * a + k] * g->Sc[3 * k + j];
            JSc[3 * a + j] = acc;
        }
    for (int a = 0; a < 2; ++a)
        for (int j = 0; j < 3; ++j) dJ[3 * a + j] = 2.0 * (dS[2 * a] * JSc[j] + dS[2 * a + 1] * JSc[3 + j]);
    /* camera point gradient: mean2d, J and depth all depend on p */
    double gp[3] = {0, 0, 0};
    gp[0] += g2[0] * fx / z;
    gp[1] += g2[1] * fy / z;
    gp[2] += -g2[0] * fx * x / (z * z) - g2[1] * fy * y / (z * z);
    /* J00 = fx/z, J02 = -fx x/z^2, J11 = fy/z, J12 = -fy y/z^2 */
    gp[2] += dJ[0] * (-fx / (z * z));
    gp[0] += dJ[2] * (-fx / (z * z));
    gp[2] += dJ[2] * (2.0 * fx * x / (z * z * z));
    gp[2] += dJ[4] * (-fy / (z * z));
    gp[1] += dJ[5] * (-fy / (z * z));
    gp[2] += dJ[5] * (2.0 * fy * y / (z * z * z));
    gp[2] += g2[5];
    gcam[0] = gp[0]; gcam[1] = gp[1]; gcam[2] = gp[2];
    /* p = R mu + t */
    for (int k = 0; k < 3; ++k) dmu[k] += R[k] * gp[0] + R[3 + k] * gp[1] + R[6 + k] * gp[2];
    /* Sc = R Sigma R^T: dL/dSigma = R^T G R */
    double Rt[9], tmp[9], dSig[9];
    mat3_T(R, Rt);
    mat3_mul(Rt, Gcam, tmp);
    mat3_mul(tmp, R, dSig);
    /* Sigma = M M^T, M = Rq diag(s): dL/dM = 2 dSig M */
    double M[9], dM[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[3 * i + j] = g->Rq[3 * i + j] * g->s[j];
    mat3_mul(dSig, M, dM);
    for (int k = 0; k < 9; ++k) dM[k] *= 2.0;
    double dR[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) dR[3 * i + j] = dM[3 * i + j] * g->s[j];
    for (int j = 0; j < 3; ++j) {
        double ds = 0;
        for (int i = 0; i < 3; ++i) ds += dM[3 * i + j] * g->Rq[3 * i + j];
        dls[j] += ds * g->s[j];
    }
    /* rotation of the unit quaternion (w, x, y, z) */
    const double w = g->qh[0], qx = g->qh[1], qy = g->qh[2], qz = g->qh[3];
    double dqh[4];
    dqh[0] = 2.0 * (-qz * dR[1] + qy * dR[2] + qz * dR[3] - qx * dR[5] - qy * dR[6] + qx * dR[7]);
    dqh[1] = 2.0 * (qy * dR[1] + qz * dR[2] + qy * dR[3] - 2.0 * qx * dR[4] - w * dR[5] + qz * dR[6] +
                    w * dR[7] - 2.0 * qx * dR[8]);
    dqh[2] = 2.0 * (-2.0 * qy * dR[0] + qx * dR[1] + w * dR[2] + qx * dR[3] + qz * dR[5] - w * dR[6] +
                    qz * dR[7] - 2.0 * qy * dR[8]);
    dqh[3] = 2.0 * (-2.0 * qz * dR[0] - w * dR[1] + qx * dR[2] + w * dR[3] - 2.0 * qz * dR[4] + qy * dR[5] +
                    qx * dR[6] + qy * dR[7]);
    /* q_hat = q / |q|:  dq = (I - q_hat q_hat^T) dq_hat / |q| */
    double dot = w * dqh[0] + qx * dqh[1] + qy * dqh[2] + qz * dqh[3];
    for (int k = 0; k < 4; ++k) dq[k] += (dqh[k] - g->qh[k] * dot) / g->qn;
}

/* Full backward.  grad_out[5+F][P]; only pixels inside tiles with
 * tile_mask[t] != 0 are processed (tile_mask may be NULL for all).
 * flags: bit0 = parameter gradients, bit1 = pose gradient.
 * Outputs (all zeroed here, then filled):
 *   grad2d[V][n][6]  dL/d(mx, my, A, B, C, d) per view
 *   gapp[n][4+F]     dL/d(o, c0, c1, c2, f...) summed over views
 *   dmu[3][n], dls[3][n], dq[4][n], dlogit[n], dcolor[3][n], dfeat[F][n]
 *   gcam[V][n][3], Gcam[V][n][6] (xx, xy, xz, yy, yz, zz), twist[V][6]. */
void orc_backward(int n, int F, const double* mu, const double* ls, const double* quat,
                  const double* logit, const double* color, const double* feat, int V,
                  const double* views, const float* cfg, int tile, const int32_t* ranges,
                  const int32_t* gids, const double* proj, const double* dproj, const double* grad_out,
                  const uint8_t* tile_mask, const uint8_t* vis, int flags,
                  double* grad2d, double* gapp, double* dmu, double* dls, double* dq, double* dlogit,
                  double* dcolor, double* dfeat, double* gcam, double* Gcam, double* twist) {
    scene_ctx s;
    setup_ctx(&s, n, F, color, feat, V, views, cfg, tile, ranges, gids, (const proj_t*)proj);
    if (dproj) s.dproj = (const proj_t*)dproj;
    const int64_t P = s.pix_base[V];
    const int NC = 5 + F, IS = IA + F, GA = 4 + F;
    int64_t total_tiles = 0;
    for (int v = 0; v < V; ++v) {
        int W = (int)views[(size_t)v * VSTRIDE], H = (int)views[(size_t)v * VSTRIDE + 1];
        total_tiles += (int64_t)((W + tile - 1) / tile) * ((H + tile - 1) / tile);
    }
    const int64_t n_inst = total_tiles > 0 ? ranges[2 * (total_tiles - 1) + 1] : 0;
    int64_t max_end = 0;
    for (int64_t t = 0; t < total_tiles; ++t)
        if (ranges[2 * t + 1] > max_end) max_end = ranges[2 * t + 1];
    (void)n_inst;
    double* inst = (double*)calloc((size_t)(max_end > 0 ? max_end : 1) * IS, sizeof(double));
    /* 1. per tile (parallel), per pixel (serial): per-instance sums */
    for (int v = 0; v < V; ++v) {
        const int W = (int)views[(size_t)v * VSTRIDE], H = (int)views[(size_t)v * VSTRIDE + 1];
        const int tx = (W + tile - 1) / tile, ty = (H + tile - 1) / tile;
#pragma omp parallel for schedule(dynamic, 1)
        for (int tt = 0; tt < tx * ty; ++tt) {
            const int64_t t = s.tile_base[v] + tt;
            if (tile_mask && !tile_mask[t]) continue;
            const int32_t beg = ranges[2 * t], end = ranges[2 * t + 1];
            if (end <= beg) continue;
            const int x0 = (tt % tx) * tile, y0 = (tt / tx) * tile;
            double gpix[5 + 256];
            for (int y = y0; y < y0 + tile && y < H; ++y)
                for (int x = x0; x < x0 + tile && x < W; ++x) {
                    const int64_t p = s.pix_base[v] + (int64_t)y * W + x;
                    for (int ch = 0; ch < NC; ++ch) gpix[ch] = grad_out[(size_t)ch * P + p];
                    pixel_backward(&s, v, x, y, gpix, inst + (size_t)beg * IS, beg, end);
                }
        }
    }
    /* 2. instance sums -> per (view, Gaussian) 2D gradients (serial, fixed order) */
    memset(grad2d, 0, sizeof(double) * (size_t)V * n * 6);
    memset(gapp, 0, sizeof(double) * (size_t)n * GA);
    for (int v = 0; v < V; ++v) {
        const int W = (int)views[(size_t)v * VSTRIDE], H = (int)views[(size_t)v * VSTRIDE + 1];
        const int ntile = ((W + tile - 1) / tile) * ((H + tile - 1) / tile);
        for (int tt = 0; tt < ntile; ++tt) {
            const int64_t t = s.tile_base[v] + tt;
            if (tile_mask && !tile_mask[t]) continue;
            for (int32_t k = ranges[2 * t]; k < ranges[2 * t + 1]; ++k) {
                const int gid = gids[k];
                const double* a = inst + (size_t)k * IS;
                double* g2 = grad2d + 6 * ((size_t)v * n + gid);
                for (int c = 0; c < 6; ++c) g2[c] += a[c];
                double* ga = gapp + (size_t)GA * gid;
                ga[0] += a[6];
                ga[1] += a[7];
                ga[2] += a[8];
                ga[3] += a[9];
                for (int f = 0; f < F; ++f) ga[4 + f] += a[IA + f];
            }
        }
    }
    free(inst);
    /* 3. projection backward per Gaussian (loop over views inside: no races) */
    memset(dmu, 0, sizeof(double) * 3 * (size_t)n);
    memset(dls, 0, sizeof(double) * 3 * (size_t)n);
    memset(dq, 0, sizeof(double) * 4 * (size_t)n);
    memset(dlogit, 0, sizeof(double) * (size_t)n);
    memset(dcolor, 0, sizeof(double) * 3 * (size_t)n);
    memset(dfeat, 0, sizeof(double) * (size_t)F * n);
    memset(gcam, 0, sizeof(double) * 3 * (size_t)V * n);
    memset(Gcam, 0, sizeof(double) * 6 * (size_t)V * n);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double m[3], l[3], q[4];
        load_gauss(n, i, mu, ls, quat, m, l, q);
        double a_mu[3] = {0, 0, 0}, a_ls[3] = {0, 0, 0}, a_q[4] = {0, 0, 0, 0};
        for (int v = 0; v < V; ++v) {
            const size_t o = (size_t)v * n + i;
            if (vis && !vis[o]) continue;
            const double* g2 = grad2d + 6 * o;
            if (g2[0] == 0 && g2[1] == 0 && g2[2] == 0 && g2[3] == 0 && g2[4] == 0 && g2[5] == 0) continue;
            const double* vw = views + (size_t)v * VSTRIDE;
            geom_t g;
            geom64(m, l, q, logit[i], vw, (double)cfg[C_BLUR], &g);
            double gc[3], Gc[9];
            project_backward(&g, vw, g2, a_mu, a_ls, a_q, gc, Gc);
            gcam[3 * o] = gc[0]; gcam[3 * o + 1] = gc[1]; gcam[3 * o + 2] = gc[2];
            double* G6 = Gcam + 6 * o;
            G6[0] = Gc[0]; G6[1] = Gc[1]; G6[2] = Gc[2]; G6[3] = Gc[4]; G6[4] = Gc[5]; G6[5] = Gc[8];
        }
        if (flags & 1) {
            for (int k = 0; k < 3; ++k) { dmu[(size_t)k * n + i] = a_mu[k]; dls[(size_t)k * n + i] = a_ls[k]; }
            for (int k = 0; k < 4; ++k) dq[(size_t)k * n + i] = a_q[k];
            const double* ga = gapp + (size_t)GA * i;
            const double o_ = 1.0 / (1.0 + exp(-logit[i]));
            dlogit[i] = ga[0] * o_ * (1.0 - o_);
            for (int k = 0; k < 3; ++k) dcolor[(size_t)k * n + i] = ga[1 + k];
            for (int f = 0; f < F; ++f) dfeat[(size_t)f * n + i] = ga[4 + f];
        }
    }
    /* 4. pose twist per view (Supp. B.1), left perturbation Exp(xi) T_CW:
     *    dL/drho = sum g,  dL/dphi = sum [p x g + 2 (Sc G - G Sc)_{(12, 20, 01)}] */
    if (flags & 2) {
        for (int v = 0; v < V; ++v) {
            const double* vw = views + (size_t)v * VSTRIDE;
            double tw[6] = {0, 0, 0, 0, 0, 0};
            for (int i = 0; i < n; ++i) {
                const size_t o = (size_t)v * n + i;
                const double* gc = gcam + 3 * o;
                const double* G6 = Gcam + 6 * o;
                if (gc[0] == 0 && gc[1] == 0 && gc[2] == 0 && G6[0] == 0 && G6[1] == 0 && G6[2] == 0 &&
                    G6[3] == 0 && G6[4] == 0 && G6[5] == 0)
                    continue;
                double m[3], l[3], q[4];
                load_gauss(n, i, mu, ls, quat, m, l, q);
                geom_t g;
                geom64(m, l, q, logit[i], vw, (double)cfg[C_BLUR], &g);
                const double G[9] = {G6[0], G6[1], G6[2], G6[1], G6[3], G6[4], G6[2], G6[4], G6[5]};
                double SG[9], GS[9];
                mat3_mul(g.Sc, G, SG);
                mat3_mul(G, g.Sc, GS);
                const double* p = g.p;
                tw[0] += gc[0];
                tw[1] += gc[1];
                tw[2] += gc[2];
                tw[3] += p[1] * gc[2] - p[2] * gc[1] + 2.0 * (SG[5] - GS[5]);
                tw[4] += p[2] * gc[0] - p[0] * gc[2] + 2.0 * (SG[6] - GS[6]);
                tw[5] += p[0] * gc[1] - p[1] * gc[0] + 2.0 * (SG[1] - GS[1]);
            }
            for (int k = 0; k < 6; ++k) twist[6 * v + k] = tw[k];
        }
    } else {
        for (int k = 0; k < 6 * V; ++k) twist[k] = 0.0;
    }
    free_ctx(&s);
}

/* ------------------------------------------------------------------------- */
/* Debug access to the FP64 geometry of one (view, Gaussian) pair, used by   */
/* the closed-form pins: out = p[3], Sigma[9], Sigma_c[9], Sigma2D[3],        */
/* Rq[9], o  (34 doubles).                                                    */
/* ------------------------------------------------------------------------- */
void orc_geom(const double* mu, const double* ls, const double* q, double logit, const double* view,
              const float* cfg, double* out) {
    geom_t g;
    geom64(mu, ls, q, logit, view, (double)cfg[C_BLUR], &g);
    memcpy(out, g.p, 3 * sizeof(double));
    memcpy(out + 3, g.Sig, 9 * sizeof(double));
    memcpy(out + 12, g.Sc, 9 * sizeof(double));
    memcpy(out + 21, g.S2, 3 * sizeof(double));
    memcpy(out + 24, g.Rq, 9 * sizeof(double));
    out[33] = g.o;
}

/* The decision-path exponential, exposed for its accuracy pin. */
void orc_dec_exp(int n, const float* x, float* y) {
    for (int i = 0; i < n; ++i) y[i] = dec_expf(x[i]);
}

/* test hooks of the decision-path logarithm and box size */
void orc_dec_log(int n, const float* x, float* y) {
    for (int i = 0; i < n; ++i) y[i] = dec_logf(x[i]);
}

void orc_box_k(int n, const float* logit, float alpha_min, float* k) {
    for (int i = 0; i < n; ++i) k[i] = box_k(logit[i], alpha_min);
}

/* ========================================================================= */
/* SLAM-loss extensions of the image-space losses (Sec. 3.3.1, Eq. (11);     */
/* Sec. 3.3.4, Eq. (15); Sec. 3.4, Eq. (21)).                                 */
/*   - the median depth error of a view (the reference value of both masks), */
/*   - the masks M_obs (Eq. 21) and M_unobs (Eq. 11),                         */
/*   - the colour term (1 - lambda) L1 + lambda (1 - SSIM) of Eq. (15),       */
/*   - every term optionally weighted per pixel by M_obs (Eq. 21).            */
/* Every decision (the depth residual that is ranked, the mask tests) is     */
/* taken in binary32 on the binary32 roundings of the inputs; the values     */
/* (losses, gradients, SSIM) are FP64.                                        */
/* ========================================================================= */

static int cmp_u32(const void* a, const void* b) {
    const uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* binary32 depth residual |fl(D - D*)| of one pixel */
static float depth_residual32(double d, double dt) {
    const float a = (float)d, b = (float)dt;
    const float r = a - b;
    return fabsf(r);
}

/* Median depth error of one view: over its pixels with a valid observed
 * depth (D* > 0), the lower median (rank floor((m - 1) / 2) of m, counted
 * from 0) of the binary32 residuals, ranked by their bit patterns (the
 * float order for non-negative values; a NaN ranks above +inf).  0 if no
 * pixel has a valid depth. */
float orc_depth_median(int64_t n, const double* depth, const double* depth_t) {
    uint32_t* u = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!((float)depth_t[i] > 0.0f)) continue;
        const float r = depth_residual32(depth[i], depth_t[i]);
        uint32_t b;
        memcpy(&b, &r, 4);
        u[m++] = b;
    }
    float med = 0.0f;
    if (m > 0) {
        qsort(u, (size_t)m, sizeof(uint32_t), cmp_u32);
        memcpy(&med, &u[(m - 1) / 2], 4);
    }
    free(u);
    return med;
}

/* Masks of one pixel, binary32 tests:
 *   bit 0  M_obs   = (O > tau_obs) and (r < obs_factor * med)            Eq. (21)
 *   bit 1  M_unobs = (O < tau_unobs) or (D > D* and r > unobs_factor * med)  Eq. (11) */
static int pixel_masks(double d, double dt, double op, float med, float tau_obs, float tau_unobs,
                       float obs_factor, float unobs_factor) {
    const float r = depth_residual32(d, dt);
    const float o = (float)op, df = (float)d, dtf = (float)dt;
    const float lim_obs = obs_factor * med, lim_unobs = unobs_factor * med;
    const int obs = (o > tau_obs) && (r < lim_obs);
    const int unobs = (o < tau_unobs) || ((df > dtf) && (r > lim_unobs));
    return obs | (unobs << 1);
}

/* The SSIM window of Wang et al. (2004) as used by Eq. (15): 11 x 11
 * samples of a Gaussian of standard deviation 1.5 pixels centred on the
 * pixel, scaled to sum to 1. */
static void ssim_window(double w[11][11]) {
    double tot = 0.0;
    for (int a = 0; a < 11; ++a)
        for (int b = 0; b < 11; ++b) {
            const double da = a - 5, db = b - 5;
            w[a][b] = exp(-(da * da + db * db) / (2.0 * 1.5 * 1.5));
            tot += w[a][b];
        }
    for (int a = 0; a < 11; ++a)
        for (int b = 0; b < 11; ++b) w[a][b] /= tot;
}

#define SSIM_C1 (0.01 * 0.01)
#define SSIM_C2 (0.03 * 0.03)

/* SSIM of one channel of one W x H image at pixel (i, j) (row i), with
 * zero padding outside the image: local means, variances and covariance
 * under the window, then
 *   s = (2 mx my + C1)(2 cxy + C2) / ((mx^2 + my^2 + C1)(vx + vy + C2)).
 * Also the partial derivatives of s with respect to the three windowed sums
 * that depend on x: mx = sum w x, sxx = sum w x^2, sxy = sum w x y (each
 * taken with the other two fixed; vx = sxx - mx^2, cxy = sxy - mx my). */
static double ssim_at(int W, int H, const double* x, const double* y, int i, int j, const double w[11][11],
                      double* d_mx, double* d_sxx, double* d_sxy) {
    double mx = 0, my = 0, sxx = 0, syy = 0, sxy = 0;
    for (int a = -5; a <= 5; ++a) {
        const int ii = i + a;
        if (ii < 0 || ii >= H) continue;
        for (int b = -5; b <= 5; ++b) {
            const int jj = j + b;
            if (jj < 0 || jj >= W) continue;
            const double wt = w[a + 5][b + 5];
            const double xv = x[(size_t)ii * W + jj], yv = y[(size_t)ii * W + jj];
            mx += wt * xv;
            my += wt * yv;
            sxx += wt * xv * xv;
            syy += wt * yv * yv;
            sxy += wt * xv * yv;
        }
    }
    const double vx = sxx - mx * mx, vy = syy - my * my, cxy = sxy - mx * my;
    const double N1 = 2.0 * mx * my + SSIM_C1, N2 = 2.0 * cxy + SSIM_C2;
    const double D1 = mx * mx + my * my + SSIM_C1, D2 = vx + vy + SSIM_C2;
    const double s = (N1 * N2) / (D1 * D2);
    if (d_mx) {
        /* dN1/dmx = 2 my, dN2/dmx = -2 my, dD1/dmx = 2 mx, dD2/dmx = -2 mx */
        *d_mx = (2.0 * my * N2 - 2.0 * my * N1) / (D1 * D2) - s * (2.0 * mx) / D1 + s * (2.0 * mx) / D2;
        *d_sxx = -s / D2;            /* dD2/dsxx = 1 */
        *d_sxy = 2.0 * N1 / (D1 * D2); /* dN2/dsxy = 2 */
    }
    return s;
}

/* SSIM map of one channel (exposed for the closed-form pins). */
void orc_ssim_map(int W, int H, const double* x, const double* y, double* s) {
    double w[11][11];
    ssim_window(w);
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) s[(size_t)i * W + j] = ssim_at(W, H, x, y, i, j, w, NULL, NULL, NULL);
}

/* sum_p m(p) (1 - s(p)) over one channel, and coef * d/dx(q) of
 * sum_p m(p) s(p) added into g: with mx(p) = sum_o w(o) x(p + o),
 *   d mx(p) / d x(q) = w(q - p),  d sxx(p) / d x(q) = 2 w(q - p) x(q),
 *   d sxy(p) / d x(q) = w(q - p) y(q). */
static double ssim_channel(int W, int H, const double* x, const double* y, const uint8_t* m, double coef,
                           double* g) {
    double w[11][11];
    ssim_window(w);
    const size_t n = (size_t)W * H;
    double* dm = (double*)calloc(n, sizeof(double));
    double* dxx = (double*)calloc(n, sizeof(double));
    double* dxy = (double*)calloc(n, sizeof(double));
    double sum = 0.0;
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            const size_t p = (size_t)i * W + j;
            if (m && !m[p]) continue;
            double a, b, c;
            const double s = ssim_at(W, H, x, y, i, j, w, &a, &b, &c);
            sum += 1.0 - s;
            dm[p] = a;
            dxx[p] = b;
            dxy[p] = c;
        }
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            const size_t q = (size_t)i * W + j;
            double acc = 0.0;
            for (int a = -5; a <= 5; ++a) {
                const int pi = i - a; /* q - p = (a, b) */
                if (pi < 0 || pi >= H) continue;
                for (int b = -5; b <= 5; ++b) {
                    const int pj = j - b;
                    if (pj < 0 || pj >= W) continue;
                    const size_t p = (size_t)pi * W + pj;
                    const double wt = w[a + 5][b + 5];
                    acc += wt * (dm[p] + 2.0 * x[q] * dxx[p] + y[q] * dxy[p]);
                }
            }
            g[q] += coef * acc;
        }
    free(dm);
    free(dxx);
    free(dxy);
    return sum;
}

/* SLAM loss of V views and its gradient d L / d out.
 *   wh[2v], wh[2v+1]: width and height of view v (its pixels are the next
 *     W*H of the planar images, row-major);
 *   norm_count[v]: the P_v the view's means divide by (normally W*H);
 *   opts: w0, w1, w2 (lambda_c, lambda_d, lambda_s), lambda (Eq. 15),
 *     tau_obs, tau_unobs, obs_factor, unobs_factor, use_obs (0/1);
 *   med_in: per-view median depth errors to use, or NULL to compute them
 *     (orc_depth_median); med_out[V] receives the ones used.
 * Per view, with M(p) = M_obs(p) if use_obs else 1:
 *   colour L1  (1 - lambda) w0 / (3 P_v) sum_p M(p) sum_c |C_c - C*_c|
 *   SSIM       lambda w0 / (3 P_v) sum_c sum_p M(p) (1 - s_c(p))
 *   depth      w1 / P_v sum_p M(p) |D - D*|
 *   semantic   w2 / P_v sum_p M(p) CE(softmax(W^T F), label)
 * terms[5] = (colour L1, SSIM, depth, semantic, total) summed over views;
 * masks[p] = M_obs | M_unobs << 1; grad_out [5+F][P] (opacity channel 0). */
void orc_slam_loss2(int F, int K, int V, const int32_t* wh, const int64_t* norm_count, const double* out,
                    const double* rgb_t, const double* depth_t, const int32_t* labels, const double* Wd,
                    const double* bias, const double* opts, const float* med_in, float* med_out, uint8_t* masks,
                    double* grad_out, double* terms, double* gW, double* gb);

/* Semantic term of one pixel through the decoder z = W^T f + b (a 1x1
 * convolution standing in for F_cnn, Eq. 8) and its gradient with respect
 * to the logits, dz[K]:
 *   CE  (bce = 0): -log softmax(z)[lab]
 *   BCE (bce = 1, Eq. 16): -sum_k [y_k log p_k + (1 - y_k) log(1 - p_k)],
 *       p = softmax(z), y the one-hot label, each log clamped at -100 (a
 *       clamped log contributes no gradient). */
static double sem_term(int F, int K, const double* f, const double* Wd, const double* bias, int lab, int bce,
                       double* dz) {
    double z[1024], pk[1024], mx = -INFINITY;
    for (int k = 0; k < K; ++k) {
        double acc = bias ? bias[k] : 0.0;
        for (int i = 0; i < F; ++i) acc += Wd[(size_t)i * K + k] * f[i];
        z[k] = acc;
        if (acc > mx) mx = acc;
    }
    double se = 0;
    for (int k = 0; k < K; ++k) se += exp(z[k] - mx);
    for (int k = 0; k < K; ++k) pk[k] = exp(z[k] - mx) / se;
    if (!bce) {
        for (int k = 0; k < K; ++k) dz[k] = pk[k] - (k == lab ? 1.0 : 0.0);
        return (mx + log(se)) - z[lab];
    }
    /* dL/dp_k, then dL/dz_j = p_j (dL/dp_j - sum_k p_k dL/dp_k) */
    double L = 0.0, dp[1024], s = 0.0;
    for (int k = 0; k < K; ++k) {
        const double y = (k == lab) ? 1.0 : 0.0;
        const double lp = log(pk[k]), lq = log(1.0 - pk[k]);
        const double cp = lp > -100.0 ? lp : -100.0, cq = lq > -100.0 ? lq : -100.0;
        L -= y * cp + (1.0 - y) * cq;
        dp[k] = (y != 0.0 && lp > -100.0 ? -y / pk[k] : 0.0) + (y != 1.0 && lq > -100.0 ? (1.0 - y) / (1.0 - pk[k]) : 0.0);
        s += pk[k] * dp[k];
    }
    for (int k = 0; k < K; ++k) dz[k] = pk[k] * (dp[k] - s);
    return L;
}

void orc_slam_loss(int F, int K, int V, const int32_t* wh, const int64_t* norm_count, const double* out,
                   const double* rgb_t, const double* depth_t, const int32_t* labels, const double* Wd,
                   const double* opts, const float* med_in, float* med_out, uint8_t* masks, double* grad_out,
                   double* terms) {
    orc_slam_loss2(F, K, V, wh, norm_count, out, rgb_t, depth_t, labels, Wd, NULL, opts, med_in, med_out, masks,
                   grad_out, terms, NULL, NULL);
}

/* As orc_slam_loss, with a decoder bias (NULL = 0), opts[9] = 1 for BCE
 * instead of CE, and the decoder gradients: gW [F][K] = sum over pixels of
 * w_sem / P_v * M(p) f(p) dz(p)^T and gb [K] the same without f (either may
 * be NULL). */
void orc_slam_loss2(int F, int K, int V, const int32_t* wh, const int64_t* norm_count, const double* out,
                    const double* rgb_t, const double* depth_t, const int32_t* labels, const double* Wd,
                    const double* bias, const double* opts, const float* med_in, float* med_out, uint8_t* masks,
                    double* grad_out, double* terms, double* gW, double* gb) {
    int64_t P = 0;
    for (int v = 0; v < V; ++v) P += (int64_t)wh[2 * v] * wh[2 * v + 1];
    const int NC = 5 + F;
    memset(grad_out, 0, sizeof(double) * (size_t)NC * P);
    const double w0 = opts[0], w1 = opts[1], w2 = opts[2], lam = opts[3];
    const float tau_obs = (float)opts[4], tau_unobs = (float)opts[5];
    const float fobs = (float)opts[6], funobs = (float)opts[7];
    const int use_obs = opts[8] != 0.0;
    const int bce = opts[9] != 0.0;
    if (gW) memset(gW, 0, sizeof(double) * (size_t)F * K);
    if (gb) memset(gb, 0, sizeof(double) * (size_t)K);
    double T[5] = {0, 0, 0, 0, 0};
    int64_t base = 0;
    for (int v = 0; v < V; ++v) {
        const int W = wh[2 * v], H = wh[2 * v + 1];
        const int64_t Pv = (int64_t)W * H;
        const double nv = (double)norm_count[v];
        const float med =
            med_in ? med_in[v] : orc_depth_median(Pv, out + 3 * (size_t)P + base, depth_t + base);
        med_out[v] = med;
        uint8_t* mv = masks + base;
        for (int64_t j = 0; j < Pv; ++j) {
            const int64_t p = base + j;
            mv[j] = (uint8_t)pixel_masks(out[3 * (size_t)P + p], depth_t[p], out[4 * (size_t)P + p], med, tau_obs,
                                         tau_unobs, fobs, funobs);
        }
        const double gc = (1.0 - lam) * w0 / (3.0 * nv), gd = w1 / nv, gs = w2 / nv;
        double lc = 0, ld = 0, lsum = 0;
        for (int64_t j = 0; j < Pv; ++j) {
            const int64_t p = base + j;
            const double M = use_obs ? (double)(mv[j] & 1) : 1.0;
            if (M == 0.0) continue;
            for (int ch = 0; ch < 3; ++ch) {
                const double r = out[(size_t)ch * P + p] - rgb_t[(size_t)ch * P + p];
                lc += fabs(r);
                grad_out[(size_t)ch * P + p] = r > 0 ? gc : (r < 0 ? -gc : 0.0);
            }
            const double rd = out[3 * (size_t)P + p] - depth_t[p];
            ld += fabs(rd);
            grad_out[3 * (size_t)P + p] = rd > 0 ? gd : (rd < 0 ? -gd : 0.0);
            if (K > 0 && F > 0 && w2 != 0.0) {
                double fv[1024], dz[1024];
                for (int f = 0; f < F; ++f) fv[f] = out[(size_t)(5 + f) * P + p];
                lsum += sem_term(F, K, fv, Wd, bias, labels[p], bce, dz);
                for (int f = 0; f < F; ++f) {
                    double g = 0;
                    for (int k = 0; k < K; ++k) g += Wd[(size_t)f * K + k] * dz[k];
                    grad_out[(size_t)(5 + f) * P + p] = gs * g;
                }
                if (gW)
                    for (int f = 0; f < F; ++f)
                        for (int k = 0; k < K; ++k) gW[(size_t)f * K + k] += gs * fv[f] * dz[k];
                if (gb)
                    for (int k = 0; k < K; ++k) gb[k] += gs * dz[k];
            }
        }
        double ls = 0.0;
        if (lam != 0.0) {
            uint8_t* m = NULL;
            if (use_obs) {
                m = (uint8_t*)malloc((size_t)Pv);
                for (int64_t j = 0; j < Pv; ++j) m[j] = mv[j] & 1;
            }
            const double coef = -lam * w0 / (3.0 * nv);
            for (int ch = 0; ch < 3; ++ch)
                ls += ssim_channel(W, H, out + (size_t)ch * P + base, rgb_t + (size_t)ch * P + base, m, coef,
                                   grad_out + (size_t)ch * P + base);
            free(m);
        }
        T[0] += gc * lc;
        T[1] += lam * w0 * ls / (3.0 * nv);
        T[2] += gd * ld;
        T[3] += gs * lsum;
        base += Pv;
    }
    terms[0] = T[0];
    terms[1] = T[1];
    terms[2] = T[2];
    terms[3] = T[3];
    terms[4] = T[0] + T[1] + T[2] + T[3];
}

/* ========================================================================= */
/* Map growth and scale regularisation (Sec. 3.3.1-3.3.2).                    */
/* ========================================================================= */

/* Adaptive expansion (Sec. 3.3.1 with the initialisation of Sec. 3.3.2):
 * every pixel with M_unobs (masks bit 1) and an observed depth D* > 0 adds
 * one Gaussian, in (view, row, column) order, appended at index n0, n0 + 1,
 * ... while below `capacity`:
 *   mean: the pixel centre (u + 1/2, v + 1/2) unprojected at D*:
 *     x_c = ((u + 1/2 - cx) / fx * D*, (v + 1/2 - cy) / fy * D*, D*),
 *     mu = R^T (x_c - t) for the view's world-to-camera [R|t];
 *   colour: the observed colour C*(p); features: feat_init[.][p] (random
 *   numbers drawn by the caller); opacity 0.5 (logit 0); log-scale
 *   log(D* / fx) on all three axes; rotation the identity (1, 0, 0, 0).
 * Arrays are structure-of-arrays with `capacity` columns.  Returns the number
 * of candidate pixels (the new count is min(n0 + that, capacity)). */
int64_t orc_expand(int F, int V, const double* views, const uint8_t* masks, const double* rgb_t,
                   const double* depth_t, const double* feat_init, int64_t n0, int64_t capacity, double* mu,
                   double* ls, double* quat, double* logit, double* color, double* feat) {
    int64_t P = 0;
    for (int v = 0; v < V; ++v) P += (int64_t)views[VSTRIDE * v] * (int64_t)views[VSTRIDE * v + 1];
    int64_t base = 0, cnt = 0;
    for (int v = 0; v < V; ++v) {
        const double* vw = views + VSTRIDE * v;
        const int W = (int)vw[0], H = (int)vw[1];
        const double fx = vw[2], fy = vw[3], cx = vw[4], cy = vw[5];
        const double* R = vw + 6;
        const double* t = vw + 15;
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                const int64_t p = base + (int64_t)y * W + x;
                const double d = depth_t[p];
                if (!((masks[p] >> 1) & 1) || !((float)d > 0.0f)) continue;
                const int64_t i = n0 + cnt++;
                if (i >= capacity) continue;
                const double xc[3] = {(x + 0.5 - cx) / fx * d, (y + 0.5 - cy) / fy * d, d};
                const double r[3] = {xc[0] - t[0], xc[1] - t[1], xc[2] - t[2]};
                for (int a = 0; a < 3; ++a) {
                    mu[(size_t)a * capacity + i] = R[a] * r[0] + R[3 + a] * r[1] + R[6 + a] * r[2];
                    ls[(size_t)a * capacity + i] = log(d / fx);
                    color[(size_t)a * capacity + i] = rgb_t[(size_t)a * P + p];
                }
                quat[i] = 1.0;
                quat[(size_t)capacity + i] = 0.0;
                quat[(size_t)2 * capacity + i] = 0.0;
                quat[(size_t)3 * capacity + i] = 0.0;
                logit[i] = 0.0;
                for (int f = 0; f < F; ++f) feat[(size_t)f * capacity + i] = feat_init[(size_t)f * P + p];
            }
        base += (int64_t)W * H;
    }
    return cnt;
}

/* Depth-adaptive scale regularisation, Eq. (12), over the 3n per-axis
 * scales s = exp(log s) (binary32, by the decision-path exponential dec_expf
 * as in the projection, so that both sides hold the same samples):
 *   mu_s, sigma_s = mean and population standard deviation of the samples,
 *   s_big = mu_s + 2 sigma_s, s_small = mu_s - 2 sigma_s,
 *   L_big = mean of s over the samples with s > s_big,
 *   L_small = mean of -log s over the samples with s < s_small,
 * each 0 when its set is empty; loss = w_big L_big + w_small L_small.
 * The thresholds and counts are constants of the gradient (they only move
 * the set boundaries): d loss / d log s = w_big s / n_big on the big set,
 * -w_small / n_small on the small set; added into grad_ls (may be NULL).
 * out[7] = (L_big, L_small, loss, mu_s, sigma_s, n_big, n_small). */
void orc_dsr(int64_t n, const float* log_scale, double w_big, double w_small, double* grad_ls, double* out) {
    const int64_t m = 3 * n;
    double sum = 0.0;
    for (int64_t j = 0; j < m; ++j) sum += (double)dec_expf(log_scale[j]);
    const double mean = m > 0 ? sum / (double)m : 0.0;
    double ss = 0.0;
    for (int64_t j = 0; j < m; ++j) {
        const double e = (double)dec_expf(log_scale[j]) - mean;
        ss += e * e;
    }
    const double sd = m > 0 ? sqrt(ss / (double)m) : 0.0;
    const double big = mean + 2.0 * sd, small = mean - 2.0 * sd;
    double sb = 0.0, sm = 0.0;
    int64_t nb = 0, ns = 0;
    for (int64_t j = 0; j < m; ++j) {
        const double s = (double)dec_expf(log_scale[j]);
        if (s > big) {
            sb += s;
            ++nb;
        }
        if (s < small) {
            sm += -log(s);
            ++ns;
        }
    }
    const double Lb = nb > 0 ? sb / (double)nb : 0.0, Ls = ns > 0 ? sm / (double)ns : 0.0;
    if (grad_ls)
        for (int64_t j = 0; j < m; ++j) {
            const double s = (double)dec_expf(log_scale[j]);
            if (s > big) grad_ls[j] += w_big * s / (double)nb;
            if (s < small) grad_ls[j] += -w_small / (double)ns;
        }
    out[0] = Lb;
    out[1] = Ls;
    out[2] = w_big * Lb + w_small * Ls;
    out[3] = mean;
    out[4] = sd;
    out[5] = (double)nb;
    out[6] = (double)ns;
}

/* ========================================================================= */
/* Optimiser steps of the SLAM loop (Supp. C.1 learning rates).              */
/* ========================================================================= */

/* Adam (Kingma and Ba, 2015) on n values with bias correction at step t
 * (from 1): m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
 * p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
void orc_adam(int64_t n, double* p, const double* g, double* m, double* v, double lr, double b1, double b2,
              double eps, int t) {
    const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}

/* SE(3) exponential of a twist (rho, phi) (translation first) as a 3x4
 * [R|t]: R = I + (sin th / th) [phi]x + ((1 - cos th) / th^2) [phi]x^2,
 * t = (I + ((1 - cos th) / th^2) [phi]x + ((th - sin th) / th^3) [phi]x^2) rho,
 * th = |phi| (series near 0). */
void orc_se3_exp(const double* xi, double* Rt) {
    const double* rho = xi;
    const double* phi = xi + 3;
    const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2], th = sqrt(th2);
    double A, B, C;
    if (th < 1e-4) {
        A = 1.0 - th2 / 6.0;
        B = 0.5 - th2 / 24.0;
        C = 1.0 / 6.0 - th2 / 120.0;
    } else {
        A = sin(th) / th;
        B = (1.0 - cos(th)) / th2;
        C = (th - sin(th)) / (th2 * th);
    }
    const double K[9] = {0, -phi[2], phi[1], phi[2], 0, -phi[0], -phi[1], phi[0], 0};
    double K2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += K[3 * i + k] * K[3 * k + j];
            K2[3 * i + j] = s;
        }
    for (int i = 0; i < 3; ++i) {
        double tv = 0.0;
        for (int j = 0; j < 3; ++j) {
            const double I = i == j ? 1.0 : 0.0;
            Rt[4 * i + j] = I + A * K[3 * i + j] + B * K2[3 * i + j];
            tv += (I + B * K[3 * i + j] + C * K2[3 * i + j]) * rho[j];
        }
        Rt[4 * i + 3] = tv;
    }
}

/* Tracking's pose step for V views: Adam on each view's twist gradient
 * (per-component learning rate lr_rho for the translation part, lr_phi for
 * the rotation part), then the left update T <- Exp(dxi) T of the view's
 * world-to-camera [R|t] (Rt [V][12], row-major 3x4). */
void orc_pose_step(int V, double* Rt, const double* grad, double* m, double* v, double lr_rho, double lr_phi,
                   double b1, double b2, double eps, int t) {
    const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int w = 0; w < V; ++w) {
        double dxi[6];
        for (int k = 0; k < 6; ++k) {
            const int i = 6 * w + k;
            m[i] = b1 * m[i] + (1.0 - b1) * grad[i];
            v[i] = b2 * v[i] + (1.0 - b2) * grad[i] * grad[i];
            dxi[k] = -(k < 3 ? lr_rho : lr_phi) * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
        }
        double E[12], T[12];
        orc_se3_exp(dxi, E);
        memcpy(T, Rt + 12 * w, sizeof(T));
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 4; ++j) {
                double s = j == 3 ? E[4 * i + 3] : 0.0;
                for (int k = 0; k < 3; ++k) s += E[4 * i + k] * T[4 * k + j];
                Rt[12 * w + 4 * i + j] = s;
            }
        }
    }
}
