// SLAM losses of GS^3LAM with their masks (Sec. 3.3.1, Eq. 11; Sec. 3.3.4,
// Eq. 15-18; Sec. 3.4, Eq. 21), all on the device and graph-capturable:
//
//   1. median depth error per view: the lower median of the binary32
//      residuals r = |D - D*| over the pixels with D* > 0, found exactly by
//      a radix select over the residual bits (non-negative floats order as
//      their bit patterns): four passes of 8 bits, each a histogram of the
//      digit among the residuals that match the prefix selected so far
//      (k_median_hist), then one block per view that locates the bucket
//      holding the wanted rank (k_median_select).  Integer counts only, so
//      the result is the same every run.
//   2. one thread per pixel (k_slam_loss): the masks M_obs (Eq. 21) and
//      M_unobs (Eq. 11) from binary32 tests, then the L1
//      colour and depth terms and the semantic cross-entropy, each weighted
//      by M_obs when the tracking mask is on, with their gradients.
//   3. with lambda > 0, the SSIM part of Eq. (15)'s colour term: per colour
//      channel and 64x16 output tile, k_ssim_fwd filters x, y, x^2, y^2 and
//      xy with the separable 11-tap Gaussian (sigma 1.5) over the tile plus
//      a 5-pixel apron staged in LDS (zero outside the view), forms SSIM and
//      its partial derivatives with respect to the three windowed sums that
//      depend on x, and writes them, scaled, as three maps; k_ssim_bwd
//      filters the maps again (the window is symmetric, so the adjoint is the
//      same filter) and adds G*m_mu + 2 x G*m_xx + y G*m_xy to the colour
//      gradient.  Both walk the tiles persistently, loading the next tile
//      while the current one is filtered.
//   4. a fixed-order sum of the per-block partial losses (deterministic).
#include "loss_common.h"

namespace sgs {

namespace {

constexpr int kSlamThreads = 256;
constexpr int kMedItems = 16;  // pixels per thread in a histogram block
constexpr int kMedChunk = kSlamThreads * kMedItems;
constexpr int kSsimTX = 64, kSsimTY = 16, kSsimR = 5;  // output tile, window radius
constexpr int kSsimIX = kSsimTX + 2 * kSsimR, kSsimIY = kSsimTY + 2 * kSsimR;

struct SlamParams {
    float w0, w1, w2, lam;
    float tau_obs, tau_unobs, obs_factor, unobs_factor;
    int use_obs, bce;
};

struct SsimConst {
    float g[2 * kSsimR + 1];  // 1-D window; the 2-D window is g[a] g[b]
    float c1, c2, lam_w0;     // lambda * w_color
};

// First SSIM tile of each view (tiles of kSsimTX x kSsimTY, row-major per view).
struct SsimTiles {
    int first[GS_MAX_VIEWS + 1];
    int n_views;
};

__device__ __forceinline__ int view_of_pixel(const gs_view* views, int n_views, int64_t p) {
    int v = 0;
    while (v + 1 < n_views && views[v + 1].pixel_offset <= p) ++v;
    return v;
}

// ---------------------------------------------------------------------------
// 1. median depth error
// ---------------------------------------------------------------------------
// sel[4 v + 0..2]: selected prefix, rank still wanted within it, number of
// valid pixels of the view.
template <int PASS>
__global__ void __launch_bounds__(kSlamThreads) k_median_hist(const float* __restrict__ depth,
                                                              const float* __restrict__ depth_t,
                                                              const gs_view* __restrict__ views,
                                                              uint32_t* __restrict__ hist,
                                                              const uint32_t* __restrict__ sel) {
    constexpr int shift = 24 - 8 * PASS;
    __shared__ uint32_t h[256];
    const int v = blockIdx.y, tid = threadIdx.x, lane = tid & (kWave - 1);
    const int64_t off = views[v].pixel_offset;
    const int64_t Pv = (int64_t)views[v].width * views[v].height;
    const int64_t b0 = (int64_t)blockIdx.x * kMedChunk;
    if (b0 >= Pv) return;  // uniform over the block
    uint32_t prefix = 0;
    if constexpr (PASS > 0) {
        if (sel[4 * v + 2] == 0) return;  // no valid pixel in the view
        prefix = sel[4 * v];
    }
    h[tid] = 0;
    __syncthreads();
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    // every load first (index clamped into the view), then the decisions
    float dtv[kMedItems], dv[kMedItems];
#pragma unroll
    for (int k = 0; k < kMedItems; ++k) {
        const int64_t j = b0 + k * kSlamThreads + tid;
        const int64_t jc = j < Pv ? j : Pv - 1;
        dtv[k] = depth_t[off + jc];
        dv[k] = depth[off + jc];
    }
#pragma unroll
    for (int k = 0; k < kMedItems; ++k) {
        const int64_t j = b0 + k * kSlamThreads + tid;
        const uint32_t u = __float_as_uint(fabsf(dv[k] - dtv[k]));
        bool ok = j < Pv && dtv[k] > 0.0f;
        if constexpr (PASS > 0) ok = ok && (u >> (shift + 8)) == prefix;
        const uint32_t d = (u >> shift) & 0xffu;
        if (__builtin_amdgcn_ballot_w64(ok) == 0) continue;  // uniform
        // one LDS add per distinct digit of the wavefront (the residuals of
        // a view mostly share a few top digits)
        const uint64_t peers = match_digit(d, ok);
        if (ok && (peers & below) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    if (h[tid] != 0) atomicAdd(&hist[256 * v + tid], h[tid]);
}

template <int PASS>
__global__ void __launch_bounds__(256) k_median_select(uint32_t* __restrict__ hist, uint32_t* __restrict__ sel,
                                                      float* __restrict__ med_ws, float* __restrict__ med_out) {
    __shared__ uint32_t s_tmp[256 / kWave];
    const int v = blockIdx.x, tid = threadIdx.x;
    const uint32_t c = hist[256 * v + tid];
    hist[256 * v + tid] = 0;  // cleared for the next pass (or the next call)
    uint32_t total;
    const uint32_t excl = block_exclusive<256>(c, s_tmp, &total);
    uint32_t prefix = 0, rank, count;
    if constexpr (PASS == 0) {
        count = total;
        rank = count > 0 ? (count - 1) / 2 : 0;
    } else {
        prefix = sel[4 * v];
        rank = sel[4 * v + 1];
        count = sel[4 * v + 2];
    }
    __syncthreads();  // every thread has read sel before one of them rewrites it
    const bool mine = count > 0 && excl <= rank && rank < excl + c;  // exactly one thread when count > 0
    if (mine) {
        sel[4 * v] = (prefix << 8) | (uint32_t)tid;
        sel[4 * v + 1] = rank - excl;
    }
    if (PASS == 0 && tid == 0) sel[4 * v + 2] = count;
    if constexpr (PASS == 3) {
        // the selected residual (whatever its bits), or 0 for a view without
        // a valid depth
        if (mine || (count == 0 && tid == 0)) {
            const float m = mine ? __uint_as_float((prefix << 8) | (uint32_t)tid) : 0.0f;
            med_ws[v] = m;
            if (med_out != nullptr) med_out[v] = m;
        }
    }
}

// ---------------------------------------------------------------------------
// 2. per-pixel masks, L1 terms and cross-entropy
// ---------------------------------------------------------------------------
// Semantic term of one pixel through the decoder z = W^T f + b (a 1x1
// convolution standing in for F_cnn, Eq. 8), K <= KC classes, logits in
// registers.  Returns the term and leaves dz = dterm/dz in z:
//   CE:  -log p_lab,  dz = p - y;
//   BCE (Eq. 16): -sum_k [y_k log p_k + (1 - y_k) log(1 - p_k)], each log
//   clamped at -100 (no gradient through a clamped log); dz_j = p_j (dp_j -
//   sum_k p_k dp_k) with dp_k the derivative in p_k.
// A class row of Wt is wavefront-uniform: scalar loads feeding the FMAs.
template <int F, int KC>
__device__ __forceinline__ float sem_dz(const float (&fv)[F], const float* __restrict__ Wt,
                                        const float* __restrict__ bias, int K, int lab, bool bce, float (&z)[KC]) {
    // z = W^T f + b, then in place z - max (the only per-class state kept,
    // so that the logits cost one register per class)
    float m = -INFINITY;
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        if (k < K) {
            const float* wr = Wt + k * F;
            float acc = bias != nullptr ? bias[k] : 0.0f;
#pragma unroll
            for (int f = 0; f < F; ++f) acc = fmaf(wr[f], fv[f], acc);
            z[k] = acc;
            m = fmaxf(m, acc);
        }
    }
    float se = 0.0f;
#pragma unroll
    for (int k = 0; k < KC; ++k)
        if (k < K) {
            z[k] -= m;
            se += __expf(z[k]);
        }
    const float inv = 1.0f / se, lse = __logf(se);
    float L = 0.0f;
    if (!bce) {
#pragma unroll
        for (int k = 0; k < KC; ++k)
            if (k < K) {
                if (k == lab) L = lse - z[k];
                z[k] = __expf(z[k]) * inv - (k == lab ? 1.0f : 0.0f);  // dz
            }
        return L;
    }
    // BCE: p_k, log p_k = z_k - lse, log(1 - p_k) = log(se - e_k) - lse;
    // z keeps p_k and one bit per class whether the log that class's
    // gradient uses is above the clamp, so dp_k = -1/p_k (label) or
    // 1/(1 - p_k) (other classes, hardware reciprocals) is rebuilt in the
    // last pass without another exp or log
    float sdp = 0.0f;
    uint64_t live = 0;
#pragma unroll
    for (int k = 0; k < KC; ++k)
        if (k < K) {
            const bool y = k == lab;
            const float e = __expf(z[k]), pk = e * inv;
            const float lp = z[k] - lse;            // log p_k
            const float lq = __logf(se - e) - lse;  // log(1 - p_k)
            L -= y ? fmaxf(lp, -100.0f) : fmaxf(lq, -100.0f);
            const bool on = y ? lp > -100.0f : lq > -100.0f;
            const float dp = on ? (y ? -__builtin_amdgcn_rcpf(pk) : __builtin_amdgcn_rcpf(1.0f - pk)) : 0.0f;
            sdp = fmaf(pk, dp, sdp);
            z[k] = pk;
            live |= (uint64_t)on << k;
        }
#pragma unroll
    for (int k = 0; k < KC; ++k)
        if (k < K) {
            const float pk = z[k];
            const float dp = ((live >> k) & 1) ? (k == lab ? -__builtin_amdgcn_rcpf(pk)
                                                            : __builtin_amdgcn_rcpf(1.0f - pk))
                                               : 0.0f;
            z[k] = pk * (dp - sdp);  // dz
        }
    return L;
}

// Decoder-gradient staging (dynamic LDS, only when the decoder gradients
// are wanted): one slot per wavefront of 32 pixel rows, f [32][F] then the
// scaled dz [32][K]; a wavefront stages and contracts its 64 pixels in two
// halves, so the area is 4 * 32 * (F + K) floats (at most 48 KiB).
constexpr int kDecRows = kWave / 2;
inline size_t dec_lds_bytes(int F, int K) { return (size_t)4 * kDecRows * (F + K) * sizeof(float); }

// MODE: kSemCE the fused cross-entropy (no decoder gradients; fewest
// registers), kSemDz the semantic term through dz (BCE), kSemDzDec the same
// plus the decoder gradients.
constexpr int kSemCE = 0, kSemDz = 1, kSemDzDec = 2;

template <int F, int KC, int MODE>
__global__ void __launch_bounds__(kSlamThreads) k_slam_loss(const float* __restrict__ out, int64_t P,
                                                            const float* __restrict__ rgb_t,
                                                            const float* __restrict__ depth_t,
                                                            const int32_t* __restrict__ labels,
                                                            const float* __restrict__ Wt,
                                                            const float* __restrict__ bias, int K, SlamParams sp,
                                                            const float* __restrict__ med,
                                                            const gs_view* __restrict__ views, int n_views,
                                                            float* __restrict__ grad_out,
                                                            uint8_t* __restrict__ masks,
                                                            double* __restrict__ partials,
                                                            float* __restrict__ dec_partials) {
    extern __shared__ float s_dyn[];
    __shared__ double s_red[3][kSlamThreads / kWave];
    __shared__ float s_db[kSlamThreads / kWave][KC > 0 ? KC : 1];  // per-wavefront bias sums
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int64_t p = (int64_t)blockIdx.x * kSlamThreads + tid;
    double lc = 0.0, ld = 0.0, ls = 0.0;
    float fv[F > 0 ? F : 1], dz[KC > 0 ? KC : 1];
    float dscale = 0.0f;  // w_sem / P_v * M(p) for the decoder gradients (0: no contribution)
    if (p < P) {
        double pc = 0.0, pd = 0.0, ps = 0.0;
        const int v = view_of_pixel(views, n_views, p);
        const float Pv = (float)((int64_t)views[v].width * views[v].height);
        const float d = out[3 * P + p], dt = depth_t[p], o = out[4 * P + p];
        // Eq. (21) / Eq. (11), binary32 tests
        const float r = fabsf(d - dt), m = med[v];
        const float lim_obs = sp.obs_factor * m, lim_unobs = sp.unobs_factor * m;
        const bool obs = (o > sp.tau_obs) && (r < lim_obs);
        const bool unobs = (o < sp.tau_unobs) || ((d > dt) && (r > lim_unobs));
        masks[p] = (uint8_t)((obs ? 1 : 0) | (unobs ? 2 : 0));
        const bool on = !sp.use_obs || obs;
        const float gc = (1.0f - sp.lam) * sp.w0 / (3.0f * Pv), gd = sp.w1 / Pv, gs = sp.w2 / Pv;
        if (on) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const float rc = out[ch * P + p] - rgb_t[ch * P + p];
                pc += (double)fabsf(rc);
                grad_out[ch * P + p] = rc > 0.0f ? gc : (rc < 0.0f ? -gc : 0.0f);
            }
            const float rd = d - dt;
            pd += (double)fabsf(rd);
            grad_out[3 * P + p] = rd > 0.0f ? gd : (rd < 0.0f ? -gd : 0.0f);
        } else {
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) grad_out[ch * P + p] = 0.0f;
        }
        grad_out[4 * P + p] = 0.0f;
        if constexpr (F > 0) {
            float gf[F];
#pragma unroll
            for (int f = 0; f < F; ++f) gf[f] = 0.0f;
#pragma unroll
            for (int f = 0; f < F; ++f) fv[f] = 0.0f;
            if (on && K > 0 && sp.w2 != 0.0f) {
#pragma unroll
                for (int f = 0; f < F; ++f) fv[f] = out[(5 + f) * P + p];
                if constexpr (MODE == kSemCE) {
                    ps = (double)semantic_ce<F, KC>(fv, Wt, K, labels[p], gf, bias);
                } else {
                    ps = (double)sem_dz<F, KC>(fv, Wt, bias, K, labels[p], sp.bce != 0, dz);
                    // dL/df = W dz
#pragma unroll
                    for (int k = 0; k < KC; ++k)
                        if (k < K) {
                            const float* wr = Wt + k * F;
#pragma unroll
                            for (int f = 0; f < F; ++f) gf[f] = fmaf(wr[f], dz[k], gf[f]);
                        }
                    dscale = gs;
                }
            }
#pragma unroll
            for (int f = 0; f < F; ++f) grad_out[(5 + f) * P + p] = gs * gf[f];
        }
        lc = pc * (double)gc;
        ld = pd * ((double)sp.w1 / (double)Pv);
        ls = ps * ((double)sp.w2 / (double)Pv);
    }
    // decoder gradients of the workgroup: dW = sum_p dscale_p f_p dz_p^T and
    // db = sum_p dscale_p dz_p.  The contraction over a wavefront's 64
    // pixels runs on MFMA (16x16x4 f32: four pixels per step; A[m][k] = f of
    // pixel k at row m, B[k][n] = scaled dz of pixel k at class n), the four
    // wavefronts' tiles and bias sums are then added in a fixed order.
    if constexpr (MODE == kSemDzDec && F > 0 && KC > 0) {
        constexpr int MT = (F + 15) / 16, NT = KC / 16;
        float* sF = s_dyn + wave * kDecRows * (F + K);  // [32][F]
        float* sZ = sF + kDecRows * F;                  // [32][K]
        using f4 = __attribute__((__vector_size__(4 * sizeof(float)))) float;
        f4 acc[MT][NT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
        const int col = lane & 15, kk = lane >> 4, row = lane & (kDecRows - 1);
        const bool c = dscale != 0.0f;
        float db = 0.0f;  // lane n < K: bias sum of this wavefront, rows in a fixed order
        for (int half = 0; half < 2; ++half) {
            if ((lane >> 5) == half) {
#pragma unroll
                for (int f = 0; f < F; ++f) sF[row * F + f] = c ? fv[f] : 0.0f;
#pragma unroll
                for (int k = 0; k < KC; ++k)
                    if (k < K) sZ[row * K + k] = c ? dscale * dz[k] : 0.0f;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // 8 steps of four pixels: A[m][k] = f of pixel k at row m, B[k][n]
            // = scaled dz of pixel k at class n (zero past F and K)
#pragma unroll 2
            for (int st = 0; st < kDecRows / 4; ++st) {
                const int pr = 4 * st + kk;
                float a[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const int m = col + 16 * mt;
                    a[mt] = m < F ? sF[pr * F + m] : 0.0f;
                }
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const int n = col + 16 * nt;
                    const float bv = n < K ? sZ[pr * K + n] : 0.0f;
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
                        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mt], bv, acc[mt][nt], 0, 0, 0);
                }
            }
            if (lane < K) {
                float t0 = 0.0f, t1 = 0.0f, t2 = 0.0f, t3 = 0.0f;  // four chains
                for (int r = 0; r < kDecRows; r += 4) {
                    t0 += sZ[r * K + lane];
                    t1 += sZ[(r + 1) * K + lane];
                    t2 += sZ[(r + 2) * K + lane];
                    t3 += sZ[(r + 3) * K + lane];
                }
                db += (t0 + t1) + (t2 + t3);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (lane < KC) s_db[wave][lane] = db;
        __syncthreads();  // every wavefront is done with its slot
        // D[m][n] with m = 4 (lane / 16) + i, n = lane % 16 per tile, into the
        // freed slots as [wave][F][K]
        float* sD = s_dyn + wave * F * K;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int mm = 16 * mt + 4 * kk + i, nn = 16 * nt + col;
                    if (mm < F && nn < K) sD[mm * K + nn] = acc[mt][nt][i];
                }
        __syncthreads();
        const int T = F * K + K;  // this workgroup's partial: dW [F][K], then db [K]
        float* dst = dec_partials + (size_t)blockIdx.x * T;
        for (int e = tid; e < F * K; e += kSlamThreads) {
            float t = 0.0f;
#pragma unroll
            for (int w = 0; w < kSlamThreads / kWave; ++w) t += s_dyn[w * F * K + e];
            dst[e] = t;
        }
        if (tid < K) {
            float t = 0.0f;
#pragma unroll
            for (int w = 0; w < kSlamThreads / kWave; ++w) t += s_db[w][tid];
            dst[F * K + tid] = t;
        }
    }
    for (int dd = kWave / 2; dd > 0; dd >>= 1) {
        lc += __shfl_xor(lc, dd, kWave);
        ld += __shfl_xor(ld, dd, kWave);
        ls += __shfl_xor(ls, dd, kWave);
    }
    if (lane == 0) {
        s_red[0][wave] = lc;
        s_red[1][wave] = ld;
        s_red[2][wave] = ls;
    }
    __syncthreads();
    if (tid < 3) {
        double a = 0;
        for (int w = 0; w < kSlamThreads / kWave; ++w) a += s_red[tid][w];
        partials[(size_t)tid * gridDim.x + blockIdx.x] = a;  // term-major
    }
}

// ---------------------------------------------------------------------------
// 3. SSIM term
// ---------------------------------------------------------------------------
struct TileIdx {
    int v, x0, y0, W, H;
};
__device__ __forceinline__ TileIdx ssim_tile(const SsimTiles& st, const gs_view* views, int t) {
    int v = 0;
    while (v + 1 < st.n_views && st.first[v + 1] <= t) ++v;
    TileIdx ti;
    ti.v = v;
    ti.W = views[v].width;
    ti.H = views[v].height;
    const int tx = ceil_div(ti.W, kSsimTX);
    const int lt = t - st.first[v];
    ti.x0 = (lt % tx) * kSsimTX;
    ti.y0 = (lt / tx) * kSsimTY;
    return ti;
}

// Staged input of one tile: rows of the output tile plus a kSsimR apron
// above and below, kSsimIX columns (the tile plus the apron left and right)
// padded to kSsimLD so that every row starts 16-byte aligned.
constexpr int kSsimLD = (kSsimIX + 3) / 4 * 4;
// horizontal pass: a thread slides the window over kSsimHX consecutive
// outputs of one staged row; vertical pass: over kSsimVY rows of one column
constexpr int kSsimHX = 8;
constexpr int kSsimVY = kSsimTY / (kSlamThreads / kSsimTX);
static_assert(kSsimTX % kSsimHX == 0 && kSsimIY * (kSsimTX / kSsimHX) <= kSlamThreads, "one horizontal item per thread");
static_assert(kSsimHX + 2 * kSsimR <= kSsimLD - kSsimHX * (kSsimTX / kSsimHX - 1), "horizontal window inside the row");

// n consecutive floats of an LDS row from a 16-byte aligned start
template <int N>
__device__ __forceinline__ void lds_row(const float* __restrict__ src, float (&v)[N]) {
    static_assert(N % 4 == 0, "whole float4");
#pragma unroll
    for (int k = 0; k < N / 4; ++k) {
        const float4 a = reinterpret_cast<const float4*>(src)[k];
        v[4 * k] = a.x;
        v[4 * k + 1] = a.y;
        v[4 * k + 2] = a.z;
        v[4 * k + 3] = a.w;
    }
}
constexpr int kSsimHN = (kSsimHX + 2 * kSsimR + 3) / 4 * 4;  // floats read per horizontal item (18 -> 20)

// Stages rows [y0 - R, y0 + TY + R) x columns [x0 - R, x0 + TX + R) of NP
// planes into LDS, zero outside the view (and in the row padding).
// Work items of the persistent SSIM kernels: (channel, tile) pairs, item =
// c * ntiles + t.  With a grid of 8k workgroups, XCD x (the workgroups whose
// linear id is x mod 8: the dispatcher places them round-robin) takes the
// x-th of eight contiguous chunks of items and its k workgroups stride
// through it, so the tiles in flight on one XCD are neighbours and share
// their aprons (and row-end cache lines) in its L2.  Other grid sizes stride
// over all items.
struct ItemWalk {
    int first, stride, end;
    __device__ explicit ItemWalk(int nitems) {
        const int G = gridDim.x, b = blockIdx.x;
        if (G >= 8 && (G & 7) == 0) {
            const int chunk = (nitems + 7) / 8, x = b & 7;
            first = x * chunk + (b >> 3);
            stride = G >> 3;
            end = min((x + 1) * chunk, nitems);
        } else {
            first = b;
            stride = G;
            end = nitems;
        }
    }
};

// Staging of one tile in two halves: ssim_load issues every global load of
// the thread into registers (one memory round trip, and in flight while the
// previous tile is filtered), ssim_store writes them to LDS.
constexpr int kSsimN = kSsimIY * kSsimLD, kSsimIT = (kSsimN + kSlamThreads - 1) / kSlamThreads;
template <int NP>
__device__ __forceinline__ void ssim_load(const float* const (&src)[NP], const TileIdx& ti, float (&v)[kSsimIT][NP]) {
#pragma unroll
    for (int it = 0; it < kSsimIT; ++it) {
        const int i = it * kSlamThreads + threadIdx.x;
        const int r = i / kSsimLD, q = i - r * kSsimLD;
        const int gy = ti.y0 - kSsimR + r, gx = ti.x0 - kSsimR + q;
        const bool in = i < kSsimN && q < kSsimIX && gx >= 0 && gx < ti.W && gy >= 0 && gy < ti.H;
        const int64_t o = in ? (int64_t)gy * ti.W + gx : 0;
#pragma unroll
        for (int k = 0; k < NP; ++k) v[it][k] = in ? src[k][o] : 0.0f;
    }
}
template <int NP>
__device__ __forceinline__ void ssim_store(const float (&v)[kSsimIT][NP], float (*dst)[kSsimIY][kSsimLD]) {
#pragma unroll
    for (int it = 0; it < kSsimIT; ++it) {
        const int i = it * kSlamThreads + threadIdx.x;
        if (i < kSsimN) {
            const int r = i / kSsimLD, q = i - r * kSsimLD;
#pragma unroll
            for (int k = 0; k < NP; ++k) dst[k][r][q] = v[it][k];
        }
    }
}

// maps: [3 channels][3 maps][P]: m_mu, m_xx, m_xy, each coef * M(p) * the
// partial derivative of SSIM(p) (coef = -lambda w0 / (3 P_v)).  Persistent:
// each workgroup walks (channel, tile) items (ItemWalk).
__global__ void __launch_bounds__(kSlamThreads) k_ssim_fwd(const float* __restrict__ out,
                                                           const float* __restrict__ rgb_t, int64_t P,
                                                           const gs_view* __restrict__ views, SsimTiles st,
                                                           SsimConst sc, const uint8_t* __restrict__ masks,
                                                           int use_obs, float* __restrict__ maps,
                                                           double* __restrict__ partials) {
    __shared__ __align__(16) float sxy[2][kSsimIY][kSsimLD];  // x, y
    __shared__ __align__(16) float hs[5][kSsimIY][kSsimTX];   // horizontal sums of x, y, xx, yy, xy
    __shared__ double s_red[kSlamThreads / kWave];
    const int tid = threadIdx.x;
    const int ntiles = st.first[st.n_views];
    const ItemWalk iw(3 * ntiles);
    double acc = 0.0;  // sum of lambda w0 / (3 P_v) M(p) (1 - s(p)) over this thread's outputs
    const int q = tid % kSsimTX, r0 = (tid / kSsimTX) * kSsimVY;  // vertical-pass outputs of the thread
    // one tile's global data: staged x, y and M(p) at the thread's outputs
    // (every load of a tile goes out together: the wait for any of them is
    // a wait for all, counts being in order)
    float pre[kSsimIT][2], mkn[kSsimVY];
    auto load_tile = [&](const TileIdx& tl, int ch) {
        const int64_t b = views[tl.v].pixel_offset;
        const float* const src[2] = {out + ch * P + b, rgb_t + ch * P + b};
        ssim_load<2>(src, tl, pre);
        const int gx = tl.x0 + q;
#pragma unroll
        for (int j = 0; j < kSsimVY; ++j) {
            const int gy = tl.y0 + r0 + j;
            // the mask plane is always written, so the load is unconditional
            const bool in = gx < tl.W && gy < tl.H;
            const uint8_t mb = masks[b + (in ? (int64_t)gy * tl.W + gx : 0)];
            mkn[j] = (!use_obs || (mb & 1)) ? 1.0f : 0.0f;
        }
    };
    int it = iw.first;
    int c = it < iw.end ? it / ntiles : 0;
    TileIdx ti = ssim_tile(st, views, it < iw.end ? it - c * ntiles : 0);
    if (it < iw.end) load_tile(ti, c);
    for (; it < iw.end; it += iw.stride) {
        const int64_t base = views[ti.v].pixel_offset;
        __syncthreads();  // the previous tile's readers of sxy and hs are done
        ssim_store<2>(pre, sxy);
        float mk[kSsimVY];
#pragma unroll
        for (int j = 0; j < kSsimVY; ++j) mk[j] = mkn[j];
        __syncthreads();
        // the next item's loads fly while this one is filtered
        const int itn = it + iw.stride;
        const int cn = itn < iw.end ? itn / ntiles : c;
        const TileIdx tin = ssim_tile(st, views, itn < iw.end ? itn - cn * ntiles : 0);
        if (itn < iw.end) load_tile(tin, cn);
        // horizontal: item (row r, outputs h0 .. h0 + HX - 1)
        if (tid < kSsimIY * (kSsimTX / kSsimHX)) {
            const int r = tid / (kSsimTX / kSsimHX), h0 = (tid - r * (kSsimTX / kSsimHX)) * kSsimHX;
            float xv[kSsimHN], yv[kSsimHN];
            lds_row<kSsimHN>(&sxy[0][r][h0], xv);
            lds_row<kSsimHN>(&sxy[1][r][h0], yv);
            float a[5][kSsimHX];
#pragma unroll
            for (int j = 0; j < kSsimHX; ++j)
#pragma unroll
                for (int k = 0; k < 5; ++k) a[k][j] = 0.0f;
#pragma unroll
            for (int i = 0; i < kSsimHX + 2 * kSsimR; ++i) {
                const float x = xv[i], y = yv[i], xx = x * x, yy = y * y, xy = x * y;
#pragma unroll
                for (int j = 0; j < kSsimHX; ++j) {
                    const int tp = i - j;  // tap of input i for output j
                    if (tp >= 0 && tp <= 2 * kSsimR) {
                        const float w = sc.g[tp];
                        a[0][j] = fmaf(w, x, a[0][j]);
                        a[1][j] = fmaf(w, y, a[1][j]);
                        a[2][j] = fmaf(w, xx, a[2][j]);
                        a[3][j] = fmaf(w, yy, a[3][j]);
                        a[4][j] = fmaf(w, xy, a[4][j]);
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < 5; ++k)
#pragma unroll
                for (int j = 0; j < kSsimHX; j += 4)
                    *reinterpret_cast<float4*>(&hs[k][r][h0 + j]) =
                        make_float4(a[k][j], a[k][j + 1], a[k][j + 2], a[k][j + 3]);
        }
        __syncthreads();
        // vertical: column q, output rows r0 .. r0 + VY - 1
        const int gx = ti.x0 + q;
        float m[5][kSsimVY];
#pragma unroll
        for (int j = 0; j < kSsimVY; ++j)
#pragma unroll
            for (int k = 0; k < 5; ++k) m[k][j] = 0.0f;
#pragma unroll
        for (int i = 0; i < kSsimVY + 2 * kSsimR; ++i) {
            float h[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) h[k] = hs[k][r0 + i][q];
#pragma unroll
            for (int j = 0; j < kSsimVY; ++j) {
                const int tp = i - j;
                if (tp >= 0 && tp <= 2 * kSsimR) {
                    const float w = sc.g[tp];
#pragma unroll
                    for (int k = 0; k < 5; ++k) m[k][j] = fmaf(w, h[k], m[k][j]);
                }
            }
        }
        const float Pv = (float)((int64_t)ti.W * ti.H);
        const float coef = -sc.lam_w0 / (3.0f * Pv);
        float part = 0.0f;
#pragma unroll
        for (int j = 0; j < kSsimVY; ++j) {
            const int gy = ti.y0 + r0 + j;
            if (gx < ti.W && gy < ti.H) {
                const int64_t p = (int64_t)gy * ti.W + gx;
                const float mx = m[0][j], my = m[1][j];
                const float vx = m[2][j] - mx * mx, vy = m[3][j] - my * my, cxy = m[4][j] - mx * my;
                const float N1 = 2.0f * mx * my + sc.c1, N2 = 2.0f * cxy + sc.c2;
                const float D1 = mx * mx + my * my + sc.c1, D2 = vx + vy + sc.c2;
                // hardware reciprocals: ~1 ulp, far inside the loss tolerance
                const float iD1 = __builtin_amdgcn_rcpf(D1), iD2 = __builtin_amdgcn_rcpf(D2);
                const float iD12 = iD1 * iD2;
                const float s = N1 * N2 * iD12;
                const float k1 = coef * mk[j];
                // partials of s with the other two windowed sums fixed
                const float d_mu = 2.0f * my * (N2 - N1) * iD12 + 2.0f * mx * s * (iD2 - iD1);
                const float d_xx = -s * iD2;
                const float d_xy = 2.0f * N1 * iD12;
                float* mp = maps + (size_t)(3 * c) * P + base + p;
                mp[0] = k1 * d_mu;
                mp[P] = k1 * d_xx;
                mp[2 * P] = k1 * d_xy;
                part += mk[j] * (1.0f - s);
            }
        }
        acc += (double)part * ((double)sc.lam_w0 / (3.0 * (double)Pv));
        ti = tin;
        c = cn;
    }
    const int lane = tid & (kWave - 1), wave = tid / kWave;
    for (int dd = kWave / 2; dd > 0; dd >>= 1) acc += __shfl_xor(acc, dd, kWave);
    if (lane == 0) s_red[wave] = acc;
    __syncthreads();
    if (tid == 0) {
        double a = 0;
        for (int w = 0; w < kSlamThreads / kWave; ++w) a += s_red[w];
        partials[blockIdx.x] = a;
    }
}

__global__ void __launch_bounds__(kSlamThreads) k_ssim_bwd(const float* __restrict__ out,
                                                           const float* __restrict__ rgb_t, int64_t P,
                                                           const gs_view* __restrict__ views, SsimTiles st,
                                                           SsimConst sc, const float* __restrict__ maps,
                                                           float* __restrict__ grad_out) {
    __shared__ __align__(16) float sm[3][kSsimIY][kSsimLD];
    __shared__ __align__(16) float hs[3][kSsimIY][kSsimTX];
    const int tid = threadIdx.x;
    const int ntiles = st.first[st.n_views];
    const ItemWalk iw(3 * ntiles);
    const int q = tid % kSsimTX, r0 = (tid / kSsimTX) * kSsimVY;  // vertical-pass outputs of the thread
    // one tile's global data: the staged maps, and x, y and the gradient so
    // far at the thread's outputs (loaded together, see k_ssim_fwd)
    float pre[kSsimIT][3], xn[kSsimVY], yn[kSsimVY], gn[kSsimVY];
    auto load_tile = [&](const TileIdx& tl, int ch) {
        const int64_t b = views[tl.v].pixel_offset;
        const float* M = maps + (size_t)(3 * ch) * P + b;
        const float* const src[3] = {M, M + P, M + 2 * P};
        ssim_load<3>(src, tl, pre);
        const int gx = tl.x0 + q;
#pragma unroll
        for (int j = 0; j < kSsimVY; ++j) {
            const int gy = tl.y0 + r0 + j;
            const bool in = gx < tl.W && gy < tl.H;
            const int64_t p = b + (in ? (int64_t)gy * tl.W + gx : 0);
            xn[j] = in ? out[ch * P + p] : 0.0f;
            yn[j] = in ? rgb_t[ch * P + p] : 0.0f;
            gn[j] = in ? grad_out[ch * P + p] : 0.0f;
        }
    };
    int it = iw.first;
    int c = it < iw.end ? it / ntiles : 0;
    TileIdx ti = ssim_tile(st, views, it < iw.end ? it - c * ntiles : 0);
    if (it < iw.end) load_tile(ti, c);
    for (; it < iw.end; it += iw.stride) {
        const int64_t base = views[ti.v].pixel_offset;
        __syncthreads();
        ssim_store<3>(pre, sm);
        float xv[kSsimVY], yv[kSsimVY], gv[kSsimVY];
#pragma unroll
        for (int j = 0; j < kSsimVY; ++j) {
            xv[j] = xn[j];
            yv[j] = yn[j];
            gv[j] = gn[j];
        }
        __syncthreads();
        const int itn = it + iw.stride;
        const int cn = itn < iw.end ? itn / ntiles : c;
        const TileIdx tin = ssim_tile(st, views, itn < iw.end ? itn - cn * ntiles : 0);
        if (itn < iw.end) load_tile(tin, cn);
        if (tid < kSsimIY * (kSsimTX / kSsimHX)) {
            const int r = tid / (kSsimTX / kSsimHX), h0 = (tid - r * (kSsimTX / kSsimHX)) * kSsimHX;
            float a[3][kSsimHX];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                float v[kSsimHN];
                lds_row<kSsimHN>(&sm[k][r][h0], v);
#pragma unroll
                for (int j = 0; j < kSsimHX; ++j) {
                    float acc = 0.0f;
#pragma unroll
                    for (int tp = 0; tp <= 2 * kSsimR; ++tp) acc = fmaf(sc.g[tp], v[j + tp], acc);
                    a[k][j] = acc;
                }
            }
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int j = 0; j < kSsimHX; j += 4)
                    *reinterpret_cast<float4*>(&hs[k][r][h0 + j]) =
                        make_float4(a[k][j], a[k][j + 1], a[k][j + 2], a[k][j + 3]);
        }
        __syncthreads();
        const int gx = ti.x0 + q;
        float b[3][kSsimVY];
#pragma unroll
        for (int j = 0; j < kSsimVY; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) b[k][j] = 0.0f;
#pragma unroll
        for (int i = 0; i < kSsimVY + 2 * kSsimR; ++i) {
            float h[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) h[k] = hs[k][r0 + i][q];
#pragma unroll
            for (int j = 0; j < kSsimVY; ++j) {
                const int tp = i - j;
                if (tp >= 0 && tp <= 2 * kSsimR) {
#pragma unroll
                    for (int k = 0; k < 3; ++k) b[k][j] = fmaf(sc.g[tp], h[k], b[k][j]);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kSsimVY; ++j) {
            const int gy = ti.y0 + r0 + j;
            if (gx < ti.W && gy < ti.H) {
                const int64_t p = base + (int64_t)gy * ti.W + gx;
                grad_out[c * P + p] = gv[j] + (b[0][j] + 2.0f * xv[j] * b[1][j] + yv[j] * b[2][j]);
            }
        }
        ti = tin;
        c = cn;
    }
}

// ---------------------------------------------------------------------------
// 4. fixed-order sum: loss = (colour L1, SSIM, depth, semantic, total)
// ---------------------------------------------------------------------------
// stage: the first-stage sums of the pixel kernel's (colour, depth,
// semantic) partials, term-major [3][nst]; ssim: the SSIM kernel's per-block
// partials.  One block; every sum in a fixed order.
__global__ void __launch_bounds__(kSumThreads) k_slam_loss_final(const double* __restrict__ stage, int nst,
                                                                 const double* __restrict__ ssim, int nssim,
                                                                 double* __restrict__ loss) {
    __shared__ double s[4][kSumThreads / kWave];
    const int t = threadIdx.x, lane = t & (kWave - 1), wave = t / kWave;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = t; i < nst; i += kSumThreads) {
        a[0] += stage[i];
        a[2] += stage[nst + i];
        a[3] += stage[2 * (size_t)nst + i];
    }
    for (int i = t; i < nssim; i += kSumThreads) a[1] += ssim[i];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        for (int d = kWave / 2; d > 0; d >>= 1) a[k] += __shfl_xor(a[k], d, kWave);
        if (lane == 0) s[k][wave] = a[k];
    }
    __syncthreads();
    if (t == 0) {
        double r[4];
        for (int k = 0; k < 4; ++k) {
            r[k] = 0.0;
            for (int w = 0; w < kSumThreads / kWave; ++w) r[k] += s[k][w];
            loss[k] = r[k];
        }
        loss[4] = ((r[0] + r[1]) + r[2]) + r[3];
    }
}

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Pixel-kernel grid: one thread per pixel.
unsigned slam_blocks(int64_t P) { return (unsigned)((P + kSlamThreads - 1) / kSlamThreads); }

struct SlamWs {
    size_t hist, sel, med, part, spart, stage, wt, mask, maps, dpart, dstage, total;
};

int ssim_tiles(const gs_view* views, int n_views, SsimTiles* st) {
    int t = 0;
    for (int v = 0; v < n_views; ++v) {
        if (st) st->first[v] = t;
        t += ceil_div(views[v].width, kSsimTX) * ceil_div(views[v].height, kSsimTY);
    }
    if (st) {
        st->first[n_views] = t;
        st->n_views = n_views;
    }
    return t;
}

// Decoder-gradient reduction: the pixel kernel's block partials, block-major
// [nblk][T] floats (T = F K + K), are summed in fixed order by chunks of
// kRowChunk rows (k_rows_stage, doubles [nchunk][T]), then over the chunks
// (k_rows_final).
constexpr int kRowChunk = 512;
int row_chunks(int64_t nblk) { return (int)((nblk + kRowChunk - 1) / kRowChunk); }

SlamWs slam_layout(int64_t P, const gs_view* views, int n_views, bool ssim, int dec_terms) {
    SlamWs L;
    size_t o = 0;
    L.hist = o;
    o += align256((size_t)n_views * 256 * 4);
    L.sel = o;
    o += align256((size_t)n_views * 4 * 4);
    L.med = o;
    o += align256((size_t)n_views * 4);
    const int64_t nblk = slam_blocks(P);
    L.part = o;
    o += align256((size_t)nblk * 3 * 8);
    const int nt = ssim ? ssim_tiles(views, n_views, nullptr) : 0;
    L.spart = o;
    o += align256((size_t)(3 * nt + 8) * 8);  // one partial per SSIM workgroup (at most 3 nt rounded up to 8)
    L.stage = o;
    o += align256((size_t)sum_stage_blocks(nblk) * 3 * 8);
    L.wt = o;
    o += align256((size_t)32 * GS_MAX_CLASSES * 4);
    L.mask = o;
    o += align256((size_t)P);
    L.maps = o;
    if (ssim) o += align256((size_t)9 * P * 4);
    L.dpart = o;
    o += align256((size_t)nblk * dec_terms * 4);
    L.dstage = o;
    o += align256((size_t)row_chunks(nblk) * dec_terms * 8);
    L.total = o;
    return L;
}

// block (c, g): column t = 64 g + lane of rows [c kRowChunk, (c + 1) kRowChunk);
// wavefront w takes rows w, w + 4, ... of the chunk, the four sums added in
// order.
__global__ void __launch_bounds__(256) k_rows_stage(const float* __restrict__ src, int64_t nrows, int T,
                                                    double* __restrict__ dst) {
    __shared__ double s[4][kWave];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int t = blockIdx.y * kWave + lane;
    const int64_t r0 = (int64_t)blockIdx.x * kRowChunk;
    double acc = 0.0;
    if (t < T) {
        constexpr int U = 16;
        for (int j0 = 0; j0 < kRowChunk / 4; j0 += U) {
            float x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t r = r0 + wave + 4 * (j0 + u);
                x[u] = src[(r < nrows ? r : nrows - 1) * T + t];
                x[u] = r < nrows ? x[u] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) acc += (double)x[u];
        }
    }
    s[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && t < T) dst[(size_t)blockIdx.x * T + t] = ((s[0][lane] + s[1][lane]) + s[2][lane]) + s[3][lane];
}

__global__ void __launch_bounds__(256) k_rows_final(const double* __restrict__ stage, int nchunk, int F, int K,
                                                    float* __restrict__ grad_w, float* __restrict__ grad_b) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int T = F * K + K;
    if (t >= T) return;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;  // four chains, fixed order
    int c = 0;
    for (; c + 3 < nchunk; c += 4) {
        a0 += stage[(size_t)c * T + t];
        a1 += stage[(size_t)(c + 1) * T + t];
        a2 += stage[(size_t)(c + 2) * T + t];
        a3 += stage[(size_t)(c + 3) * T + t];
    }
    for (; c < nchunk; ++c) a0 += stage[(size_t)c * T + t];
    const double a = (a0 + a1) + (a2 + a3);
    if (t < F * K) {
        if (grad_w != nullptr) grad_w[t] = (float)a;
    } else if (grad_b != nullptr) {
        grad_b[t - F * K] = (float)a;
    }
}

// Workgroups of a persistent SSIM launch: as many as are resident on the
// device at once, rounded down to a multiple of the 8 XCDs (ItemWalk), at
// least 8, at most the items rounded up to 8.
unsigned ssim_grid(const void* kern, int nitems) {
    int dev = 0, cus = 0, per_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kSlamThreads, 0);
    if (cus < 1) cus = 1;
    if (per_cu < 1) per_cu = 1;
    int g = cus * per_cu / 8 * 8;
    const int cap = (nitems + 7) / 8 * 8;
    if (g > cap) g = cap;
    return (unsigned)(g >= 8 ? g : 8);
}

template <int F, int KC>
void launch_slam_pixels(unsigned nblk, hipStream_t s, const float* out, int64_t P, const float* rgb_t,
                        const float* depth_t, const int32_t* labels, const float* Wt, const float* bias, int K,
                        const SlamParams& sp, const float* med, const gs_view* views, int n_views, float* grad_out,
                        uint8_t* masks, double* partials, float* dec_partials) {
    // the decoder-gradient path is its own instantiation, so that the plain
    // loss keeps its register budget
    const size_t lds = dec_lds_bytes(F, K);
    if (dec_partials != nullptr && F > 0)
        hipLaunchKernelGGL((k_slam_loss<F, KC, kSemDzDec>), dim3(nblk), dim3(kSlamThreads), lds, s, out, P, rgb_t,
                           depth_t, labels, Wt, bias, K, sp, med, views, n_views, grad_out, masks, partials,
                           dec_partials);
    else if (sp.bce)
        hipLaunchKernelGGL((k_slam_loss<F, KC, kSemDz>), dim3(nblk), dim3(kSlamThreads), 0, s, out, P, rgb_t, depth_t,
                           labels, Wt, bias, K, sp, med, views, n_views, grad_out, masks, partials, nullptr);
    else
        hipLaunchKernelGGL((k_slam_loss<F, KC, kSemCE>), dim3(nblk), dim3(kSlamThreads), 0, s, out, P, rgb_t, depth_t,
                           labels, Wt, bias, K, sp, med, views, n_views, grad_out, masks, partials, nullptr);
}

int dec_terms_of(int F, const gs_decoder* dec) {
    if (dec == nullptr || F == 0 || dec->n_classes == 0) return 0;
    if (dec->grad_weight == nullptr && dec->grad_bias == nullptr) return 0;
    return F * dec->n_classes + dec->n_classes;
}

template <int F>
hipError_t launch_slam_t(const float* out, const float* rgb_t, const float* depth_t, const int32_t* labels,
                         const gs_decoder* dec, const gs_slam_loss_opts& o, const gs_view* views_host,
                         const gs_view* views_dev, int n_views, int64_t P, float* grad_out, double* loss,
                         float* median, uint8_t* masks, char* ws, hipStream_t s) {
    const bool ssim = o.ssim_lambda != 0.0f;
    const int dterms = dec_terms_of(F, dec);
    const SlamWs L = slam_layout(P, views_host, n_views, ssim, dterms);
    uint32_t* hist = reinterpret_cast<uint32_t*>(ws + L.hist);
    uint32_t* sel = reinterpret_cast<uint32_t*>(ws + L.sel);
    float* med = reinterpret_cast<float*>(ws + L.med);
    double* part = reinterpret_cast<double*>(ws + L.part);
    double* spart = reinterpret_cast<double*>(ws + L.spart);
    float* Wt = reinterpret_cast<float*>(ws + L.wt);
    uint8_t* mk = masks != nullptr ? masks : reinterpret_cast<uint8_t*>(ws + L.mask);
    float* maps = reinterpret_cast<float*>(ws + L.maps);
    float* dpart = dterms > 0 ? reinterpret_cast<float*>(ws + L.dpart) : nullptr;
    double* dstage = reinterpret_cast<double*>(ws + L.dstage);

    // 1. median depth error per view
    hipError_t e = fill_u32(hist, 0u, (int64_t)n_views * (256 + 4), s);  // hist and sel are adjacent
    if (e != hipSuccess) return e;
    int64_t pmax = 0;
    for (int v = 0; v < n_views; ++v) {
        const int64_t pv = (int64_t)views_host[v].width * views_host[v].height;
        pmax = pv > pmax ? pv : pmax;
    }
    const dim3 hg((unsigned)((pmax + kMedChunk - 1) / kMedChunk), (unsigned)n_views);
    const float* dep = out + 3 * P;
    hipLaunchKernelGGL(k_median_hist<0>, hg, dim3(kSlamThreads), 0, s, dep, depth_t, views_dev, hist, sel);
    hipLaunchKernelGGL(k_median_select<0>, dim3(n_views), dim3(256), 0, s, hist, sel, med, median);
    hipLaunchKernelGGL(k_median_hist<1>, hg, dim3(kSlamThreads), 0, s, dep, depth_t, views_dev, hist, sel);
    hipLaunchKernelGGL(k_median_select<1>, dim3(n_views), dim3(256), 0, s, hist, sel, med, median);
    hipLaunchKernelGGL(k_median_hist<2>, hg, dim3(kSlamThreads), 0, s, dep, depth_t, views_dev, hist, sel);
    hipLaunchKernelGGL(k_median_select<2>, dim3(n_views), dim3(256), 0, s, hist, sel, med, median);
    hipLaunchKernelGGL(k_median_hist<3>, hg, dim3(kSlamThreads), 0, s, dep, depth_t, views_dev, hist, sel);
    hipLaunchKernelGGL(k_median_select<3>, dim3(n_views), dim3(256), 0, s, hist, sel, med, median);

    // 2. masks, L1 and the semantic term (with the decoder gradients' block partials)
    SlamParams sp;
    sp.w0 = o.w_color;
    sp.w1 = o.w_depth;
    sp.w2 = o.w_sem;
    sp.lam = o.ssim_lambda;
    sp.tau_obs = o.tau_obs;
    sp.tau_unobs = o.tau_unobs;
    sp.obs_factor = o.obs_factor;
    sp.unobs_factor = o.unobs_factor;
    sp.use_obs = (o.flags & GS_LOSS_OBS_MASK) != 0;
    sp.bce = (o.flags & GS_LOSS_BCE) != 0;
    const int K = dec != nullptr ? dec->n_classes : 0;
    const bool sem = F > 0 && K > 0 && sp.w2 != 0.0f;
    if (sem)
        hipLaunchKernelGGL(k_transpose_decoder, dim3((unsigned)ceil_div(F * K, 256)), dim3(256), 0, s, dec->weight,
                           F, K, Wt);
    const unsigned nblk = slam_blocks(P);
    const int Ke = sem ? K : 0;
    const float* bias = sem ? dec->bias : nullptr;
    float* dp = sem ? dpart : nullptr;
    if (Ke > 32)
        launch_slam_pixels<F, 64>(nblk, s, out, P, rgb_t, depth_t, labels, Wt, bias, Ke, sp, med, views_dev, n_views,
                                  grad_out, mk, part, dp);
    else
        launch_slam_pixels<F, 32>(nblk, s, out, P, rgb_t, depth_t, labels, Wt, bias, Ke, sp, med, views_dev, n_views,
                                  grad_out, mk, part, dp);
    if (dterms > 0) {
        // dL/dW and dL/db (zero when the semantic term is off)
        if (!sem) {
            e = fill_u32(reinterpret_cast<uint32_t*>(dpart), 0u, (int64_t)nblk * dterms, s);
            if (e != hipSuccess) return e;
        }
        const int nch = row_chunks(nblk);
        hipLaunchKernelGGL(k_rows_stage, dim3((unsigned)nch, (unsigned)ceil_div(dterms, kWave)), dim3(256), 0, s,
                           dpart, (int64_t)nblk, dterms, dstage);
        hipLaunchKernelGGL(k_rows_final, dim3((unsigned)ceil_div(dterms, 256)), dim3(256), 0, s, dstage, nch, F,
                           dec->n_classes, dec->grad_weight, dec->grad_bias);
    }

    // 3. SSIM
    int nssim = 0;
    if (ssim) {
        SsimTiles st;
        const int nt = ssim_tiles(views_host, n_views, &st);
        SsimConst sc;
        double g[2 * kSsimR + 1], tot = 0.0;
        for (int t = 0; t <= 2 * kSsimR; ++t) {
            const double d = t - kSsimR;
            g[t] = exp(-d * d / (2.0 * 1.5 * 1.5));
            tot += g[t];
        }
        for (int t = 0; t <= 2 * kSsimR; ++t) sc.g[t] = (float)(g[t] / tot);
        sc.c1 = (float)(0.01 * 0.01);
        sc.c2 = (float)(0.03 * 0.03);
        sc.lam_w0 = o.ssim_lambda * o.w_color;
        // persistent grids walking the (channel, tile) items
        const unsigned gf = ssim_grid(reinterpret_cast<const void*>(&k_ssim_fwd), 3 * nt);
        const unsigned gb = ssim_grid(reinterpret_cast<const void*>(&k_ssim_bwd), 3 * nt);
        if (nt > 0) {
            hipLaunchKernelGGL(k_ssim_fwd, dim3(gf), dim3(kSlamThreads), 0, s, out, rgb_t, P, views_dev, st, sc, mk,
                               sp.use_obs, maps, spart);
            hipLaunchKernelGGL(k_ssim_bwd, dim3(gb), dim3(kSlamThreads), 0, s, out, rgb_t, P, views_dev, st, sc, maps,
                               grad_out);
        }
        nssim = nt > 0 ? (int)gf : 0;
    }
    // 4. loss terms: the per-block partials summed in two fixed-order stages
    double* stage = reinterpret_cast<double*>(ws + L.stage);
    const int nst = sum_stage_blocks(nblk);
    hipLaunchKernelGGL(k_sum_stage, dim3((unsigned)nst), dim3(kSumThreads), 0, s, part, (int)nblk, 3, stage);
    hipLaunchKernelGGL(k_slam_loss_final, dim3(1), dim3(kSumThreads), 0, s, stage, nst, spart, nssim, loss);
    return hipGetLastError();
}

}  // namespace

size_t slam_loss_workspace_bytes(int64_t P, const gs_view* views_host, int n_views, int n_feat,
                                 const gs_decoder* dec, const gs_slam_loss_opts& o) {
    return slam_layout(P, views_host, n_views, o.ssim_lambda != 0.0f, dec_terms_of(n_feat, dec)).total;
}

hipError_t launch_slam_loss(const float* out, int n_feat, const float* rgb_t, const float* depth_t,
                            const int32_t* labels, const gs_decoder* dec, const gs_slam_loss_opts& o,
                            const gs_view* views_host, const gs_view* views_dev, int n_views, int64_t P,
                            float* grad_out, double* loss, float* median, uint8_t* masks, void* ws, hipStream_t s) {
    char* w = static_cast<char*>(ws);
    switch (n_feat) {
        case 0:
            return launch_slam_t<0>(out, rgb_t, depth_t, labels, dec, o, views_host, views_dev, n_views, P, grad_out,
                                    loss, median, masks, w, s);
        case 8:
            return launch_slam_t<8>(out, rgb_t, depth_t, labels, dec, o, views_host, views_dev, n_views, P, grad_out,
                                    loss, median, masks, w, s);
        case 32:
            return launch_slam_t<32>(out, rgb_t, depth_t, labels, dec, o, views_host, views_dev, n_views, P, grad_out,
                                     loss, median, masks, w, s);
        default:
            return launch_slam_t<16>(out, rgb_t, depth_t, labels, dec, o, views_host, views_dev, n_views, P,
                                     grad_out, loss, median, masks, w, s);
    }
}

}  // namespace sgs
