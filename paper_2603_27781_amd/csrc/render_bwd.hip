// Backward of the compositing (GS^3LAM Sec. 3.2.1-3.2.2, differentiated for
// the gradient-descent updates of Sec. 3.3.4 and 3.4).
//
// Same launch shape as the forward.  Each pixel starts from T_final and its
// `last` count and walks its tile list from the back, rebuilding the
// transmittance before every contributor by division, T_i = T_{i+1}/(1-a_i),
// instead of storing it.  With g the pixel's upstream gradient (5+F
// channels) and x_i the Gaussian's channel values (colour, depth, 1, f),
//   dL/dalpha_i = T_i (g . x_i) - sum_{j>i} (g . x_j) alpha_j T_j / (1 - alpha_i)
//               = T_i ((g . x_i) - R_i),
//   R_i = sum_{j>i} (g . x_j) alpha_j prod_{i<k<j} (1 - alpha_k)
// (one scalar per pixel), accumulated from the back as
// R_{i-1} = R_i + alpha_i ((g . x_i) - R_i): a convex combination per step,
// with no division by 1 - alpha_i, so the error of the rebuilt T_i scales
// the (small) difference instead of two large terms before they cancel;
// then through alpha = min(alpha_max, o 2^q'), q' = A'dx^2 + B2'dx dy + C'dy^2,
// to the projected mean, the conic, the opacity, and linearly to colour,
// depth and feature.  The 10+F per-Gaussian values of the 64 pixels of a
// wavefront are summed with a transposing butterfly (each exchange halves
// the values a lane keeps, so after log2 steps every lane holds a different
// total); one LDS atomic instruction per wavefront and Gaussian adds them to
// the batch's per-instance accumulator (the four wavefronts of the tile).
// Wavefronts with no contributing pixel skip the reduction.
//
// No global atomics: every (view, tile, Gaussian) instance belongs to exactly
// one tile, so after each batch the workgroup writes the instance's totals as
// one contiguous record at its emission index.  The instances of a (view,
// Gaussian) pair are contiguous in emission order, so k_reduce_records then
// sums each pair's records in a fixed order, and the scattered
// read-modify-write traffic of global atomics (which dominated this kernel)
// is replaced by streaming writes and reads.  The only order left to the
// hardware is that of the (at most TS*TS/64) wavefront totals added into an
// instance's LDS accumulator, which can change the last bits between runs.
#include "raster_common.h"

namespace sgs {

// Transposing butterfly over NV (a power of two) values per lane.  Each
// halving step, across one lane bit, halves the CNT values a lane keeps: a
// lane with the bit set keeps the upper half and receives its partner's
// upper half, the partner the opposite, and both add.  After log2(NV)
// halving steps each lane holds one partial total, and the remaining bits
// of the order finish the sum.  Two bit orders:
//   full wavefront (ORD 0): 5, 4 (permlane swaps: one swap + one add per
//     pair), 2 (DPP half-row mirror, valid because bits 0 and 1 are still
//     unused), 0, 1 (DPP quad permutations), 3 (DPP row rotation);
//   within the 16 lanes that share bits 4 and 5 (ORD 1): 2, 0, 1, 3.
// No step goes through LDS.  Every index is a compile-time constant
// (template recursion), so the values stay in registers.
template <int ORD>
__host__ __device__ constexpr int bfly_bit(int s) {
    return ORD == 0 ? (s == 0 ? 5 : (s == 1 ? 4 : (s == 2 ? 2 : (s == 3 ? 0 : (s == 4 ? 1 : 3)))))
                    : (s == 0 ? 2 : (s == 1 ? 0 : (s == 2 ? 1 : 3)));
}
template <int ORD>
__host__ __device__ constexpr int bfly_nbits() { return ORD == 0 ? 6 : 4; }

template <int D>
__device__ __forceinline__ float bfly_partner(float x) {
    if constexpr (D == 4) return mirror8_lane(x);
    else return xor_lane<D>(x);
}

// NR: the values v[NR ..] are padding.  In the first step a pair whose
// upper value is padding needs no selects: the lanes with the bit clear get
// the pair total of the lower value from one add, and the lanes with the bit
// set, which would carry the padding slot, get a value nobody reads (the
// slots never mix, so it cannot reach a real total).
template <int ORD, int NV, int CNT, int S, int NR>
struct BflyStep {
    __device__ __forceinline__ static void run(float (&v)[NV], int lane) {
        if constexpr (S < bfly_nbits<ORD>()) {
            constexpr int D = 1 << bfly_bit<ORD>(S);
            if constexpr (CNT > 1) {
                constexpr int HALF = CNT / 2;
                if constexpr (D >= 16) {
#pragma unroll
                    for (int k = 0; k < HALF; ++k) v[k] = swap_halves_add<D>(v[k], v[k + HALF]);
                } else {
                    // both pair totals (one DPP add each), then the lane's
                    // half; selecting between computed values rather than
                    // between array elements keeps the compiler from turning
                    // the selects into a lane-dependent index into v
                    const bool up = (lane & D) != 0;
#pragma unroll
                    for (int k = 0; k < HALF; ++k) {
                        const float lo = v[k] + bfly_partner<D>(v[k]);
                        if (S == 0 && k + HALF >= NR) {
                            v[k] = lo;
                        } else {
                            const float hi = v[k + HALF] + bfly_partner<D>(v[k + HALF]);
                            v[k] = up ? hi : lo;
                        }
                    }
                }
                BflyStep<ORD, NV, HALF, S + 1, NR>::run(v, lane);
            } else {
                // full reduction across this bit; the mirror partner is only
                // valid while bits 0 and 1 are unused, which holds here since
                // bit 2 comes before them in both orders
                v[0] += bfly_partner<D>(v[0]);
                BflyStep<ORD, NV, 1, S + 1, NR>::run(v, lane);
            }
        }
    }
};

template <int NV, int ORD = 0, int NR = NV>
struct Butterfly {
    static constexpr int steps() {
        int b = 0;
        while ((1 << b) < NV) ++b;
        return b;
    }
    // After the call, the lane holds in v[0] the total (over the lanes the
    // order covers) of value index slot(lane).
    __device__ __forceinline__ static float reduce(float (&v)[NV], int lane) {
        BflyStep<ORD, NV, NV, 0, NR>::run(v, lane);
        return v[0];
    }
    __device__ __forceinline__ static int slot(int lane) {
        int s = 0, cnt = NV;
#pragma unroll
        for (int st = 0; st < steps(); ++st) {
            cnt >>= 1;
            if (lane & (1 << bfly_bit<ORD>(st))) s += cnt;
        }
        return s;
    }
    // Lane bits summed over after the halving steps; lanes with all of them
    // clear hold one copy of each slot total.
    static constexpr int reduced_mask() {
        int m = 0;
        for (int st = steps(); st < bfly_nbits<ORD>(); ++st) m |= 1 << bfly_bit<ORD>(st);
        return m;
    }
};

// Sum over the 64 lanes of six values per lane, transposed: afterwards the
// lanes with bits 0, 1 and 3 clear hold one total each, of value
// geo6_slot(lane) (6: none).  Bit 5 pairs (0, 4), (1, 5) and (2, 3), so the
// lower half keeps values 0, 1, 2 and the upper half 4, 5, 3 and no swap is
// spent on padding; bit 4 pairs (a, c) and (b, dead register); bit 2 is the
// DPP half-row mirror (valid while bits 0 and 1 are unused), then bits 0, 1
// and 3 finish with DPP adds.
__device__ __forceinline__ int geo6_slot(int lane) {
    const int b5 = (lane >> 5) & 1, b4 = (lane >> 4) & 1, b2 = (lane >> 2) & 1;
    if (b4 == 0) return b2 == 0 ? 4 * b5 : 1 + 4 * b5;
    return b2 == 0 ? 2 + b5 : 6;
}

// Bits 5 and 4 of the six-value sum: afterwards a2 holds value
// A(b5, b4) = b4 ? 2 + b5 : 4 b5 and b2 value B(b5, b4) = 1 + 4 b5 (garbage
// where b4 is set), each still to be summed over bits 0-3.
__device__ __forceinline__ void geo6_bits54(const float (&v)[6], float& a2, float& b2) {
    const float a = swap_halves_add<32>(v[0], v[4]);
    const float b = swap_halves_add<32>(v[1], v[5]);
    const unsigned cu = __float_as_uint(v[2]), du = __float_as_uint(v[3]);
    const auto r = __builtin_amdgcn_permlane32_swap(cu, du, false, false);
    const float c = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    // bit 4: the second operand of b's swap is r[1], dead after the add above
    const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(c), false, false);
    a2 = __uint_as_float(p[0]) + __uint_as_float(p[1]);
    const auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(b), r[1], false, false);
    b2 = __uint_as_float(q[0]) + __uint_as_float(q[1]);
}

__device__ __forceinline__ float geo6_reduce(const float (&v)[6], int lane) {
    float a2, b2;
    geo6_bits54(v, a2, b2);
    // bit 2
    const bool up = (lane & 4) != 0;
    const float lo = a2 + mirror8_lane(a2), hi = b2 + mirror8_lane(b2);
    float t = up ? hi : lo;
    t += xor_lane<1>(t);
    t += xor_lane<2>(t);
    t += xor_lane<8>(t);
    return t;
}

// The weights w of the four lanes that share this lane's bits 0-3.  W[t] is
// w of the lane whose bits 4-5 are t: a permlane32 swap of w with itself
// gives the lanes l & ~32 and l | 32, a permlane16 swap of each of those
// with itself their bit-4 pairs.  Register swaps only: the LDS crossbar
// (ds_swizzle) would spare the three vector instructions, but the backward
// is held by LDS issue as much as by vector issue.
__device__ __forceinline__ void quad_row_weights(float w, float (&W)[4]) {
    const unsigned u = __float_as_uint(w);
    const auto h = __builtin_amdgcn_permlane32_swap(u, u, false, false);  // w(l & ~32), w(l | 32)
    const auto p0 = __builtin_amdgcn_permlane16_swap(h[0], h[0], false, false);
    const auto p1 = __builtin_amdgcn_permlane16_swap(h[1], h[1], false, false);
    W[0] = __uint_as_float(p0[0]);
    W[1] = __uint_as_float(p0[1]);
    W[2] = __uint_as_float(p1[0]);
    W[3] = __uint_as_float(p1[1]);
}

// Staged appearance records of the backward.  With parameter gradients a
// lane reads only its channels c = 4 m + q (q = lane bits 4-5); with more
// than five per lane (32 feature channels) each quarter q is staged
// contiguously, QS floats 16-byte aligned, so a step reads its NL values with
// ceil(NL / 4) wide loads instead of about NL / 2 paired ones.  Otherwise the
// record is staged as the projection wrote it.
template <int F, bool PARAMS>
struct BwdApp {
    static constexpr int AV = AppRec<F>::vec;
    static constexpr int NL = PARAMS ? (4 + F) / 4 : 0;
    static constexpr bool qmajor = PARAMS && NL > 5;
    static constexpr int QS = (NL + 3) / 4 * 4;   // floats per quarter when quarter-major
    static constexpr int vec = qmajor ? QS : AV;  // float4 per staged record
};

template <int N>
struct Pow2 {
    static constexpr int value = N <= 1 ? 1 : 2 * Pow2<(N + 1) / 2>::value;
};
template <>
struct Pow2<1> {
    static constexpr int value = 1;
};

// Geometry record values of one instance from its moments.  With h the
// per-pixel factor dL/dalpha * alpha (zero where alpha is clamped or the
// pixel does not contribute) and (dx, dy) a pixel centre from the projected
// mean, the backward accumulates S = sum_p h {1, dx, dy, dx^2, dx dy, dy^2}
// in slots 0-4 and 6; with the staged g0 = (mx, my, A', B2'),
// g1 = (C', o, ...) the record holds
//   -ln2 (2A' Sx + B2' Sy), -ln2 (B2' Sx + 2C' Sy)   (mean: -ln2 sum h dq'/ddx, ...)
//   -Sxx / 2, -Sxy, -Syy / 2                          (conic)
//   S1 / o = sum dL/dalpha G                           (opacity, alpha = o G where unclamped)
// The derivatives of q' are linear in dx and dy, so their sums follow from
// the first moments exactly; the step forms six products of h instead of
// the derivatives and their products.
__device__ __forceinline__ void moments_to_geometry(const float4& g0, const float4& g1, float* r) {
    const float s1 = r[0], sx = r[1], sy = r[2], sxx = r[3], sxy = r[4], syy = r[6];
    r[0] = -kLn2 * fmaf(2.0f * g0.z, sx, g0.w * sy);
    r[1] = -kLn2 * fmaf(g0.w, sx, 2.0f * g1.x * sy);
    r[2] = -0.5f * sxx;
    r[3] = -sxy;
    r[4] = -0.5f * syy;
    r[6] = s1 / g1.y;
}

template <int TS, int F, int B, bool PARAMS>
__device__ __forceinline__ void bwd_tile(int t, const float4* __restrict__ rec, const float4* __restrict__ app, int n,
                                         const int32_t* __restrict__ inst, const int32_t* __restrict__ inst_gid,
                                         const int2* __restrict__ ranges, const gs_view* __restrict__ views,
                                         int n_views, int64_t P, const RasterConst& c,
                                         const float* __restrict__ T_final, const int32_t* __restrict__ last,
                                         const float* __restrict__ grad_out, float* __restrict__ records,
                                         float4* s_g0, float4* s_g1, float4* s_app, int* s_max, float* s_acc) {
    constexpr int NT = TS * TS;
    constexpr int AV = AppRec<F>::vec;
    static_assert((3 + F) % 4 == 3, "the staged appearance record needs its padding slot for the depth");
    constexpr int NREAL = PARAMS ? 10 + F : 6;  // record slots
    constexpr int NBF = 6;                      // full-wavefront butterfly: mean, conic, opacity | depth
    constexpr int LIN = PARAMS ? 4 + F : 0;     // linear channels: depth, colour, feature
    constexpr int NL = LIN / 4;                 // linear channels per lane (a multiple of 4 channels)
    constexpr int RS = (NREAL + 3) / 4 * 4;  // record stride (floats), float4-aligned
    constexpr int AST = NREAL + 1;           // accumulator stride (odd: spreads LDS banks)
    constexpr int NQ = B / 64;               // 64-bit candidate masks per batch
    using BA = BwdApp<F, PARAMS>;
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

    const int64_t p = inside ? vw.pixel_offset + (int64_t)y * vw.width + x : 0;
    float T = inside ? T_final[p] : 1.0f;
    const int lastp = inside ? last[p] : 0;
    // the pixel's upstream gradient: all 5+F channels in pose-only mode; with
    // parameter gradients only the opacity channel (the others live in gq)
    constexpr int NG = PARAMS ? 1 : 5 + F;
    float g[NG];
    if constexpr (PARAMS) {
        g[0] = inside ? grad_out[4 * P + p] : 0.0f;
    } else {
#pragma unroll
        for (int ch = 0; ch < 5 + F; ++ch) g[ch] = inside ? grad_out[ch * P + p] : 0.0f;
    }
    // R of the Gaussian about to be visited.  With parameter gradients the
    // opacity channel (x = 1 for every Gaussian) is left out of g . x and R
    // starts at -g_opacity instead: R + g_opacity is then the full R, and
    // g . x - R is unchanged.
    float Rg = PARAMS ? -g[0] : 0.0f;
    const float log2_amin = __log2f(c.alpha_min);
    const float amin = c.alpha_min, amax = c.alpha_max;

    if (tid == 0) *s_max = 0;
    __syncthreads();
    if (lastp > 0) atomicMax(s_max, lastp);
    __syncthreads();
    const int end = rg.x + *s_max;
    // the wavefront's own bound: no lane contributes from position wlast on
    int wlast = lastp;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) wlast = max(wlast, __shfl_xor(wlast, d, kWave));

    // instances past every pixel's last contributor: zero records
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int k = end + tid; k < rg.y; k += NT) {
        float4* r4 = reinterpret_cast<float4*>(records + (size_t)inst[k] * RS);
#pragma unroll
        for (int q = 0; q < RS / 4; ++q) r4[q] = z4;
    }

    // full-wavefront butterfly value k -> record slot: 0..4 (mean, conic) as
    // they are; value 5 is the opacity (slot 6) with parameter gradients,
    // else the depth (slot 5).  Scales: dmx, dmy <- -ln2; dA, dC <- -1/2;
    // dB <- -1.
    const int bslot = geo6_slot(lane);
    const bool writer = (lane & 0xB) == 0 && bslot < NBF;
    const int my_slot = bslot < 5 ? bslot : (PARAMS ? 6 : 5);
    float scale = 1.0f;
    if (bslot < 2) scale = -kLn2;
    else if (bslot == 2 || bslot == 4) scale = -0.5f;
    else if (bslot == 3) scale = -1.0f;

    // Linear channels c (0 depth, 1-3 colour, 4+ feature): their gradient is
    // sum_p g_c(p) w(p) with g constant over the tile.  A lane owns the
    // channels c = 4 m + q (q = lane bits 4-5) and keeps, for them, g of the
    // four lanes sharing its bits 0-3 (index t = the lane's bits 4-5, the
    // order of quad_row_weights); per Gaussian it takes those lanes' weights
    // (three permlane swaps), forms the four-lane sums with FMAs and finishes
    // over the 16 lanes of its row group with the ORD 1 butterfly.
    const int q4 = (lane >> 4) & 3, b4 = q4 & 1;
    float gq[NL > 0 ? NL : 1][4];
    if constexpr (PARAMS) {
#pragma unroll
        for (int t4 = 0; t4 < 4; ++t4) {
            const int lp = (lane & 15) | (t4 << 4);  // the order of quad_row_weights
            const int xx = tx * TS + sbx + (lp & 7), yy = ty * TS + sby + (lp >> 3);
            const bool in = xx < vw.width && yy < vw.height;
            const int64_t pp = vw.pixel_offset + (int64_t)yy * vw.width + xx;
#pragma unroll
            for (int m = 0; m < NL; ++m) {
                const int ch = 4 * m + q4;
                const int plane = ch == 0 ? 3 : (ch < 4 ? ch - 1 : ch + 1);
                gq[m][t4] = in ? grad_out[plane * P + pp] : 0.0f;
            }
        }
    }
    // With parameter gradients the last four steps of the six-value sum
    // (bits 2, 0, 1, 3) and the sum of the linear channels over the 16 lanes
    // of a row group run as one ORD 1 butterfly over NC values per lane:
    // the two geometry values still open after bits 5 and 4, then the NL
    // linear channels.  The six geometry values are the moments (see
    // moments_to_geometry), accumulated in slots 0-4 and 6 and turned into
    // the record's values when it is written.  Value index -> record slot of
    // this lane:
    constexpr int NC = Pow2<2 + NL>::value;
    const int cs = Butterfly<NC, 1>::slot(lane);
    int cslot = -1;
    {
        const int b5 = (lane >> 5) & 1;
        int gi = -1;  // geometry value index
        if (cs == 0) gi = b4 ? 2 + b5 : 4 * b5;
        else if (cs == 1 && !b4) gi = 1 + 4 * b5;
        if (gi >= 0) {
            cslot = gi < 5 ? gi : 6;
        } else if (cs >= 2 && cs < 2 + NL) {
            const int ch = 4 * (cs - 2) + q4;
            cslot = ch == 0 ? 5 : 6 + ch;
        }
    }
    const bool cwriter = PARAMS && (lane & Butterfly<NC, 1>::reduced_mask()) == 0 && cslot >= 0;
    // float index, within a staged appearance record, of this lane's channels
    // c = 4 m + q (depth sits in the record's padding slot)
    int xidx[NL > 0 ? NL : 1];
#pragma unroll
    for (int m = 0; m < NL; ++m) {
        const int ch = 4 * m + q4;
        xidx[m] = ch == 0 ? AV * 4 - 1 : ch - 1;
    }

    for (int bend = end; bend > rg.x; bend -= B) {
        const int bstart = max(rg.x, bend - B);
        const int nb = bend - bstart;
        __syncthreads();
        for (int k = tid; k < nb; k += NT) {
            const int gid = inst_gid[inst[bstart + k]];
            float4 a0, a1;
            stage_geometry(rec, vbase + gid, a0, a1);
            s_g0[k] = a0;
            s_g1[k] = a1;
            if constexpr (BA::qmajor) {
                // quarter q holds channels q, 4 + q, 8 + q, ... (channel 0 is
                // the depth, channel c >= 1 the record's float c - 1)
                float4 in[AV];
#pragma unroll
                for (int q = 0; q < AV; ++q) in[q] = app[(size_t)gid * AV + q];
                const float* f = reinterpret_cast<const float*>(in);
#pragma unroll
                for (int qd = 0; qd < 4; ++qd) {
#pragma unroll
                    for (int v4 = 0; v4 < BA::QS / 4; ++v4) {
                        float e[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int m = 4 * v4 + u, ch = 4 * m + qd;
                            e[u] = m < NL ? (ch == 0 ? a1.z : f[ch - 1]) : 0.0f;
                        }
                        s_app[k * BA::vec + qd * (BA::QS / 4) + v4] = make_float4(e[0], e[1], e[2], e[3]);
                    }
                }
            } else {
#pragma unroll
                for (int q = 0; q < AV; ++q) s_app[k * AV + q] = app[(size_t)gid * AV + q];
                // the record's last float is padding (3 + F is 3 mod 4): depth goes there
                reinterpret_cast<float*>(s_app)[(k + 1) * AV * 4 - 1] = a1.z;
            }
        }
        for (int k = tid; k < nb * AST; k += NT) s_acc[k] = 0.0f;
        __syncthreads();
        // Candidates of this wavefront: Gaussians of the batch before its
        // last contributor whose box reaches its 8x8 block, one bit each
        // (lane k tests Gaussian 64 q + k).  The loop below visits only
        // these, from the back, with the next candidate's geometry already
        // in flight.
        uint64_t cand[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int k = 64 * q + lane;
            bool ok = false;
            if (k < nb && bstart + k - rg.x < wlast) {
                const float4 a0 = s_g0[k], a1 = s_g1[k];
                ok = !box_misses(a0, a1, wx0, wy0) && !ellipse_misses(a0, a1, wx0, wy0, log2_amin);
            }
            cand[q] = __builtin_amdgcn_ballot_w64(ok);
        }
#pragma unroll
        for (int q = NQ - 1; q >= 0; --q) {
            uint64_t m = cand[q];
            if (m == 0) continue;
            int j = 64 * q + 63 - __builtin_clzll(m);
            float4 g0 = s_g0[j], g1 = s_g1[j];
            for (;;) {
                m &= ~(1ull << (j - 64 * q));
                const int jn = m ? 64 * q + 63 - __builtin_clzll(m) : -1;
                // appearance of Gaussian j: with parameter gradients only this
                // lane's channels, else the whole record
                float xs[PARAMS ? (NL > 0 ? NL : 1) : AV * 4];
                if constexpr (BA::qmajor) {
                    const float4* sq = s_app + j * BA::vec + q4 * (BA::QS / 4);
#pragma unroll
                    for (int v4 = 0; v4 < NL / 4; ++v4) {
                        const float4 t = sq[v4];
                        xs[4 * v4] = t.x;
                        xs[4 * v4 + 1] = t.y;
                        xs[4 * v4 + 2] = t.z;
                        xs[4 * v4 + 3] = t.w;
                    }
#pragma unroll
                    for (int m = NL / 4 * 4; m < NL; ++m) xs[m] = reinterpret_cast<const float*>(sq)[m];
                    __builtin_amdgcn_sched_barrier(0);
                } else if constexpr (PARAMS) {
                    const float* sa = reinterpret_cast<const float*>(s_app) + j * AV * 4;
#pragma unroll
                    for (int m = 0; m < NL; ++m) xs[m] = sa[xidx[m]];
                    // issue these loads at the top of the step (the g . x
                    // below waits on them; left alone, the scheduler sinks
                    // some past the exponential)
                    __builtin_amdgcn_sched_barrier(0);
                } else {
#pragma unroll
                    for (int qq = 0; qq < AV; ++qq) {
                        const float4 a4 = s_app[j * AV + qq];
                        xs[4 * qq] = a4.x;
                        xs[4 * qq + 1] = a4.y;
                        xs[4 * qq + 2] = a4.z;
                        xs[4 * qq + 3] = a4.w;
                    }
                }
                const int jl = bstart + j - rg.x;
                float dx, dy, G, qx, qy;
                bool unc;
                const float a = pair_alpha(g0, g1, px, py, amax, dx, dy, G, unc, qx, qy);
                // The values the geometry sums need (dx, dy with parameter
                // gradients; without, qx, qy: the derivatives of q' along dx
                // and dy, up to the factors the record scales apply) are
                // kept here by an empty statement (no instruction): sunk
                // further down they would keep g0 and g1 alive.  g0 and g1
                // are dead from here -- the next candidate's geometry is
                // loaded into them (no register copies at the end of the
                // step), unconditionally with a clamped index (a conditional
                // load becomes a pointer select that leaves LDS addressing)
                if constexpr (PARAMS) __asm__ volatile("" : "+v"(dx), "+v"(dy));
                else __asm__ volatile("" : "+v"(qx), "+v"(qy));
                const int jp = jn >= 0 ? jn : j;
                g0 = s_g0[jp];
                g1 = s_g1[jp];
                // issue those loads here, most of a step ahead of their use
                // (left alone, the scheduler sinks them towards the end)
                __builtin_amdgcn_sched_barrier(0);
                const bool contrib = jl < lastp && a >= amin;
                // No branch on whether any lane contributes (nearly every
                // candidate step has a contributor).  Branch-free over the
                // wavefront: lanes without a contribution take alpha = 0 (T
                // unchanged, exact since rcp(1) = 1, w = 0) and zero
                // multipliers, so a step without contributors adds zeros.
                {
                    const float ac = contrib ? a : 0.0f;
                    T = T * __builtin_amdgcn_rcpf(1.0f - ac);  // transmittance before this Gaussian
                    const float w = ac * T;
                    // g . x over the 5+F channels of this lane's pixel
                    float gx;
                    if constexpr (PARAMS) {
                        // partial dot products over this lane's channel quarter
                        // for the four lanes of its group, then a transposing
                        // reduce over lane bits 5 and 4 hands each lane its own
                        float pt[4];
#pragma unroll
                        for (int t4 = 0; t4 < 4; ++t4) {
                            float acc = gq[0][t4] * xs[0];
#pragma unroll
                            for (int m = 1; m < NL; ++m) acc = fmaf(gq[m][t4], xs[m], acc);
                            pt[t4] = acc;
                        }
                        // pt[t] is for the pixel of the lane with bits 4-5 = t:
                        // bit 5 pairs pt[0] with pt[2] (bit-4 clear) and pt[1]
                        // with pt[3], bit 4 the two results; the opacity
                        // channel is not in gx (it is in Rg)
                        gx = swap_halves_add<16>(swap_halves_add<32>(pt[0], pt[2]),
                                                 swap_halves_add<32>(pt[1], pt[3]));
                    } else {
                        gx = fmaf(g[0], xs[0], fmaf(g[1], xs[1], fmaf(g[2], xs[2], fmaf(g[3], xs[AV * 4 - 1], g[4]))));
#pragma unroll
                        for (int f = 0; f < F; ++f) gx = fmaf(g[5 + f], xs[3 + f], gx);
                    }
                    const float dg = gx - Rg;
                    const float dA = T * dg;
                    Rg = fmaf(ac, dg, Rg);
                    const float hm = (contrib && unc) ? dA : 0.0f;
                    const float h = hm * a;
                    float val[NBF];
                    if constexpr (PARAMS) {
                        // the moments h {1, dx, dy, dx^2, dx dy, dy^2}
                        const float hx = h * dx, hy = h * dy;
                        val[0] = h;
                        val[1] = hx;
                        val[2] = hy;
                        val[3] = hx * dx;
                        val[4] = hx * dy;
                        val[5] = hy * dy;
                    } else {
                        val[0] = h * qx;
                        val[1] = h * qy;
                        val[2] = h * dx * dx;
                        val[3] = h * dx * dy;
                        val[4] = h * dy * dy;
                        val[5] = g[3] * w;
                    }
                    if constexpr (PARAMS) {
                        float cv[NC];
                        geo6_bits54(val, cv[0], cv[1]);
                        float W[4];
                        quad_row_weights(w, W);
#pragma unroll
                        for (int m = 0; m < NL; ++m)
                            cv[2 + m] =
                                fmaf(gq[m][3], W[3], fmaf(gq[m][2], W[2], fmaf(gq[m][1], W[1], gq[m][0] * W[0])));
#pragma unroll
                        for (int m = 2 + NL; m < NC; ++m) cv[m] = 0.0f;
                        const float tot = Butterfly<NC, 1, 2 + NL>::reduce(cv, lane);
                        if (cwriter) atomicAdd(&s_acc[j * AST + cslot], tot);
                    } else {
                        const float tot = geo6_reduce(val, lane);
                        if (writer) atomicAdd(&s_acc[j * AST + my_slot], tot * scale);
                    }
                }
                if (jn < 0) break;
                j = jn;
            }
        }
        __syncthreads();
        // one contiguous record per instance of the batch (zeros if untouched)
        for (int k = tid; k < nb; k += NT) {
            float4* r4 = reinterpret_cast<float4*>(records + (size_t)inst[bstart + k] * RS);
            const float* a = s_acc + k * AST;
            float r[RS];
#pragma unroll
            for (int b = 0; b < RS; ++b) r[b] = b < NREAL ? a[b] : 0.0f;
            if constexpr (PARAMS) moments_to_geometry(s_g0[k], s_g1[k], r);
#pragma unroll
            for (int q = 0; q < RS / 4; ++q) r4[q] = make_float4(r[4 * q], r[4 * q + 1], r[4 * q + 2], r[4 * q + 3]);
        }
    }
}

// Occupancy: the kernel is latency-bound (LDS reads and cross-lane steps on
// every Gaussian), so the register budget is capped at five wavefronts per
// SIMD with up to 16 feature channels and at four with 32 (with 64
// Gaussians per LDS batch, which keeps the LDS from capping it at three):
// the values fit without spills.  Launch shapes whose LDS batch caps
// residency below that anyway (tile 8, larger batches) get no cap.
template <int TS, int F, int B>
constexpr int bwd_waves_target() {
    return TS < 16 ? 1 : (F <= 16 ? (B <= 128 ? 5 : 1) : (B <= 64 ? 4 : 1));
}
template <int TS, int F, int B, bool PARAMS>
__global__ void __launch_bounds__(TS* TS) __attribute__((amdgpu_waves_per_eu(bwd_waves_target<TS, F, B>(), 8))) k_render_bwd(const float4* __restrict__ rec, const float4* __restrict__ app,
                                                       int n, const int32_t* __restrict__ inst,
                                                       const int32_t* __restrict__ inst_gid,
                                                       const int2* __restrict__ ranges,
                                                       const gs_view* __restrict__ views, int n_views,
                                                       int total_tiles, int64_t P, RasterConst c,
                                                       const float* __restrict__ T_final,
                                                       const int32_t* __restrict__ last,
                                                       const float* __restrict__ grad_out,
                                                       float* __restrict__ records, int32_t* queue, int persistent) {
    constexpr int NREAL = PARAMS ? 10 + F : 6;
    __shared__ float4 s_g0[B];
    __shared__ float4 s_g1[B];
    __shared__ float4 s_app[B * BwdApp<F, PARAMS>::vec];
    __shared__ float s_acc[B * (NREAL + 1)];
    __shared__ int s_tile;
    __shared__ int s_max;
    if (!persistent) {
        const int t = tile_of_block<TS>(blockIdx.x, total_tiles);
        if (t < 0) return;
        bwd_tile<TS, F, B, PARAMS>(t, rec, app, n, inst, inst_gid, ranges, views, n_views, P, c, T_final,
                                   last, grad_out, records, s_g0, s_g1, s_app, &s_max, s_acc);
        return;
    }
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_tile = atomicAdd(queue + 1, 1);
        __syncthreads();
        const int t = s_tile;
        if (t >= total_tiles) break;
        bwd_tile<TS, F, B, PARAMS>(t, rec, app, n, inst, inst_gid, ranges, views, n_views, P, c, T_final, last,
                                   grad_out, records, s_g0, s_g1, s_app, &s_max, s_acc);
    }
}

// Sum of the records of every (view, Gaussian) pair (contiguous emission
// indices, fixed order).  VP lanes per Gaussian, adjacent in one wavefront
// (VP a power of two, VP <= 64; the launcher uses VP <= 2); with more views
// than VP the lanes take views vl, vl + VP, ... in rounds.  Few
// pairs are visible and their record counts vary widely, so a wavefront
// flattens the records of its pairs (an exclusive scan of the counts) and
// loads them STG at a time, one record per lane (consecutive records of a
// pair are adjacent in memory), into LDS; each owner lane then adds its own
// records from LDS in emission order.  grad_geo[V][n][8] <- (dmx, dmy, dA,
// dB, dC, dd, 0, 0) for visible pairs (others are not written); the
// appearance part is summed over the Gaussian's lanes by a fixed xor tree
// and grad_app[n][4+F] written by its first lane (fixed order).
//
// Residency: the staged records take STG x 4 x RS bytes of LDS per
// wavefront.  With 32 feature channels (176-byte records) a full wavefront
// of them (45 KB per workgroup) and the 130 registers the kernel would take
// both stop at three wavefronts per SIMD; staging 48 at a time (37 KB) and
// capping the registers at 128 allow four.
template <int F, bool PARAMS>
struct ReduceShape {
    static constexpr int STG = PARAMS && F > 16 ? 48 : kWave;  // records staged per pass
    static constexpr int waves = PARAMS && F > 16 ? 4 : 1;     // occupancy target (1: none)
};
template <int F, bool PARAMS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ReduceShape<F, PARAMS>::waves, 8)))
k_reduce_records(const float* __restrict__ records,
                                                        const int32_t* __restrict__ pair_first,
                                                        const int32_t* __restrict__ touched, int n, int n_views,
                                                        int vp_log2, int64_t capacity, float* __restrict__ grad_geo,
                                                        float* __restrict__ grad_app) {
    constexpr int NREAL = PARAMS ? 10 + F : 6;
    constexpr int RS = (NREAL + 3) / 4 * 4;
    constexpr int NA = PARAMS ? 4 + F : 1;
    constexpr int STG = ReduceShape<F, PARAMS>::STG;
    __shared__ float4 s_rec[256 / kWave][STG][RS / 4];
    __shared__ int s_start[256 / kWave][kWave];
    __shared__ int s_first[256 / kWave][kWave];
    __shared__ int s_mark[256 / kWave][kWave];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int vp = 1 << vp_log2;
    const int64_t i64 = t >> vp_log2;
    const int vl = (int)(t & (vp - 1));
    const int i = (int)(i64 < n ? i64 : n);
    float appacc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) appacc[q] = 0.0f;
    for (int v0 = 0; v0 < n_views; v0 += vp) {
        const int v = v0 + vl;
        const size_t pair = (size_t)v * n + i;
        const bool in = i64 < n && v < n_views;
        // both loads in one round trip (pair_first is only meaningful, and
        // only used, for visible pairs)
        const int tc = in ? touched[pair] : 0;
        const int pf = in ? pair_first[pair] : 0;
        const bool vis = tc > 0;
        int cnt = 0, first = 0;
        if (vis) {
            first = pf;
            const int64_t stop = (int64_t)first + tc;
            cnt = (int)((stop < capacity ? stop : capacity) - first);  // truncated lists
            cnt = cnt > 0 ? cnt : 0;
        }
        // exclusive scan of the counts over the wavefront
        const int incl = wave_add_scan(cnt);
        const int start = incl - cnt;
        const int total = __builtin_amdgcn_readlane(incl, kWave - 1);
        s_start[wave][lane] = start;
        s_first[wave][lane] = first;
        // the pair's records are summed in FP64: a Gaussian spanning many
        // tiles adds many partials of both signs (float only at the end)
        double geo[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int carry = -1;  // owner of the last record before the current 64
        for (int base = 0; base < total; base += STG) {
            // owner of record base + lane: the last lane with records whose
            // start is at or before it -- each such lane marks its start's
            // slot (starts of lanes with records are distinct) and a
            // max-scan carries the marks forward
            s_mark[wave][lane] = -1;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (cnt > 0 && start >= base && start < base + STG) s_mark[wave][start - base] = lane;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int lo = max(wave_max_scan(s_mark[wave][lane]), carry);
            carry = __builtin_amdgcn_readlane(lo, kWave - 1);
            // (lanes from STG on mark nothing, so the scan's last lane holds
            // the owner of record base + STG - 1)
            const int idx = base + lane;
            if (lane < STG && idx < total) {
                const int64_t e = (int64_t)s_first[wave][lo] + (idx - s_start[wave][lo]);
                const float4* r4 = reinterpret_cast<const float4*>(records + (size_t)e * RS);
#pragma unroll
                for (int q = 0; q < RS / 4; ++q) s_rec[wave][lane][q] = r4[q];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int r0 = start > base ? start : base;
            const int r1 = start + cnt < base + STG ? start + cnt : base + STG;
            for (int r = r0; r < r1; ++r) {
                float rr[RS];
#pragma unroll
                for (int q = 0; q < RS / 4; ++q) {
                    const float4 a = s_rec[wave][r - base][q];
                    rr[4 * q] = a.x;
                    rr[4 * q + 1] = a.y;
                    rr[4 * q + 2] = a.z;
                    rr[4 * q + 3] = a.w;
                }
#pragma unroll
                for (int q = 0; q < 6; ++q) geo[q] += (double)rr[q];
                if (PARAMS) {
#pragma unroll
                    for (int q = 0; q < NA; ++q) appacc[q] += rr[6 + q];
                }
            }
        }
        if (vis) {
            float4* gg = reinterpret_cast<float4*>(grad_geo + pair * 8);
            gg[0] = make_float4((float)geo[0], (float)geo[1], (float)geo[2], (float)geo[3]);
            gg[1] = make_float4((float)geo[4], (float)geo[5], 0.f, 0.f);
        }
        // the next round reuses this wavefront's LDS
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (PARAMS) {
        // sum over the Gaussian's VP lanes (bits 0 .. vp_log2-1), DPP and
        // swizzles; the half-row mirror serves bit 2 once bits 0 and 1 are
        // summed (every lane of a quad then holds the quad's total)
        if (vp_log2 > 0)
#pragma unroll
            for (int q = 0; q < NA; ++q) appacc[q] += xor_lane<1>(appacc[q]);
        if (vp_log2 > 1)
#pragma unroll
            for (int q = 0; q < NA; ++q) appacc[q] += xor_lane<2>(appacc[q]);
        if (vp_log2 > 2)
#pragma unroll
            for (int q = 0; q < NA; ++q) appacc[q] += mirror8_lane(appacc[q]);
        if (vp_log2 > 3)
#pragma unroll
            for (int q = 0; q < NA; ++q) appacc[q] += xor_lane<8>(appacc[q]);
        if (vp_log2 > 4)
#pragma unroll
            for (int q = 0; q < NA; ++q) appacc[q] += xor_lane<16>(appacc[q]);
        if (vp_log2 > 5)
#pragma unroll
            for (int q = 0; q < NA; ++q) appacc[q] += xor_lane<32>(appacc[q]);
        if (i64 < n && vl == 0) {
            // the row of 4+F floats is 16-byte aligned (4+F is a multiple of 4)
            float4* ga = reinterpret_cast<float4*>(grad_app + (size_t)i * (4 + F));
#pragma unroll
            for (int q = 0; q < NA / 4; ++q)
                ga[q] = make_float4(appacc[4 * q], appacc[4 * q + 1], appacc[4 * q + 2], appacc[4 * q + 3]);
        }
    }
}

__global__ void k_reset_queue_bwd(int32_t* q) {
    if (threadIdx.x < 4) q[threadIdx.x] = 0;
}

template <int TS, int F, int B, bool PARAMS>
hipError_t launch_bwd_t(const float* rec, const float* app, int n, const int32_t* inst, const int32_t* inst_gid,
                        const int32_t* ranges, const gs_view* views, int n_views, int total_tiles, int64_t P,
                        const RasterConst& c, int persistent, const float* T_final, const int32_t* last,
                        const float* grad_out, float* records, int32_t* queue, hipStream_t s) {
    auto kern = k_render_bwd<TS, F, B, PARAMS>;
    unsigned grid = total_tiles > 0 ? tile_grid<TS>(total_tiles) : 0u;
    if (persistent) {
        int dev = 0, cus = 0, per_cu = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, TS * TS, 0);
        if (per_cu < 1) per_cu = 1;
        if (cus < 1) cus = 1;  // a failed query still drains the queue, with fewer workgroups
        const unsigned cap = (unsigned)(cus * per_cu);
        grid = cap < (unsigned)total_tiles ? cap : (unsigned)total_tiles;
        hipLaunchKernelGGL(k_reset_queue_bwd, dim3(1), dim3(64), 0, s, queue);
    }
    if (grid == 0) return hipGetLastError();
    hipLaunchKernelGGL(kern, dim3(grid), dim3(TS * TS), 0, s, reinterpret_cast<const float4*>(rec),
                       reinterpret_cast<const float4*>(app), n, inst, inst_gid, reinterpret_cast<const int2*>(ranges),
                       views, n_views, total_tiles, P, c, T_final, last, grad_out, records, queue, persistent);
    return hipGetLastError();
}

template <int TS, int F, bool PARAMS>
hipError_t launch_bwd_b(int B, const float* rec, const float* app, int n, const int32_t* inst, const int32_t* inst_gid,
                        const int32_t* ranges, const gs_view* views, int n_views, int total_tiles, int64_t P,
                        const RasterConst& c, int persistent, const float* T_final, const int32_t* last,
                        const float* grad_out, float* records, int32_t* queue, hipStream_t s) {
    switch (B) {
        case 64:
            return launch_bwd_t<TS, F, 64, PARAMS>(rec, app, n, inst, inst_gid, ranges, views, n_views, total_tiles,
                                                   P, c, persistent, T_final, last, grad_out, records, queue, s);
        case 128:
            return launch_bwd_t<TS, F, 128, PARAMS>(rec, app, n, inst, inst_gid, ranges, views, n_views, total_tiles,
                                                    P, c, persistent, T_final, last, grad_out, records, queue, s);
        default:
            return launch_bwd_t<TS, F, 256, PARAMS>(rec, app, n, inst, inst_gid, ranges, views, n_views, total_tiles,
                                                    P, c, persistent, T_final, last, grad_out, records, queue, s);
    }
}

template <int F, bool PARAMS>
hipError_t launch_bwd_ts(int TS, int B, const float* rec, const float* app, int n, const int32_t* inst,
                         const int32_t* inst_gid, const int32_t* ranges, const gs_view* views, int n_views,
                         int total_tiles, int64_t P, const RasterConst& c, int persistent, const float* T_final,
                         const int32_t* last, const float* grad_out, float* records, int32_t* queue, hipStream_t s) {
    switch (TS) {
        case 8:
            return launch_bwd_b<8, F, PARAMS>(B, rec, app, n, inst, inst_gid, ranges, views, n_views, total_tiles, P,
                                              c, persistent, T_final, last, grad_out, records, queue, s);
        case 32:
            return launch_bwd_b<32, F, PARAMS>(B, rec, app, n, inst, inst_gid, ranges, views, n_views, total_tiles, P,
                                               c, persistent, T_final, last, grad_out, records, queue, s);
        default:
            return launch_bwd_b<16, F, PARAMS>(B, rec, app, n, inst, inst_gid, ranges, views, n_views, total_tiles, P,
                                               c, persistent, T_final, last, grad_out, records, queue, s);
    }
}

template <int F>
hipError_t launch_bwd_f(bool params, int TS, int B, const float* rec, const float* app, int n, const int32_t* inst,
                        const int32_t* inst_gid, const int32_t* ranges, const gs_view* views, int n_views,
                        int total_tiles, int64_t P, const RasterConst& c, int persistent, const float* T_final,
                        const int32_t* last, const float* grad_out, float* records, int32_t* queue, hipStream_t s) {
    if (params)
        return launch_bwd_ts<F, true>(TS, B, rec, app, n, inst, inst_gid, ranges, views, n_views, total_tiles, P, c,
                                      persistent, T_final, last, grad_out, records, queue, s);
    return launch_bwd_ts<F, false>(TS, B, rec, app, n, inst, inst_gid, ranges, views, n_views, total_tiles, P, c,
                                   persistent, T_final, last, grad_out, records, queue, s);
}

int bwd_record_floats(int n_feat, bool params) {
    const int nreal = params ? 10 + n_feat : 6;
    return (nreal + 3) / 4 * 4;
}

hipError_t launch_render_bwd(const float* rec, const float* app, int n, int n_feat, const int32_t* inst,
                             const int32_t* inst_gid, const int32_t* ranges, const gs_view* views_dev, int n_views,
                             int total_tiles, int64_t total_pixels, const RasterConst& c, int lds_batch,
                             int persistent, const float* T_final, const int32_t* last, const float* grad_out,
                             bool params, float* records, int32_t* queue, hipStream_t s) {
    const int TS = c.tile;
#define SGS_BWD_CASE(FF)                                                                                            \
    return launch_bwd_f<FF>(params, TS, lds_batch, rec, app, n, inst, inst_gid, ranges, views_dev, n_views,         \
                            total_tiles, total_pixels, c, persistent, T_final, last, grad_out, records, queue, s)
    switch (n_feat) {
        case 0: SGS_BWD_CASE(0);
        case 8: SGS_BWD_CASE(8);
        case 32: SGS_BWD_CASE(32);
        default: SGS_BWD_CASE(16);
    }
#undef SGS_BWD_CASE
}

template <int F>
hipError_t launch_reduce_t(bool params, const float* records, const int32_t* pair_first, const int32_t* touched,
                           int n, int n_views, int64_t capacity, float* grad_geo, float* grad_app, hipStream_t s) {
    // two lanes per Gaussian, the views taken in rounds: a wavefront then
    // covers 32 consecutive Gaussians, so its pair loads are two coalesced
    // runs and its records two contiguous ranges of emission indices (the
    // instances of consecutive visible pairs of one view are adjacent).  A
    // lane per view was as fast at 8 views and F = 16 (147 against 149 us)
    // and much slower at 16 views and F = 32 (809 against 599 us).
    int vp_log2 = 0;
    while ((1 << vp_log2) < n_views && vp_log2 < 1) ++vp_log2;
    const int64_t lanes = (int64_t)n << vp_log2;
    const dim3 grid((unsigned)((lanes + 255) / 256));
    if (params)
        hipLaunchKernelGGL((k_reduce_records<F, true>), grid, dim3(256), 0, s, records, pair_first, touched, n, n_views,
                           vp_log2, capacity, grad_geo, grad_app);
    else
        hipLaunchKernelGGL((k_reduce_records<F, false>), grid, dim3(256), 0, s, records, pair_first, touched, n,
                           n_views, vp_log2, capacity, grad_geo, grad_app);
    return hipGetLastError();
}

hipError_t launch_reduce_records(const float* records, const int32_t* pair_first, const int32_t* touched, int n,
                                 int n_feat, int n_views, int64_t capacity, bool params, float* grad_geo,
                                 float* grad_app, hipStream_t s) {
    if (n == 0) return hipSuccess;
    switch (n_feat) {
        case 0: return launch_reduce_t<0>(params, records, pair_first, touched, n, n_views, capacity, grad_geo, grad_app, s);
        case 8: return launch_reduce_t<8>(params, records, pair_first, touched, n, n_views, capacity, grad_geo, grad_app, s);
        case 32: return launch_reduce_t<32>(params, records, pair_first, touched, n, n_views, capacity, grad_geo, grad_app, s);
        default: return launch_reduce_t<16>(params, records, pair_first, touched, n, n_views, capacity, grad_geo, grad_app, s);
    }
}

}  // namespace sgs
