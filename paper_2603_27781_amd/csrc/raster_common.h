// Pieces shared by the forward and backward compositing kernels.
#pragma once

#include "sgs_common.h"

namespace sgs {

// -1/2 log2(e): the conic is staged pre-scaled so that
// alpha = o * 2^(A' dx^2 + B2' dx dy + C' dy^2) with A' = kq A, B2' = 2 kq B, C' = kq C.
constexpr float kQ = -0.72134752044448170f;
constexpr float kLn2 = 0.69314718055994531f;

template <int F>
struct AppRec {
    static constexpr int stride = ((3 + F) + 3) / 4 * 4;  // floats per Gaussian
    static constexpr int vec = stride / 4;                // float4 per Gaussian
};

// Staging of one instance into LDS: geometry in two float4
//   g0 = (mx, my, A', B2'),  g1 = (C', o, d, packed radii)
__device__ __forceinline__ void stage_geometry(const float4* __restrict__ rec, size_t pair, float4& g0, float4& g1) {
    const float4 r0 = rec[2 * pair];
    const float4 r1 = rec[2 * pair + 1];
    g0 = make_float4(r0.x, r0.y, kQ * r0.z, (2.0f * kQ) * r0.w);
    g1 = make_float4(kQ * r1.x, r1.y, r1.z, r1.w);
}

// Wavefront votes on a lane condition.  The condition goes to the ballot as
// it is, so it stays a lane mask in scalar registers (the int-typed library
// votes turn it into a 0/1 vector value and compare it back first).
__device__ __forceinline__ bool wave_any(bool c) { return __builtin_amdgcn_ballot_w64(c) != 0; }
__device__ __forceinline__ bool wave_all(bool c) { return __builtin_amdgcn_ballot_w64(!c) == 0; }

// Lane selects driven by a wavefront lane mask held in scalar registers
// (bit l of m decides lane l): one v_cndmask, where a bool derived from the
// mask would first cost a vector shift and compare.  Plain register
// operands only, no memory access.
__device__ __forceinline__ float mask_select(uint64_t m, float if_set, float if_clear) {
    float r;
    __asm__("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(if_clear), "v"(if_set), "s"(m));
    return r;
}
__device__ __forceinline__ int mask_select(uint64_t m, int if_set, int if_clear) {
    int r;
    __asm__("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(if_clear), "v"(if_set), "s"(m));
    return r;
}

// alpha of one (pixel, Gaussian) pair.  The forward and the backward kernels
// both call this with the same staged values, so every alpha_min / T_min
// decision of the backward reproduces the forward exactly.
//   G = 2^q' (the Gaussian factor), returns min(alpha_max, o G) as a median
// of three (o G >= 0; one instruction with alpha_max in a scalar register; a
// NaN product stays NaN and so fails every alpha test).  q' <= 0 for the
// positive definite conic; its binary32 evaluation can land above 0 only by
// its rounding error, where G then exceeds 1 by as little as it would fall
// short of the true value below 0, so q' is not clamped.
// qx, qy: the derivatives of q' along dx and dy, 2A'dx + B2'dy and
// B2'dx + 2C'dy, formed from the intermediates of q' (the forward does not
// read them, so they cost it nothing).
__device__ __forceinline__ float pair_alpha(const float4& g0, const float4& g1, float px, float py, float amax,
                                            float& dx, float& dy, float& G, bool& unclamped, float& qx,
                                            float& qy) {
    dx = px - g0.x;
    dy = py - g0.y;
    const float adx = g0.z * dx, cdy = g1.x * dy;
    const float v = fmaf(g0.w, dx, cdy);  // B2'dx + C'dy
    float q = fmaf(adx, dx, dy * v);
    qx = fmaf(2.0f, adx, g0.w * dy);
    qy = v + cdy;
    G = __builtin_amdgcn_exp2f(q);
    const float a = g1.y * G;
    unclamped = a < amax;
    return __builtin_amdgcn_fmed3f(a, 0.0f, amax);
}

// Value of `x` held by lane (lane ^ D) of the wavefront.  D = 1, 2: DPP
// quad permutation; D = 8: DPP row rotation by 8 (within a row of 16 lanes
// that is lane ^ 8); all three are VALU operand modifiers, no LDS traffic.
// Their source lanes always exist, so bound_ctrl (read 0 for a missing
// source) changes nothing but lets the compiler fold the move into the
// consuming add.
// D = 4, 16: ds_swizzle in xor mode (within 32-lane halves); D = 32:
// ds_bpermute.
template <int D>
__device__ __forceinline__ float xor_lane(float x) {
    const int v = __float_as_int(x);
    if constexpr (D == 1) {
        return __int_as_float(__builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true));  // quad_perm [1,0,3,2]
    } else if constexpr (D == 2) {
        return __int_as_float(__builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true));  // quad_perm [2,3,0,1]
    } else if constexpr (D == 8) {
        return __int_as_float(__builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, true));  // row_ror:8
    } else if constexpr (D < 32) {
        return __int_as_float(__builtin_amdgcn_ds_swizzle(v, (D << 10) | 0x1F));  // xor_mask D, and_mask 31
    } else {
        const int lane = __lane_id();
        return __int_as_float(__builtin_amdgcn_ds_bpermute((lane ^ D) << 2, v));
    }
}

// Value of `x` held by lane 7 - (lane & 7) of the same group of 8 (DPP
// row_half_mirror): the partner differs in lane bit 2, and also in bits 0
// and 1, so it serves as the bit-2 exchange of a butterfly only while the
// values do not yet depend on bits 0 and 1.
__device__ __forceinline__ float mirror8_lane(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x141, 0xF, 0xF, true));
}

// One exchange of the transposing butterfly across lane bit log2(D) for
// D = 16, 32 (gfx950 permlane swaps): returns, in every lane, the pair total
// of lo (lanes with the bit clear) or of hi (lanes with the bit set).  The
// swap moves the upper lanes of `lo` and the lower lanes of `hi` across, so
// one swap and one add replace two selects, a permute and an add.
template <int D>
__device__ __forceinline__ float swap_halves_add(float lo, float hi) {
    static_assert(D == 16 || D == 32, "swap exchange is for lane bits 4 and 5");
    const unsigned a = __float_as_uint(lo), b = __float_as_uint(hi);
    if constexpr (D == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
        return __uint_as_float(r[0]) + __uint_as_float(r[1]);
    } else {
        const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        return __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
}

// Minimum over t in [lo, hi] of a t^2 + b t + c0 (a > 0), given inv2a =
// 1 / (2a).  The vertex comes from a hardware reciprocal: any t in [lo, hi]
// gives a value at least the true minimum, and a relative error e in t
// raises it by only a (e t)^2, far inside the test's margin.
__device__ __forceinline__ float quad_min_on(float a, float b, float c0, float lo, float hi, float inv2a) {
    const float t = fminf(fmaxf(-b * inv2a, lo), hi);
    return fmaf(fmaf(a, t, b), t, c0);
}

// Exact (up to a margin) wavefront-level test: does the region where
// alpha >= alpha_min reach a pixel centre of the 8x8 block whose first
// centre is (x0, y0)?  With the staged conic, alpha = o 2^(-Q(dx, dy)),
// Q = a dx^2 + b dx dy + c dy^2 positive definite (a = -A', b = -B2',
// c = -C'), so alpha >= alpha_min needs Q <= log2(o / alpha_min).  Q is
// convex, so its minimum over the rectangle of pixel centres is 0 if the
// mean lies inside, else on one of the four edges (a clamped 1-D quadratic
// each).  The margin (1e-3 absolute in Q) covers the rounding of both
// evaluations, so the test only prunes pairs with alpha < alpha_min.
__device__ __forceinline__ bool ellipse_misses(const float4& g0, const float4& g1, float x0, float y0,
                                               float log2_amin) {
    const float a = -g0.z, b = -g0.w, c = -g1.x;
    const float K = __log2f(g1.y) - log2_amin;  // log2(o / alpha_min)
    const float xl = x0 - g0.x, xh = xl + 7.0f, yl = y0 - g0.y, yh = yl + 7.0f;
    if (xl <= 0.0f && xh >= 0.0f && yl <= 0.0f && yh >= 0.0f) return K < 0.0f;
    // edges x = xl, xh: Q = c y^2 + (b x) y + a x^2; edges y = yl, yh likewise
    const float i2c = __builtin_amdgcn_rcpf(2.0f * c), i2a = __builtin_amdgcn_rcpf(2.0f * a);
    float q = quad_min_on(c, b * xl, a * xl * xl, yl, yh, i2c);
    q = fminf(q, quad_min_on(c, b * xh, a * xh * xh, yl, yh, i2c));
    q = fminf(q, quad_min_on(a, b * yl, c * yl * yl, xl, xh, i2a));
    q = fminf(q, quad_min_on(a, b * yh, c * yh * yh, xl, xh, i2a));
    return q > K + 1e-3f;
}

// Conservative wavefront-level test: can the Gaussian reach any pixel centre
// of the 8x8 block whose first centre is (x0, y0)?  Only prunes; a Gaussian
// outside its box has alpha < alpha_min at every pixel centre.
__device__ __forceinline__ bool box_misses(const float4& g0, const float4& g1, float x0, float y0) {
    const float2 r = unpack_radii(g1.w);
    return (g0.x + r.x < x0) || (g0.x - r.x > x0 + 7.0f) || (g0.y + r.y < y0) || (g0.y - r.y > y0 + 7.0f);
}

}  // namespace sgs
