// The decision-path exponential and logarithm, shared by the projection
// (scales, opacity and box size of the binary32 decision path) and the
// scale regularisation (its samples): explicit sequences of binary32
// operations, so any IEEE implementation of the same sequences gives the
// same bits (the library is built without contraction).
#pragma once

#include <hip/hip_runtime.h>

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

// ln(y) for a positive normal y: y = m 2^e with m in [sqrt(1/2), sqrt(2))
// (frexp, then one doubling below sqrt(1/2)), f = m - 1 (exact), s = f/(2+f),
// ln m = 2 atanh(s) = 2s + 2s z (1/3 + z/5 + z^2/7 + z^3/9 + z^4/11) with
// z = s^2 (Horner), ln y = e ln2_hi + (ln m + e ln2_lo), ln 2 split as above.
__device__ __forceinline__ float dec_log(float y) {
    int e;
    float m = frexpf(y, &e);
    if (m < 0x1.6a09e6p-1f) {
        m = m + m;
        e = e - 1;
    }
    const float f = m - 1.0f;
    const float s = f / (2.0f + f);
    const float z = s * s;
    float p = 0x1.745d18p-4f;     // 1/11
    p = 0x1.c71c72p-4f + z * p;   // 1/9
    p = 0x1.24924ap-3f + z * p;   // 1/7
    p = 0x1.99999ap-3f + z * p;   // 1/5
    p = 0x1.555556p-2f + z * p;   // 1/3
    const float t = s + s;
    const float lnm = t + (t * z) * p;
    const float fe = (float)e;
    return fe * 0x1.62e4p-1f + (lnm + fe * 0x1.7f7d1cp-20f);
}

// Squared box radius in standard deviations of a Gaussian of opacity logit
// l: alpha = o exp(-q/2) >= alpha_min needs q <= 2 ln(o / alpha_min),
// with o = 1 / (1 + exp(-l)) taken on the decision path; plus 2^-8 so that
// the box covers the binary32 rounding of q and alpha at any opacity.
// Returns a value <= 0 when o / alpha_min <= 1 (the pair is culled).
__device__ __forceinline__ float dec_box_k(float logit, float alpha_min) {
    const float o = 1.0f / (1.0f + dec_exp(-logit));
    const float y = o / alpha_min;
    if (!(y > 1.0f)) return 0.0f;
    return 2.0f * dec_log(y) + 0x1p-8f;
}

}  // namespace sgs
