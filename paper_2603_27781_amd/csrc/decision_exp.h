// The decision-path exponential, shared by the projection (scales of the
// binary32 decision path) and the scale regularisation (its samples): an
// explicit sequence of binary32 operations, so any IEEE implementation of
// the same sequence gives the same bits (the library is built without
// contraction).
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

}  // namespace sgs
