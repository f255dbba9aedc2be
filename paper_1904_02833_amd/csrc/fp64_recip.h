// FP64 reciprocal and reciprocal square root for the double-precision
// chain kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace snake {

// 1/x and 1/sqrt(x) in FP64 from the hardware estimates refined by two
// Newton-Raphson steps each (every step squares the relative error, so two
// take the estimate to the last bits of FP64); in place of the IEEE
// division and square-root sequences, for finite positive x
__device__ __forceinline__ double rcp64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ double rsqrt64(double x)
{
    // Goldschmidt form: g -> sqrt(x), h -> 1 / (2 sqrt(x))
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    double e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    e = fma(-g, h, 0.5);
    h = fma(h, e, h);
    return 2.0 * h;
}

}  // namespace snake
