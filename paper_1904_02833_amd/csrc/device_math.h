// FP32 vector / quaternion helpers for the snake kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace snake {

struct V3 {
    float x, y, z;
};
struct Q4 {
    float w, x, y, z;
};

__device__ __forceinline__ V3 mk(float a, float b, float c) { return V3{a, b, c}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return V3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator-(V3 a) { return V3{-a.x, -a.y, -a.z}; }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return V3{s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b)
{
    return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ float amax3(V3 a) { return fmaxf(fabsf(a.x), fmaxf(fabsf(a.y), fabsf(a.z))); }
__device__ __forceinline__ V3 sel(bool c, V3 a, V3 b) { return c ? a : b; }
// s a + b with one rounding per component (fused multiply-add)
__device__ __forceinline__ V3 fma3(float s, V3 a, V3 b)
{
    return V3{fmaf(s, a.x, b.x), fmaf(s, a.y, b.y), fmaf(s, a.z, b.z)};
}

__device__ __forceinline__ Q4 qmul(Q4 a, Q4 b)
{
    return Q4{a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z,
              a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
              a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x,
              a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}
__device__ __forceinline__ Q4 qconj(Q4 a) { return Q4{a.w, -a.x, -a.y, -a.z}; }
__device__ __forceinline__ Q4 qnormalize(Q4 a)
{
    float r = rsqrtf(a.w * a.w + a.x * a.x + a.y * a.y + a.z * a.z);
    return Q4{a.w * r, a.x * r, a.y * r, a.z * r};
}
// body x axis in the world: R(q) e_x
__device__ __forceinline__ V3 qaxis(Q4 q)
{
    return V3{1.f - 2.f * (q.y * q.y + q.z * q.z), 2.f * (q.x * q.y + q.w * q.z),
              2.f * (q.x * q.z - q.w * q.y)};
}
// R(q) v = v + 2 (w (u x v) + u x (u x v)), u = (q.x, q.y, q.z)
__device__ __forceinline__ V3 qrot(Q4 q, V3 v)
{
    const V3 u{q.x, q.y, q.z};
    const V3 t = cross(u, v);
    return fma3(2.f, fma3(q.w, t, cross(u, t)), v);
}
// q <- normalize(q + 1/2 [0, dth] (x) q); the product [0, dth] (x) q is
// (-dth . u, w dth + dth x u)
__device__ __forceinline__ Q4 qturn(Q4 q, V3 dth)
{
    const V3 u{q.x, q.y, q.z};
    const float tw = -dot(dth, u);
    const V3 tv = fma3(q.w, dth, cross(dth, u));
    return qnormalize(Q4{fmaf(0.5f, tw, q.w), fmaf(0.5f, tv.x, q.x), fmaf(0.5f, tv.y, q.y), fmaf(0.5f, tv.z, q.z)});
}

// x = K^{-1} b for a symmetric 3x3 K = [[a,b,c],[b,d,e],[c,e,f]] (adjugate)
__device__ __forceinline__ V3 sym3_solve(float a, float b, float c, float d, float e, float f, V3 r)
{
    float c00 = d * f - e * e;
    float c01 = c * e - b * f;
    float c02 = b * e - c * d;
    float c11 = a * f - c * c;
    float c12 = b * c - a * e;
    float c22 = a * d - b * b;
    // hardware reciprocal (1 ulp): the determinant of an SPD block is far
    // from the FP32 limits, and the solve's rounding is at that level anyway
    float inv = __builtin_amdgcn_rcpf(a * c00 + b * c01 + c * c02);
    return V3{(c00 * r.x + c01 * r.y + c02 * r.z) * inv, (c01 * r.x + c11 * r.y + c12 * r.z) * inv,
              (c02 * r.x + c12 * r.y + c22 * r.z) * inv};
}

// wave64 lane shifts: value of lane+1 / lane-1 (edges are masked by callers)
__device__ __forceinline__ float lane_next(float v) { return __shfl_down(v, 1, 64); }
__device__ __forceinline__ float lane_prev(float v) { return __shfl_up(v, 1, 64); }
__device__ __forceinline__ V3 lane_next(V3 v) { return V3{lane_next(v.x), lane_next(v.y), lane_next(v.z)}; }
__device__ __forceinline__ V3 lane_prev(V3 v) { return V3{lane_prev(v.x), lane_prev(v.y), lane_prev(v.z)}; }
__device__ __forceinline__ Q4 lane_next(Q4 v)
{
    return Q4{lane_next(v.w), lane_next(v.x), lane_next(v.y), lane_next(v.z)};
}

// max over aligned groups of SEG lanes (NaN must be mapped to +inf first)
template <int SEG>
__device__ __forceinline__ float seg_max(float v)
{
#pragma unroll
    for (int off = SEG / 2; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

}  // namespace snake
