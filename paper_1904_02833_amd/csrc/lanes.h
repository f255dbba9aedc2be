// Lane-per-body helpers of the double-precision chain kernels: small
// vector and quaternion types, the cylinder's inverse inertia, the paper's
// pressure law, and the exchanges and reductions along a chain whose body i
// sits in lane i (DPP moves inside a wave, LDS across the waves of a
// workgroup).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "kernels.h"

namespace snake {
namespace {

struct D3 {
    double x, y, z;
};
struct DQ {
    double w, x, y, z;
};
__device__ __forceinline__ D3 d3(double a, double b, double c) { return D3{a, b, c}; }
__device__ __forceinline__ D3 operator+(D3 a, D3 b) { return D3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ D3 operator-(D3 a, D3 b) { return D3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ D3 operator-(D3 a) { return D3{-a.x, -a.y, -a.z}; }
__device__ __forceinline__ D3 operator*(double s, D3 a) { return D3{s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ D3 cross(D3 a, D3 b)
{
    return D3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ DQ qmul(DQ a, DQ b)
{
    return DQ{a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z, a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
              a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x, a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}
__device__ __forceinline__ DQ qconj(DQ a) { return DQ{a.w, -a.x, -a.y, -a.z}; }
// body x axis in the world, R(q) e_x
__device__ __forceinline__ D3 qaxis(DQ q)
{
    return D3{1.0 - 2.0 * (q.y * q.y + q.z * q.z), 2.0 * (q.x * q.y + q.w * q.z), 2.0 * (q.x * q.z - q.w * q.y)};
}
// q <- normalize(q + 1/2 [0, dth] (x) q)
__device__ __forceinline__ DQ qturn(DQ q, D3 dth)
{
    const DQ t = qmul(DQ{0.0, dth.x, dth.y, dth.z}, q);
    DQ r{q.w + 0.5 * t.w, q.x + 0.5 * t.x, q.y + 0.5 * t.y, q.z + 0.5 * t.z};
    const double n = sqrt(r.w * r.w + r.x * r.x + r.y * r.y + r.z * r.z);
    return DQ{r.w / n, r.x / n, r.y / n, r.z / n};
}
// inverse inertia of a cylinder with axis a: c1 t + c2 (a.t) a
__device__ __forceinline__ D3 inv_inertia(D3 t, D3 a, double c1, double c2) { return c1 * t + (c2 * dot(a, t)) * a; }
__device__ __forceinline__ double inv_inertia_form(D3 s, D3 a, double c1, double c2)
{
    const double as = dot(a, s);
    return c1 * dot(s, s) + c2 * as * as;
}
// rows of the skew matrix [r]x (so [r]x v = r x v)
__device__ __forceinline__ D3 skew_row(D3 r, int k)
{
    return k == 0 ? D3{0.0, -r.z, r.y} : (k == 1 ? D3{r.z, 0.0, -r.x} : D3{-r.y, r.x, 0.0});
}

__device__ __forceinline__ double paper_pressure(const NParams& Q, double pf, double uf)
{
    // eq. delta_p_i / eq. deflation, once per step, in psi
    double p = pf * Q.amp, u = uf * Q.amp;
    if (u > p) {
        const double dp = (u - p) / Q.p_s;
        p = p + Q.p_s * dp * dp * Q.k_i;
    } else if (u < p) {
        p = fmax(p - fmin(p * Q.k_d, Q.T_p), u);
    }
    return p / Q.amp;
}

// One DPP move of a double (its two halves): lane permutations that run on
// the VALU with a few cycles of latency, where a lane shuffle goes through the
// LDS pipe and waits on its round trip.  Sources outside the wave read 0.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// the value of lane l (uniform across the wave)
__device__ __forceinline__ double row_value(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int kDppWaveShl1 = 0x130;   // lane i takes lane i+1
constexpr int kDppWaveShr1 = 0x138;   // lane i takes lane i-1

// Exchanges along the chain.  A snake of SEG <= 64 lanes sits inside one
// wave; a longer one spans SEG / 64 waves of its own workgroup and passes
// the boundary lanes through LDS (every lane of the workgroup calls these
// together, so the barriers are uniform).
template <int SEG, int K>
__device__ __forceinline__ void from_next(double (&v)[K], int lane, int wv, double* buf, int& ph)
{
    double r[K];
#pragma unroll
    for (int k = 0; k < K; ++k) r[k] = dpp_move<kDppWaveShl1>(v[k]);
    if constexpr (SEG > 64) {
        // two buffers used in turn: the one written here was last read
        // before the previous exchange's barrier
        double* b = buf + (ph & 1) * (SEG / 64) * 8;
        ++ph;
        if (lane == 0)
#pragma unroll
            for (int k = 0; k < K; ++k) b[wv * 8 + k] = v[k];
        __syncthreads();
        if (lane == 63 && wv + 1 < SEG / 64)
#pragma unroll
            for (int k = 0; k < K; ++k) r[k] = b[(wv + 1) * 8 + k];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = r[k];
}

template <int SEG, int K>
__device__ __forceinline__ void from_prev(double (&v)[K], int lane, int wv, double* buf, int& ph)
{
    double r[K];
#pragma unroll
    for (int k = 0; k < K; ++k) r[k] = dpp_move<kDppWaveShr1>(v[k]);
    if constexpr (SEG > 64) {
        double* b = buf + (ph & 1) * (SEG / 64) * 8;
        ++ph;
        if (lane == 63)
#pragma unroll
            for (int k = 0; k < K; ++k) b[wv * 8 + k] = v[k];
        __syncthreads();
        if (lane == 0 && wv > 0)
#pragma unroll
            for (int k = 0; k < K; ++k) r[k] = b[(wv - 1) * 8 + k];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = r[k];
}

// Sum (MAX = false) or maximum over the snake's lanes, the same bits in
// every lane: within rows of 16 lanes (8 for an 8-lane snake) by DPP swaps
// (quad [1,0,3,2], quad [2,3,0,1], then the half-row and row mirrors, which
// pair lanes already holding equal values, so each stage combines disjoint
// sets and every lane adds the same two operands), the rows of the snake
// read lane by lane and joined in a fixed order, then the waves' partials
// in order.
template <int SEG, bool MAX>
__device__ __forceinline__ double seg_reduce(double v, int lane, int wv, double* red, int& ph)
{
    constexpr int W = SEG < 64 ? SEG : 64;
    auto join = [](double a, double b) { return MAX ? fmax(a, b) : a + b; };
    v = join(v, dpp_move<0xB1>(v));
    v = join(v, dpp_move<0x4E>(v));
    v = join(v, dpp_move<0x141>(v));
    if constexpr (W >= 16) v = join(v, dpp_move<0x140>(v));
    if constexpr (W >= 32) {
        // every lane of a row now holds its row's value: read the four rows
        // into scalar registers and join them in a fixed order
        const double r0 = row_value(v, 0), r1 = row_value(v, 16);
        if constexpr (W == 32) {
            const double r2 = row_value(v, 32), r3 = row_value(v, 48);
            v = lane < 32 ? join(r0, r1) : join(r2, r3);
        } else {
            const double r2 = row_value(v, 32), r3 = row_value(v, 48);
            v = join(join(r0, r1), join(r2, r3));
        }
    }
    if constexpr (SEG > 64) {
        // two partial arrays used in turn, as the exchange buffers
        double* r = red + (ph & 1) * (SEG / 64);
        ++ph;
        if (lane == 0) r[wv] = v;
        __syncthreads();
        double a = r[0];
#pragma unroll
        for (int w = 1; w < SEG / 64; ++w) a = MAX ? fmax(a, r[w]) : a + r[w];
        v = a;
    }
    return v;
}

}  // namespace
}  // namespace snake
