// Block evaluations shared by the FP32 solver kernels (block Jacobi and
// block Gauss-Seidel): the stretch and bend-twist blocks of a joint with
// their local solutions, the forces and torques a joint's increments put on
// its two bodies, the inverse inertia of a segment and the projected
// increments of a contact block.  Also the paper's chamber latency law.
#pragma once

#include "device_math.h"
#include "kernels.h"

namespace snake {

// geometry of joint i needed again by the increment application
struct Geo {
    V3 aA, aB;   // body axes; the attachment offsets are +-L/2 along them
    Q4 e, qA0;   // joint error quaternion; qA q0 (body A's frame turned by the rest rotation)
};

__device__ __forceinline__ float paper_update(const KParams& P, float pf, float uf)
{
    // eq. delta_p_i / eq. deflation, applied once per step, in psi
    float p = pf * P.amp, u = uf * P.amp;
    if (u > p) {
        float dp = (u - p) / P.p_s;
        p = p + P.p_s * dp * dp * P.k_i;
    } else if (u < p) {
        float cut = fminf(p * P.k_d, P.T_p);
        p = fmaxf(p - cut, u);
    }
    return p / P.amp;
}

// Stretch and bend-twist blocks of joint (A = i, B = i+1) at the current
// iterate.  Returns the unscaled local solutions -(K + alpha~)^-1 (C + alpha~ l)
// and the block residuals.
__device__ __forceinline__ void joint_eval(V3 dxp, V3 dA, V3 dB, Q4 qA, Q4 qB, V3 aA, V3 aB,
                                           float c0h, float s0h, float ct, float st, float wA,
                                           float c1A, float c2A, float wB, float c1B, float c2B,
                                           float hl, float inv_L, float comp_s, float comp_b,
                                           float comp_t, V3 ls, V3 lb, Geo& g, V3& Dls, V3& Dlb,
                                           float& rs, float& rb)
{
    g.aA = aA;   // body x axes R(q) e_x of A and B
    g.aB = aB;

    // stretch: end point of A minus start point of B (eq. rigid_to_particle
    // form), the attachment offsets rA = hl aA and rB = -hl aB
    const V3 C = fma3(hl, aA + aB, dxp + (dA - dB));
    const V3 rhs = fma3(comp_s, ls, C);
    // K + alpha~ = (wA + wB + comp_s) I + kA (I - a a^T) + kB (I - b b^T) with the unit
    // axes a, b and kX = c1X hl^2, i.e. dg I - U diag(kA, kB) U^T with U = [a b].
    // Woodbury: (K + alpha~)^-1 r = (r + U M^-1 diag(kA, kB) U^T r) / dg with the
    // 2x2 matrix M = [[dg - kA, -kA g], [-kB g, dg - kB]], g = a.b (det M > 0).
    const float kA = c1A * (hl * hl), kB = c1B * (hl * hl);
    const float dg = wA + wB + kA + kB + comp_s;
    const V3 a = g.aA, b = g.aB;
    const float ar = dot(a, rhs), br = dot(b, rhs), gab = dot(a, b);
    const float pA = dg - kA, pB = dg - kB;
    const float det = pA * pB - (kA * kB) * (gab * gab);
    const float u1 = kA * ar, u2 = kB * br;
    const float f = __builtin_amdgcn_rcpf(det * dg);
    const float y1 = (pB * u1 + (kA * gab) * u2) * f;
    const float y2 = ((kB * gab) * u1 + pA * u2) * f;
    const float inv_dg = __builtin_amdgcn_rcpf(dg);
    Dls = fma3(-y2, b, fma3(-y1, a, (-inv_dg) * rhs));
    rs = amax3(rhs) * inv_L;

    // bend-twist: e = conj(qA q0) qB with q0 = (c0h, 0, 0, s0h)
    const Q4 qA0{qA.w * c0h - qA.z * s0h, qA.x * c0h + qA.y * s0h, qA.y * c0h - qA.x * s0h,
                 qA.z * c0h + qA.w * s0h};
    g.qA0 = qA0;
    Q4 e = qmul(qconj(qA0), qB);
    if (e.w < 0.f) e = Q4{-e.w, -e.x, -e.y, -e.z};
    g.e = e;
    const V3 ev{e.x, e.y, e.z};
    const V3 rhsb = fma3(2.f, ev, mk(comp_t * lb.x, comp_b * lb.y, comp_b * lb.z));
    // K = G F^T (IA^-1 + IB^-1) F G^T, G = e_w I - [e]x, F = R(qA q0):
    //   (c1A + c1B)(|e|^2 I - e e^T) + c2A gA gA^T + c2B gB gB^T
    // with gX = G uX and uA = R(q0)^T e_x = (ct, -st, 0), uB = R(e) e_x
    const V3 ga{fmaf(e.w, ct, -(ev.z * st)), fmaf(-e.w, st, -(ev.z * ct)), fmaf(ev.x, st, ev.y * ct)};
    const V3 ub = qaxis(e);
    const V3 gb = fma3(e.w, ub, -cross(ev, ub));
    const float M1 = c1A + c1B;
    const float n2 = e.w * e.w + dot(ev, ev);
    Dlb = -sym3_solve(M1 * (n2 - ev.x * ev.x) + c2A * ga.x * ga.x + c2B * gb.x * gb.x + comp_t,
                      -M1 * ev.x * ev.y + c2A * ga.x * ga.y + c2B * gb.x * gb.y,
                      -M1 * ev.x * ev.z + c2A * ga.x * ga.z + c2B * gb.x * gb.z,
                      M1 * (n2 - ev.y * ev.y) + c2A * ga.y * ga.y + c2B * gb.y * gb.y + comp_b,
                      -M1 * ev.y * ev.z + c2A * ga.y * ga.z + c2B * gb.y * gb.z,
                      M1 * (n2 - ev.z * ev.z) + c2A * ga.z * ga.z + c2B * gb.z * gb.z + comp_b, rhsb);
    rb = amax3(rhsb);
}

// J^T of joint increments (dls, dlb): the force on body A is dls (on B, -dls);
// the torques on A and B are tA, tB.  Stretch: rA x dl with rA = hl aA (and
// -rB x dl with rB = -hl aB); bend-twist: -/+ z with z = R(qA q0) G^T dlb,
// G = e_w I - [e]x.  Each body applies its inverse mass and inertia to the
// sum of what its joints send it.
__device__ __forceinline__ void joint_torques(const Geo& g, V3 dls, V3 dlb, float hl, V3& tA, V3& tB)
{
    const V3 ev{g.e.x, g.e.y, g.e.z};
    const V3 z = qrot(g.qA0, fma3(g.e.w, dlb, cross(ev, dlb)));
    tA = fma3(hl, cross(g.aA, dls), -z);
    tB = fma3(hl, cross(g.aB, dls), z);
}

// I^-1 t = c1 t + c2 (a . t) a for a body with axis a (c1 = c2 = 0: fixed)
__device__ __forceinline__ V3 inv_inertia(V3 t, V3 a, float c1, float c2)
{
    return fma3(c2 * dot(a, t), a, c1 * t);
}

// increments of the contact block of a body (normal, tangent x, tangent y)
__device__ __forceinline__ V3 contact_incr(V3 lc, float cn, V3 d, float sc, float m, float mu)
{
    const float ln = fmaxf(0.f, lc.x - sc * m * cn);
    float t0 = lc.y - sc * m * d.x;
    float t1 = lc.z - sc * m * d.y;
    const float cap = mu * ln;
    const float n2 = t0 * t0 + t1 * t1;
    if (ln <= 0.f) {
        t0 = 0.f;
        t1 = 0.f;
    } else if (n2 > cap * cap) {
        // onto the disc of radius cap: scale by cap / |t| (hardware rsqrt)
        const float f = cap * __builtin_amdgcn_rsqf(n2);
        t0 *= f;
        t1 *= f;
    }
    return V3{ln - lc.x, t0 - lc.y, t1 - lc.z};
}

// Command of module m of snake s for the end of step stepc (eq.
// snake_control): clamp(sin(2 pi f t + alpha m + phase0) + offset, -1, 1),
// t = (stepc + 1) dt, evaluated in double.
__device__ __forceinline__ double serpenoid_command(const KParams& P, int s, int m, long long stepc)
{
    const double freq = P.freq[s], ph0 = P.phase0[s];
    const double t = (double)(stepc + 1) * P.dt;
    const double a = sin(6.283185307179586476925286766559 * freq * t + P.ctrl_alpha * m + ph0) + P.ctrl_offset;
    return fmin(1.0, fmax(-1.0, a));
}

// Command of global module gm at step stepc from a piecewise-constant
// schedule: the last piece starting at or before stepc (binary search).
__device__ __forceinline__ float schedule_command(const KParams& P, int gm, long long stepc)
{
    int lo = P.sched_off[gm], hi = P.sched_off[gm + 1] - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((long long)P.sched_start[mid] <= stepc)
            lo = mid;
        else
            hi = mid - 1;
    }
    return P.sched_val[lo];
}

}  // namespace snake
