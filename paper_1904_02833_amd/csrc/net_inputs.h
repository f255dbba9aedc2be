// Inputs of the warm-start network for joint gj, shared by the feature
// kernel and the solver's fused warm start: two rows (stretch, bend-twist),
// evaluated at the predicted state of the current substep in the predicted
// frame of the joint's first body (layout in snake.h, sim_step_record).
#pragma once

#include "device_math.h"
#include "kernels.h"

namespace snake {

// Snake of joint gj: the last s in [lo, hi] with joint_off[s] <= gj (the
// caller's range must hold it).
__device__ __forceinline__ int snake_of_joint(const KParams& P, int gj, int lo, int hi)
{
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (P.joint_off[mid] <= gj)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// f: the stretch row (entry 30 = 0); the bend-twist row is f with entries
// 19..21 replaced by lbn and entry 30 = 1.  The joint's snake is searched in
// [lo, hi].
__device__ __forceinline__ void joint_features(const KParams& P, int gj, int lo, int hi, float (&f)[32], V3& lbn)
{
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (P.joint_off[mid] <= gj)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int s = lo;
    const int i = gj - P.joint_off[s];
    const int B = P.Bn[s], S = P.Sn[s];
    const int a = P.body_off[s] + i, b = a + 1;
    const int gm = P.module_off[s] + i / S;
    const int N = P.N, J = P.J, n = P.n_snakes;
    auto ld3 = [&](const float* arr, int k) { return mk(arr[k], arr[N + k], arr[2 * N + k]); };
    auto ldq = [&](const float* arr, int k) { return Q4{arr[k], arr[N + k], arr[2 * N + k], arr[3 * N + k]}; };
    const V3 xa = ld3(P.x, a), xb = ld3(P.x, b);
    const V3 va = ld3(P.v, a), vb = ld3(P.v, b);
    const V3 wa = ld3(P.w, a), wb = ld3(P.w, b);
    const Q4 qa = ldq(P.q_pred, a), qb = ldq(P.q_pred, b);
    const float p0 = P.p[gm], p1 = P.p[P.Mt + gm];
    const bool intra = (i + 1) % S != 0;
    const float th0 = intra ? P.kappa_max * (p0 - p1) * P.L : 0.f;
    const float h = P.h, hl = P.half_L;
    const V3 aA = qaxis(qa), aB = qaxis(qb);
    const V3 rA = hl * aA, rB = (-hl) * aB;
    const Q4 qac = qconj(qa);
    // stretch violation at the predicted positions, then in body-A axes
    const V3 Cs = ((xa - xb) + h * (va - vb)) + (rA - rB);
    float s0h, c0h;
    sincosf(0.5f * th0, &s0h, &c0h);
    const Q4 t = qmul(qac, qb);
    Q4 e{c0h * t.w + s0h * t.z, c0h * t.x + s0h * t.y, c0h * t.y - s0h * t.x, c0h * t.z - s0h * t.w};
    if (e.w < 0.f) e = Q4{-e.w, -e.x, -e.y, -e.z};
    const V3 rel_v = (va + cross(wa, rA)) - (vb + cross(wb, rB));
    const float ref = P.lam_ref, refb = P.lam_ref * P.L;
    const V3 ls = mk(P.lam_j[gj], P.lam_j[J + gj], P.lam_j[2 * J + gj]);
    const V3 lb = mk(P.lam_j[3 * J + gj], P.lam_j[4 * J + gj], P.lam_j[5 * J + gj]);
    const V3 c = (1.f / P.L) * qrot(qac, Cs);
    f[0] = c.x; f[1] = c.y; f[2] = c.z;
    f[3] = 2.f * e.x; f[4] = 2.f * e.y; f[5] = 2.f * e.z;
    const V3 rv = (h / P.L) * qrot(qac, rel_v);
    f[6] = rv.x; f[7] = rv.y; f[8] = rv.z;
    const V3 rw = h * qrot(qac, wb - wa);
    f[9] = rw.x; f[10] = rw.y; f[11] = rw.z;
    const V3 gz = qrot(qac, mk(0.f, 0.f, 1.f));
    f[12] = gz.x; f[13] = gz.y; f[14] = gz.z;
    f[15] = p0; f[16] = p1; f[17] = P.cmd[gm]; f[18] = th0;
    f[22] = log10f(fmaxf(P.comp[s], 1e-30f));
    f[23] = log10f(fmaxf(P.comp[n + s], 1e-30f));
    f[24] = log10f(fmaxf(P.comp[2 * n + s], 1e-30f));
    f[25] = P.mu[s];
    f[26] = P.lam_c[a] / ref;
    f[27] = P.lam_c[b] / ref;
    f[28] = ((xa.z + h * va.z) - P.R) * P.inv_L;
    f[29] = ((xb.z + h * vb.z) - P.R) * P.inv_L;
    f[31] = B > 1 ? (float)i / (float)(B - 1) : 0.f;
    // stretch row; the bend-twist row differs in entries 19..21 and 30
    const V3 lsl = (1.f / ref) * qrot(qac, ls);
    f[19] = lsl.x; f[20] = lsl.y; f[21] = lsl.z; f[30] = 0.f;
    lbn = mk(lb.x / refb, lb.y / refb, lb.z / refb);
}

}  // namespace snake
