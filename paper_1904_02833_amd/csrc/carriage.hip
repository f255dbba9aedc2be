// Block-Jacobi iterations for the wheeled carriage (section "Rigid Body
// Joints and Contact"; section "Soft robotic snake model": the wheels give
// the snake its anisotropic friction).
//
// Blocks: the chain's stretch and bend-twist joints; per wheel a hinge
// position block (the attachment form of eq. rigid_to_particle, wheel centre
// at a fixed point of its segment), a hinge axis block (the bend-twist form
// at rest angle 0 with its spin row free: two rigid rows) and a contact
// block with the ground (normal row at the wheel's lowest rim point,
// friction rows on the material point that touched at the start of the
// substep, projected onto the Coulomb disc).  Each block takes its local
// solution scaled by relax over the larger degree of its bodies, as in the
// chain's Jacobi solver.  A wheel rolls at the cost of its spin inertia and
// slides sideways against the full friction cone.
//
// Layout: lane i holds segment i, joint i (bodies i, i+1) and the two
// wheels of segment i with their blocks, so the wheels add no exchange:
// only the joints talk to the neighbouring lanes, as in the Newton kernel
// (snakes of up to 64 lanes share a wave, longer ones take a workgroup).
// Everything runs in double; the state stays in the library's FP32 arrays
// between launches.
#include <hip/hip_runtime.h>
#include <math.h>

#include "blocks.h"
#include "carriage.h"
#include "fp64_recip.h"
#include "kernels.h"
#include "lanes.h"

namespace snake {

namespace {

// R(q) e_y and R(q) e_z
__device__ __forceinline__ D3 qcol1(DQ f)
{
    return D3{2.0 * (f.x * f.y - f.w * f.z), 1.0 - 2.0 * (f.x * f.x + f.z * f.z), 2.0 * (f.y * f.z + f.w * f.x)};
}
__device__ __forceinline__ D3 qcol2(DQ f)
{
    return D3{2.0 * (f.x * f.z + f.w * f.y), 2.0 * (f.y * f.z - f.w * f.x), 1.0 - 2.0 * (f.x * f.x + f.y * f.y)};
}

// Symmetric 3x3 system K u = b by the adjugate (K = J W J^T + E of a block,
// positive definite).
struct S3 {
    double a00, a01, a02, a11, a12, a22;
};

__device__ __forceinline__ D3 solve_sym3(const S3& K, D3 b)
{
    const double c00 = K.a11 * K.a22 - K.a12 * K.a12;
    const double c01 = K.a02 * K.a12 - K.a01 * K.a22;
    const double c02 = K.a01 * K.a12 - K.a02 * K.a11;
    const double c11 = K.a00 * K.a22 - K.a02 * K.a02;
    const double c12 = K.a01 * K.a02 - K.a00 * K.a12;
    const double c22 = K.a00 * K.a11 - K.a01 * K.a01;
    const double id = rcp64(K.a00 * c00 + K.a01 * c01 + K.a02 * c02);
    return D3{(c00 * b.x + c01 * b.y + c02 * b.z) * id, (c01 * b.x + c11 * b.y + c12 * b.z) * id,
              (c02 * b.x + c12 * b.y + c22 * b.z) * id};
}

// (alpha I + d0 u0 u0^T + d1 u1 u1^T)^-1 b through the 2x2 capacitance
// system (Woodbury): z = (I + D U^T U / alpha)^-1 D U^T b / alpha,
// u = (b - U z) / alpha, U = [u0 u1], D = diag(d0, d1).
__device__ __forceinline__ D3 solve_rank2(double alpha, D3 u0, double d0, D3 u1, double d1, D3 b)
{
    const double ia = rcp64(alpha);
    const double g00 = dot(u0, u0), g01 = dot(u0, u1), g11 = dot(u1, u1);
    const double y0 = d0 * dot(u0, b) * ia, y1 = d1 * dot(u1, b) * ia;
    const double m00 = 1.0 + d0 * g00 * ia, m01 = d0 * g01 * ia;
    const double m10 = d1 * g01 * ia, m11 = 1.0 + d1 * g11 * ia;
    const double idet = rcp64(m00 * m11 - m01 * m10);
    const double z0 = (m11 * y0 - m01 * y1) * idet, z1 = (m00 * y1 - m10 * y0) * idet;
    return ia * (b - (z0 * u0 + z1 * u1));
}

// s^T M t for the inverse inertia M of a body with symmetry axis a
__device__ __forceinline__ double iform(D3 s, D3 t, D3 a, double c1, double c2)
{
    return c1 * dot(s, t) + c2 * dot(a, s) * dot(a, t);
}

// q <- normalize(q + 1/2 [0, dth] (x) q), one reciprocal of the norm
__device__ __forceinline__ DQ qturn1(DQ q, D3 dth)
{
    const DQ t = qmul(DQ{0.0, dth.x, dth.y, dth.z}, q);
    const DQ r{q.w + 0.5 * t.w, q.x + 0.5 * t.x, q.y + 0.5 * t.y, q.z + 0.5 * t.z};
    const double in = rsqrt64(r.w * r.w + r.x * r.x + r.y * r.y + r.z * r.z);
    return DQ{r.w * in, r.x * in, r.y * in, r.z * in};
}

// larger of a and b, NaN kept
__device__ __forceinline__ double rmax(double a, double b) { return (b > a || b != b) ? b : a; }

// Lowest rim point of a wheel of radius rw with axle a, relative to its
// centre: -rw (e_z - a_z a) / |e_z - a_z a| (0 for a wheel lying flat).
__device__ __forceinline__ D3 low_point(D3 a, double rw)
{
    const D3 u{-a.z * a.x, -a.z * a.y, 1.0 - a.z * a.z};
    const double n2 = dot(u, u);
    return n2 > 0.0 ? (-rw * rsqrt64(n2)) * u : D3{0.0, 0.0, 0.0};
}

template <int SEG>
__global__ void __launch_bounds__(SEG > 64 ? SEG : 256) __attribute__((amdgpu_waves_per_eu(1)))
k_carriage(KParams P, NParams Q, WParams Wp, const int* __restrict__ list, int count, int n_steps)
{
    constexpr int WG = SEG > 64 ? SEG : 256;
    constexpr int NWV = SEG > 64 ? SEG / 64 : 1;
    __shared__ double xbuf[2 * NWV * 8];   // two buffers used in turn
    __shared__ double red[2 * NWV];
    int xph = 0, rph = 0;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int idx = blockIdx.x * (WG / SEG) + t / SEG;
    const int i = t % SEG;
    const int s = idx < count ? list[idx] : -1;
    const bool live = s >= 0;

    int B = 0, S = 1, bo = 0, mo = 0;
    double comp_s = 0.0, comp_b = 0.0, comp_t = 0.0, mu = 0.0;
    if (live) {
        B = P.Bn[s];
        S = P.Sn[s];
        bo = P.body_off[s];
        mo = P.module_off[s];
        comp_s = Q.comp[s];
        comp_b = Q.comp[P.n_snakes + s];
        comp_t = Q.comp[2 * P.n_snakes + s];
        mu = Q.mu[s];
    }
    const bool hasb = i < B;
    const bool hasj = i + 1 < B;
    const bool gnd = !(P.flags & kNoGround);
    const bool fixed = (P.flags & kFixedRoot) && i == 0;
    const int N = P.N, N2 = 2 * P.N, J = P.J, Mt = P.Mt;
    const int gb = bo + i, gj = bo - s + i;
    const int m = i / S, gm = mo + m;
    const bool intra = hasj && ((i + 1) % S != 0);
    const double h = Q.h, hl = 0.5 * Q.L, inv_L = 1.0 / Q.L;
    const double c1 = 1.0 / Q.I_pe, c2 = 1.0 / Q.I_ax - 1.0 / Q.I_pe;
    const double wA = (hasb && !fixed) ? 1.0 / Q.m : 0.0;
    const double c1A = (hasb && !fixed) ? c1 : 0.0, c2A = (hasb && !fixed) ? c2 : 0.0;
    const double wB = 1.0 / Q.m;
    const double wW = 1.0 / Wp.mw, c1W = 1.0 / Wp.Ip, c2W = 1.0 / Wp.Ia - 1.0 / Wp.Ip;
    // degrees: a segment has two blocks per joint and two per wheel, a
    // wheel its hinge position, hinge axis and contact
    const int degA = (i > 0 ? 2 : 0) + (hasj ? 2 : 0) + 4;
    const int degB = 2 + (i + 2 < B ? 2 : 0) + 4;
    const int degW = 2 + (gnd ? 1 : 0);
    const double scj = Wp.relax / (double)(degA > degB ? degA : degB);
    const double sch = Wp.relax / (double)(degA > degW ? degA : degW);
    const double scc = Wp.relax / (double)degW;
    const D3 zero{0.0, 0.0, 0.0};

    D3 x = zero, v = zero, w = zero;
    DQ q{1.0, 0.0, 0.0, 0.0};
    D3 ls = zero, lb = zero;
    D3 xw[2], vw[2], ww[2], lh[2], la[2], lc[2];
    DQ qw[2];
    double p0 = 0.0, p1 = 0.0, cmdv = 0.0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        xw[k] = vw[k] = ww[k] = lh[k] = la[k] = lc[k] = zero;
        qw[k] = DQ{1.0, 0.0, 0.0, 0.0};
    }
    if (hasb) {
        x = d3(P.x[gb], P.x[N + gb], P.x[2 * N + gb]);
        q = DQ{P.q[gb], P.q[N + gb], P.q[2 * N + gb], P.q[3 * N + gb]};
        v = d3(P.v[gb], P.v[N + gb], P.v[2 * N + gb]);
        w = d3(P.w[gb], P.w[N + gb], P.w[2 * N + gb]);
        p0 = P.p[gm];
        p1 = P.p[Mt + gm];
        cmdv = P.cmd[gm];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int g = 2 * gb + k;
            xw[k] = d3(Wp.x[g], Wp.x[N2 + g], Wp.x[2 * N2 + g]);
            qw[k] = DQ{Wp.q[g], Wp.q[N2 + g], Wp.q[2 * N2 + g], Wp.q[3 * N2 + g]};
            vw[k] = d3(Wp.v[g], Wp.v[N2 + g], Wp.v[2 * N2 + g]);
            ww[k] = d3(Wp.w[g], Wp.w[N2 + g], Wp.w[2 * N2 + g]);
        }
    }
    if (hasj) {
        ls = d3(P.lam_j[gj], P.lam_j[J + gj], P.lam_j[2 * J + gj]);
        lb = d3(P.lam_j[3 * J + gj], P.lam_j[4 * J + gj], P.lam_j[5 * J + gj]);
    }

    float rstep = 0.f;
    int itstep = 0, status = 0, itsum = 0;
    for (int st = 0; st < n_steps; ++st) {
        const long long stepc = (live ? P.step[s] : 0) + st;
        // command for the end of this step (eq. snake_control or a schedule)
        if (hasb && P.controller == kCtrlSerpenoid)
            cmdv = serpenoid_command(P, s, m, stepc);
        else if (hasb && P.controller == kCtrlSchedule)
            cmdv = schedule_command(P, gm, stepc);
        if (P.law == kLawPaper) {
            p0 = paper_pressure(Q, p0, fmax(cmdv, 0.0));
            p1 = paper_pressure(Q, p1, fmax(-cmdv, 0.0));
        }
        const double u0 = fmax(cmdv, 0.0), u1 = fmax(-cmdv, 0.0);
        rstep = 0.f;
        itstep = 0;
        status = 0;
        for (int sub = 0; sub < P.substeps; ++sub) {
            if (P.law == kLawLag) {
                p0 = u0 + (p0 - u0) * (u0 > p0 ? Q.lag_in : Q.lag_de);
                p1 = u1 + (p1 - u1) * (u1 > p1 ? Q.lag_in : Q.lag_de);
            }
            const double th0 = intra ? Q.kappa_max * (p0 - p1) * Q.L : 0.0;
            const DQ q0{cos(0.5 * th0), 0.0, 0.0, sin(0.5 * th0)};

            // start of the substep; the wheels' friction anchors (contact
            // point in the world, its arm in the wheel frame)
            const D3 xp = x;
            const DQ qp = q;
            D3 xpw[2], anc[2], arm[2];
            DQ qpw[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                xpw[k] = xw[k];
                qpw[k] = qw[k];
                const D3 r = low_point(qcol1(qw[k]), Wp.rw);
                anc[k] = xw[k] + r;
                arm[k] = d3(dot(qaxis(qw[k]), r), dot(qcol1(qw[k]), r), dot(qcol2(qw[k]), r));
            }

            // predicted positions: gravity, gyroscopic torque, one step of h
            if (hasb && !fixed) {
                v.z -= h * Q.g;
                x = x + h * v;
                const D3 ax = qaxis(q);
                const D3 Iw = Q.I_pe * w + ((Q.I_ax - Q.I_pe) * dot(ax, w)) * ax;
                const D3 tq = -cross(w, Iw);
                w = w + h * inv_inertia(tq, ax, c1, c2);
                q = qturn(q, h * w);
            } else if (fixed) {
                v = zero;
                w = zero;
            }
            if (hasb) {
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    vw[k].z -= h * Q.g;
                    xw[k] = xw[k] + h * vw[k];
                    const D3 ay = qcol1(qw[k]);
                    const D3 Iw = Wp.Ip * ww[k] + ((Wp.Ia - Wp.Ip) * dot(ay, ww[k])) * ay;
                    const D3 tq = -cross(ww[k], Iw);
                    ww[k] = ww[k] + h * inv_inertia(tq, ay, c1W, c2W);
                    qw[k] = qturn(qw[k], h * ww[k]);
                }
            }
            ls = zero;
            lb = zero;
#pragma unroll
            for (int k = 0; k < 2; ++k) lh[k] = la[k] = lc[k] = zero;

            int its = 0;
            double r = 0.0;
            for (;; ++its) {
                // ---- evaluate every block at the current iterate ----
                double nbq[7] = {x.x, x.y, x.z, q.w, q.x, q.y, q.z};
                from_next<SEG, 7>(nbq, lane, wv, xbuf, xph);
                const D3 xB = d3(nbq[0], nbq[1], nbq[2]);
                const DQ qB{nbq[3], nbq[4], nbq[5], nbq[6]};
                const D3 aA = qaxis(q), aB = qaxis(qB);
                const D3 ra = hl * aA, rb = -hl * aB;
                double rl = 0.0;
                D3 dls = zero, dlb = zero, A0 = zero, A1 = zero, A2 = zero;
                if (hasj) {
                    // stretch: end point of body i on start point of body i+1
                    const D3 Cs = (x + ra) - (xB + rb);
                    DQ e = qmul(qmul(qconj(q0), qconj(q)), qB);
                    if (e.w < 0.0) e = DQ{-e.w, -e.x, -e.y, -e.z};
                    const D3 Cb = d3(2.0 * e.x, 2.0 * e.y, 2.0 * e.z);
                    const DQ f = qmul(q, q0);
                    const D3 F0 = qaxis(f), F1 = qcol1(f), F2 = qcol2(f);
                    const D3 G0{e.w, e.z, -e.y}, G1{-e.z, e.w, e.x}, G2{e.y, -e.x, e.w};
                    A0 = G0.x * F0 + G0.y * F1 + G0.z * F2;
                    A1 = G1.x * F0 + G1.y * F1 + G1.z * F2;
                    A2 = G2.x * F0 + G2.y * F1 + G2.z * F2;
                    // stretch block: K = (wA + wB + comp) I + [ra]x IA [ra]x^T + [rb]x IB [rb]x^T;
                    // each arm lies on its body's axis, so [r]x I^-1 [r]x^T = c1 (|r|^2 I - r r^T)
                    const D3 rs = Cs + comp_s * ls;
                    rl = rmax(rl, rmax(rmax(fabs(rs.x), fabs(rs.y)), fabs(rs.z)) * inv_L);
                    dls = -scj * solve_rank2(wA + wB + comp_s + c1A * dot(ra, ra) + c1 * dot(rb, rb), ra, -c1A, rb,
                                             -c1, rs);
                    // bend-twist block: K = A (IA + IB) A^T + comp
                    auto kb = [&](D3 u, D3 vv) { return iform(u, vv, aA, c1A, c2A) + iform(u, vv, aB, c1, c2); };
                    const S3 Kb{kb(A0, A0) + comp_t, kb(A0, A1), kb(A0, A2), kb(A1, A1) + comp_b, kb(A1, A2),
                                kb(A2, A2) + comp_b};
                    const D3 rbv = d3(Cb.x + comp_t * lb.x, Cb.y + comp_b * lb.y, Cb.z + comp_b * lb.z);
                    rl = rmax(rl, rmax(rmax(fabs(rbv.x), fabs(rbv.y)), fabs(rbv.z)));
                    dlb = -scj * solve_sym3(Kb, rbv);
                }
                D3 dlh[2], dla[2], dlc[2], rh[2], H0[2], H2[2], rlow[2], sarm[2];
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    dlh[k] = dla[k] = dlc[k] = rh[k] = H0[k] = H2[k] = rlow[k] = sarm[k] = zero;
                    if (!hasb) continue;
                    const D3 aW = qcol1(qw[k]);
                    // hinge position: x + R(q) (0, +-dw, -hw) - x_wheel
                    rh[k] = (k == 0 ? Wp.dw : -Wp.dw) * qcol1(q) - Wp.hw * qcol2(q);
                    const D3 Ch = (x + rh[k]) - xw[k];
                    {
                        // K = (wA + wW) I + [rh]x IA [rh]x^T
                        //   = (wA + wW + c1 |rh|^2) I - c1 rh rh^T + c2 (rh x a)(rh x a)^T
                        rl = rmax(rl, rmax(rmax(fabs(Ch.x), fabs(Ch.y)), fabs(Ch.z)) * inv_L);
                        dlh[k] = -sch * solve_rank2(wA + wW + c1A * dot(rh[k], rh[k]), rh[k], -c1A, cross(rh[k], aA),
                                                    c2A, Ch);
                    }
                    // hinge axis: e = conj(q) q_wheel, rows x and z rigid
                    {
                        DQ e = qmul(qconj(q), qw[k]);
                        if (e.w < 0.0) e = DQ{-e.w, -e.x, -e.y, -e.z};
                        const D3 F0 = qaxis(q), F1 = qcol1(q), F2 = qcol2(q);
                        const D3 G0{e.w, e.z, -e.y}, G2{e.y, -e.x, e.w};
                        H0[k] = G0.x * F0 + G0.y * F1 + G0.z * F2;
                        H2[k] = G2.x * F0 + G2.y * F1 + G2.z * F2;
                        const double k00 = iform(H0[k], H0[k], aA, c1A, c2A) + iform(H0[k], H0[k], aW, c1W, c2W);
                        const double k02 = iform(H0[k], H2[k], aA, c1A, c2A) + iform(H0[k], H2[k], aW, c1W, c2W);
                        const double k22 = iform(H2[k], H2[k], aA, c1A, c2A) + iform(H2[k], H2[k], aW, c1W, c2W);
                        const double r0 = 2.0 * e.x, r2 = 2.0 * e.z;
                        rl = rmax(rl, rmax(fabs(r0), fabs(r2)));
                        const double id = rcp64(k00 * k22 - k02 * k02);
                        dla[k] = d3(-sch * (k22 * r0 - k02 * r2) * id, 0.0, -sch * (k00 * r2 - k02 * r0) * id);
                    }
                    // contact: lowest rim point; friction on the anchored material point
                    if (gnd) {
                        rlow[k] = low_point(aW, Wp.rw);
                        sarm[k] = arm[k].x * qaxis(qw[k]) + arm[k].y * aW + arm[k].z * qcol2(qw[k]);
                        const D3 jn = cross(rlow[k], d3(0.0, 0.0, 1.0));
                        const D3 j0 = cross(sarm[k], d3(1.0, 0.0, 0.0));
                        const D3 j1 = cross(sarm[k], d3(0.0, 1.0, 0.0));
                        const double cn = xw[k].z + rlow[k].z;
                        const double c0 = xw[k].x + sarm[k].x - anc[k].x;
                        const double c1t = xw[k].y + sarm[k].y - anc[k].y;
                        const double rc = lc[k].x > 0.0 ? fabs(cn) : (cn < 0.0 ? -cn : 0.0);
                        rl = rmax(rl, rc * inv_L);
                        const double knn = wW + iform(jn, jn, aW, c1W, c2W);
                        const double k11 = wW + iform(j0, j0, aW, c1W, c2W);
                        const double k12 = iform(j0, j1, aW, c1W, c2W);
                        const double k22 = wW + iform(j1, j1, aW, c1W, c2W);
                        double ln = lc[k].x + scc * (-cn * rcp64(knn));
                        if (ln < 0.0) ln = 0.0;
                        const double idet = rcp64(k11 * k22 - k12 * k12);
                        const double y0 = (k22 * c0 - k12 * c1t) * idet;
                        const double y1 = (k11 * c1t - k12 * c0) * idet;
                        double lt0 = lc[k].y - scc * y0, lt1 = lc[k].z - scc * y1;
                        const double cap = mu * ln;
                        const double nt2 = lt0 * lt0 + lt1 * lt1;
                        if (ln <= 0.0) {
                            lt0 = lt1 = 0.0;
                        } else if (nt2 > cap * cap) {
                            const double f = cap * rsqrt64(nt2);
                            lt0 *= f;
                            lt1 *= f;
                        }
                        dlc[k] = d3(ln - lc[k].x, lt0 - lc[k].y, lt1 - lc[k].z);
                    }
                }
                r = seg_reduce<SEG, true>(rl != rl ? INFINITY : rl, lane, wv, red, rph);
                if (!(r < INFINITY)) {
                    status |= kStatusNonfinite;
                    break;
                }
                const bool stop = Q.tol > 0.0 ? (r <= Q.tol || its >= P.iters) : (its >= P.iters);
                if (stop) {
                    if (Q.tol > 0.0 && r > Q.tol) status |= kStatusNotConverged;
                    break;
                }

                // ---- apply: multipliers, then every body by W J^T dl ----
                ls = ls + dls;
                lb = lb + dlb;
                // joint i's share of body i+1, passed on to the next lane
                const D3 Atb = dlb.x * A0 + dlb.y * A1 + dlb.z * A2;
                double nb6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                if (hasj) {
                    const D3 tB = Atb - cross(rb, dls);
                    nb6[0] = -dls.x;
                    nb6[1] = -dls.y;
                    nb6[2] = -dls.z;
                    nb6[3] = tB.x;
                    nb6[4] = tB.y;
                    nb6[5] = tB.z;
                }
                from_prev<SEG, 6>(nb6, lane, wv, xbuf, xph);
                D3 f = zero, tq = zero;
                if (hasb && i > 0) {
                    f = d3(nb6[0], nb6[1], nb6[2]);
                    tq = d3(nb6[3], nb6[4], nb6[5]);
                }
                if (hasj) {
                    f = f + dls;
                    tq = tq + (cross(ra, dls) - Atb);
                }
                if (hasb) {
#pragma unroll
                    for (int k = 0; k < 2; ++k) {
                        lh[k] = lh[k] + dlh[k];
                        la[k] = la[k] + dla[k];
                        lc[k] = lc[k] + dlc[k];
                        const D3 Ath = dla[k].x * H0[k] + dla[k].z * H2[k];
                        f = f + dlh[k];
                        tq = tq + (cross(rh[k], dlh[k]) - Ath);
                        // the wheel: hinge position, hinge axis, contact
                        D3 fw = -dlh[k], tw = Ath;
                        if (gnd) {
                            fw = fw + d3(dlc[k].y, dlc[k].z, dlc[k].x);
                            tw = tw + dlc[k].x * cross(rlow[k], d3(0.0, 0.0, 1.0)) +
                                 dlc[k].y * cross(sarm[k], d3(1.0, 0.0, 0.0)) +
                                 dlc[k].z * cross(sarm[k], d3(0.0, 1.0, 0.0));
                        }
                        xw[k] = xw[k] + wW * fw;
                        qw[k] = qturn1(qw[k], inv_inertia(tw, qcol1(qw[k]), c1W, c2W));
                    }
                    if (!fixed) {
                        x = x + wA * f;
                        q = qturn1(q, inv_inertia(tq, aA, c1A, c2A));
                    }
                }
            }
            itstep += its;
            rstep = fmaxf(rstep, (float)r);

            // velocities of the implicit step
            if (hasb && !fixed) {
                v = (1.0 / h) * (x - xp);
                const DQ dq = qmul(q, qconj(qp));
                const double sg = dq.w >= 0.0 ? 2.0 / h : -2.0 / h;
                w = d3(sg * dq.x, sg * dq.y, sg * dq.z);
            }
            if (hasb) {
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    vw[k] = (1.0 / h) * (xw[k] - xpw[k]);
                    const DQ dq = qmul(qw[k], qconj(qpw[k]));
                    const double sg = dq.w >= 0.0 ? 2.0 / h : -2.0 / h;
                    ww[k] = d3(sg * dq.x, sg * dq.y, sg * dq.z);
                }
            }
        }
        itsum += itstep;
    }

    if (hasb) {
        P.x[gb] = (float)x.x;
        P.x[N + gb] = (float)x.y;
        P.x[2 * N + gb] = (float)x.z;
        P.q[gb] = (float)q.w;
        P.q[N + gb] = (float)q.x;
        P.q[2 * N + gb] = (float)q.y;
        P.q[3 * N + gb] = (float)q.z;
        P.v[gb] = (float)v.x;
        P.v[N + gb] = (float)v.y;
        P.v[2 * N + gb] = (float)v.z;
        P.w[gb] = (float)w.x;
        P.w[N + gb] = (float)w.y;
        P.w[2 * N + gb] = (float)w.z;
        if (i % S == 0) {
            P.p[gm] = (float)p0;
            P.p[Mt + gm] = (float)p1;
            P.cmd[gm] = (float)cmdv;
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int g = 2 * gb + k;
            Wp.x[g] = (float)xw[k].x;
            Wp.x[N2 + g] = (float)xw[k].y;
            Wp.x[2 * N2 + g] = (float)xw[k].z;
            Wp.q[g] = (float)qw[k].w;
            Wp.q[N2 + g] = (float)qw[k].x;
            Wp.q[2 * N2 + g] = (float)qw[k].y;
            Wp.q[3 * N2 + g] = (float)qw[k].z;
            Wp.v[g] = (float)vw[k].x;
            Wp.v[N2 + g] = (float)vw[k].y;
            Wp.v[2 * N2 + g] = (float)vw[k].z;
            Wp.w[g] = (float)ww[k].x;
            Wp.w[N2 + g] = (float)ww[k].y;
            Wp.w[2 * N2 + g] = (float)ww[k].z;
            const double lw[9] = {lh[k].x, lh[k].y, lh[k].z, la[k].x, la[k].y, la[k].z, lc[k].x, lc[k].y, lc[k].z};
#pragma unroll
            for (int c = 0; c < 9; ++c) Wp.lam[c * N2 + g] = (float)lw[c];
        }
    }
    if (hasj) {
        P.lam_j[gj] = (float)ls.x;
        P.lam_j[J + gj] = (float)ls.y;
        P.lam_j[2 * J + gj] = (float)ls.z;
        P.lam_j[3 * J + gj] = (float)lb.x;
        P.lam_j[4 * J + gj] = (float)lb.y;
        P.lam_j[5 * J + gj] = (float)lb.z;
    }
    if constexpr (SEG > 64) __syncthreads();   // every lane has read step[s] before it moves
    if (live && i == 0) {
        P.residual[s] = rstep;
        P.iters_out[s] = itstep;
        P.status[s] = status;
        P.step[s] = P.step[s] + n_steps;
        P.iters_total[s] = P.iters_total[s] + itsum;
    }
}

__global__ void k_init_wheels(KParams P, WParams Wp)
{
    const int gb = blockIdx.x * blockDim.x + threadIdx.x;
    if (gb >= P.N) return;
    const int N = P.N, N2 = 2 * P.N;
    for (int k = 0; k < 2; ++k) {
        const int g = 2 * gb + k;
        Wp.x[g] = P.x[gb];
        Wp.x[N2 + g] = (float)((double)P.x[N + gb] + (k == 0 ? Wp.dw : -Wp.dw));
        Wp.x[2 * N2 + g] = (float)((double)P.x[2 * N + gb] - Wp.hw);
        Wp.q[g] = 1.f;
        Wp.q[N2 + g] = Wp.q[2 * N2 + g] = Wp.q[3 * N2 + g] = 0.f;
        for (int d = 0; d < 3; ++d) Wp.v[d * N2 + g] = Wp.w[d * N2 + g] = 0.f;
        for (int c = 0; c < 9; ++c) Wp.lam[c * N2 + g] = 0.f;
    }
}

}  // namespace

hipError_t launch_init_wheels(const KParams& P, const WParams& Wp, hipStream_t stream)
{
    hipLaunchKernelGGL(k_init_wheels, dim3((P.N + 255) / 256), dim3(256), 0, stream, P, Wp);
    return hipGetLastError();
}

hipError_t launch_carriage(const KParams& P, const NParams& Q, const WParams& Wp, const int* list, const int* off,
                           int n_steps, hipStream_t stream)
{
    if (n_steps <= 0) return hipSuccess;
#define CARRIAGE_CLASS(C, SEGV)                                                                           \
    if (off[C + 1] > off[C]) {                                                                            \
        const int cnt = off[C + 1] - off[C];                                                              \
        constexpr int wg = SEGV > 64 ? SEGV : 256;                                                        \
        const int per = wg / SEGV;                                                                        \
        hipLaunchKernelGGL((k_carriage<SEGV>), dim3((cnt + per - 1) / per), dim3(wg), 0, stream, P, Q, Wp, \
                           list + off[C], cnt, n_steps);                                                  \
        hipError_t e = hipGetLastError();                                                                 \
        if (e != hipSuccess) return e;                                                                    \
    }
    CARRIAGE_CLASS(0, 8)
    CARRIAGE_CLASS(1, 16)
    CARRIAGE_CLASS(2, 32)
    CARRIAGE_CLASS(3, 64)
    CARRIAGE_CLASS(4, 128)
    CARRIAGE_CLASS(5, 256)
    CARRIAGE_CLASS(6, 512)
    CARRIAGE_CLASS(7, 1024)
#undef CARRIAGE_CLASS
    return hipSuccess;
}

}  // namespace snake
