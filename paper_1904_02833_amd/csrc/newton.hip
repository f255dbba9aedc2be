// The paper's own solver for the implicit step (section "Time-Stepping"):
// Newton iterations, each solving the Schur-complement system of
// eq. schur_system, [J W J^T + E] dl = b, with a fixed number of
// preconditioned conjugate-residual iterations (diagonal preconditioner),
// contact through a Fischer-Burmeister reformulation.
//
// Everything runs in double (commands and pressures too): the system's
// conditioning (compliant stretch rows next to contact rows) is far beyond
// what a Krylov iteration keeps in single precision.  State stays in the
// library's FP32 arrays between launches.
//
// Layout: a snake takes SEG lanes (a power of two >= its body count, at
// least 8), lane i holding body i, joint i (bodies i, i+1: the stretch and
// bend-twist blocks) and contact i.  Snakes of up to 64 lanes share a wave
// and exchange through lane shuffles only; longer ones take a workgroup of
// SEG / 64 waves joined through LDS at the wave boundaries.  The matrix is
// never formed: a product is the gather W J^T v onto the bodies (one
// exchange with the previous lane) followed by J u per block (one exchange
// with the next lane), as in the Jacobi update.
#include <hip/hip_runtime.h>
#include <math.h>

#include "blocks.h"
#include "fp64_recip.h"
#include "kernels.h"
#include "lanes.h"

namespace snake {

namespace {

// Below this the derivative of a contact row's reformulation with respect to
// the constraint value counts as zero (the row then fixes its increment).
constexpr double kEps = 1e-6;
// Scale of the friction natural map's trial, in body masses (every positive
// scale has the same roots; this one keeps the iterates of the workloads'
// contacts from cycling between stick and slip).
constexpr double kFrictionTrial = 10.0;

template <int SEG>
__global__ void __launch_bounds__(SEG > 64 ? SEG : 256) __attribute__((amdgpu_waves_per_eu(2)))
k_newton(KParams P, NParams Q, const int* __restrict__ list, int count, int n_steps)
{
    constexpr int WG = SEG > 64 ? SEG : 256;
    constexpr int NWV = SEG > 64 ? SEG / 64 : 1;
    __shared__ double xbuf[2 * NWV * 8];   // two buffers used in turn
    __shared__ double red[2 * NWV];
    // the kept (best) iterate of each lane: x, q, stretch, bend-twist and
    // contact multipliers (each lane reads and writes only its own row)
    __shared__ double kept[WG][16];
    int xph = 0, rph = 0;   // which buffer the next exchange / reduction takes
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
    const bool hasc = hasb && gnd;
    const bool fixed = (P.flags & kFixedRoot) && i == 0;
    const int N = P.N, J = P.J, Mt = P.Mt;
    const int gb = bo + i, gj = bo - s + i;
    const int m = i / S, gm = mo + m;
    const bool intra = hasj && ((i + 1) % S != 0);
    const double h = Q.h, hl = 0.5 * Q.L, inv_L = 1.0 / Q.L;
    const double c1 = 1.0 / Q.I_pe, c2 = 1.0 / Q.I_ax - 1.0 / Q.I_pe;
    // body i (may be fixed) and body i+1 (never the fixed root)
    const double wA = (hasb && !fixed) ? 1.0 / Q.m : 0.0;
    const double c1A = (hasb && !fixed) ? c1 : 0.0, c2A = (hasb && !fixed) ? c2 : 0.0;
    const double wB = 1.0 / Q.m;
    const D3 zero{0.0, 0.0, 0.0};

    D3 x = zero, v = zero, w = zero;
    DQ q{1.0, 0.0, 0.0, 0.0};
    D3 ls = zero, lb = zero, lc = zero;
    double p0 = 0.0, p1 = 0.0, cmdv = 0.0;
    if (hasb) {
        x = d3(P.x[gb], P.x[N + gb], P.x[2 * N + gb]);
        q = DQ{P.q[gb], P.q[N + gb], P.q[2 * N + gb], P.q[3 * N + gb]};
        v = d3(P.v[gb], P.v[N + gb], P.v[2 * N + gb]);
        w = d3(P.w[gb], P.w[N + gb], P.w[2 * N + gb]);
        lc = d3(P.lam_c[gb], P.lam_c[N + gb], P.lam_c[2 * N + gb]);
        p0 = P.p[gm];
        p1 = P.p[Mt + gm];
        cmdv = P.cmd[gm];
    }
    if (hasj) {
        ls = d3(P.lam_j[gj], P.lam_j[J + gj], P.lam_j[2 * J + gj]);
        lb = d3(P.lam_j[3 * J + gj], P.lam_j[4 * J + gj], P.lam_j[5 * J + gj]);
    }

    // y = [J W J^T + E] v over the snake (v, y: stretch, bend-twist, contact
    // rows of this lane); also returns the body displacement u = W J^T v.
    D3 ra = zero, rb = zero, A0 = zero, A1 = zero, A2 = zero, aA = zero, aB = zero;
    double En = 0.0, Et00 = 0.0, Et01 = 0.0, Et11 = 0.0;
    auto gather = [&](D3 vs, D3 vb, D3 vc, D3& uf, D3& ut) {
        // joint i on body i (A) and on body i+1 (B)
        const D3 Atvb = vb.x * A0 + vb.y * A1 + vb.z * A2;   // A^T v_b
        D3 fA = zero, tA = zero;
        double nb6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (hasj) {
            fA = vs;
            tA = cross(ra, vs) - Atvb;
            const D3 tB = Atvb - cross(rb, vs);
            nb6[0] = -vs.x;
            nb6[1] = -vs.y;
            nb6[2] = -vs.z;
            nb6[3] = tB.x;
            nb6[4] = tB.y;
            nb6[5] = tB.z;
        }
        from_prev<SEG, 6>(nb6, lane, wv, xbuf, xph);
        D3 f = fA, tq = tA;
        if (hasb && i > 0) {
            f = d3(nb6[0], nb6[1], nb6[2]) + f;
            tq = d3(nb6[3], nb6[4], nb6[5]) + tq;
        }
        if (hasc) f = f + d3(vc.y, vc.z, vc.x);
        uf = hasb ? wA * f : zero;
        ut = hasb ? inv_inertia(tq, aA, c1A, c2A) : zero;
    };
    auto apply = [&](const double (&vin)[9], double (&y)[9]) {
        const D3 vs = d3(vin[0], vin[1], vin[2]), vb = d3(vin[3], vin[4], vin[5]), vc = d3(vin[6], vin[7], vin[8]);
        D3 uf, ut;
        gather(vs, vb, vc, uf, ut);
        double un[6] = {uf.x, uf.y, uf.z, ut.x, ut.y, ut.z};
        from_next<SEG, 6>(un, lane, wv, xbuf, xph);
        const D3 ufn = d3(un[0], un[1], un[2]), utn = d3(un[3], un[4], un[5]);
        if (hasj) {
            const D3 ys = (uf - cross(ra, ut)) - (ufn - cross(rb, utn)) + comp_s * vs;
            const D3 dt = utn - ut;
            y[0] = ys.x;
            y[1] = ys.y;
            y[2] = ys.z;
            y[3] = dot(A0, dt) + comp_t * vb.x;
            y[4] = dot(A1, dt) + comp_b * vb.y;
            y[5] = dot(A2, dt) + comp_b * vb.z;
        } else {
            for (int k = 0; k < 6; ++k) y[k] = 0.0;
        }
        if (hasc) {
            y[6] = uf.z + En * vc.x;
            y[7] = uf.x + Et00 * vc.y + Et01 * vc.z;
            y[8] = uf.y + Et01 * vc.y + Et11 * vc.z;
        } else {
            y[6] = y[7] = y[8] = 0.0;
        }
    };

    // Joint blocks at the current (x, q): constraint values, and the
    // geometry the products use (axes, attachment arms, bend Jacobian rows).
    auto evaluate = [&](DQ q0, D3& Cs, D3& Cb) {
        double nbq[7] = {x.x, x.y, x.z, q.w, q.x, q.y, q.z};
        from_next<SEG, 7>(nbq, lane, wv, xbuf, xph);
        const D3 xB = d3(nbq[0], nbq[1], nbq[2]);
        const DQ qB{nbq[3], nbq[4], nbq[5], nbq[6]};
        aA = qaxis(q);
        aB = qaxis(qB);
        ra = hl * aA;
        rb = -hl * aB;
        Cs = zero;
        Cb = zero;
        if (hasj) {
            Cs = (x + ra) - (xB + rb);
            DQ e = qmul(qmul(qconj(q0), qconj(q)), qB);
            if (e.w < 0.0) e = DQ{-e.w, -e.x, -e.y, -e.z};
            Cb = d3(2.0 * e.x, 2.0 * e.y, 2.0 * e.z);
            // d C_b = G F^T (dth_B - dth_A), G = e_w I - [e_xyz]x, F = R(q q0)
            const DQ f = qmul(q, q0);
            const D3 F0 = qaxis(f);   // columns of R(f)
            const D3 F1{2.0 * (f.x * f.y - f.w * f.z), 1.0 - 2.0 * (f.x * f.x + f.z * f.z),
                        2.0 * (f.y * f.z + f.w * f.x)};
            const D3 F2{2.0 * (f.x * f.z + f.w * f.y), 2.0 * (f.y * f.z - f.w * f.x),
                        1.0 - 2.0 * (f.x * f.x + f.y * f.y)};
            // row k of G F^T = sum_c G[k][c] F_c^T
            const D3 G0{e.w, e.z, -e.y}, G1{-e.z, e.w, e.x}, G2{e.y, -e.x, e.w};
            A0 = G0.x * F0 + G0.y * F1 + G0.z * F2;
            A1 = G1.x * F0 + G1.y * F1 + G1.z * F2;
            A2 = G2.x * F0 + G2.y * F1 + G2.z * F2;
        }
    };

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
            // rest rotation of joint i about body z, angle kappa_max (p0 - p1) L
            const double th0 = intra ? Q.kappa_max * (p0 - p1) * Q.L : 0.0;
            const DQ q0{cos(0.5 * th0), 0.0, 0.0, sin(0.5 * th0)};

            // predicted positions
            const D3 xp = x;
            const DQ qp = q;
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
            if (P.warm == kWarmPrev) {
                // the previous substep's multipliers, bodies moved by
                // W J(x~)^T lambda0 at the predicted state
                D3 Cs, Cb, uf, ut;
                evaluate(q0, Cs, Cb);
                gather(hasj ? ls : zero, hasj ? lb : zero, hasb && gnd ? lc : zero, uf, ut);
                if (hasb && !fixed) {
                    x = x + uf;
                    q = qturn(q, ut);
                }
            } else {
                ls = zero;
                lb = zero;
                lc = zero;
            }

            double r = 0.0, best = INFINITY;
            int its = 0;
            for (int k = 0;; ++k) {
                // blocks at the current iterate
                D3 Cs, Cb;
                evaluate(q0, Cs, Cb);
                const D3 Cc = d3(x.z - Q.R, x.x - xp.x, x.y - xp.y);

                // residual: the block-Jacobi measure and the friction natural map
                double rl = 0.0;
                if (hasj) {
                    const D3 es = Cs + comp_s * ls;
                    const D3 eb = Cb + d3(comp_t * lb.x, comp_b * lb.y, comp_b * lb.z);
                    rl = fmax(fmax(fabs(es.x), fmax(fabs(es.y), fabs(es.z))) * inv_L,
                              fmax(fabs(eb.x), fmax(fabs(eb.y), fabs(eb.z))));
                }
                if (hasc) {
                    rl = fmax(rl, (lc.x > 0.0 ? fabs(Cc.x) : fmax(-Cc.x, 0.0)) * inv_L);
                    if (wA != 0.0) {
                        const double mm = 1.0 / wA;
                        double y0 = lc.y - mm * Cc.y, y1 = lc.z - mm * Cc.z;
                        const double cap = mu * fmax(lc.x, 0.0);
                        const double ny = sqrt(y0 * y0 + y1 * y1);
                        if (ny > cap) {
                            const double f = ny > 0.0 ? cap / ny : 0.0;
                            y0 *= f;
                            y1 *= f;
                        }
                        const double e0 = lc.y - y0, e1 = lc.z - y1;
                        rl = fmax(rl, sqrt(e0 * e0 + e1 * e1) * wA * inv_L);
                    }
                }
                if (!(rl <= INFINITY)) rl = INFINITY;   // NaN
                r = seg_reduce<SEG, true>(rl, lane, wv, red, rph);
                if (Q.keep_best && r < best) {
                    best = r;
                    double* kp = kept[t];
                    kp[0] = x.x; kp[1] = x.y; kp[2] = x.z;
                    kp[3] = q.w; kp[4] = q.x; kp[5] = q.y; kp[6] = q.z;
                    kp[7] = ls.x; kp[8] = ls.y; kp[9] = ls.z;
                    kp[10] = lb.x; kp[11] = lb.y; kp[12] = lb.z;
                    kp[13] = lc.x; kp[14] = lc.y; kp[15] = lc.z;
                }
                if (!(r < INFINITY)) {
                    status |= kStatusNonfinite;
                    break;
                }
                if ((Q.tol > 0.0 && r <= Q.tol) || k >= Q.newton_iters) {
                    if (Q.tol > 0.0 && r > Q.tol) status |= kStatusNotConverged;
                    break;
                }

                // rows of eq. schur_system: right-hand side, compliance, free-row
                // projector, fixed increments, preconditioner diagonal
                double rhs[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, dg[9] = {1, 1, 1, 1, 1, 1, 1, 1, 1};
                double fixd[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
                const double pj = hasj ? 1.0 : 0.0;
                double pn = 0.0, pt00 = 0.0, pt01 = 0.0, pt11 = 0.0;
                En = Et00 = Et01 = Et11 = 0.0;
                if (hasj) {
                    rhs[0] = -(Cs.x + comp_s * ls.x);
                    rhs[1] = -(Cs.y + comp_s * ls.y);
                    rhs[2] = -(Cs.z + comp_s * ls.z);
                    rhs[3] = -(Cb.x + comp_t * lb.x);
                    rhs[4] = -(Cb.y + comp_b * lb.y);
                    rhs[5] = -(Cb.z + comp_b * lb.z);
#pragma unroll
                    for (int k2 = 0; k2 < 3; ++k2) {
                        dg[k2] = wA + wB + inv_inertia_form(skew_row(ra, k2), aA, c1A, c2A) +
                                 inv_inertia_form(skew_row(rb, k2), aB, c1, c2) + comp_s;
                    }
                    dg[3] = inv_inertia_form(A0, aA, c1A, c2A) + inv_inertia_form(A0, aB, c1, c2) + comp_t;
                    dg[4] = inv_inertia_form(A1, aA, c1A, c2A) + inv_inertia_form(A1, aB, c1, c2) + comp_b;
                    dg[5] = inv_inertia_form(A2, aA, c1A, c2A) + inv_inertia_form(A2, aB, c1, c2) + comp_b;
                }
                if (hasc && wA != 0.0) {
                    // normal: Fischer-Burmeister phi(a, b) of a = C_n, b = w l_n
                    const double a = Cc.x, bb = wA * lc.x;
                    const double rr = sqrt(a * a + bb * bb);
                    double fa, fb;
                    if (rr > 0.0) {
                        fa = 1.0 - a / rr;
                        fb = 1.0 - bb / rr;
                    } else {
                        fa = fb = 1.0 - sqrt(0.5);
                    }
                    const double phi = (a + bb > 0.0) ? 2.0 * a * bb / (a + bb + rr) : a + bb - rr;
                    if (fa > kEps) {
                        pn = 1.0;
                        En = wA * fb / fa;
                        rhs[6] = -phi / fa;
                    } else {
                        fixd[6] = -lc.x;   // a > 0 here: the root is b = 0
                    }
                    // friction: natural map onto the disc of radius mu max(l_n, 0)
                    const double mm = kFrictionTrial / wA;
                    const double y0 = lc.y - mm * Cc.y, y1 = lc.z - mm * Cc.z;
                    const double cap = mu * fmax(lc.x, 0.0);
                    const double ny = sqrt(y0 * y0 + y1 * y1);
                    if (cap > 0.0 && ny <= cap) {
                        pt00 = pt11 = 1.0;
                        rhs[7] = -Cc.y;
                        rhs[8] = -Cc.z;
                    } else if (!(cap > 0.0)) {
                        fixd[7] = -lc.y;
                        fixd[8] = -lc.z;
                    } else {
                        const double sl = cap / ny;
                        const double u0 = y0 / ny, u1 = y1 / ny, v0 = -u1, v1 = u0;
                        const double fpar = lc.y * u0 + lc.z * u1 - cap;
                        const double fper = lc.y * v0 + lc.z * v1;
                        const double eper = (1.0 - sl) / (mm * sl), bper = -fper / (mm * sl);
                        fixd[7] = -fpar * u0;
                        fixd[8] = -fpar * u1;
                        pt00 = v0 * v0;
                        pt01 = v0 * v1;
                        pt11 = v1 * v1;
                        Et00 = eper * v0 * v0;
                        Et01 = eper * v0 * v1;
                        Et11 = eper * v1 * v1;
                        rhs[7] = bper * v0;
                        rhs[8] = bper * v1;
                    }
                    dg[6] = wA + En;
                    dg[7] = wA + Et00;
                    dg[8] = wA + Et11;
                }
                // the preconditioner as reciprocals, once per Newton iteration
#pragma unroll
                for (int k2 = 0; k2 < 9; ++k2) dg[k2] = dg[k2] > 0.0 ? rcp64(dg[k2]) : 1.0;
                auto project = [&](double (&u)[9]) {
#pragma unroll
                    for (int k2 = 0; k2 < 6; ++k2) u[k2] *= pj;
                    u[6] *= pn;
                    const double t0 = pt00 * u[7] + pt01 * u[8], t1 = pt01 * u[7] + pt11 * u[8];
                    u[7] = t0;
                    u[8] = t1;
                };
                auto precondition = [&](const double (&u)[9], double (&o)[9]) {
#pragma unroll
                    for (int k2 = 0; k2 < 9; ++k2) o[k2] = u[k2];
                    project(o);
#pragma unroll
                    for (int k2 = 0; k2 < 9; ++k2) o[k2] *= dg[k2];
                    project(o);
                };
                auto sdot = [&](const double (&a)[9], const double (&b)[9]) {
                    double acc = 0.0;
#pragma unroll
                    for (int k2 = 0; k2 < 9; ++k2) acc += a[k2] * b[k2];
                    return seg_reduce<SEG, false>(acc, lane, wv, red, rph);
                };

                // preconditioned conjugate residual on the free rows
                double xs[9], z[9], pv[9], Ap[9], Az[9], Mq[9];
                apply(fixd, Az);
#pragma unroll
                for (int k2 = 0; k2 < 9; ++k2) Ap[k2] = rhs[k2] - Az[k2];
                project(Ap);
                precondition(Ap, z);
#pragma unroll
                for (int k2 = 0; k2 < 9; ++k2) {
                    xs[k2] = 0.0;
                    pv[k2] = z[k2];
                }
                apply(z, Az);
                project(Az);
#pragma unroll
                for (int k2 = 0; k2 < 9; ++k2) Ap[k2] = Az[k2];
                double rho = sdot(z, Az);
                for (int it = 0; it < Q.pcr_iters; ++it) {
                    if (!(rho > 0.0)) break;
                    precondition(Ap, Mq);
                    const double den = sdot(Ap, Mq);
                    if (!(den > 0.0)) break;
                    const double alpha = rho * rcp64(den);
#pragma unroll
                    for (int k2 = 0; k2 < 9; ++k2) {
                        xs[k2] += alpha * pv[k2];
                        z[k2] -= alpha * Mq[k2];
                    }
                    if (it == Q.pcr_iters - 1) break;
                    apply(z, Az);
                    project(Az);
                    const double rho1 = sdot(z, Az);
                    const double beta = rho1 * rcp64(rho);
                    rho = rho1;
#pragma unroll
                    for (int k2 = 0; k2 < 9; ++k2) {
                        pv[k2] = z[k2] + beta * pv[k2];
                        Ap[k2] = Az[k2] + beta * Ap[k2];
                    }
                }
#pragma unroll
                for (int k2 = 0; k2 < 9; ++k2) xs[k2] += fixd[k2];
                its += Q.pcr_iters;

                // lambda += dl, bodies += W J^T dl
                const D3 ds = d3(xs[0], xs[1], xs[2]), db = d3(xs[3], xs[4], xs[5]), dc = d3(xs[6], xs[7], xs[8]);
                D3 uf, ut;
                gather(ds, db, dc, uf, ut);
                if (hasj) {
                    ls = ls + ds;
                    lb = lb + db;
                }
                if (hasc) lc = lc + dc;
                if (hasb && !fixed) {
                    x = x + uf;
                    q = qturn(q, ut);
                }
            }
            if (Q.keep_best && !(r <= best) && best < INFINITY) {
                // end at the best evaluated iterate instead of the last
                r = best;
                const double* kp = kept[t];
                x = d3(kp[0], kp[1], kp[2]);
                q = DQ{kp[3], kp[4], kp[5], kp[6]};
                ls = d3(kp[7], kp[8], kp[9]);
                lb = d3(kp[10], kp[11], kp[12]);
                lc = d3(kp[13], kp[14], kp[15]);
                // (no status change: an iterate at or below tol ends the loop
                // itself, so the best one here is above tol whenever tol > 0)
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
        P.lam_c[gb] = (float)lc.x;
        P.lam_c[N + gb] = (float)lc.y;
        P.lam_c[2 * N + gb] = (float)lc.z;
        if (i % S == 0) {
            P.p[gm] = (float)p0;
            P.p[Mt + gm] = (float)p1;
            P.cmd[gm] = (float)cmdv;
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

}  // namespace

hipError_t launch_newton(const KParams& P, const NParams& Q, const int* list, const int* off, int n_steps,
                         hipStream_t stream)
{
    if (n_steps <= 0) return hipSuccess;
#define NEWTON_CLASS(C, SEGV)                                                                          \
    if (off[C + 1] > off[C]) {                                                                         \
        const int cnt = off[C + 1] - off[C];                                                           \
        constexpr int wg = SEGV > 64 ? SEGV : 256;                                                     \
        const int per = wg / SEGV;                                                                     \
        hipLaunchKernelGGL((k_newton<SEGV>), dim3((cnt + per - 1) / per), dim3(wg), 0, stream, P, Q,   \
                           list + off[C], cnt, n_steps);                                               \
        hipError_t e = hipGetLastError();                                                              \
        if (e != hipSuccess) return e;                                                                 \
    }
    NEWTON_CLASS(0, 8)
    NEWTON_CLASS(1, 16)
    NEWTON_CLASS(2, 32)
    NEWTON_CLASS(3, 64)
    NEWTON_CLASS(4, 128)
    NEWTON_CLASS(5, 256)
    NEWTON_CLASS(6, 512)
    NEWTON_CLASS(7, 1024)
#undef NEWTON_CLASS
    return hipSuccess;
}

}  // namespace snake
