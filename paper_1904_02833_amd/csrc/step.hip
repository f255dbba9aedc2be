// Solver kernels: one fused launch advances a tile of snakes by whole steps.
//
// Mapping (wave64, gfx950): a snake of B <= SEG bodies owns an aligned group
// of SEG lanes; lane i holds body i (its state stays in VGPRs for the whole
// launch), joint i (bodies i, i+1) and the ground contact of body i.  Each
// iteration a lane fetches the displacement and orientation of body i+1 from
// lane i+1, evaluates its three blocks, sends the increments of joint i that
// land on body i+1 to lane i+1, and gathers in a fixed order.  The snake's
// residual is an xor-butterfly max over its SEG lanes, so a snake stops at
// its own tolerance while its wave continues for the others.
//
// Every substep: chamber pressure -> rest rotation of intra-module joints ->
// predicted positions (first-order implicit step, section "Time-Stepping")
// -> multiplier initialisation -> block-Jacobi iterations on the compliant
// system (equations of motion with c + E lambda = 0, contact and Coulomb
// cone, section "Simulator"; linearisation eq. schur_system) -> velocities.
//
// Precision: positions are kept as start-of-substep position xp plus a small
// displacement d, so constraint values are formed from differences of
// nearby FP32 numbers and the multipliers do not inherit the ulp of the
// absolute coordinates.
#include "device_math.h"
#include "kernels.h"

namespace snake {

namespace {

// geometry of joint i needed again by the increment application
struct Geo {
    V3 rA, rB, aA, aB;
    Q4 e, qA;
    float ct, st;
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
__device__ __forceinline__ void joint_eval(V3 dxp, V3 dA, V3 dB, Q4 qA, Q4 qB, float c0h, float s0h,
                                           float ct, float st, float wA, float c1A, float c2A,
                                           float wB, float c1B, float c2B, float hl, float inv_L,
                                           float comp_s, float comp_b, float comp_t, V3 ls, V3 lb,
                                           Geo& g, V3& Dls, V3& Dlb, float& rs, float& rb)
{
    g.aA = qaxis(qA);
    g.aB = qaxis(qB);
    g.rA = hl * g.aA;
    g.rB = (-hl) * g.aB;
    g.qA = qA;
    g.ct = ct;
    g.st = st;

    // stretch: end point of A minus start point of B (eq. rigid_to_particle form)
    const V3 C = (dxp + (dA - dB)) + (g.rA - g.rB);
    const V3 rhs = C + comp_s * ls;
    // K = (wA + wB) I + c1A hl^2 (I - aA aA^T) + c1B hl^2 (I - aB aB^T)
    const float kA = c1A * (hl * hl), kB = c1B * (hl * hl);
    const float dg = wA + wB + kA + kB + comp_s;
    const V3 a = g.aA, b = g.aB;
    Dls = -sym3_solve(dg - kA * a.x * a.x - kB * b.x * b.x, -kA * a.x * a.y - kB * b.x * b.y,
                      -kA * a.x * a.z - kB * b.x * b.z, dg - kA * a.y * a.y - kB * b.y * b.y,
                      -kA * a.y * a.z - kB * b.y * b.z, dg - kA * a.z * a.z - kB * b.z * b.z, rhs);
    rs = amax3(rhs) * inv_L;

    // bend-twist: e = conj(q0) conj(qA) qB with q0 = (c0h, 0, 0, s0h)
    const Q4 t = qmul(qconj(qA), qB);
    Q4 e{c0h * t.w + s0h * t.z, c0h * t.x + s0h * t.y, c0h * t.y - s0h * t.x, c0h * t.z - s0h * t.w};
    if (e.w < 0.f) e = Q4{-e.w, -e.x, -e.y, -e.z};
    g.e = e;
    const V3 ev{e.x, e.y, e.z};
    const V3 rhsb = 2.f * ev + mk(comp_t * lb.x, comp_b * lb.y, comp_b * lb.z);
    // K = G F^T (IA^-1 + IB^-1) F G^T, G = e_w I - [e]x, F = R(qA q0):
    //   (c1A + c1B)(|e|^2 I - e e^T) + c2A gA gA^T + c2B gB gB^T
    // with gX = G uX and uA = R(q0)^T e_x, uB = R(e) e_x
    const V3 ua{ct, -st, 0.f};
    const V3 ub = qaxis(e);
    const V3 ga = e.w * ua - cross(ev, ua);
    const V3 gb = e.w * ub - cross(ev, ub);
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

// W J^T of joint increments (dls, dlb) on bodies A and B
__device__ __forceinline__ void joint_corr(const Geo& g, V3 dls, V3 dlb, float wA, float c1A,
                                           float c2A, float wB, float c1B, float c2B, V3& dxA,
                                           V3& dthA, V3& dxB, V3& dthB)
{
    dxA = wA * dls;
    dxB = (-wB) * dls;
    const V3 thsA = c1A * cross(g.rA, dls);
    const V3 thsB = (-c1B) * cross(g.rB, dls);
    const V3 ev{g.e.x, g.e.y, g.e.z};
    const V3 y = g.e.w * dlb + cross(ev, dlb);
    const V3 y0{g.ct * y.x - g.st * y.y, g.st * y.x + g.ct * y.y, y.z};
    const V3 z = qrot(g.qA, y0);
    const V3 thbA = -(c1A * z + (c2A * dot(g.aA, z)) * g.aA);
    const V3 thbB = c1B * z + (c2B * dot(g.aB, z)) * g.aB;
    dthA = thsA + thbA;
    dthB = thsB + thbB;
}

// increments of the contact block of a body (normal, tangent x, tangent y)
__device__ __forceinline__ V3 contact_incr(V3 lc, float cn, V3 d, float sc, float m, float mu)
{
    const float ln = fmaxf(0.f, lc.x - sc * m * cn);
    float t0 = lc.y - sc * m * d.x;
    float t1 = lc.z - sc * m * d.y;
    const float cap = mu * ln;
    const float nt = sqrtf(t0 * t0 + t1 * t1);
    if (ln <= 0.f) {
        t0 = 0.f;
        t1 = 0.f;
    } else if (nt > cap) {
        const float f = cap / nt;
        t0 *= f;
        t1 *= f;
    }
    return V3{ln - lc.x, t0 - lc.y, t1 - lc.z};
}

template <int SEG>
__global__ void __launch_bounds__(64) k_step(KParams P, const int* __restrict__ tiles, int n_steps)
{
    constexpr int PER = 64 / SEG;
    const int lane = threadIdx.x;
    const int i = lane & (SEG - 1);
    const int s = tiles[blockIdx.x * PER + lane / SEG];
    const bool live = s >= 0;
    int B = 0, S = 1, bo = 0, mo = 0;
    float comp_s = 0.f, comp_b = 0.f, comp_t = 0.f, mu = 0.f;
    double freq = 0.0, ph0 = 0.0;
    if (live) {
        B = P.Bn[s];
        S = P.Sn[s];
        bo = P.body_off[s];
        mo = P.module_off[s];
        comp_s = P.comp[s];
        comp_b = P.comp[P.n_snakes + s];
        comp_t = P.comp[2 * P.n_snakes + s];
        mu = P.mu[s];
        freq = P.freq[s];
        ph0 = P.phase0[s];
    }
    const bool hasb = i < B;
    const bool hasj = i + 1 < B;
    const int gnd = (P.flags & kNoGround) ? 0 : 1;
    const bool fixed = (P.flags & kFixedRoot) && i == 0;
    const int N = P.N, J = P.J, Mt = P.Mt;
    const int gb = bo + i;
    const int gj = bo - s + i;
    const int m = i / S;
    const int gm = mo + m;
    const bool intra = hasj && ((i + 1) % S != 0);
    // blocks on body i and body i+1; scale of a joint block uses the larger
    const int dA = gnd + (i > 0 ? 2 : 0) + (i + 1 < B ? 2 : 0);
    const int dB = gnd + 2 + (i + 2 < B ? 2 : 0);
    const float sj = P.relax / (float)max(dA, dB);
    const float sc = P.relax / (float)max(dA, 1);
    const float wA = fixed ? 0.f : P.inv_m, c1A = fixed ? 0.f : P.c1, c2A = fixed ? 0.f : P.c2;
    const float wB = P.inv_m, c1B = P.c1, c2B = P.c2;
    const float hl = P.half_L, h = P.h, mass = 1.f / P.inv_m;

    V3 x{0.f, 0.f, 0.f}, v{0.f, 0.f, 0.f}, w{0.f, 0.f, 0.f};
    Q4 q{1.f, 0.f, 0.f, 0.f};
    V3 ls{0.f, 0.f, 0.f}, lb{0.f, 0.f, 0.f}, lc{0.f, 0.f, 0.f};
    float p0 = 0.f, p1 = 0.f, cmdv = 0.f;
    if (hasb) {
        x = mk(P.x[gb], P.x[N + gb], P.x[2 * N + gb]);
        q = Q4{P.q[gb], P.q[N + gb], P.q[2 * N + gb], P.q[3 * N + gb]};
        v = mk(P.v[gb], P.v[N + gb], P.v[2 * N + gb]);
        w = mk(P.w[gb], P.w[N + gb], P.w[2 * N + gb]);
        lc = mk(P.lam_c[gb], P.lam_c[N + gb], P.lam_c[2 * N + gb]);
        p0 = P.p[gm];
        p1 = P.p[Mt + gm];
        cmdv = P.cmd[gm];
    }
    if (hasj) {
        ls = mk(P.lam_j[gj], P.lam_j[J + gj], P.lam_j[2 * J + gj]);
        lb = mk(P.lam_j[3 * J + gj], P.lam_j[4 * J + gj], P.lam_j[5 * J + gj]);
    }
    long long stepc = live ? P.step[s] : 0;
    long long itot = live ? P.iters_total[s] : 0;
    float rstep = 0.f;
    int itstep = 0, status = 0;

    for (int st = 0; st < n_steps; ++st) {
        // command for the end of this step (eq. snake_control or a schedule)
        if (hasb && P.controller == kCtrlSerpenoid) {
            const double t = (double)(stepc + 1) * P.dt;
            double a = sin(6.283185307179586476925286766559 * freq * t + P.ctrl_alpha * m + ph0) +
                       P.ctrl_offset;
            a = fmin(1.0, fmax(-1.0, a));
            cmdv = (float)a;
        } else if (hasb && P.controller == kCtrlSchedule) {
            int lo = P.sched_off[gm], hi = P.sched_off[gm + 1] - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if ((long long)P.sched_start[mid] <= stepc)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            cmdv = P.sched_val[lo];
        }
        const float u0 = fmaxf(cmdv, 0.f), u1 = fmaxf(-cmdv, 0.f);
        if (P.law == kLawPaper) {
            p0 = paper_update(P, p0, u0);
            p1 = paper_update(P, p1, u1);
        }
        rstep = 0.f;
        itstep = 0;
        status = 0;
        for (int sub = 0; sub < P.substeps; ++sub) {
            if (P.law == kLawLag) {
                p0 = u0 + (p0 - u0) * (u0 > p0 ? P.lag_in : P.lag_de);
                p1 = u1 + (p1 - u1) * (u1 > p1 ? P.lag_in : P.lag_de);
            }
            // rest rotation of joint i about body z, angle kappa_max (p0 - p1) L
            const float th0 = intra ? P.kappa_max * (p0 - p1) * P.L : 0.f;
            float s0h, c0h;
            sincosf(0.5f * th0, &s0h, &c0h);
            const float ct = c0h * c0h - s0h * s0h, stt = 2.f * s0h * c0h;

            // predicted positions
            const V3 xp = x;
            const Q4 qp = q;
            V3 d{0.f, 0.f, 0.f};
            if (hasb && !fixed) {
                v.z -= h * P.g;
                d = h * v;
                const V3 ax = qaxis(q);
                const V3 Iw = P.I_pe * w + ((P.I_ax - P.I_pe) * dot(ax, w)) * ax;
                const V3 tq = -cross(w, Iw);
                const V3 dw = P.c1 * tq + (P.c2 * dot(ax, tq)) * ax;
                w = w + h * dw;
                q = qturn(q, h * w);
            } else if (fixed) {
                v = V3{0.f, 0.f, 0.f};
                w = V3{0.f, 0.f, 0.f};
            }
            const float zp = xp.z - P.R;
            const V3 dxp = xp - lane_next(xp);

            // multiplier initialisation
            if (P.warm == kWarmPrev) {
                // x <- x~ + W J(x~)^T lambda0 with lambda0 = previous multipliers
                const V3 dn = lane_next(d);
                const Q4 qn = lane_next(q);
                Geo g;
                V3 Dls, Dlb;
                float rs, rb;
                joint_eval(dxp, d, dn, q, qn, c0h, s0h, ct, stt, wA, c1A, c2A, wB, c1B, c2B, hl,
                           P.inv_L, comp_s, comp_b, comp_t, ls, lb, g, Dls, Dlb, rs, rb);
                V3 dxA, dthA, dxB, dthB;
                joint_corr(g, ls, lb, wA, c1A, c2A, wB, c1B, c2B, dxA, dthA, dxB, dthB);
                V3 inx = lane_prev(dxB), inth = lane_prev(dthB);
                const bool recv = hasb && i > 0;
                inx = sel(recv, inx, V3{0.f, 0.f, 0.f});
                inth = sel(recv, inth, V3{0.f, 0.f, 0.f});
                const V3 ownx = sel(hasj, dxA, V3{0.f, 0.f, 0.f});
                const V3 ownth = sel(hasj, dthA, V3{0.f, 0.f, 0.f});
                const V3 dxc = (gnd && !fixed) ? P.inv_m * mk(lc.y, lc.z, lc.x) : V3{0.f, 0.f, 0.f};
                if (hasb && !fixed) {
                    d = d + ((inx + ownx) + dxc);
                    q = qturn(q, inth + ownth);
                }
            } else {
                ls = V3{0.f, 0.f, 0.f};
                lb = V3{0.f, 0.f, 0.f};
                lc = V3{0.f, 0.f, 0.f};
            }

            bool done = !live;
            int kdone = 0;
            float rdone = 0.f;
            for (int k = 0;; ++k) {
                const V3 dn = lane_next(d);
                const Q4 qn = lane_next(q);
                Geo g;
                V3 Dls, Dlb;
                float rs, rb;
                joint_eval(dxp, d, dn, q, qn, c0h, s0h, ct, stt, wA, c1A, c2A, wB, c1B, c2B, hl,
                           P.inv_L, comp_s, comp_b, comp_t, ls, lb, g, Dls, Dlb, rs, rb);
                const float cn = zp + d.z;
                const float rc = (lc.x > 0.f ? fabsf(cn) : fmaxf(-cn, 0.f)) * P.inv_L;
                float rl = fmaxf(hasj ? fmaxf(rs, rb) : 0.f, (hasb && gnd) ? rc : 0.f);
                rl = (rl == rl) ? rl : INFINITY;
                const float r = seg_max<SEG>(rl);
                if (!done) {
                    const bool bad = !(r < INFINITY);
                    const bool stop = bad || (P.tol > 0.f ? (r <= P.tol || k >= P.iters) : (k >= P.iters));
                    if (stop) {
                        done = true;
                        kdone = k;
                        rdone = r;
                        if (bad)
                            status |= kStatusNonfinite;
                        else if (P.tol > 0.f && r > P.tol)
                            status |= kStatusNotConverged;
                    }
                }
                if (__all(done)) break;

                const V3 dls = sj * Dls, dlb = sj * Dlb;
                V3 dxA, dthA, dxB, dthB;
                joint_corr(g, dls, dlb, wA, c1A, c2A, wB, c1B, c2B, dxA, dthA, dxB, dthB);
                V3 dlc{0.f, 0.f, 0.f};
                if (gnd && !fixed) dlc = contact_incr(lc, cn, d, sc, mass, mu);
                const V3 dxc = P.inv_m * mk(dlc.y, dlc.z, dlc.x);
                // gather in the fixed order: joint i-1 (from lane i-1), joint i, contact
                V3 inx = lane_prev(dxB), inth = lane_prev(dthB);
                const bool recv = hasb && i > 0;
                inx = sel(recv, inx, V3{0.f, 0.f, 0.f});
                inth = sel(recv, inth, V3{0.f, 0.f, 0.f});
                const V3 ownx = sel(hasj, dxA, V3{0.f, 0.f, 0.f});
                const V3 ownth = sel(hasj, dthA, V3{0.f, 0.f, 0.f});
                if (!done) {
                    if (hasj) {
                        ls = ls + dls;
                        lb = lb + dlb;
                    }
                    if (hasb && gnd) lc = lc + dlc;
                    if (hasb && !fixed) {
                        d = d + ((inx + ownx) + dxc);
                        q = qturn(q, inth + ownth);
                    }
                }
            }
            itstep += kdone;
            rstep = fmaxf(rstep, rdone);

            // velocities of the implicit step
            if (hasb && !fixed) {
                x = xp + d;
                v = P.inv_h * d;
                const Q4 dq = qmul(q, qconj(qp));
                const float sg = dq.w >= 0.f ? 2.f * P.inv_h : -2.f * P.inv_h;
                w = mk(sg * dq.x, sg * dq.y, sg * dq.z);
            }
        }
        stepc += 1;
        itot += itstep;
    }

    if (hasb) {
        P.x[gb] = x.x;
        P.x[N + gb] = x.y;
        P.x[2 * N + gb] = x.z;
        P.q[gb] = q.w;
        P.q[N + gb] = q.x;
        P.q[2 * N + gb] = q.y;
        P.q[3 * N + gb] = q.z;
        P.v[gb] = v.x;
        P.v[N + gb] = v.y;
        P.v[2 * N + gb] = v.z;
        P.w[gb] = w.x;
        P.w[N + gb] = w.y;
        P.w[2 * N + gb] = w.z;
        P.lam_c[gb] = lc.x;
        P.lam_c[N + gb] = lc.y;
        P.lam_c[2 * N + gb] = lc.z;
        if (i % S == 0) {
            P.p[gm] = p0;
            P.p[Mt + gm] = p1;
            P.cmd[gm] = cmdv;
        }
    }
    if (hasj) {
        P.lam_j[gj] = ls.x;
        P.lam_j[J + gj] = ls.y;
        P.lam_j[2 * J + gj] = ls.z;
        P.lam_j[3 * J + gj] = lb.x;
        P.lam_j[4 * J + gj] = lb.y;
        P.lam_j[5 * J + gj] = lb.z;
    }
    if (live && i == 0) {
        P.residual[s] = rstep;
        P.iters_out[s] = itstep;
        P.status[s] = status;
        P.step[s] = stepc;
        P.iters_total[s] = itot;
    }
}

// straight chains at rest on the ground along +x, zero pressure
__global__ void k_init_state(KParams P)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int stride = gridDim.x * blockDim.x;
    const int N = P.N, J = P.J, Mt = P.Mt;
    for (int gb = tid; gb < N; gb += stride) {
        // snake of body gb: last s with body_off[s] <= gb
        int lo = 0, hi = P.n_snakes - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (P.body_off[mid] <= gb)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int i = gb - P.body_off[lo];
        P.x[gb] = ((float)i + 0.5f) * P.L;
        P.x[N + gb] = 0.f;
        P.x[2 * N + gb] = P.R;
        P.q[gb] = 1.f;
        P.q[N + gb] = 0.f;
        P.q[2 * N + gb] = 0.f;
        P.q[3 * N + gb] = 0.f;
        for (int k = 0; k < 3; ++k) {
            P.v[k * N + gb] = 0.f;
            P.w[k * N + gb] = 0.f;
            P.lam_c[k * N + gb] = 0.f;
        }
    }
    for (int j = tid; j < 6 * J; j += stride) P.lam_j[j] = 0.f;
    for (int j = tid; j < Mt; j += stride) {
        P.p[j] = 0.f;
        P.p[Mt + j] = 0.f;
        P.cmd[j] = 0.f;
    }
    for (int s = tid; s < P.n_snakes; s += stride) {
        P.residual[s] = 0.f;
        P.iters_out[s] = 0;
        P.status[s] = 0;
        P.step[s] = 0;
        P.iters_total[s] = 0;
    }
}

__global__ void k_set_cmd(float* dst, const float* src, int n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) {
        const float a = src[t];
        dst[t] = (a == a) ? fminf(1.f, fmaxf(-1.f, a)) : 0.f;
    }
}

}  // namespace

hipError_t launch_step(int seg, const KParams& P, const int* tiles, int n_tiles, int n_steps,
                       hipStream_t stream)
{
    if (n_tiles <= 0) return hipSuccess;
    const dim3 grid(n_tiles), block(64);
    switch (seg) {
        case 16: hipLaunchKernelGGL(k_step<16>, grid, block, 0, stream, P, tiles, n_steps); break;
        case 32: hipLaunchKernelGGL(k_step<32>, grid, block, 0, stream, P, tiles, n_steps); break;
        case 64: hipLaunchKernelGGL(k_step<64>, grid, block, 0, stream, P, tiles, n_steps); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_init_state(const KParams& P, hipStream_t stream)
{
    const int work = P.N > 6 * P.J ? P.N : 6 * P.J;
    int blocks = (work + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_init_state, dim3(blocks), dim3(256), 0, stream, P);
    return hipGetLastError();
}

hipError_t launch_set_cmd(float* dst, const float* src, int n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_set_cmd, dim3((n + 255) / 256), dim3(256), 0, stream, dst, src, n);
    return hipGetLastError();
}

}  // namespace snake
