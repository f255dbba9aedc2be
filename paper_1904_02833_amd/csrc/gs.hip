// Block Gauss-Seidel on the compliant system: the blocks of a snake are
// visited colour by colour over the greedy block colouring of the index
// work (blocks of one colour share no body), each colour's blocks taking
// their local solutions (scaled by relax, no averaging) at the current state
// and applying them at once.  FP32, the block evaluations of the Jacobi
// kernel, the same residual and stopping rule; zero multipliers at each
// substep.
//
// Layout: one body per lane as in the Newton kernel (a snake takes SEG
// lanes, a power of two >= B, at least 8; up to 64 lanes per snake several
// snakes share a wave and exchange by lane shuffles; longer snakes take a
// workgroup of SEG / 64 waves joined through LDS).  A sweep is the residual
// pass of the iterate followed by five colour passes; each pass fetches the
// next body's state and sends the increments of joint i to body i+1.
#include <hip/hip_runtime.h>

#include "blocks.h"
#include "device_math.h"
#include "kernels.h"

namespace snake {

namespace {

constexpr int kColours = 5;   // greedy colouring of a chain: at most 5

template <int SEG, int K>
__device__ __forceinline__ void gs_from_next(float (&v)[K], int lane, int wv, float* buf, int& ph)
{
    float r[K];
#pragma unroll
    for (int k = 0; k < K; ++k) r[k] = __shfl_down(v[k], 1, 64);
    if constexpr (SEG > 64) {
        // two buffers used in turn: the one written here was last read
        // before the previous exchange's barrier
        float* b = buf + (ph & 1) * (SEG / 64) * 12;
        ++ph;
        if (lane == 0)
#pragma unroll
            for (int k = 0; k < K; ++k) b[wv * 12 + k] = v[k];
        __syncthreads();
        if (lane == 63 && wv + 1 < SEG / 64)
#pragma unroll
            for (int k = 0; k < K; ++k) r[k] = b[(wv + 1) * 12 + k];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = r[k];
}

template <int SEG, int K>
__device__ __forceinline__ void gs_from_prev(float (&v)[K], int lane, int wv, float* buf, int& ph)
{
    float r[K];
#pragma unroll
    for (int k = 0; k < K; ++k) r[k] = __shfl_up(v[k], 1, 64);
    if constexpr (SEG > 64) {
        float* b = buf + (ph & 1) * (SEG / 64) * 12;
        ++ph;
        if (lane == 63)
#pragma unroll
            for (int k = 0; k < K; ++k) b[wv * 12 + k] = v[k];
        __syncthreads();
        if (lane == 0 && wv > 0)
#pragma unroll
            for (int k = 0; k < K; ++k) r[k] = b[(wv - 1) * 12 + k];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = r[k];
}

// maximum over the snake's lanes of non-negative values (NaN mapped to +inf
// before), the same in every lane
template <int SEG>
__device__ __forceinline__ float gs_seg_max(float v, int lane, int wv, float* red, int& ph)
{
    constexpr int W = SEG < 64 ? SEG : 64;
#pragma unroll
    for (int o = 1; o < W; o <<= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    if constexpr (SEG > 64) {
        // two partial arrays used in turn, as the exchange buffers
        float* r = red + (ph & 1) * (SEG / 64);
        ++ph;
        if (lane == 0) r[wv] = v;
        __syncthreads();
        float a = r[0];
#pragma unroll
        for (int w = 1; w < SEG / 64; ++w) a = fmaxf(a, r[w]);
        v = a;
    }
    return v;
}

template <int SEG>
__global__ void __launch_bounds__(SEG > 64 ? SEG : 256) __attribute__((amdgpu_waves_per_eu(3)))
k_gs(KParams P, const int* __restrict__ block_off, const int* __restrict__ blk_color,
     const int* __restrict__ list, int count, int n_steps)
{
    constexpr int WG = SEG > 64 ? SEG : 256;
    constexpr int NWV = SEG > 64 ? SEG / 64 : 1;
    __shared__ float xbuf[2 * NWV * 12];   // two buffers used in turn
    __shared__ float red[2 * NWV];
    int xph = 0, rph = 0;   // which buffer the next exchange / reduction takes
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int idx = blockIdx.x * (WG / SEG) + t / SEG;
    const int i = t % SEG;
    const int s = idx < count ? list[idx] : -1;
    const bool live = s >= 0;

    int B = 0, S = 1, bo = 0, mo = 0;
    float comp_s = 0.f, comp_b = 0.f, comp_t = 0.f, mu = 0.f;
    if (live) {
        B = P.Bn[s];
        S = P.Sn[s];
        bo = P.body_off[s];
        mo = P.module_off[s];
        comp_s = P.comp[s];
        comp_b = P.comp[P.n_snakes + s];
        comp_t = P.comp[2 * P.n_snakes + s];
        mu = P.mu[s];
    }
    const bool hasb = i < B;
    const bool hasj = i + 1 < B;
    const bool gnd = !(P.flags & kNoGround);
    const bool fixed = (P.flags & kFixedRoot) && i == 0;
    const int N = P.N, J = P.J, Mt = P.Mt;
    const int gb = bo + i, gj = bo - s + i;
    const int m = i / S, gm = mo + m;
    const bool intra = hasj && ((i + 1) % S != 0);
    // colours of this lane's blocks (-1: no such block)
    int cs = -1, cb = -1, cc = -1;
    if (live) {
        const int b0 = block_off[s];
        if (hasj) {
            cs = blk_color[b0 + 2 * i];
            cb = blk_color[b0 + 2 * i + 1];
        }
        if (hasb && gnd) cc = blk_color[b0 + 2 * (B - 1) + i];
    }
    const float wA = fixed ? 0.f : P.inv_m, c1A = fixed ? 0.f : P.c1, c2A = fixed ? 0.f : P.c2;
    const float wB = P.inv_m, c1B = P.c1, c2B = P.c2;
    const float hl = P.half_L, h = P.h, mass = 1.f / P.inv_m, sc = P.relax;
    const V3 zero{0.f, 0.f, 0.f};

    V3 x = zero, v = zero, w = zero;
    Q4 q{1.f, 0.f, 0.f, 0.f};
    V3 ls = zero, lb = zero, lc = zero;
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

    float rstep = 0.f;
    int itstep = 0, status = 0, itsum = 0;
    for (int st = 0; st < n_steps; ++st) {
        const long long stepc = (live ? P.step[s] : 0) + st;
        // command for the end of this step (eq. snake_control or a schedule)
        if (hasb && P.controller == kCtrlSerpenoid)
            cmdv = (float)serpenoid_command(P, s, m, stepc);
        else if (hasb && P.controller == kCtrlSchedule)
            cmdv = schedule_command(P, gm, stepc);
        if (P.law == kLawPaper) {
            p0 = paper_update(P, p0, fmaxf(cmdv, 0.f));
            p1 = paper_update(P, p1, fmaxf(-cmdv, 0.f));
        }
        const float u0 = fmaxf(cmdv, 0.f), u1 = fmaxf(-cmdv, 0.f);
        rstep = 0.f;
        itstep = 0;
        status = 0;
        for (int sub = 0; sub < P.substeps; ++sub) {
            if (P.law == kLawLag) {
                p0 = u0 + (p0 - u0) * (u0 > p0 ? P.lag_in : P.lag_de);
                p1 = u1 + (p1 - u1) * (u1 > p1 ? P.lag_in : P.lag_de);
            }
            const float th0 = intra ? P.kappa_max * (p0 - p1) * P.L : 0.f;
            float s0h, c0h;
            sincosf(0.5f * th0, &s0h, &c0h);
            const float ct = c0h * c0h - s0h * s0h, stt = 2.f * s0h * c0h;

            // predicted positions (displacement d from the start xp)
            const V3 xp = x;
            const Q4 qp = q;
            V3 d = zero;
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
                v = zero;
                w = zero;
            }
            ls = zero;
            lb = zero;
            lc = zero;
            const float zp = xp.z - P.R;
            V3 dxp;
            {
                float e[3] = {xp.x, xp.y, xp.z};
                gs_from_next<SEG, 3>(e, lane, wv, xbuf, xph);
                dxp = xp - mk(e[0], e[1], e[2]);
            }
            // state of body i+1 at the current iterate
            auto next_body = [&](V3& dn, Q4& qn, V3& an, V3 aA) {
                float e[10] = {d.x, d.y, d.z, q.w, q.x, q.y, q.z, aA.x, aA.y, aA.z};
                gs_from_next<SEG, 10>(e, lane, wv, xbuf, xph);
                dn = mk(e[0], e[1], e[2]);
                qn = Q4{e[3], e[4], e[5], e[6]};
                an = mk(e[7], e[8], e[9]);
            };

            float r = 0.f;
            int k = 0;
            for (;; ++k) {
                // residual of iterate k
                {
                    const V3 aA = qaxis(q);
                    V3 dn, an;
                    Q4 qn;
                    next_body(dn, qn, an, aA);
                    Geo g;
                    V3 Dls, Dlb;
                    float rs, rb;
                    joint_eval(dxp, d, dn, q, qn, aA, an, c0h, s0h, ct, stt, wA, c1A, c2A, wB, c1B, c2B, hl,
                               P.inv_L, comp_s, comp_b, comp_t, ls, lb, g, Dls, Dlb, rs, rb);
                    const float cn = zp + d.z;
                    const float rc = (lc.x > 0.f ? fabsf(cn) : fmaxf(-cn, 0.f)) * P.inv_L;
                    float rl = fmaxf(hasj ? fmaxf(rs, rb) : 0.f, (hasb && gnd) ? rc : 0.f);
                    rl = (rl == rl) ? rl : INFINITY;
                    r = gs_seg_max<SEG>(rl, lane, wv, red, rph);
                }
                if (!(r < INFINITY)) {
                    status |= kStatusNonfinite;
                    break;
                }
                const bool stop = P.tol > 0.f ? (r <= P.tol || k >= P.iters) : (k >= P.iters);
                if (stop) {
                    if (P.tol > 0.f && r > P.tol) status |= kStatusNotConverged;
                    break;
                }
                // one sweep: the colour passes in order
                for (int col = 0; col < kColours; ++col) {
                    const V3 aA = qaxis(q);
                    V3 dn, an;
                    Q4 qn;
                    next_body(dn, qn, an, aA);
                    V3 fA = zero, tA = zero;
                    float out[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                    if (cs == col || cb == col) {
                        Geo g;
                        V3 Dls, Dlb;
                        float rs, rb;
                        joint_eval(dxp, d, dn, q, qn, aA, an, c0h, s0h, ct, stt, wA, c1A, c2A, wB, c1B, c2B, hl,
                                   P.inv_L, comp_s, comp_b, comp_t, ls, lb, g, Dls, Dlb, rs, rb);
                        const V3 dls = cs == col ? sc * Dls : zero;
                        const V3 dlb = cb == col ? sc * Dlb : zero;
                        V3 tB;
                        joint_torques(g, dls, dlb, hl, tA, tB);
                        fA = dls;
                        ls = ls + dls;
                        lb = lb + dlb;
                        out[0] = -dls.x;
                        out[1] = -dls.y;
                        out[2] = -dls.z;
                        out[3] = tB.x;
                        out[4] = tB.y;
                        out[5] = tB.z;
                    }
                    V3 dlc = zero;
                    if (cc == col && !fixed) dlc = contact_incr(lc, zp + d.z, d, sc, mass, mu);
                    gs_from_prev<SEG, 6>(out, lane, wv, xbuf, xph);
                    if (hasb && i > 0) {
                        fA = fA + mk(out[0], out[1], out[2]);
                        tA = tA + mk(out[3], out[4], out[5]);
                    }
                    if (cc == col) lc = lc + dlc;
                    if (hasb && !fixed) {
                        d = d + wA * (fA + mk(dlc.y, dlc.z, dlc.x));
                        q = qturn(q, inv_inertia(tA, aA, c1A, c2A));
                    }
                }
            }
            itstep += k;
            rstep = fmaxf(rstep, r);

            // velocities of the implicit step
            if (hasb && !fixed) {
                x = xp + d;
                v = P.inv_h * d;
                const Q4 dq = qmul(q, qconj(qp));
                const float sg = dq.w >= 0.f ? 2.f * P.inv_h : -2.f * P.inv_h;
                w = mk(sg * dq.x, sg * dq.y, sg * dq.z);
            }
        }
        itsum += itstep;
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

hipError_t launch_gs(const KParams& P, const int* block_off, const int* blk_color, const int* list, const int* off,
                     int n_steps, hipStream_t stream)
{
    if (n_steps <= 0) return hipSuccess;
#define GS_CLASS(C, SEGV)                                                                               \
    if (off[C + 1] > off[C]) {                                                                          \
        const int cnt = off[C + 1] - off[C];                                                            \
        constexpr int wg = SEGV > 64 ? SEGV : 256;                                                      \
        const int per = wg / SEGV;                                                                      \
        hipLaunchKernelGGL((k_gs<SEGV>), dim3((cnt + per - 1) / per), dim3(wg), 0, stream, P, block_off, \
                           blk_color, list + off[C], cnt, n_steps);                                     \
        hipError_t e = hipGetLastError();                                                               \
        if (e != hipSuccess) return e;                                                                  \
    }
    GS_CLASS(0, 8)
    GS_CLASS(1, 16)
    GS_CLASS(2, 32)
    GS_CLASS(3, 64)
    GS_CLASS(4, 128)
    GS_CLASS(5, 256)
    GS_CLASS(6, 512)
    GS_CLASS(7, 1024)
#undef GS_CLASS
    return hipSuccess;
}

}  // namespace snake
