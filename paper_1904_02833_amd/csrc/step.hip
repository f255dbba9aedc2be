// Solver kernel: one launch advances every snake by whole steps.
//
// Mapping (wave64, gfx950): a snake of B bodies owns an aligned segment of
// 2^k >= B lanes; lane i holds body i (its state stays in VGPRs for the whole
// launch), joint i (bodies i, i+1) and the ground contact of body i.  Each
// iteration a lane fetches the displacement, orientation and axis of body
// i+1 from lane i+1, evaluates its three blocks, sends the increments of
// joint i that land on body i+1 to lane i+1, and gathers in a fixed order.
// Lane shifts use ds_bpermute (the LDS pipe), leaving the VALU, which bounds
// the kernel, to the arithmetic.  The snake's residual is an xor-butterfly
// max over its segment, so a snake stops at its own tolerance while its wave
// continues for the others.
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
#include "blocks.h"
#include "device_math.h"
#include "net_inputs.h"
#include "kernels.h"

namespace snake {

namespace {

// Copy NW floats from 16-byte aligned LDS into registers with vector reads.
template <int NW>
__device__ __forceinline__ void lds_row(const float* src, float* dst)
{
    if constexpr (NW % 4 == 0) {
#pragma unroll
        for (int k = 0; k < NW / 4; ++k) {
            const float4 t = reinterpret_cast<const float4*>(src)[k];
            dst[4 * k] = t.x;
            dst[4 * k + 1] = t.y;
            dst[4 * k + 2] = t.z;
            dst[4 * k + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < NW; ++k) dst[k] = src[k];
    }
}

// Tile kernel.  A workgroup of NW waves takes tiles from the cost-ordered
// tile list (grid-stride, so a grid smaller than the list is persistent).
// A tile holds snakes in lane segments made of whole 16-lane rows, in one of
// two layouts: power-of-two segments placed largest first, so each is
// aligned to its size (segments of <= 64 lanes stay inside a wave), or
// segments of the snake's length rounded up to 16 lanes, placed one after
// another (fewer idle lanes, and a segment may cross a wave boundary);
// ROWS = 2 is the latter with 8-lane half rows for snakes of up to 8 bodies.  A
// segment that crosses a wave boundary exchanges the boundary body and the
// residual through LDS (two workgroup barriers per iteration, only in tiles
// that have such a snake).
template <int NW, int PHASE, int ROWS>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(4)))
k_tile(KParams P, const int4* __restrict__ hdr, const int2* __restrict__ slots, int n_tiles,
       int n_steps, int sub_only)
{
    constexpr int phase = PHASE;
    // lane 0 of each wave: u(3), q(4), axis(3), wave done.  Buffer 2 is used
    // at the start of a substep, buffers 0/1 alternate between iterations (and
    // buffer 1 serves the warm start): a buffer is written again only after a
    // barrier that every reader of its previous contents has passed.
    __shared__ float xnext[3][NW][12];
    __shared__ __align__(16) float xdone[3][NW];   // wave done flags, buffered as xnext
    __shared__ float xprev[NW][6];   // lane 63 of each wave: increments on the next body
    __shared__ __align__(16) float xfirst[NW];     // residual maximum of the segment piece holding lane 0
    __shared__ float xlast[NW];      // ... and of the piece holding lane 63
    const int L = threadIdx.x;
    const int lane = L & 63;
    const int wv = L >> 6;

    for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int4 H = hdr[tile];
        const bool xw = (NW > 1) && H.z != 0;
        if (NW > 1) __syncthreads();

        // slot: snake, lane offset << 16 | segment lanes; lanes outside every
        // segment form whole rows of their own
        int s = -1, i = 0, seg = 16, off = L & ~15;
        for (int k = 0; k < H.y; ++k) {
            const int2 sl = slots[H.x + k];
            const int o = sl.y >> 16, n = sl.y & 0xffff;
            if (L >= o && L < o + n) {
                s = sl.x;
                i = L - o;
                seg = n;
                off = o;
            }
        }
        const bool live = s >= 0;
        constexpr bool packed = ROWS != 0;  // rows layout (segments not aligned)
        // waves wa..wb hold the segment; in this wave it covers rows ra..rb
        const int wa = off >> 6, wb = (off + seg - 1) >> 6;
        const int wbase = wv << 6, row = lane >> 4;
        const int ra = (max(off, wbase) - wbase) >> 4;
        const int rb = (min(off + seg, wbase + 64) - 1 - wbase) >> 4;

        // neighbour exchange: body i+1 of the same snake lives in lane+1, or
        // for lane 63 of a spanning segment in lane 0 of the next wave
        auto fetch_next = [&](int buf, V3 u, Q4 qq, V3 a, bool wave_done, V3& un, Q4& qn,
                              V3& an) -> bool {
            un = lane_next(u);
            qn = lane_next(qq);
            an = lane_next(a);
            if (!xw) return false;
            if (lane == 0) {
                float* e = xnext[buf][wv];
                e[0] = u.x; e[1] = u.y; e[2] = u.z;
                e[3] = qq.w; e[4] = qq.x; e[5] = qq.y; e[6] = qq.z;
                e[7] = a.x; e[8] = a.y; e[9] = a.z;
                xdone[buf][wv] = wave_done ? 1.f : 0.f;
            }
            __syncthreads();
            // all flags in vector reads, so the latencies overlap
            // (each flag is 1.0f or +0.0f, so the and of the bit patterns is
            // nonzero exactly when every flag is set)
            float fl[NW];
            lds_row<NW>(xdone[buf], fl);
            int fa = -1;
#pragma unroll
            for (int w = 0; w < NW; ++w) fa &= __float_as_int(fl[w]);
            const bool all = fa != 0;
            if (lane == 63 && wv + 1 < NW) {
                const float* e = xnext[buf][wv + 1];
                un = mk(e[0], e[1], e[2]);
                qn = Q4{e[3], e[4], e[5], e[6]};
                an = mk(e[7], e[8], e[9]);
            }
            return all;
        };
        // increments of joint i-1 arriving at body i, and the segment maximum
        auto fetch_prev = [&](V3 dxB, V3 dthB, float rw, V3& inx, V3& inth) -> float {
            inx = lane_prev(dxB);
            inth = lane_prev(dthB);
            if (!xw) return rw;
            if (lane == 63) {
                float* e = xprev[wv];
                e[0] = dxB.x; e[1] = dxB.y; e[2] = dxB.z;
                e[3] = dthB.x; e[4] = dthB.y; e[5] = dthB.z;
            }
            if (lane == 0) xfirst[wv] = rw;
            if (lane == 63) xlast[wv] = rw;
            __syncthreads();
            if (lane == 0 && wv > 0) {
                const float* e = xprev[wv - 1];
                inx = mk(e[0], e[1], e[2]);
                inth = mk(e[3], e[4], e[5]);
            }
            float r = rw;
            if (wa != wb) {
                // the segment's piece in wave wa holds that wave's lane 63, the
                // pieces in the following waves hold their lane 0 (all NW
                // entries are read at once, so the reads overlap)
                // (non-negative values and +inf: the integer order of the bit
                // patterns is the float order, with no NaN canonicalisation)
                float fv[NW];
                lds_row<NW>(xfirst, fv);
                int ri = __float_as_int(xlast[wa]);
#pragma unroll
                for (int w = 1; w < NW; ++w)
                    if (w > wa && w <= wb) ri = max(ri, __float_as_int(fv[w]));
                r = __int_as_float(ri);
            }
            return r;
        };
        // Max over the segment's piece in this wave of non-negative values
        // (NaN already mapped to +inf): on their bit patterns the integer
        // order is the float order.  Rows of 16 lanes reduce by xor swaps
        // (aligned layout: lane shuffles; rows layout: DPP quad swaps and
        // half-row / row mirrors, which reach the same lanes within a row);
        // aligned power-of-two segments join rows by xor swaps too, packed
        // segments by a prefix and a suffix maximum over their rows.
        auto seg_reduce = [&](float v) -> float {
            int b = __float_as_int(v);
            if (packed) {
                b = max(b, __builtin_amdgcn_update_dpp(0, b, 0xB1, 0xf, 0xf, false));   // quad [1,0,3,2]
                b = max(b, __builtin_amdgcn_update_dpp(0, b, 0x4E, 0xf, 0xf, false));   // quad [2,3,0,1]
                b = max(b, __builtin_amdgcn_update_dpp(0, b, 0x141, 0xf, 0xf, false));  // half-row mirror
                if constexpr (ROWS == 2) {
                    // an 8-lane segment shares its row with another snake
                    const int t = __builtin_amdgcn_update_dpp(0, b, 0x140, 0xf, 0xf, false);
                    if (seg > 8) b = max(b, t);
                } else {
                    b = max(b, __builtin_amdgcn_update_dpp(0, b, 0x140, 0xf, 0xf, false));  // row mirror
                }
            } else {
#pragma unroll
                for (int o = 8; o >= 1; o >>= 1) b = max(b, __shfl_xor(b, o, 64));
            }
            if (!packed) {
#pragma unroll
                for (int o = 16; o <= 32; o <<= 1) {
                    const int t = __shfl_xor(b, o, 64);
                    if (o < seg) b = max(b, t);
                }
            } else {
                int p = b, q = b, t;
                t = __shfl_up(p, 16, 64);
                if (row > ra) p = max(p, t);
                t = __shfl_up(p, 32, 64);
                if (row > ra + 1) p = max(p, t);
                t = __shfl_down(q, 16, 64);
                if (row < rb) q = max(q, t);
                t = __shfl_down(q, 32, 64);
                if (row < rb - 1) q = max(q, t);
                b = max(p, q);
            }
            return __int_as_float(b);
        };

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
        const int gnd = (P.flags & kNoGround) ? 0 : 1;
        const bool fixed = (P.flags & kFixedRoot) && i == 0;
        const int N = P.N, J = P.J, Mt = P.Mt;
        const int gb = bo + i;
        const int gj = bo - s + i;
        const int m = i / S;
        const int gm = mo + m;
        const bool intra = hasj && ((i + 1) % S != 0);
        // blocks on body i and body i+1; a joint block is scaled by the larger
        const int dA = gnd + (i > 0 ? 2 : 0) + (i + 1 < B ? 2 : 0);
        const int dB = gnd + 2 + (i + 2 < B ? 2 : 0);
        // zero on a lane without a joint, whose increments are then zero and
        // its multiplier updates need no mask (its joint with whatever lies
        // in the next lane is evaluated and discarded)
        const float sj = hasj ? P.relax / (float)max(dA, dB) : 0.f;
        // lane masks (all ones / zero) for the joint's and the received
        // increments: a bitwise and (a full-rate VALU operation) zeroes what a
        // lane does not own, NaN included; the empty asm keeps the compiler
        // from turning the and back into a select
        int mj = hasj ? -1 : 0, mr = (hasb && i > 0) ? -1 : 0;
        asm volatile("" : "+v"(mj), "+v"(mr));
        auto andz = [](int m, V3 a) {
            return mk(__int_as_float(__float_as_int(a.x) & m), __int_as_float(__float_as_int(a.y) & m),
                      __int_as_float(__float_as_int(a.z) & m));
        };
        const float sc = P.relax / (float)max(dA, 1);
        const float wA = fixed ? 0.f : P.inv_m, c1A = fixed ? 0.f : P.c1, c2A = fixed ? 0.f : P.c2;
        const float wB = P.inv_m, c1B = P.c1, c2B = P.c2;
        const float hl = P.half_L, h = P.h, mass = 1.f / P.inv_m;
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
        // a split substep continues the counters of its step
        if (phase == kPhaseSolve && sub_only > 0 && live) {
            rstep = P.residual[s];
            itstep = P.iters_out[s];
            status = P.status[s];
        }
        const int it_before = itstep;

        // residual of the current iterate (one evaluation pass, no update)
        auto eval_residual = [&](int buf, V3 dxp, float zp, V3 d, Q4 qq, V3 l_s, V3 l_b, V3 l_c, float c0h,
                                 float s0h, float ct, float stt) -> float {
            const V3 aA = qaxis(qq);
            V3 dn, an;
            Q4 qn;
            fetch_next(buf, d, qq, aA, false, dn, qn, an);
            Geo g;
            V3 Dls, Dlb;
            float rs, rb;
            joint_eval(dxp, d, dn, qq, qn, aA, an, c0h, s0h, ct, stt, wA, c1A, c2A, wB, c1B, c2B, hl,
                       P.inv_L, comp_s, comp_b, comp_t, l_s, l_b, g, Dls, Dlb, rs, rb);
            const float cn = zp + d.z;
            const float rc = (l_c.x > 0.f ? fabsf(cn) : fmaxf(-cn, 0.f)) * P.inv_L;
            float rl = fmaxf(hasj ? fmaxf(rs, rb) : 0.f, (hasb && gnd) ? rc : 0.f);
            rl = (rl == rl) ? rl : INFINITY;
            rl = seg_reduce(rl);
            V3 inx, inth;
            return fetch_prev(zero, zero, rl, inx, inth);
        };

        const int steps = phase == kPhaseFull ? n_steps : 1;
        for (int st = 0; st < steps; ++st) {
            const long long stepc = (live ? P.step[s] : 0) + st;
            const int sub0 = phase == kPhaseFull ? 0 : sub_only;
            const int sub1 = phase == kPhaseFull ? P.substeps : sub_only + 1;
            if (phase != kPhaseSolve && sub0 == 0) {
                // command for the end of this step (eq. snake_control or a schedule)
                if (hasb && P.controller == kCtrlSerpenoid)
                    cmdv = (float)serpenoid_command(P, s, m, stepc);
                else if (hasb && P.controller == kCtrlSchedule)
                    cmdv = schedule_command(P, gm, stepc);
                if (P.law == kLawPaper) {
                    p0 = paper_update(P, p0, fmaxf(cmdv, 0.f));
                    p1 = paper_update(P, p1, fmaxf(-cmdv, 0.f));
                }
            }
            const float u0 = fmaxf(cmdv, 0.f), u1 = fmaxf(-cmdv, 0.f);
            if (phase == kPhaseFull) {
                rstep = 0.f;
                itstep = 0;
                status = 0;
            }
            for (int sub = sub0; sub < sub1; ++sub) {
                if (phase != kPhaseSolve && P.law == kLawLag) {
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
                V3 d = zero;
                if (phase == kPhaseSolve) {
                    if (hasb && !fixed) {
                        d = h * v;
                        q = Q4{P.q_pred[gb], P.q_pred[N + gb], P.q_pred[2 * N + gb], P.q_pred[3 * N + gb]};
                    }
                } else if (hasb && !fixed) {
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
                if (phase == kPhasePre) {
                    // the predicted orientation goes to its own array; the state
                    // keeps the start-of-substep orientation for the solve
                    if (hasb) {
                        P.q_pred[gb] = q.w;
                        P.q_pred[N + gb] = q.x;
                        P.q_pred[2 * N + gb] = q.y;
                        P.q_pred[3 * N + gb] = q.z;
                    }
                    q = qp;
                    continue;
                }
                const float zp = xp.z - P.R;
                V3 dxp;
                {
                    V3 xpn, an;
                    Q4 qn;
                    fetch_next(2, xp, q, zero, false, xpn, qn, an);
                    dxp = xp - xpn;
                }

                // multiplier initialisation
                const bool learned = PHASE == kPhaseSolve && P.warm == kWarmMlp;
                // fallback after K iterations (below): keep lambda0 aside
                const bool probe = learned && P.fallback && P.fallback_k > 0;
                V3 ls0 = zero, lb0 = zero;
                V3 d_zero = d;
                Q4 q_zero = q;
                if (P.warm == kWarmPrev || learned) {
                    if (learned) {
                        // network outputs: stretch in the predicted frame of body i,
                        // bend-twist in the joint frame, both in units of lam_ref
                        ls = zero;
                        lb = zero;
                        if (hasj) {
                            const float* y = P.mlp_y + 6 * (size_t)gj;
                            ls = P.lam_ref * qrot(q, mk(y[0], y[1], y[2]));
                            lb = (P.lam_ref * P.L) * mk(y[3], y[4], y[5]);
                        }
                        lc = zero;
                    }
                    if (probe) {
                        ls0 = ls;
                        lb0 = lb;
                        ls = zero;
                        lb = zero;
                    } else {
                        float r_zero = 0.f;
                        if (learned && P.fallback)
                            r_zero = eval_residual(0, dxp, zp, d, q, zero, zero, zero, c0h, s0h, ct, stt);
                        // x <- x~ + W J(x~)^T lambda0
                        {
                            const V3 aA = qaxis(q);
                            V3 dn, an;
                            Q4 qn;
                            fetch_next(1, d, q, aA, false, dn, qn, an);
                            Geo g;
                            V3 Dls, Dlb;
                            float rs, rb;
                            joint_eval(dxp, d, dn, q, qn, aA, an, c0h, s0h, ct, stt, wA, c1A, c2A, wB, c1B,
                                       c2B, hl, P.inv_L, comp_s, comp_b, comp_t, ls, lb, g, Dls, Dlb, rs, rb);
                            V3 tA, tB;
                            joint_torques(g, ls, lb, hl, tA, tB);
                            V3 inf, intq;
                            fetch_prev(sel(hasj, -ls, zero), sel(hasj, tB, zero), 0.f, inf, intq);
                            const bool recv = hasb && i > 0;
                            const V3 fsum = sel(recv, inf, zero) + sel(hasj, ls, zero);
                            const V3 tsum = sel(recv, intq, zero) + sel(hasj, tA, zero);
                            const V3 dxc = (gnd && !fixed) ? P.inv_m * mk(lc.y, lc.z, lc.x) : zero;
                            if (hasb && !fixed) {
                                d = d + fma3(wA, fsum, dxc);
                                q = qturn(q, inv_inertia(tsum, aA, c1A, c2A));
                            }
                        }
                        if (learned && P.fallback) {
                            // keep the learned start only if it begins closer than zero
                            const float r_nn = eval_residual(0, dxp, zp, d, q, ls, lb, lc, c0h, s0h, ct, stt);
                            if (live && !(r_nn <= r_zero)) {
                                d = d_zero;
                                q = q_zero;
                                ls = zero;
                                lb = zero;
                                lc = zero;
                                status |= kStatusFellBack;
                            }
                        }
                    }
                } else {
                    ls = zero;
                    lb = zero;
                    lc = zero;
                }

                // Fallback after K iterations: the zero start, then the learned
                // start, K iterations each (solve phase only; the full-step
                // kernels never take the learned start).  run_probe repeats the
                // iteration below for exactly kprobe iterations, without status,
                // and returns the residual of iterate kprobe.
                int koff = 0, extra = 0;
                if constexpr (PHASE == kPhaseSolve) {
                    if (probe) {
                        // x <- x~ + W J(x~)^T lambda0 for the multipliers in ls, lb, lc
                        auto apply_start = [&]() {
                            const V3 aA = qaxis(q);
                            V3 dn, an;
                            Q4 qn;
                            fetch_next(1, d, q, aA, false, dn, qn, an);
                            Geo g;
                            V3 Dls, Dlb;
                            float rs, rb;
                            joint_eval(dxp, d, dn, q, qn, aA, an, c0h, s0h, ct, stt, wA, c1A, c2A, wB, c1B,
                                       c2B, hl, P.inv_L, comp_s, comp_b, comp_t, ls, lb, g, Dls, Dlb, rs, rb);
                            V3 tA, tB;
                            joint_torques(g, ls, lb, hl, tA, tB);
                            V3 inf, intq;
                            fetch_prev(sel(hasj, -ls, zero), sel(hasj, tB, zero), 0.f, inf, intq);
                            const bool recv = hasb && i > 0;
                            const V3 fsum = sel(recv, inf, zero) + sel(hasj, ls, zero);
                            const V3 tsum = sel(recv, intq, zero) + sel(hasj, tA, zero);
                            const V3 dxc = (gnd && !fixed) ? P.inv_m * mk(lc.y, lc.z, lc.x) : zero;
                            if (hasb && !fixed) {
                                d = d + fma3(wA, fsum, dxc);
                                q = qturn(q, inv_inertia(tsum, aA, c1A, c2A));
                            }
                        };
                        auto run_probe = [&](int kprobe) -> float {
                    bool done = !live;
                    float rdone = 0.f;
                for (int k = 0;; ++k) {
                    const V3 aA = qaxis(q);
                    V3 dn, an;
                    Q4 qn;
                    const bool wave_done = __all(done);
                    const bool all_done = fetch_next(k & 1, d, q, aA, wave_done, dn, qn, an);
                    if (xw ? all_done : wave_done) break;
                    Geo g;
                    V3 Dls, Dlb;
                    float rs, rb;
                    joint_eval(dxp, d, dn, q, qn, aA, an, c0h, s0h, ct, stt, wA, c1A, c2A, wB, c1B,
                               c2B, hl, P.inv_L, comp_s, comp_b, comp_t, ls, lb, g, Dls, Dlb, rs, rb);
                    const float cn = zp + d.z;
                    const float rc = (lc.x > 0.f ? fabsf(cn) : fmaxf(-cn, 0.f)) * P.inv_L;
                    float rl = fmaxf(hasj ? fmaxf(rs, rb) : 0.f, (hasb && gnd) ? rc : 0.f);
                    rl = (rl == rl) ? rl : INFINITY;
                    rl = seg_reduce(rl);

                    const V3 dls = sj * Dls, dlb = sj * Dlb;
                    V3 tA, tB;
                    joint_torques(g, dls, dlb, hl, tA, tB);
                    V3 inf, intq;
                    const float r = fetch_prev(andz(mj, -dls), andz(mj, tB), rl, inf, intq);

                    if (!done) {
                        const bool bad = !(r < INFINITY);
                        if (bad || k >= kprobe) {
                            done = true;
                            rdone = bad ? INFINITY : r;
                        }
                    }
                    if (!done) {
                        V3 dlc = zero;
                        if (gnd && !fixed) dlc = contact_incr(lc, cn, d, sc, mass, mu);
                        // gather in a fixed order: forces of joint i-1 (received),
                        // joint i and the contact through the inverse mass; torques
                        // of the two joints through the inverse inertia
                        const V3 fsum = andz(mr, inf) + andz(mj, dls);
                        const V3 tsum = andz(mr, intq) + andz(mj, tA);
                        // unmasked: zero increments without a joint, the
                        // fixed root's zero inverse mass, and an empty lane's
                        // state, read only by the joints that are discarded
                        ls = ls + dls;
                        lb = lb + dlb;
                        if (gnd) lc = lc + dlc;
                        d = fma3(wA, fsum + mk(dlc.y, dlc.z, dlc.x), d);
                        if (!fixed) q = qturn(q, inv_inertia(tsum, aA, c1A, c2A));
                    }
                }
                            return rdone;
                        };
                        const float rz = run_probe(P.fallback_k);   // zero start
                        // keep the zero start's iterate K for a fallback
                        if (hasb) {
                            float* ps = P.probe + gb;
                            const float keep[16] = {d.x, d.y, d.z, q.w, q.x, q.y, q.z, ls.x, ls.y, ls.z,
                                                    lb.x, lb.y, lb.z, lc.x, lc.y, lc.z};
#pragma unroll
                            for (int c = 0; c < 16; ++c) ps[(size_t)c * N] = keep[c];
                        }
                        d = d_zero;
                        q = q_zero;
                        ls = ls0;
                        lb = lb0;
                        lc = zero;
                        if (xw) __syncthreads();   // every wave has read the last exchange
                        apply_start();
                        const float rw = run_probe(P.fallback_k);   // learned start
                        // keep the learned start if it is finite and not farther than zero
                        if (rw < INFINITY && (rz >= INFINITY || rw <= rz)) {
                            koff = P.fallback_k;
                            extra = P.fallback_k;
                        } else {
                            // continue from the zero start's iterate K
                            if (hasb) {
                                const float* ps = P.probe + gb;
                                float kept[16];
#pragma unroll
                                for (int c = 0; c < 16; ++c) kept[c] = ps[(size_t)c * N];
                                d = mk(kept[0], kept[1], kept[2]);
                                q = Q4{kept[3], kept[4], kept[5], kept[6]};
                                ls = mk(kept[7], kept[8], kept[9]);
                                lb = mk(kept[10], kept[11], kept[12]);
                                lc = mk(kept[13], kept[14], kept[15]);
                            }
                            if (live) status |= kStatusFellBack;
                            koff = P.fallback_k;
                            extra = P.fallback_k;
                        }
                        if (xw) __syncthreads();
                    }
                }

                bool done = !live;
                int kdone = 0;
                float rdone = 0.f;
                for (int k = 0;; ++k) {
                    const V3 aA = qaxis(q);
                    V3 dn, an;
                    Q4 qn;
                    const bool wave_done = __all(done);
                    const bool all_done = fetch_next(k & 1, d, q, aA, wave_done, dn, qn, an);
                    if (xw ? all_done : wave_done) break;
                    Geo g;
                    V3 Dls, Dlb;
                    float rs, rb;
                    joint_eval(dxp, d, dn, q, qn, aA, an, c0h, s0h, ct, stt, wA, c1A, c2A, wB, c1B,
                               c2B, hl, P.inv_L, comp_s, comp_b, comp_t, ls, lb, g, Dls, Dlb, rs, rb);
                    const float cn = zp + d.z;
                    const float rc = (lc.x > 0.f ? fabsf(cn) : fmaxf(-cn, 0.f)) * P.inv_L;
                    float rl = fmaxf(hasj ? fmaxf(rs, rb) : 0.f, (hasb && gnd) ? rc : 0.f);
                    rl = (rl == rl) ? rl : INFINITY;
                    rl = seg_reduce(rl);

                    const V3 dls = sj * Dls, dlb = sj * Dlb;
                    V3 tA, tB;
                    joint_torques(g, dls, dlb, hl, tA, tB);
                    V3 inf, intq;
                    const float r = fetch_prev(andz(mj, -dls), andz(mj, tB), rl, inf, intq);

                    if (!done) {
                        const int kl = k + koff;
                        const bool bad = !(r < INFINITY);
                        const bool stop = bad || (P.tol > 0.f ? (r <= P.tol || kl >= P.iters) : (kl >= P.iters));
                        if (stop) {
                            done = true;
                            kdone = kl;
                            rdone = r;
                            if (bad)
                                status |= kStatusNonfinite;
                            else if (P.tol > 0.f && r > P.tol)
                                status |= kStatusNotConverged;
                        }
                    }
                    if (!done) {
                        V3 dlc = zero;
                        if (gnd && !fixed) dlc = contact_incr(lc, cn, d, sc, mass, mu);
                        // gather in a fixed order: forces of joint i-1 (received),
                        // joint i and the contact through the inverse mass; torques
                        // of the two joints through the inverse inertia
                        const V3 fsum = andz(mr, inf) + andz(mj, dls);
                        const V3 tsum = andz(mr, intq) + andz(mj, tA);
                        // unmasked: zero increments without a joint, the
                        // fixed root's zero inverse mass, and an empty lane's
                        // state, read only by the joints that are discarded
                        ls = ls + dls;
                        lb = lb + dlb;
                        if (gnd) lc = lc + dlc;
                        d = fma3(wA, fsum + mk(dlc.y, dlc.z, dlc.x), d);
                        if (!fixed) q = qturn(q, inv_inertia(tsum, aA, c1A, c2A));
                    }
                }
                if (live) kdone += extra;
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
        if (NW > 1) __syncthreads();   // every lane has read step[s] before it moves
        if (live && i == 0 && phase != kPhasePre) {
            P.residual[s] = rstep;
            P.iters_out[s] = itstep;
            P.status[s] = status;
            const bool last = phase == kPhaseFull || sub_only == P.substeps - 1;
            if (last) P.step[s] = P.step[s] + (phase == kPhaseFull ? n_steps : 1);
            P.iters_total[s] = P.iters_total[s] + (phase == kPhaseFull ? itsum : itstep - it_before);
        }
    }
}

// Inputs of the warm-start network, two rows (stretch, bend-twist) per joint
// (joint_features).
__global__ void k_features(KParams P, float* __restrict__ feat)
{
    const int gj = blockIdx.x * blockDim.x + threadIdx.x;
    if (gj >= P.J) return;
    float f[32];
    V3 lbn;
    joint_features(P, gj, 0, P.n_snakes - 1, f, lbn);
    float* out = feat + (size_t)64 * gj;
    for (int k = 0; k < 32; ++k) out[k] = f[k];
    f[19] = lbn.x; f[20] = lbn.y; f[21] = lbn.z; f[30] = 1.f;
    for (int k = 0; k < 32; ++k) out[32 + k] = f[k];
}

// Training targets: the substep's final multipliers in network units
// (stretch in the predicted frame of body A over lam_ref, bend-twist over
// lam_ref L), two rows of 3 per joint.
__global__ void k_targets(KParams P, float* __restrict__ tgt)
{
    const int gj = blockIdx.x * blockDim.x + threadIdx.x;
    if (gj >= P.J) return;
    int lo = 0, hi = P.n_snakes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (P.joint_off[mid] <= gj)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int a = P.body_off[lo] + (gj - P.joint_off[lo]);
    const int N = P.N, J = P.J;
    const Q4 qa{P.q_pred[a], P.q_pred[N + a], P.q_pred[2 * N + a], P.q_pred[3 * N + a]};
    const V3 ls = mk(P.lam_j[gj], P.lam_j[J + gj], P.lam_j[2 * J + gj]);
    const V3 y = (1.f / P.lam_ref) * qrot(qconj(qa), ls);
    const float refb = P.lam_ref * P.L;
    float* out = tgt + (size_t)6 * gj;
    out[0] = y.x; out[1] = y.y; out[2] = y.z;
    out[3] = P.lam_j[3 * J + gj] / refb;
    out[4] = P.lam_j[4 * J + gj] / refb;
    out[5] = P.lam_j[5 * J + gj] / refb;
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

hipError_t launch_tiles(int nw, int rows, const KParams& P, const int4* hdr, const int2* slots,
                        int n_tiles, int grid, int n_steps, int phase, int sub, hipStream_t stream)
{
    if (n_tiles <= 0) return hipSuccess;
    if (grid <= 0 || grid > n_tiles) grid = n_tiles;
    const dim3 g(grid), b(64 * nw);
#define SNAKE_LAUNCH(NWV, PH, RW) \
    hipLaunchKernelGGL((k_tile<NWV, PH, RW>), g, b, 0, stream, P, hdr, slots, n_tiles, n_steps, sub)
#define SNAKE_PHASES(NWV, RW)                                        \
    if (phase == kPhaseFull) SNAKE_LAUNCH(NWV, kPhaseFull, RW);     \
    else if (phase == kPhasePre) SNAKE_LAUNCH(NWV, kPhasePre, RW);  \
    else SNAKE_LAUNCH(NWV, kPhaseSolve, RW);
#define SNAKE_LAYOUTS(NWV)                   \
    if (rows == 2) { SNAKE_PHASES(NWV, 2) }     \
    else if (rows) { SNAKE_PHASES(NWV, 1) }   \
    else { SNAKE_PHASES(NWV, 0) }
    switch (nw) {
        case 1: SNAKE_LAYOUTS(1) break;
        case 2: SNAKE_LAYOUTS(2) break;
        case 4: SNAKE_LAYOUTS(4) break;
        case 8: SNAKE_LAYOUTS(8) break;
        case 16: SNAKE_LAYOUTS(16) break;
        default: return hipErrorInvalidValue;
    }
#undef SNAKE_LAYOUTS
#undef SNAKE_PHASES
#undef SNAKE_LAUNCH
    return hipGetLastError();
}

hipError_t launch_features(const KParams& P, float* feat, hipStream_t stream)
{
    if (P.J <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_features, dim3((P.J + 127) / 128), dim3(128), 0, stream, P, feat);
    return hipGetLastError();
}

hipError_t launch_targets(const KParams& P, float* tgt, hipStream_t stream)
{
    if (P.J <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_targets, dim3((P.J + 127) / 128), dim3(128), 0, stream, P, tgt);
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
