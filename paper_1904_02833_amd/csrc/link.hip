// Full-resolution soft links (include/link.h): particles on a tetrahedral
// mesh per link, rigid frames between links, solved by block Jacobi in FP32.
//
// Mapping (gfx950): one workgroup of 1024 threads (16 wave64) per snake.
// Thread i owns link i (i < links) and the blocks b = i and b = i + 1024 of
// the snake's block list (tetrahedra, distance rows, attachments).  Each
// particle has an aligned group of 1, 2, 4 or 8 lanes (a host-built plan,
// more lanes for the particles with more incident blocks), whose first lane
// holds the particle; each frame has a group of eight lanes in the last wave.  A block keeps its multipliers, its pending
// increment and its start-of-substep geometry in registers for the whole
// launch; the per-mesh constants (shared by every link of every snake) are
// read through the caches.  One iteration: every block evaluates itself at
// the current iterate and writes what its bodies need to LDS (a tetrahedron
// the 3x3 matrix R T, T the increment as a symmetric strain tensor, so the
// impulse on vertex m is R T g_m; a distance row its impulse on the first
// particle; an attachment its increment); the workgroup's residual maximum
// decides the stop; then every particle gathers its blocks in the fixed
// order of the mesh's incidence list (tetrahedra, distance rows,
// attachment, its own contact) and every frame its attachments, each group
// summing its members' ranges of the list and adding the partial sums
// pairwise.  Two barriers per iteration.  Positions are the start-of-substep position plus
// a displacement: edges and attachment gaps are formed from the
// start-of-substep differences (computed once per substep) plus
// displacement differences, so they keep FP32 precision far from the
// origin.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "device_math.h"
#include "link.h"

using snake::cross;
using snake::dot;
using snake::mk;
using snake::Q4;
using snake::qconj;
using snake::qmul;
using snake::qrot;
using snake::qturn;
using snake::V3;

namespace lk {

constexpr int kThreads = 1024;
constexpr int kSlots = 2;          // blocks per thread
constexpr int kWaves = kThreads / 64;
constexpr int kMaxLinks = 4;
constexpr int kLdsLimit = 163840;  // bytes of LDS a gfx950 workgroup may take

constexpr int kCentre = 0, kRadial = 1, kChamber0 = 2, kChamber1 = 3;
// incidence entries: type << 28 | block << 2 | slot
constexpr int kIncTet = 0, kIncDist = 1, kIncAtt = 2;

struct Params {
    int n_snakes, L, P1, Tm, D1, A1, ring;
    int P, F, NB;                   // per snake: particles, frames, blocks
    int ground, fixed0, tol_mode, iters, substeps;
    float h, inv_h, g, tol, lag_in, lag_de, young_inv_pmax, frame_w, Lref_inv, a_rigid;
    float I_ax_inv, I_pe_inv, I_ax, I_pe, relax;
    // state (SoA, batch totals in the comments)
    float *x, *v, *lam_c;           // [3][NP]
    float *fx, *fq, *fv, *fw;       // [3|4][NF]
    float *p, *cmd;                 // [2][NL], [NL]
    float *lam_tet, *lam_dist, *lam_att;  // [6][NT], [ND], [3][NA]
    float* residual;
    int *iters_out, *status, *iters_total;
    const float* mu;                // [n_snakes]
    int64_t NP, NF, NL, NT, ND, NA;
    // per-mesh constants
    const int* tet_v;               // [Tm] four 8-bit local particle indices
    const float* tet_g;             // [12][Tm] g_0..g_3 (g_0 = -(g_1+g_2+g_3))
    const float* tet_ldl;           // [21][Tm] unit-lower L (15, row-major below the diagonal) then 1/D (6)
    const float* tet_alpha;         // [3][Tm] E/h^2: normal diagonal, normal off-diagonal, shear
    const float* tet_scale;         // [Tm] relax / largest vertex degree
    const int* dist_ij;             // [D1] i | j << 16 (local)
    const int* dist_kind;           // [D1]
    const float* dist_c;            // [4][D1] rest, w_i, w_j, scale
    const int* att_p;               // [A1] local particle
    const float* att_c;             // [5][A1] r (3), w_p, particle degree
    const float* part_w;            // [P1] inverse masses
    const float* part_m;            // [P1] masses
    const int* part_deg;            // [P1] blocks touching the particle
    const int* inc;                 // incidence entries, particle by particle
    const int* gplan;               // [2][1024] per lane: particle | log2 group << 16 (-1: none),
                                    // first | end << 16 of its range of the incidence entries
    int gmax;                       // largest particle group
};

__device__ __forceinline__ V3 lane_xor(V3 v, int m)
{
    return mk(__shfl_xor(v.x, m, 64), __shfl_xor(v.y, m, 64), __shfl_xor(v.z, m, 64));
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

// rotation of the polar decomposition F = R S (det F > 0) by Newton's
// iteration R <- (R + R^-T) / 2 from R = F; returns false for det F <= 0.
// Convergence is quadratic: with the iterate R (I + E), E symmetric, one
// step leaves about E^2 / 2 and moves the iterate by about |E|, so a step
// that moved no entry by more than 1e-4 (|E| below 3e-4 in norm) leaves an
// error below 5e-8, under FP32 rounding, and ends the iteration.  The first
// two steps are not tested: from F at the strains of a link's elements one
// step never suffices and two rarely do, so a wave (whose lanes run until
// the last one stops) would pay for the test without ending sooner.  The iterate is kept as Z_k = 2^k R_k, so
// that Z_{k+1} = Z_k + 4^k cof(Z_k) / det Z_k takes one fused multiply-add
// per entry (R^-T = cof R / det R; the powers of two are exact).
__device__ __forceinline__ bool polar_step(float* Z, float sc, float& diff, bool test)
{
    const float c00 = Z[4] * Z[8] - Z[5] * Z[7], c01 = Z[5] * Z[6] - Z[3] * Z[8], c02 = Z[3] * Z[7] - Z[4] * Z[6];
    const float c10 = Z[2] * Z[7] - Z[1] * Z[8], c11 = Z[0] * Z[8] - Z[2] * Z[6], c12 = Z[1] * Z[6] - Z[0] * Z[7];
    const float c20 = Z[1] * Z[5] - Z[2] * Z[4], c21 = Z[2] * Z[3] - Z[0] * Z[5], c22 = Z[0] * Z[4] - Z[1] * Z[3];
    const float det = Z[0] * c00 + Z[1] * c01 + Z[2] * c02;
    // hardware reciprocal (1 ulp): the iteration's fixed point is the
    // rotation either way, within the convergence test
    const float id = sc * __builtin_amdgcn_rcpf(det);
    const float c[9] = {c00, c01, c02, c10, c11, c12, c20, c21, c22};
    diff = 0.f;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const float n = fmaf(c[k], id, Z[k]);
        if (test) diff = fmaxf(diff, fabsf(fmaf(-2.f, Z[k], n)));
        Z[k] = n;
    }
    return det > 0.f;
}

__device__ __forceinline__ bool polar(const float* F, float* R)
{
    float Z[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Z[k] = F[k];
    float diff;
    bool ok = polar_step(Z, 1.f, diff, false);
    ok = ok && polar_step(Z, 4.f, diff, false);
    // after step k + 1: 4^(k+1), 2^-(k+1), and the bound on |Z_{k+1} - 2 Z_k|
    float sc = 16.f, inv = 0.25f, lim = 8e-4f;
#pragma unroll 2
    for (int it = 2; ok && it < 12; ++it) {
        ok = polar_step(Z, sc, diff, true);
        sc *= 4.f;
        inv *= 0.5f;
        if (diff <= lim) break;
        lim *= 2.f;
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) R[k] = Z[k] * inv;
    return ok;
}

// world inverse inertia of a frame (solid cylinder along body x) applied to t
__device__ __forceinline__ V3 frame_inv_inertia(const Params& P, Q4 q, V3 t)
{
    const V3 a = snake::qaxis(q);
    return P.I_pe_inv * t + ((P.I_ax_inv - P.I_pe_inv) * dot(a, t)) * a;
}

// LDS of one snake's workgroup.  Per-block and per-particle data are
// records (array of structures with odd strides, free of bank conflicts for
// consecutive blocks), so one address per record serves all its fields
// through the instructions' immediate offsets.
// element record: g_1..g_3 (9), L (15), -scale / D (6), E/h^2 (3), vertices,
// the gather slots of its four vertices (4), pad
constexpr int kTR = 39;
// distance row: rest, w_i, w_j, scale, i | j << 16, kind, slots of i and j,
// -scale / (w_i + w_j + rigid compliance)
constexpr int kDR = 9;
// attachment: r (3), w_p, -relax / max(particle degree, frame degree) at an
// end frame and at an inner frame, particle, slot, pad
constexpr int kAR = 9;
constexpr int kPR = 7;    // particle: start-of-substep position (3), displacement (3), pad
constexpr int kFr = 20;   // frame: xp (3), d (3), q (4), v (3), w (3), q at the substep start (4)

struct Lds {
    float* tr;    // [Tm][kTR]
    float* dr;    // [D1][kDR]
    float* ar;    // [A1][kAR]
    float* pr;    // [P][kPR]
    float* V;     // [L][n_inc][3] what each block sends each of its particles, in the
                  // particles' gather order (slot = incidence entry)
    float* da;    // [A][6] attachment increments and their torques about the frame (the frames' side)
    float* fr;    // [F][kFr]
    float* lk;    // [4][L] p0, p1, chamber 0 commanded, chamber 1 commanded
    float* red;   // [kWaves] residual maxima of the waves
};

// words of LDS for a snake (the layout of Lds)
__host__ __device__ inline int lds_words(int L, int P1, int Tm, int D1, int A1, int n_inc)
{
    const int P = L * P1, T = L * Tm, D = L * D1, A = L * A1;
    return kTR * Tm + kDR * D1 + kAR * A1 + kPR * P + 3 * L * n_inc + 6 * A + kFr * (L + 1) + 4 * L + kWaves;
}

__device__ __forceinline__ V3 ld3(const float* a) { return mk(a[0], a[1], a[2]); }
__device__ __forceinline__ void st3(float* a, V3 v)
{
    a[0] = v.x;
    a[1] = v.y;
    a[2] = v.z;
}

__global__ void __launch_bounds__(kThreads) k_link(Params P, int n_steps)
{
    extern __shared__ float smem[];
    const int s = blockIdx.x;
    const int tid = threadIdx.x;
    const int L = P.L, NP = P.P, NF = P.F, Tm = P.Tm, D1 = P.D1, A1 = P.A1, P1 = P.P1;
    const int T = L * Tm, D = L * D1, A = L * A1;
    const int n_inc = 4 * Tm + 2 * D1 + A1;
    Lds S;
    {
        float* w = smem;
        S.tr = w, w += kTR * Tm;
        S.dr = w, w += kDR * D1;
        S.ar = w, w += kAR * A1;
        S.pr = w, w += kPR * NP;
        S.V = w, w += 3 * L * n_inc;
        S.da = w, w += 6 * A;
        S.fr = w, w += kFr * NF;
        S.lk = w, w += 4 * L;
        S.red = w;
    }
    // per-mesh constants into records (the slot fields are filled below)
    for (int i = tid; i < kTR * Tm; i += kThreads) {
        const int t = i / kTR, f = i - t * kTR;
        if (f >= 34 && f < 38) continue;
        float val = 0.f;
        if (f < 9)
            val = P.tet_g[(f + 3) * Tm + t];
        else if (f < 24)
            val = P.tet_ldl[(f - 9) * Tm + t];
        else if (f < 30)
            val = -P.tet_scale[t] * P.tet_ldl[(f - 9) * Tm + t];
        else if (f < 33)
            val = P.tet_alpha[(f - 30) * Tm + t];
        else if (f == 33)
            val = __int_as_float(P.tet_v[t]);
        S.tr[i] = val;
    }
    for (int i = tid; i < kDR * D1; i += kThreads) {
        const int e = i / kDR, f = i - e * kDR;
        if (f == 6 || f == 7) continue;
        S.dr[i] = f < 4 ? P.dist_c[f * D1 + e] : f == 4 ? __int_as_float(P.dist_ij[e])
                  : f == 5 ? __int_as_float(P.dist_kind[e])
                           : -P.dist_c[3 * D1 + e] / (P.dist_c[D1 + e] + P.dist_c[2 * D1 + e] + P.a_rigid);
    }
    for (int i = tid; i < kAR * A1; i += kThreads) {
        const int e = i / kAR, f = i - e * kAR;
        if (f == 7) continue;
        const int dpart = (int)P.att_c[4 * A1 + e], dend = A1 / 2 > dpart ? A1 / 2 : dpart,
                  dmid = A1 > dpart ? A1 : dpart;
        S.ar[i] = f < 4 ? P.att_c[f * A1 + e] : f == 4 ? -P.relax / (float)dend : f == 5 ? -P.relax / (float)dmid
                : f == 6 ? __int_as_float(P.att_p[e]) : 0.f;
    }
    // incidence entry i is gather slot i: each block records the slots of
    // its particles (one entry per block and particle)
    for (int i = tid; i < n_inc; i += kThreads) {
        const int ent = P.inc[i];
        const int type = ent >> 28, blk = (ent >> 2) & 0x3ffffff, slot = ent & 3;
        if (type == kIncTet)
            S.tr[kTR * blk + 34 + slot] = __int_as_float(i);
        else if (type == kIncDist)
            S.dr[kDR * blk + 6 + slot] = __int_as_float(i);
        else
            S.ar[kAR * blk + 7] = __int_as_float(i);
    }

    // this lane's particle group: the particle, the group's size, the
    // lane's range of the particle's incidence entries; the group's first
    // lane holds the particle
    const int gw0 = P.gplan[tid], gw1 = P.gplan[kThreads + tid];
    const bool isg = gw0 >= 0;
    const int pidx = isg ? gw0 & 0xffff : 0, gsize = isg ? 1 << (gw0 >> 16) : 1;
    const int e0 = gw1 & 0xffff, e1 = gw1 >> 16;
    const bool isp = isg && (tid & (gsize - 1)) == 0;
    const int64_t gp = (int64_t)s * NP + pidx;    // particle
    // frame groups of eight lanes in the last wave, which holds no particle
    // when the snake has at most 960: their sums run beside the particles'
    const int fj = tid - (kThreads - 64), fi = fj >> 3, fsub = fj & 7;
    const bool isfg = fj >= 0 && fi < NF, isf = isfg && fsub == 0;
    const int64_t gf = (int64_t)s * NF + fi;      // frame
    const int64_t gl = (int64_t)s * L + tid;      // link
    const bool isl = tid < L;
    const bool ffix = P.fixed0 && fi == 0;

    // particle state in registers
    V3 x = mk(0.f, 0.f, 0.f), v = x, lc = x, d = x, dlc = x;
    float wp = 0.f, pmass = 0.f, cscale = 0.f;
    const int pl = pidx / P1, pk = pidx - pl * P1;
    if (isp) {
        x = mk(P.x[gp], P.x[P.NP + gp], P.x[2 * P.NP + gp]);
        v = mk(P.v[gp], P.v[P.NP + gp], P.v[2 * P.NP + gp]);
        lc = mk(P.lam_c[gp], P.lam_c[P.NP + gp], P.lam_c[2 * P.NP + gp]);
        wp = P.part_w[pk];
        pmass = P.part_m[pk];
        cscale = P.relax / (float)P.part_deg[pk];
    }
    float* const my = S.pr + kPR * pidx;   // this group's particle record
    const float mu = P.mu[s];
    // frame and link state in LDS
    if (isf) {
        float* f = S.fr + kFr * fi;
        f[0] = P.fx[gf], f[1] = P.fx[P.NF + gf], f[2] = P.fx[2 * P.NF + gf];
        f[6] = P.fq[gf], f[7] = P.fq[P.NF + gf], f[8] = P.fq[2 * P.NF + gf], f[9] = P.fq[3 * P.NF + gf];
        f[10] = P.fv[gf], f[11] = P.fv[P.NF + gf], f[12] = P.fv[2 * P.NF + gf];
        f[13] = P.fw[gf], f[14] = P.fw[P.NF + gf], f[15] = P.fw[2 * P.NF + gf];
    }
    if (isl) {
        S.lk[tid] = P.p[gl];
        S.lk[L + tid] = P.p[P.NL + gl];
    }
    // blocks: kind 0 element, 1 distance row, 2 attachment, 3 none
    int bkind[kSlots], bidx[kSlots], blink[kSlots];
    float lam[kSlots][6], pend[kSlots][6];
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
        const int b = tid + k * kThreads;
        bkind[k] = b < T ? 0 : b < T + D ? 1 : b < T + D + A ? 2 : 3;
        const int loc = bkind[k] == 0 ? b : bkind[k] == 1 ? b - T : b - T - D;
        const int per = bkind[k] == 0 ? Tm : bkind[k] == 1 ? D1 : A1;
        blink[k] = bkind[k] < 3 ? loc / per : 0;
        bidx[k] = bkind[k] < 3 ? loc - blink[k] * per : 0;
#pragma unroll
        for (int r = 0; r < 6; ++r) lam[k][r] = 0.f;
#pragma unroll
        for (int r = 0; r < 6; ++r) pend[k][r] = 0.f;
    }
    __syncthreads();

    float rstep = 0.f;
    int itstep = 0, status = 0, itsum = 0;
    for (int st = 0; st < n_steps; ++st) {
        rstep = 0.f;
        itstep = 0;
        status = 0;
        for (int sub = 0; sub < P.substeps; ++sub) {
            // chamber pressures: first-order lag toward the commanded chamber
            if (isl) {
                const float c = P.cmd[gl];
                const float u0 = fmaxf(c, 0.f), u1 = fmaxf(-c, 0.f);
                float p0 = S.lk[tid], p1 = S.lk[L + tid];
                p0 = u0 + (p0 - u0) * (u0 > p0 ? P.lag_in : P.lag_de);
                p1 = u1 + (p1 - u1) * (u1 > p1 ? P.lag_in : P.lag_de);
                S.lk[tid] = p0;
                S.lk[L + tid] = p1;
                S.lk[2 * L + tid] = u0 > 0.f ? 1.f : 0.f;
                S.lk[3 * L + tid] = u1 > 0.f ? 1.f : 0.f;
            }
            // prediction
            if (isp) {
                v.z -= P.h * P.g;
                d = P.h * v;
                lc = mk(0.f, 0.f, 0.f);
                st3(my, x);
                st3(my + 3, d);
            }
            if (isf) {
                float* f = S.fr + kFr * fi;
                Q4 q{f[6], f[7], f[8], f[9]};
                f[16] = q.w, f[17] = q.x, f[18] = q.y, f[19] = q.z;
                V3 fv = mk(f[10], f[11], f[12]), fw = mk(f[13], f[14], f[15]), fd = mk(0.f, 0.f, 0.f);
                if (ffix) {
                    fv = fw = fd;
                } else {
                    fv.z -= P.h * P.g;
                    fd = P.h * fv;
                    const V3 ax = snake::qaxis(q);
                    const V3 Iw = P.I_pe * fw + ((P.I_ax - P.I_pe) * dot(ax, fw)) * ax;
                    const V3 tq = -cross(fw, Iw);
                    fw = fw + P.h * frame_inv_inertia(P, q, tq);
                    q = qturn(q, P.h * fw);
                }
                f[3] = fd.x, f[4] = fd.y, f[5] = fd.z;
                f[6] = q.w, f[7] = q.x, f[8] = q.y, f[9] = q.z;
                f[10] = fv.x, f[11] = fv.y, f[12] = fv.z;
                f[13] = fw.x, f[14] = fw.y, f[15] = fw.z;
            }
#pragma unroll
            for (int k = 0; k < kSlots; ++k)
#pragma unroll
                for (int r = 0; r < 6; ++r) lam[k][r] = 0.f;
            __syncthreads();

            int k_it = 0;
            float r = 0.f;
            for (;;) {
                // ---- every block at the current iterate
                float res = 0.f;
#pragma unroll
                for (int k = 0; k < kSlots; ++k) {
                    const int t = bidx[k];
                    if (bkind[k] == 0) {
                        const float* c = S.tr + kTR * t;
                        const int vv = __float_as_int(c[33]), base = blink[k] * P1;
                        const float* p0 = S.pr + kPR * (base + (vv & 255));
                        float F[9];
                        {
                            float E[3][3];   // edges x_m - x_0, m = 1..3, as columns
#pragma unroll
                            for (int m = 1; m < 4; ++m) {
                                const float* pm = S.pr + kPR * (base + ((vv >> (8 * m)) & 255));
#pragma unroll
                                for (int q = 0; q < 3; ++q) E[q][m - 1] = (pm[q] - p0[q]) + (pm[3 + q] - p0[3 + q]);
                            }
                            // F = sum_m (x_m - x_0) g_m^T
#pragma unroll
                            for (int j = 0; j < 3; ++j)
#pragma unroll
                                for (int i = 0; i < 3; ++i)
                                    F[3 * i + j] = E[i][0] * c[j] + E[i][1] * c[3 + j] + E[i][2] * c[6 + j];
                        }
                        float R[9];
                        const bool ok = polar(F, R);
                        // strain sym(R^T F) - I in Voigt order (xx yy zz yz xz xy);
                        // R^T F is symmetric at the polar factor, so one of each
                        // off-diagonal pair serves
                        float y[6];
                        {
                            const float s00 = R[0] * F[0] + R[3] * F[3] + R[6] * F[6];
                            const float s11 = R[1] * F[1] + R[4] * F[4] + R[7] * F[7];
                            const float s22 = R[2] * F[2] + R[5] * F[5] + R[8] * F[8];
                            const float s12 = R[1] * F[2] + R[4] * F[5] + R[7] * F[8];
                            const float s02 = R[0] * F[2] + R[3] * F[5] + R[6] * F[8];
                            const float s01 = R[0] * F[1] + R[3] * F[4] + R[6] * F[7];
                            const float ad = c[30], ao = c[31], as = c[32];
                            const float* l = lam[k];
                            y[0] = (s00 - 1.f) + ad * l[0] + ao * (l[1] + l[2]);
                            y[1] = (s11 - 1.f) + ad * l[1] + ao * (l[0] + l[2]);
                            y[2] = (s22 - 1.f) + ad * l[2] + ao * (l[0] + l[1]);
                            y[3] = s12 + as * l[3];
                            y[4] = s02 + as * l[4];
                            y[5] = s01 + as * l[5];
                        }
                        float rm = 0.f;
#pragma unroll
                        for (int q = 0; q < 6; ++q) rm = fmaxf(rm, fabsf(y[q]));
                        res = fmaxf(res, ok ? rm : INFINITY);
                        // -scale (L D L^T)^-1 y: forward, diagonal (with -scale), backward
#pragma unroll
                        for (int q = 1; q < 6; ++q)
#pragma unroll
                            for (int cc = 0; cc < q; ++cc) y[q] -= c[9 + q * (q - 1) / 2 + cc] * y[cc];
#pragma unroll
                        for (int q = 0; q < 6; ++q) y[q] *= c[24 + q];
#pragma unroll
                        for (int q = 4; q >= 0; --q)
#pragma unroll
                            for (int cc = q + 1; cc < 6; ++cc) y[q] -= c[9 + cc * (cc - 1) / 2 + q] * y[cc];
#pragma unroll
                        for (int q = 0; q < 6; ++q) pend[k][q] = y[q];
                        // U = R T, T the increment as a symmetric tensor; vertex m
                        // receives U g_m, written to its gather slot (g_0 = -(g_1 +
                        // g_2 + g_3), so vertex 0 the negated sum of the others)
                        const float Tn[9] = {y[0], 0.5f * y[5], 0.5f * y[4], 0.5f * y[5], y[1], 0.5f * y[3],
                                             0.5f * y[4], 0.5f * y[3], y[2]};
                        float u[9];
#pragma unroll
                        for (int i = 0; i < 3; ++i)
#pragma unroll
                            for (int j = 0; j < 3; ++j)
                                u[3 * i + j] = R[3 * i] * Tn[j] + R[3 * i + 1] * Tn[3 + j] + R[3 * i + 2] * Tn[6 + j];
                        float* vb = S.V + 3 * blink[k] * n_inc;
                        V3 sum = mk(0.f, 0.f, 0.f);
#pragma unroll
                        for (int m = 1; m < 4; ++m) {
                            const float g0 = c[3 * m - 3], g1 = c[3 * m - 2], g2 = c[3 * m - 1];
                            const V3 o = mk(u[0] * g0 + u[1] * g1 + u[2] * g2, u[3] * g0 + u[4] * g1 + u[5] * g2,
                                            u[6] * g0 + u[7] * g1 + u[8] * g2);
                            st3(vb + 3 * __float_as_int(c[34 + m]), o);
                            sum = m == 1 ? o : sum + o;
                        }
                        st3(vb + 3 * __float_as_int(c[34]), -sum);
                    } else if (bkind[k] == 1) {
                        const float* c = S.dr + kDR * t;
                        const int ij = __float_as_int(c[4]), base = blink[k] * P1;
                        const float* pi = S.pr + kPR * (base + (ij & 0xffff));
                        const float* pj = S.pr + kPR * (base + (ij >> 16));
                        const int kind = __float_as_int(c[5]);
                        // a chamber row acts while its chamber is commanded (S.lk rows
                        // 2 and 3), at that chamber's pressure (rows 0 and 1)
                        const int ch = kind - kChamber0;
                        const bool on = ch < 0 || S.lk[(2 + ch) * L + blink[k]] > 0.f;
                        float* vb = S.V + 3 * blink[k] * n_inc;
                        pend[k][0] = 0.f;
                        V3 im = mk(0.f, 0.f, 0.f);
                        if (on) {
                            const float press = ch < 0 ? 0.f : S.lk[ch * L + blink[k]];
                            const V3 df = (ld3(pi) - ld3(pj)) + (ld3(pi + 3) - ld3(pj + 3));
                            // hardware reciprocal square root (1 ulp)
                            const float dd = dot(df, df), il = __builtin_amdgcn_rsqf(dd), len = dd * il;
                            const float rest = c[0] * (1.f + press * P.young_inv_pmax);
                            const float rr = (len - rest) + P.a_rigid * lam[k][0];
                            res = fmaxf(res, fabsf(rr) * P.Lref_inv);
                            const float dl = c[8] * rr;
                            pend[k][0] = dl;
                            im = (dl * il) * df;
                        }
                        // + on the first particle, - on the second
                        st3(vb + 3 * __float_as_int(c[6]), im);
                        st3(vb + 3 * __float_as_int(c[7]), -im);
                    } else if (bkind[k] == 2) {
                        const float* c = S.ar + kAR * t;
                        const int a = t;
                        const float* pi = S.pr + kPR * (blink[k] * P1 + __float_as_int(c[6]));
                        const int f = blink[k] + (a < A1 / 2 ? 0 : 1);
                        const float* fr = S.fr + kFr * f;
                        const Q4 q{fr[6], fr[7], fr[8], fr[9]};
                        const V3 u = qrot(q, ld3(c));
                        const V3 gap = (ld3(fr) - ld3(pi)) + (ld3(fr + 3) - ld3(pi + 3));
                        const V3 rr = gap + u + P.a_rigid * mk(lam[k][0], lam[k][1], lam[k][2]);
                        res = fmaxf(res, snake::amax3(rr) * P.Lref_inv);
                        // K = (w_f + w_p + a) I + [u]x I^-1 [u]x^T; row k of [u]x is -(e_k x u)
                        const bool fixedf = P.fixed0 && f == 0;
                        const float wdiag = (fixedf ? 0.f : P.frame_w) + c[3] + P.a_rigid;
                        const V3 cx = mk(0.f, -u.z, u.y), cy = mk(u.z, 0.f, -u.x), cz = mk(-u.y, u.x, 0.f);
                        const V3 z0 = mk(0.f, 0.f, 0.f);
                        const V3 ix = fixedf ? z0 : frame_inv_inertia(P, q, cx);
                        const V3 iy = fixedf ? z0 : frame_inv_inertia(P, q, cy);
                        const V3 iz = fixedf ? z0 : frame_inv_inertia(P, q, cz);
                        const V3 sol = snake::sym3_solve(wdiag + dot(cx, ix), dot(cx, iy), dot(cx, iz), wdiag + dot(cy, iy),
                                                         dot(cy, iz), wdiag + dot(cz, iz), rr);
                        const float sc = (f == 0 || f == L) ? c[4] : c[5];
                        pend[k][0] = sc * sol.x;
                        pend[k][1] = sc * sol.y;
                        pend[k][2] = sc * sol.z;
                        const V3 inc_a = mk(pend[k][0], pend[k][1], pend[k][2]);
                        float* dao = S.da + 6 * (blink[k] * A1 + a);                     // to the frame
                        st3(dao, inc_a);
                        st3(dao + 3, cross(u, inc_a));
                        st3(S.V + 3 * (blink[k] * n_inc + __float_as_int(c[7])), -inc_a);   // to the particle
                    }
                }
                // the particle's ground contact: normal, then the slip since the
                // substep start projected on the Coulomb disc of the new normal
                if (isp && P.ground) {
                    const float z = x.z + d.z;
                    res = fmaxf(res, (lc.x > 0.f ? fabsf(z) : fmaxf(-z, 0.f)) * P.Lref_inv);
                    const float ln = fmaxf(0.f, lc.x + cscale * (-pmass * z));
                    float tx = lc.y + cscale * (-pmass * d.x), ty = lc.z + cscale * (-pmass * d.y);
                    const float cap = mu * ln, n2 = tx * tx + ty * ty;
                    if (!(ln > 0.f)) {
                        tx = ty = 0.f;
                    } else if (n2 > cap * cap) {
                        // hardware reciprocal square root (1 ulp)
                        const float f = cap * __builtin_amdgcn_rsqf(n2);
                        tx *= f;
                        ty *= f;
                    }
                    dlc = mk(ln - lc.x, tx - lc.y, ty - lc.z);
                }
                res = (res == res) ? res : INFINITY;
                res = wave_max(res);
                if ((tid & 63) == 0) S.red[tid >> 6] = res;
                __syncthreads();
                r = 0.f;
#pragma unroll
                for (int w = 0; w < kWaves; ++w) r = fmaxf(r, S.red[w]);
                const bool bad = !(r < INFINITY);
                const bool stop = bad || (P.tol_mode ? (r <= P.tol || k_it >= P.iters) : (k_it >= P.iters));
                if (stop) {
                    if (bad)
                        status |= LINK_STATUS_NONFINITE;
                    else if (P.tol_mode && r > P.tol)
                        status |= LINK_STATUS_NOT_CONVERGED;
                    break;
                }
                // ---- apply: multipliers, then every body's gather in its fixed order
#pragma unroll
                for (int k = 0; k < kSlots; ++k) {
                    if (bkind[k] == 0) {
#pragma unroll
                        for (int q = 0; q < 6; ++q) lam[k][q] += pend[k][q];
                    } else {
#pragma unroll
                        for (int q = 0; q < 3; ++q) lam[k][q] += pend[k][q];
                    }
                }
                // particles: every lane of a group sums its range of the
                // particle's slots in list order (four read ahead), the group
                // adds the partial sums pairwise, the first lane applies
                V3 fsum = mk(0.f, 0.f, 0.f);
                if (isg) {
                    const float* vb = S.V + 3 * pl * n_inc;
                    int e = e0;
                    for (; e + 4 <= e1; e += 4) {
                        const V3 v0 = ld3(vb + 3 * e), v1 = ld3(vb + 3 * e + 3);
                        const V3 v2 = ld3(vb + 3 * e + 6), v3 = ld3(vb + 3 * e + 9);
                        fsum = fsum + v0;
                        fsum = fsum + v1;
                        fsum = fsum + v2;
                        fsum = fsum + v3;
                    }
                    if (e < e1) {
                        // the last one to three entries, read together
                        const V3 v0 = ld3(vb + 3 * e);
                        const V3 v1 = ld3(vb + 3 * min(e + 1, e1 - 1)), v2 = ld3(vb + 3 * min(e + 2, e1 - 1));
                        fsum = fsum + v0;
                        if (e + 1 < e1) fsum = fsum + v1;
                        if (e + 2 < e1) fsum = fsum + v2;
                    }
                }
                for (int off = 1; off < P.gmax; off <<= 1) {
                    const V3 o = lane_xor(fsum, off);
                    if (off < gsize) fsum = fsum + o;
                }
                if (isp) {
                    if (P.ground) {
                        lc = lc + dlc;
                        fsum = fsum + mk(dlc.y, dlc.z, dlc.x);
                    }
                    d = d + wp * fsum;
                    st3(my + 3, d);
                }
                // frames (the last wave): lanes 0-3 of a frame's group sum
                // quarters of link f-1's last section's attachments, lanes
                // 4-7 quarters of link f's first section's, in list order
                if (fj >= 0) {
                    V3 F = mk(0.f, 0.f, 0.f), tq = F;
                    const int l = fi - 1 + (fsub >> 2);
                    if (isfg && !ffix && l >= 0 && l < L) {
                        const int a0 = fsub < 4 ? A1 / 2 : 0, a1 = fsub < 4 ? A1 : A1 / 2;
                        const int ch = (a1 - a0 + 3) >> 2;
                        const int lo = min(a1, a0 + (fsub & 3) * ch), hi = min(a1, lo + ch);
                        int o = 6 * (l * A1 + lo);
                        int a = lo;
                        for (; a + 3 <= hi; a += 3, o += 18) {
                            const V3 d0 = ld3(S.da + o), t0 = ld3(S.da + o + 3);
                            const V3 d1 = ld3(S.da + o + 6), t1 = ld3(S.da + o + 9);
                            const V3 d2 = ld3(S.da + o + 12), t2 = ld3(S.da + o + 15);
                            F = F + d0, tq = tq + t0;
                            F = F + d1, tq = tq + t1;
                            F = F + d2, tq = tq + t2;
                        }
                        for (; a < hi; ++a, o += 6) {
                            F = F + ld3(S.da + o);
                            tq = tq + ld3(S.da + o + 3);
                        }
                    }
#pragma unroll
                    for (int off = 1; off < 8; off <<= 1) {
                        F = F + lane_xor(F, off);
                        tq = tq + lane_xor(tq, off);
                    }
                    if (isf && !ffix) {
                        float* f = S.fr + kFr * fi;
                        const Q4 q{f[6], f[7], f[8], f[9]};
                        const V3 th = frame_inv_inertia(P, q, tq);
                        const Q4 qn = qturn(q, th);
                        f[3] += P.frame_w * F.x, f[4] += P.frame_w * F.y, f[5] += P.frame_w * F.z;
                        f[6] = qn.w, f[7] = qn.x, f[8] = qn.y, f[9] = qn.z;
                    }
                }
                __syncthreads();
                ++k_it;
            }
            itstep += k_it;
            rstep = fmaxf(rstep, r);
            // velocities of the implicit step
            if (isp) {
                x = x + d;
                v = P.inv_h * d;
            }
            if (isf && !ffix) {
                float* f = S.fr + kFr * fi;
                const V3 fd = mk(f[3], f[4], f[5]);
                f[0] += fd.x, f[1] += fd.y, f[2] += fd.z;
                f[10] = P.inv_h * fd.x, f[11] = P.inv_h * fd.y, f[12] = P.inv_h * fd.z;
                const Q4 dq = qmul(Q4{f[6], f[7], f[8], f[9]}, qconj(Q4{f[16], f[17], f[18], f[19]}));
                const float sg = dq.w >= 0.f ? 2.f * P.inv_h : -2.f * P.inv_h;
                f[13] = sg * dq.x, f[14] = sg * dq.y, f[15] = sg * dq.z;
            }
            __syncthreads();
        }
        itsum += itstep;
    }

    if (isp) {
        P.x[gp] = x.x, P.x[P.NP + gp] = x.y, P.x[2 * P.NP + gp] = x.z;
        P.v[gp] = v.x, P.v[P.NP + gp] = v.y, P.v[2 * P.NP + gp] = v.z;
        P.lam_c[gp] = lc.x, P.lam_c[P.NP + gp] = lc.y, P.lam_c[2 * P.NP + gp] = lc.z;
    }
    if (isf) {
        const float* f = S.fr + kFr * fi;
        P.fx[gf] = f[0], P.fx[P.NF + gf] = f[1], P.fx[2 * P.NF + gf] = f[2];
        P.fq[gf] = f[6], P.fq[P.NF + gf] = f[7], P.fq[2 * P.NF + gf] = f[8], P.fq[3 * P.NF + gf] = f[9];
        P.fv[gf] = f[10], P.fv[P.NF + gf] = f[11], P.fv[2 * P.NF + gf] = f[12];
        P.fw[gf] = f[13], P.fw[P.NF + gf] = f[14], P.fw[2 * P.NF + gf] = f[15];
    }
    if (isl) {
        P.p[gl] = S.lk[tid];
        P.p[P.NL + gl] = S.lk[L + tid];
    }
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
        if (bkind[k] == 0) {
            const int64_t b = (int64_t)s * T + blink[k] * Tm + bidx[k];
#pragma unroll
            for (int q = 0; q < 6; ++q) P.lam_tet[q * P.NT + b] = lam[k][q];
        } else if (bkind[k] == 1) {
            P.lam_dist[(int64_t)s * D + blink[k] * D1 + bidx[k]] = lam[k][0];
        } else if (bkind[k] == 2) {
            const int64_t b = (int64_t)s * A + blink[k] * A1 + bidx[k];
#pragma unroll
            for (int q = 0; q < 3; ++q) P.lam_att[q * P.NA + b] = lam[k][q];
        }
    }
    if (tid == 0) {
        P.residual[s] = rstep;
        P.iters_out[s] = itstep;
        P.status[s] = status;
        P.iters_total[s] = P.iters_total[s] + itsum;
    }
}

}  // namespace lk

// ------------------------------------------------------------------ setup kernels (FP64)

namespace lk {

struct Setup {
    int P1, Tm;
    double young, poisson, density, h2, relax;
    const double* X;          // [P1][3]
    const int* tets;          // [Tm][4]
    const int* deg;           // [P1]
    double* mass;             // [P1] out
    float *part_w, *part_m;   // [P1] out
    float *tet_g, *tet_ldl, *tet_alpha, *tet_scale;  // out
};

__device__ double tet_rest(const double* X, const int* v, double* Di)
{
    double Dm[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) Dm[3 * r + k] = X[3 * v[k + 1] + r] - X[3 * v[0] + r];
    const double c00 = Dm[4] * Dm[8] - Dm[5] * Dm[7], c01 = Dm[5] * Dm[6] - Dm[3] * Dm[8],
                 c02 = Dm[3] * Dm[7] - Dm[4] * Dm[6];
    const double det = Dm[0] * c00 + Dm[1] * c01 + Dm[2] * c02;
    if (Di) {
        Di[0] = c00 / det, Di[3] = c01 / det, Di[6] = c02 / det;
        Di[1] = (Dm[2] * Dm[7] - Dm[1] * Dm[8]) / det, Di[4] = (Dm[0] * Dm[8] - Dm[2] * Dm[6]) / det,
        Di[7] = (Dm[1] * Dm[6] - Dm[0] * Dm[7]) / det;
        Di[2] = (Dm[1] * Dm[5] - Dm[2] * Dm[4]) / det, Di[5] = (Dm[2] * Dm[3] - Dm[0] * Dm[5]) / det,
        Di[8] = (Dm[0] * Dm[4] - Dm[1] * Dm[3]) / det;
    }
    return fabs(det) / 6.0;
}

// lumped masses: each particle a quarter of every element it belongs to,
// summed in element order
__global__ void k_link_mass(Setup S)
{
    for (int p = threadIdx.x; p < S.P1; p += blockDim.x) {
        double m = 0.0;
        for (int t = 0; t < S.Tm; ++t) {
            const int* v = S.tets + 4 * t;
            if (v[0] == p || v[1] == p || v[2] == p || v[3] == p) m += 0.25 * S.density * tet_rest(S.X, v, nullptr);
        }
        S.mass[p] = m;
        S.part_w[p] = (float)(1.0 / m);
        S.part_m[p] = (float)m;
    }
}

// per element: g_m (gradients of the barycentric coordinates), the
// compliance E/h^2 and the LDL^T factors of K + E/h^2, K = J W J^T, which
// depends on the g_m and the inverse masses only (the rotation of the
// Jacobian cancels in J W J^T)
__global__ void k_link_tets(Setup S)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= S.Tm) return;
    const int* v = S.tets + 4 * t;
    double Di[9];
    const double V = tet_rest(S.X, v, Di);
    double g[4][3];
    for (int c = 0; c < 3; ++c) {
        g[1][c] = Di[c], g[2][c] = Di[3 + c], g[3][c] = Di[6 + c];
        g[0][c] = -(g[1][c] + g[2][c] + g[3][c]);
    }
    double G[3][3] = {};
    for (int m = 0; m < 4; ++m) {
        const double w = 1.0 / S.mass[v[m]];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) G[i][j] += w * g[m][i] * g[m][j];
    }
    const int va[6] = {0, 1, 2, 1, 0, 0}, vb[6] = {0, 1, 2, 2, 2, 1};
    double K[6][6];
    for (int p = 0; p < 6; ++p)
        for (int q = 0; q < 6; ++q) {
            const int a = va[p], b = vb[p], c = va[q], e = vb[q];
            K[p][q] = 0.25 * ((a == c ? G[b][e] : 0.0) + (a == e ? G[b][c] : 0.0) + (b == c ? G[a][e] : 0.0) +
                              (b == e ? G[a][c] : 0.0));
        }
    const double s = 1.0 / (V * S.young * S.h2);
    const double ad = s, ao = -S.poisson * s, as = (1.0 + S.poisson) * s;
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) K[p][q] += p == q ? ad : ao;
    for (int p = 3; p < 6; ++p) K[p][p] += as;
    // K = L D L^T
    double Lm[6][6] = {}, Dd[6];
    for (int j = 0; j < 6; ++j) {
        double dj = K[j][j];
        for (int k = 0; k < j; ++k) dj -= Lm[j][k] * Lm[j][k] * Dd[k];
        Dd[j] = dj;
        for (int i = j + 1; i < 6; ++i) {
            double a = K[i][j];
            for (int k = 0; k < j; ++k) a -= Lm[i][k] * Lm[j][k] * Dd[k];
            Lm[i][j] = a / dj;
        }
    }
    int li = 0;
    for (int q = 0; q < 6; ++q)
        for (int c = 0; c < q; ++c) S.tet_ldl[(li++) * S.Tm + t] = (float)Lm[q][c];
    for (int q = 0; q < 6; ++q) S.tet_ldl[(15 + q) * S.Tm + t] = (float)(1.0 / Dd[q]);
    for (int m = 0; m < 4; ++m)
        for (int c = 0; c < 3; ++c) S.tet_g[(3 * m + c) * S.Tm + t] = (float)g[m][c];
    S.tet_alpha[t] = (float)ad;
    S.tet_alpha[S.Tm + t] = (float)ao;
    S.tet_alpha[2 * S.Tm + t] = (float)as;
    int dm = 0;
    for (int m = 0; m < 4; ++m) dm = S.deg[v[m]] > dm ? S.deg[v[m]] : dm;
    S.tet_scale[t] = (float)(S.relax / dm);
}

struct Init {
    int n_snakes, L, P1;
    double link_length, radius;
    const double* X;
    float *x, *v, *lam_c, *fx, *fq, *fv, *fw, *p, *cmd, *lam_tet, *lam_dist, *lam_att, *residual;
    int *iters, *status, *iters_total;
    int64_t NP, NF, NL, NT, ND, NA;
};

// every snake straight along +x at rest, zero pressures, commands, multipliers
__global__ void k_link_init(Init I)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < I.NP) {
        const int64_t l = i / I.P1;
        const int k = (int)(i - l * I.P1);
        const int lk = (int)(l % I.L);
        I.x[i] = (float)(I.X[3 * k] + lk * I.link_length);
        I.x[I.NP + i] = (float)I.X[3 * k + 1];
        I.x[2 * I.NP + i] = (float)(I.X[3 * k + 2] + I.radius);
        for (int c = 0; c < 3; ++c) I.v[c * I.NP + i] = I.lam_c[c * I.NP + i] = 0.f;
    }
    if (i < I.NF) {
        const int f = (int)(i % (I.L + 1));
        I.fx[i] = (float)(f * I.link_length);
        I.fx[I.NF + i] = 0.f;
        I.fx[2 * I.NF + i] = (float)I.radius;
        I.fq[i] = 1.f;
        for (int c = 1; c < 4; ++c) I.fq[c * I.NF + i] = 0.f;
        for (int c = 0; c < 3; ++c) I.fv[c * I.NF + i] = I.fw[c * I.NF + i] = 0.f;
    }
    if (i < I.NL) I.p[i] = I.p[I.NL + i] = I.cmd[i] = 0.f;
    if (i < I.NT)
        for (int c = 0; c < 6; ++c) I.lam_tet[c * I.NT + i] = 0.f;
    if (i < I.ND) I.lam_dist[i] = 0.f;
    if (i < I.NA)
        for (int c = 0; c < 3; ++c) I.lam_att[c * I.NA + i] = 0.f;
    if (i < I.n_snakes) {
        I.residual[i] = 0.f;
        I.iters[i] = I.status[i] = I.iters_total[i] = 0;
    }
}

__global__ void k_link_set_cmd(float* cmd, const float* src, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const float a = src[i];
        cmd[i] = a == a ? fminf(fmaxf(a, -1.f), 1.f) : 0.f;
    }
}

}  // namespace lk

// ------------------------------------------------------------------ host runtime

namespace {

thread_local std::string g_lerr;

int lfail(int code, const std::string& msg)
{
    g_lerr = msg;
    return code;
}

int lhip(hipError_t e, const char* what) { return lfail(LINK_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)); }

struct Topo {
    int P1 = 0, Tm = 0, D1 = 0, A1 = 0;
    std::vector<int> dist_ij, dist_kind, dist_i, dist_j, att_p, deg_p, deg_f, inc_off, inc, tet_v, tets;
    std::vector<float> dist_c, att_c;
    std::vector<int> gplan;   // [2][1024] the kernel's per-lane particle groups
    int gmax = 1;
};

int axial_kind(int ring, int slot)
{
    if (slot == 0) return lk::kCentre;
    const int k = slot - 1, q = ring / 4;
    if (k == q || k == 3 * q) return lk::kCentre;
    return (k < q || k > 3 * q) ? lk::kChamber0 : lk::kChamber1;
}

struct Sz {
    int64_t n = 0, L = 0, P1 = 0, Tm = 0, D1 = 0, A1 = 0;
    int64_t NP = 0, NF = 0, NL = 0, NT = 0, ND = 0, NA = 0;
    size_t lds = 0;
};

bool fpos(double v) { return std::isfinite(v) && v > 0.0; }

int validate(const link_desc_t* d, Sz* z)
{
    if (!d) return lfail(LINK_EINVAL, "descriptor is NULL");
    if (d->n_snakes < 1) return lfail(LINK_EINVAL, "n_snakes must be >= 1");
    if (d->n_links < 1 || d->n_links > lk::kMaxLinks) return lfail(LINK_EINVAL, "n_links must be in [1, 4]");
    if (d->sections < 3) return lfail(LINK_EINVAL, "sections must be >= 3");
    if (d->ring < 4 || d->ring > 28 || d->ring % 4) return lfail(LINK_EINVAL, "ring must be a multiple of 4 in [4, 28]");
    if (d->n_tets < 1) return lfail(LINK_EINVAL, "n_tets must be >= 1");
    if (!d->X || !d->tets || !d->mu) return lfail(LINK_EINVAL, "X, tets or mu is NULL");
    if (!fpos(d->link_length) || !fpos(d->radius) || !fpos(d->young) || !fpos(d->density) ||
        !(d->poisson >= 0.0 && d->poisson < 0.5) || !std::isfinite(d->p_max) || d->p_max < 0.0 ||
        !fpos(d->frame_mass) || !fpos(d->frame_length))
        return lfail(LINK_EINVAL, "material, geometry or frame constants out of range");
    if (!std::isfinite(d->gravity)) return lfail(LINK_EINVAL, "gravity must be finite");
    if (!fpos(d->dt) || d->substeps < 1) return lfail(LINK_EINVAL, "dt must be > 0 and substeps >= 1");
    if (d->iters < 0 || d->iters > 1000000) return lfail(LINK_EINVAL, "iters must be in [0, 1e6]");
    if (!std::isfinite(d->tol)) return lfail(LINK_EINVAL, "tol must be finite");
    if (!(d->relax > 0.0 && d->relax <= 1.0)) return lfail(LINK_EINVAL, "relax must be in (0, 1]");
    if (!fpos(d->tau_inflate) || !fpos(d->tau_deflate)) return lfail(LINK_EINVAL, "tau_inflate and tau_deflate must be > 0");
    if (!std::isfinite(d->rigid_compliance) || d->rigid_compliance < 0.0)
        return lfail(LINK_EINVAL, "rigid_compliance must be finite and >= 0");
    if (d->flags & ~(LINK_FLAG_FIXED_FRAME0 | LINK_FLAG_NO_GROUND)) return lfail(LINK_EINVAL, "unknown flag bits");
    for (int s = 0; s < d->n_snakes; ++s)
        if (!std::isfinite(d->mu[s]) || d->mu[s] < 0.0) return lfail(LINK_EINVAL, "mu must be finite and >= 0");
    z->n = d->n_snakes;
    z->L = d->n_links;
    z->P1 = (int64_t)d->sections * (d->ring + 1);
    if (z->P1 > 255) return lfail(LINK_EINVAL, "a link mesh holds at most 255 particles");
    z->Tm = d->n_tets;
    for (int64_t k = 0; k < 4 * z->Tm; ++k)
        if (d->tets[k] < 0 || d->tets[k] >= z->P1) return lfail(LINK_EINVAL, "tetrahedron index out of range");
    z->D1 = (int64_t)(d->sections - 1) * (d->ring + 1) + (int64_t)(d->sections - 2) * d->ring;
    z->A1 = 2 * (d->ring + 1);
    const int64_t P = z->L * z->P1, NB = z->L * (z->Tm + z->D1 + z->A1);
    if (P > lk::kThreads) return lfail(LINK_EINVAL, "a snake may hold at most 1024 particles");
    if (NB > (int64_t)lk::kThreads * lk::kSlots) return lfail(LINK_EINVAL, "a snake may hold at most 2048 blocks");
    z->lds = sizeof(float) * (size_t)lk::lds_words((int)z->L, (int)z->P1, (int)z->Tm, (int)z->D1, (int)z->A1,
                                                   (int)(4 * z->Tm + 2 * z->D1 + z->A1));
    if (z->lds > (size_t)lk::kLdsLimit)
        return lfail(LINK_EINVAL, "a snake needs " + std::to_string(z->lds) + " bytes of LDS (limit 163840)");
    if ((int64_t)d->n_snakes * P > ((int64_t)1 << 28)) return lfail(LINK_EINVAL, "too many particles (limit 2^28)");
    z->NP = z->n * P;
    z->NF = z->n * (z->L + 1);
    z->NL = z->n * z->L;
    z->NT = z->n * z->L * z->Tm;
    z->ND = z->n * z->L * z->D1;
    z->NA = z->n * z->L * z->A1;
    return LINK_OK;
}

// constraint lists of one link, degrees and the particles' incidence lists
// The particles' lane groups of the link kernel.  Particle p's incidence
// list of c entries is cut into g equal ranges, one per lane of an aligned
// group of g lanes (g a power of two up to 8, so a group lies in one wave),
// g the least that keeps every range within K entries, K the least for
// which the groups fit below the frames' wave (when the particles need
// more lanes, one lane each over the whole workgroup).
void gather_plan(int L, Topo* t)
{
    const int P = L * t->P1, avail = P <= lk::kThreads - 64 ? lk::kThreads - 64 : lk::kThreads;
    auto count = [&](int p) { return t->inc_off[p % t->P1 + 1] - t->inc_off[p % t->P1]; };
    auto group = [](int c, int K) {
        int g = 1;
        while (g < 8 && g * K < c) g <<= 1;
        return g;
    };
    auto lanes = [&](int K) {
        int cur = 0;
        for (int p = 0; p < P; ++p) {
            const int g = group(count(p), K);
            cur = ((cur + g - 1) & ~(g - 1)) + g;
        }
        return cur;
    };
    int cmax = 1;
    for (int p = 0; p < t->P1; ++p) cmax = std::max(cmax, count(p));
    int K = 1;
    while (K < cmax && lanes(K) > avail) ++K;
    t->gplan.assign(2 * lk::kThreads, 0);
    for (int i = 0; i < lk::kThreads; ++i) t->gplan[i] = -1;
    t->gmax = 1;
    int cur = 0;
    for (int p = 0; p < P; ++p) {
        const int c = count(p), g = group(c, K), ch = (c + g - 1) / g, first = t->inc_off[p % t->P1];
        const int lg = g == 1 ? 0 : g == 2 ? 1 : g == 4 ? 2 : 3;
        cur = (cur + g - 1) & ~(g - 1);
        for (int j = 0; j < g; ++j) {
            t->gplan[cur + j] = p | lg << 16;
            t->gplan[lk::kThreads + cur + j] = (first + std::min(c, j * ch)) | (first + std::min(c, (j + 1) * ch)) << 16;
        }
        cur += g;
        t->gmax = std::max(t->gmax, g);
    }
}

void topology(const link_desc_t* d, const Sz& z, Topo* t)
{
    const int n = d->ring + 1, S = d->sections;
    const bool ground = !(d->flags & LINK_FLAG_NO_GROUND);
    t->P1 = (int)z.P1, t->Tm = (int)z.Tm, t->D1 = (int)z.D1, t->A1 = (int)z.A1;
    for (int g = 0; g + 1 < S; ++g)
        for (int s = 0; s < n; ++s) {
            t->dist_i.push_back(g * n + s);
            t->dist_j.push_back((g + 1) * n + s);
            t->dist_kind.push_back(axial_kind(d->ring, s));
        }
    for (int g = 1; g + 1 < S; ++g)
        for (int k = 0; k < d->ring; ++k) {
            t->dist_i.push_back(g * n);
            t->dist_j.push_back(g * n + 1 + k);
            t->dist_kind.push_back(lk::kRadial);
        }
    for (int s = 0; s < n; ++s) t->att_p.push_back(s);
    for (int s = 0; s < n; ++s) t->att_p.push_back((S - 1) * n + s);
    t->tets.assign(d->tets, d->tets + 4 * z.Tm);
    t->deg_p.assign(t->P1, ground ? 1 : 0);
    for (int k = 0; k < 4 * t->Tm; ++k) t->deg_p[t->tets[k]] += 1;
    for (int e = 0; e < t->D1; ++e) {
        t->deg_p[t->dist_i[e]] += 1;
        t->deg_p[t->dist_j[e]] += 1;
    }
    for (int a = 0; a < t->A1; ++a) t->deg_p[t->att_p[a]] += 1;
    const int L = (int)z.L;
    for (int f = 0; f <= L; ++f) t->deg_f.push_back((f == 0 || f == L) ? n : 2 * n);
    // incidence lists in the gather order: elements, distance rows, attachment
    std::vector<std::vector<int>> inc(t->P1);
    for (int e = 0; e < t->Tm; ++e)
        for (int m = 0; m < 4; ++m) inc[t->tets[4 * e + m]].push_back(lk::kIncTet << 28 | e << 2 | m);
    for (int e = 0; e < t->D1; ++e) {
        inc[t->dist_i[e]].push_back(lk::kIncDist << 28 | e << 2 | 0);
        inc[t->dist_j[e]].push_back(lk::kIncDist << 28 | e << 2 | 1);
    }
    for (int a = 0; a < t->A1; ++a) inc[t->att_p[a]].push_back(lk::kIncAtt << 28 | a << 2);
    t->inc_off.push_back(0);
    for (int p = 0; p < t->P1; ++p) {
        t->inc.insert(t->inc.end(), inc[p].begin(), inc[p].end());
        t->inc_off.push_back((int)t->inc.size());
    }
    for (int e = 0; e < t->Tm; ++e) {
        const int* v = d->tets + 4 * e;
        t->tet_v.push_back(v[0] | v[1] << 8 | v[2] << 16 | v[3] << 24);
    }
    for (int e = 0; e < t->D1; ++e) t->dist_ij.push_back(t->dist_i[e] | t->dist_j[e] << 16);
    gather_plan(L, t);
}

struct Carve {
    char* base;
    size_t pos = 0;
    template <class T>
    T* take(int64_t count)
    {
        pos = (pos + 255) & ~(size_t)255;
        T* p = base ? reinterpret_cast<T*>(base + pos) : nullptr;
        pos += (size_t)(count > 0 ? count : 1) * sizeof(T);
        return p;
    }
};

struct Arrays {
    // state (contiguous, first)
    float *x, *v, *lam_c, *fx, *fq, *fv, *fw, *p, *cmd, *lam_tet, *lam_dist, *lam_att, *residual;
    int *iters, *status, *iters_total;
    // constants and setup data
    float* mu;
    int *tet_v, *dist_ij, *dist_kind, *att_p, *part_deg, *gplan, *inc, *tets;
    float *tet_g, *tet_ldl, *tet_alpha, *tet_scale, *dist_c, *att_c, *part_w, *part_m;
    double *X, *mass;
};

size_t carve(const Sz& z, int64_t n_inc, char* base, Arrays* a)
{
    Carve c{base};
    a->x = c.take<float>(3 * z.NP);
    a->v = c.take<float>(3 * z.NP);
    a->lam_c = c.take<float>(3 * z.NP);
    a->fx = c.take<float>(3 * z.NF);
    a->fq = c.take<float>(4 * z.NF);
    a->fv = c.take<float>(3 * z.NF);
    a->fw = c.take<float>(3 * z.NF);
    a->p = c.take<float>(2 * z.NL);
    a->cmd = c.take<float>(z.NL);
    a->lam_tet = c.take<float>(6 * z.NT);
    a->lam_dist = c.take<float>(z.ND);
    a->lam_att = c.take<float>(3 * z.NA);
    a->residual = c.take<float>(z.n);
    a->iters = c.take<int>(z.n);
    a->status = c.take<int>(z.n);
    a->iters_total = c.take<int>(z.n);
    a->mu = c.take<float>(z.n);
    a->tet_v = c.take<int>(z.Tm);
    a->dist_ij = c.take<int>(z.D1);
    a->dist_kind = c.take<int>(z.D1);
    a->att_p = c.take<int>(z.A1);
    a->part_deg = c.take<int>(z.P1);
    a->gplan = c.take<int>(2 * lk::kThreads);
    a->inc = c.take<int>(n_inc);
    a->tets = c.take<int>(4 * z.Tm);
    a->tet_g = c.take<float>(12 * z.Tm);
    a->tet_ldl = c.take<float>(21 * z.Tm);
    a->tet_alpha = c.take<float>(3 * z.Tm);
    a->tet_scale = c.take<float>(z.Tm);
    a->dist_c = c.take<float>(4 * z.D1);
    a->att_c = c.take<float>(5 * z.A1);
    a->part_w = c.take<float>(z.P1);
    a->part_m = c.take<float>(z.P1);
    a->X = c.take<double>(3 * z.P1);
    a->mass = c.take<double>(z.P1);
    return c.pos;
}

int64_t incidence_count(const link_desc_t* d, const Sz& z)
{
    (void)d;
    return 4 * z.Tm + 2 * z.D1 + z.A1;
}

}  // namespace

struct link {
    Sz z;
    Topo topo;
    Arrays a;
    lk::Params kp;
    hipStream_t stream;
};

extern "C" {

int link_workspace_bytes(const link_desc_t* d, size_t* bytes)
{
    Sz z;
    if (int rc = validate(d, &z)) return rc;
    if (!bytes) return lfail(LINK_EINVAL, "bytes is NULL");
    Arrays a;
    *bytes = carve(z, incidence_count(d, z), nullptr, &a);
    return LINK_OK;
}

int link_create(const link_desc_t* d, void* workspace, size_t bytes, void* hip_stream, link_t** out)
{
    if (!out) return lfail(LINK_EINVAL, "out is NULL");
    *out = nullptr;
    Sz z;
    if (int rc = validate(d, &z)) return rc;
    if (!workspace) return lfail(LINK_EINVAL, "workspace is NULL");
    Arrays a;
    const size_t need = carve(z, incidence_count(d, z), nullptr, &a);
    if (bytes < need) return lfail(LINK_ENOMEM, "workspace holds " + std::to_string(bytes) + " bytes, need " +
                                                    std::to_string(need));
    link* s = new link();
    s->z = z;
    s->stream = (hipStream_t)hip_stream;
    carve(z, incidence_count(d, z), (char*)workspace, &s->a);
    topology(d, z, &s->topo);
    const Topo& t = s->topo;
    const Arrays& A = s->a;
    const double h = d->dt / d->substeps;
    // distance and attachment constants (host, from the rest mesh in double)
    std::vector<float> dist_c(4 * t.D1), att_c(5 * t.A1), mu(z.n);
    std::vector<double> mass(t.P1, 0.0);
    for (int64_t i = 0; i < z.n; ++i) mu[i] = (float)d->mu[i];
    hipError_t e = hipSuccess;
    auto up = [&](void* dst, const void* src, size_t n) {
        if (e == hipSuccess) e = hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, s->stream);
    };
    up(A.X, d->X, sizeof(double) * 3 * t.P1);
    up(A.tets, t.tets.data(), sizeof(int) * t.tets.size());
    up(A.part_deg, t.deg_p.data(), sizeof(int) * t.P1);
    up(A.mu, mu.data(), sizeof(float) * z.n);
    up(A.tet_v, t.tet_v.data(), sizeof(int) * t.Tm);
    up(A.dist_ij, t.dist_ij.data(), sizeof(int) * t.D1);
    up(A.dist_kind, t.dist_kind.data(), sizeof(int) * t.D1);
    up(A.att_p, t.att_p.data(), sizeof(int) * t.A1);
    up(A.gplan, t.gplan.data(), sizeof(int) * t.gplan.size());
    up(A.inc, t.inc.data(), sizeof(int) * t.inc.size());
    lk::Setup su{};
    su.P1 = t.P1, su.Tm = t.Tm;
    su.young = d->young, su.poisson = d->poisson, su.density = d->density, su.h2 = h * h, su.relax = d->relax;
    su.X = A.X, su.tets = A.tets, su.deg = A.part_deg, su.mass = A.mass, su.part_w = A.part_w, su.part_m = A.part_m;
    su.tet_g = A.tet_g, su.tet_ldl = A.tet_ldl, su.tet_alpha = A.tet_alpha, su.tet_scale = A.tet_scale;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(lk::k_link_mass, dim3(1), dim3(256), 0, s->stream, su);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(lk::k_link_tets, dim3((t.Tm + 63) / 64), dim3(64), 0, s->stream, su);
        e = hipGetLastError();
    }
    // the distance and attachment constants need the masses
    if (e == hipSuccess) e = hipMemcpyAsync(mass.data(), A.mass, sizeof(double) * t.P1, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        delete s;
        return lhip(e, "link setup");
    }
    for (int k = 0; k < t.D1; ++k) {
        const int i = t.dist_i[k], j = t.dist_j[k];
        double r2 = 0.0;
        for (int c = 0; c < 3; ++c) r2 += (d->X[3 * i + c] - d->X[3 * j + c]) * (d->X[3 * i + c] - d->X[3 * j + c]);
        dist_c[k] = (float)std::sqrt(r2);
        dist_c[t.D1 + k] = (float)(1.0 / mass[i]);
        dist_c[2 * t.D1 + k] = (float)(1.0 / mass[j]);
        dist_c[3 * t.D1 + k] = (float)(d->relax / std::max(t.deg_p[i], t.deg_p[j]));
    }
    const int n = d->ring + 1;
    for (int k = 0; k < t.A1; ++k) {
        const int p = t.att_p[k];
        // rest position relative to the frame: section 0 sits at the link's
        // start, the last section at its end (frame at x = 0 or link_length)
        const double fxr = k < n ? 0.0 : d->link_length;
        att_c[k] = (float)(d->X[3 * p] - fxr);
        att_c[t.A1 + k] = (float)d->X[3 * p + 1];
        att_c[2 * t.A1 + k] = (float)d->X[3 * p + 2];
        att_c[3 * t.A1 + k] = (float)(1.0 / mass[p]);
        att_c[4 * t.A1 + k] = (float)t.deg_p[p];
    }
    up(A.dist_c, dist_c.data(), sizeof(float) * dist_c.size());
    up(A.att_c, att_c.data(), sizeof(float) * att_c.size());
    lk::Init in{};
    in.n_snakes = (int)z.n, in.L = (int)z.L, in.P1 = t.P1;
    in.link_length = d->link_length, in.radius = d->radius, in.X = A.X;
    in.x = A.x, in.v = A.v, in.lam_c = A.lam_c, in.fx = A.fx, in.fq = A.fq, in.fv = A.fv, in.fw = A.fw;
    in.p = A.p, in.cmd = A.cmd, in.lam_tet = A.lam_tet, in.lam_dist = A.lam_dist, in.lam_att = A.lam_att;
    in.residual = A.residual, in.iters = A.iters, in.status = A.status, in.iters_total = A.iters_total;
    in.NP = z.NP, in.NF = z.NF, in.NL = z.NL, in.NT = z.NT, in.ND = z.ND, in.NA = z.NA;
    const int64_t most = std::max({z.NP, z.NF, z.NL, z.NT, z.ND, z.NA, z.n});
    if (e == hipSuccess) {
        hipLaunchKernelGGL(lk::k_link_init, dim3((unsigned)((most + 255) / 256)), dim3(256), 0, s->stream, in);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        delete s;
        return lhip(e, "link create");
    }
    if (z.lds > 65536) {   // dynamic LDS past 64 KB has to be requested
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(lk::k_link), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)z.lds);
        if (e != hipSuccess) {
            delete s;
            return lhip(e, "link LDS request");
        }
    }
    lk::Params& P = s->kp;
    P = lk::Params{};
    P.n_snakes = (int)z.n, P.L = (int)z.L, P.P1 = t.P1, P.Tm = t.Tm, P.D1 = t.D1, P.A1 = t.A1, P.ring = d->ring;
    P.P = (int)(z.L * t.P1), P.F = (int)(z.L + 1), P.NB = (int)(z.L * (t.Tm + t.D1 + t.A1));
    P.ground = (d->flags & LINK_FLAG_NO_GROUND) ? 0 : 1;
    P.fixed0 = (d->flags & LINK_FLAG_FIXED_FRAME0) ? 1 : 0;
    P.tol_mode = d->tol > 0.0 ? 1 : 0;
    P.iters = d->iters, P.substeps = d->substeps;
    P.h = (float)h, P.inv_h = (float)(1.0 / h), P.g = (float)d->gravity, P.tol = (float)d->tol;
    P.lag_in = (float)std::exp(-h / d->tau_inflate), P.lag_de = (float)std::exp(-h / d->tau_deflate);
    P.young_inv_pmax = (float)(d->p_max / d->young);
    P.frame_w = (float)(1.0 / d->frame_mass);
    P.Lref_inv = (float)((d->sections - 1) / d->link_length);
    P.a_rigid = (float)(d->rigid_compliance / (h * h));
    const double m = d->frame_mass, R = d->radius, Lf = d->frame_length;
    const double I_ax = 0.5 * m * R * R, I_pe = m * (3 * R * R + Lf * Lf) / 12.0;
    P.I_ax = (float)I_ax, P.I_pe = (float)I_pe, P.I_ax_inv = (float)(1.0 / I_ax), P.I_pe_inv = (float)(1.0 / I_pe);
    P.relax = (float)d->relax;
    P.x = A.x, P.v = A.v, P.lam_c = A.lam_c, P.fx = A.fx, P.fq = A.fq, P.fv = A.fv, P.fw = A.fw;
    P.p = A.p, P.cmd = A.cmd, P.lam_tet = A.lam_tet, P.lam_dist = A.lam_dist, P.lam_att = A.lam_att;
    P.residual = A.residual, P.iters_out = A.iters, P.status = A.status, P.iters_total = A.iters_total;
    P.mu = A.mu;
    P.NP = z.NP, P.NF = z.NF, P.NL = z.NL, P.NT = z.NT, P.ND = z.ND, P.NA = z.NA;
    P.tet_v = A.tet_v, P.tet_g = A.tet_g, P.tet_ldl = A.tet_ldl, P.tet_alpha = A.tet_alpha, P.tet_scale = A.tet_scale;
    P.dist_ij = A.dist_ij, P.dist_kind = A.dist_kind, P.dist_c = A.dist_c, P.att_p = A.att_p, P.att_c = A.att_c;
    P.part_w = A.part_w, P.part_m = A.part_m, P.part_deg = A.part_deg, P.inc = A.inc;
    P.gplan = A.gplan, P.gmax = t.gmax;
    *out = s;
    return LINK_OK;
}

int link_set_commands(link_t* s, const float* cmd, int64_t n, int mem)
{
    if (!s || !cmd) return lfail(LINK_EINVAL, "link or cmd is NULL");
    if (n != s->z.NL) return lfail(LINK_EINVAL, "expected one command per link (" + std::to_string(s->z.NL) + ")");
    hipError_t e;
    if (mem == LINK_MEM_HOST) {
        std::vector<float> c(cmd, cmd + n);
        for (float& v : c) {
            if (std::isnan(v)) return lfail(LINK_EINVAL, "command is NaN");
            v = std::min(1.f, std::max(-1.f, v));
        }
        e = hipMemcpyAsync(s->a.cmd, c.data(), sizeof(float) * n, hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    } else if (mem == LINK_MEM_DEVICE) {
        hipLaunchKernelGGL(lk::k_link_set_cmd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s->stream, s->a.cmd,
                           cmd, n);
        e = hipGetLastError();
    } else {
        return lfail(LINK_EINVAL, "unknown memory kind");
    }
    return e == hipSuccess ? LINK_OK : lhip(e, "set commands");
}

int link_step(link_t* s, int32_t n_steps)
{
    if (!s) return lfail(LINK_EINVAL, "link is NULL");
    if (n_steps < 0) return lfail(LINK_EINVAL, "n_steps must be >= 0");
    if (n_steps == 0) return LINK_OK;
    hipLaunchKernelGGL(lk::k_link, dim3((unsigned)s->z.n), dim3(lk::kThreads), s->z.lds, s->stream, s->kp, n_steps);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LINK_OK : lhip(e, "link step");
}

static int copy_fields(link_t* s, uint32_t fields, void* const* ptrs, int mem, bool read)
{
    if (!s || !ptrs) return lfail(LINK_EINVAL, "link or pointer table is NULL");
    if (mem != LINK_MEM_HOST && mem != LINK_MEM_DEVICE) return lfail(LINK_EINVAL, "unknown memory kind");
    if (fields >> LINK_F_COUNT) return lfail(LINK_EINVAL, "unknown field bits");
    const Sz& z = s->z;
    const Arrays& A = s->a;
    void* dev[LINK_F_COUNT] = {A.x, A.v, A.fx, A.fq, A.fv, A.fw, A.p, A.cmd, A.lam_tet, A.lam_dist, A.lam_att,
                               A.lam_c, A.residual, A.iters, A.status, A.iters_total};
    const int64_t cnt[LINK_F_COUNT] = {3 * z.NP, 3 * z.NP, 3 * z.NF, 4 * z.NF, 3 * z.NF, 3 * z.NF, 2 * z.NL, z.NL,
                                       6 * z.NT, z.ND, 3 * z.NA, 3 * z.NP, z.n, z.n, z.n, z.n};
    const hipMemcpyKind kind = mem == LINK_MEM_HOST ? (read ? hipMemcpyDeviceToHost : hipMemcpyHostToDevice)
                                                    : hipMemcpyDeviceToDevice;
    hipError_t e = hipSuccess;
    for (int k = 0; k < LINK_F_COUNT && e == hipSuccess; ++k) {
        if (!(fields >> k & 1u)) continue;
        if (!ptrs[k]) return lfail(LINK_EINVAL, "pointer of a selected field is NULL");
        const size_t n = sizeof(float) * (size_t)cnt[k];
        e = read ? hipMemcpyAsync(ptrs[k], dev[k], n, kind, s->stream) : hipMemcpyAsync(dev[k], ptrs[k], n, kind, s->stream);
    }
    if (e == hipSuccess && mem == LINK_MEM_HOST) e = hipStreamSynchronize(s->stream);
    return e == hipSuccess ? LINK_OK : lhip(e, read ? "read state" : "write state");
}

int link_read_state(link_t* s, uint32_t fields, void* const* dst, int mem)
{
    return copy_fields(s, fields, dst, mem, true);
}

int link_write_state(link_t* s, uint32_t fields, const void* const* src, int mem)
{
    return copy_fields(s, fields, const_cast<void* const*>(src), mem, false);
}

int link_read_index(link_t* s, int32_t which, int32_t* dst, int64_t count)
{
    if (!s || !dst) return lfail(LINK_EINVAL, "link or dst is NULL");
    const Topo& t = s->topo;
    const int L = (int)s->z.L;
    std::vector<int> out;
    switch (which) {
    case LINK_IDX_DIST_I:
    case LINK_IDX_DIST_J:
    case LINK_IDX_DIST_KIND:
        for (int l = 0; l < L; ++l)
            for (int k = 0; k < t.D1; ++k)
                out.push_back(which == LINK_IDX_DIST_KIND ? t.dist_kind[k]
                                                          : l * t.P1 + (which == LINK_IDX_DIST_I ? t.dist_i[k] : t.dist_j[k]));
        break;
    case LINK_IDX_DEG_PARTICLE:
        for (int l = 0; l < L; ++l) out.insert(out.end(), t.deg_p.begin(), t.deg_p.end());
        break;
    case LINK_IDX_DEG_FRAME:
        out = t.deg_f;
        break;
    default:
        return lfail(LINK_EINVAL, "unknown index array");
    }
    if (count != (int64_t)out.size()) return lfail(LINK_EINVAL, "count does not match the index array's length");
    std::memcpy(dst, out.data(), sizeof(int32_t) * out.size());
    return LINK_OK;
}

int link_plan_gathers(const link_desc_t* d, int32_t* out2048, int32_t* gmax)
{
    Sz z;
    if (int rc = validate(d, &z)) return rc;
    if (!out2048 || !gmax) return lfail(LINK_EINVAL, "out2048 or gmax is NULL");
    Topo t;
    topology(d, z, &t);
    std::memcpy(out2048, t.gplan.data(), sizeof(int32_t) * t.gplan.size());
    *gmax = t.gmax;
    return LINK_OK;
}

int link_sizes(const link_t* s, int64_t* out10)
{
    if (!s || !out10) return lfail(LINK_EINVAL, "link or out is NULL");
    const Sz& z = s->z;
    const int64_t v[10] = {z.n, z.NP, z.NF, z.NT, z.ND, z.NA, z.L, z.L * z.P1, z.D1 * z.L, z.A1 * z.L};
    std::memcpy(out10, v, sizeof v);
    return LINK_OK;
}

void link_destroy(link_t* s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    delete s;
}

const char* link_last_error(void) { return g_lerr.c_str(); }

}  // extern "C"
