/*
 * FP64 CPU oracle of the compliant-constraint snake solve.
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the CPU
 * baseline leg of the benchmark.  Shares no code with the GPU library.
 * Plain scalar loops, double precision, no reordering beyond what each
 * formula states, so each step can be read against the paper:
 *
 *   step      paper passage
 *   --------  -----------------------------------------------------------
 *   command   eq. snake_control (clamped sine per module)
 *   pressure  first-order lag, or eq. delta_p_i + eq. deflation
 *   rest      eq. expansion: strain linear in pressure -> rest curvature
 *             linear in the chamber pressure difference
 *   predict   section "Time-Stepping" (first-order implicit), rigid bodies
 *             as centre + quaternion (section "Rigid Bodies")
 *   blocks    compliant constraints c + E lambda = 0 (section "Simulator");
 *             stretch in the form of eq. rigid_to_particle; contact
 *             c_n >= 0 with a Coulomb cone (sections "Simulator" and
 *             "Rigid Body Joints and Contact")
 *   solve     block Jacobi on the system of eq. schur_system, each block
 *             increment scaled by relax / (number of blocks on its busiest
 *             body), applied to both lambda and the bodies
 *   finalize  velocities from the implicit step's displacement
 */
#include "snake_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* small fp64 algebra                                                   */
/* ------------------------------------------------------------------ */

static void cross3(const double* a, const double* b, double* o)
{
    double t0 = a[1] * b[2] - a[2] * b[1];
    double t1 = a[2] * b[0] - a[0] * b[2];
    double t2 = a[0] * b[1] - a[1] * b[0];
    o[0] = t0;
    o[1] = t1;
    o[2] = t2;
}

/* row-major 3x3 */
static void m3_mul(const double* A, const double* B, double* O)
{
    double T[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
            T[3 * i + j] = s;
        }
    memcpy(O, T, sizeof T);
}

static void m3_transpose(const double* A, double* O)
{
    double T[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) T[3 * j + i] = A[3 * i + j];
    memcpy(O, T, sizeof T);
}

static void m3_vec(const double* A, const double* v, double* o)
{
    double t[3];
    for (int i = 0; i < 3; ++i) t[i] = A[3 * i] * v[0] + A[3 * i + 1] * v[1] + A[3 * i + 2] * v[2];
    memcpy(o, t, sizeof t);
}

/* S such that S u = v x u */
static void skew3(const double* v, double* S)
{
    S[0] = 0.0;   S[1] = -v[2]; S[2] = v[1];
    S[3] = v[2];  S[4] = 0.0;   S[5] = -v[0];
    S[6] = -v[1]; S[7] = v[0];  S[8] = 0.0;
}

/* Hamilton product, q = (w, x, y, z) */
static void q_mul(const double* a, const double* b, double* o)
{
    double w = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    double x = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    double y = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    double z = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    o[0] = w;
    o[1] = x;
    o[2] = y;
    o[3] = z;
}

static void q_conj(const double* a, double* o)
{
    o[0] = a[0];
    o[1] = -a[1];
    o[2] = -a[2];
    o[3] = -a[3];
}

static void q_normalize(double* q)
{
    double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; ++k) q[k] /= n;
}

/* rotation matrix of a unit quaternion (body -> world) */
static void q_to_matrix(const double* q, double* R)
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* q <- normalize(q + 1/2 [0, dtheta] (x) q): a world-frame rotation vector
 * applied to a quaternion to first order, then renormalised */
static void q_apply_rotvec(double* q, const double* dth)
{
    double p[4] = {0.0, dth[0], dth[1], dth[2]};
    double t[4];
    q_mul(p, q, t);
    for (int k = 0; k < 4; ++k) q[k] += 0.5 * t[k];
    q_normalize(q);
}

/* solve A x = b for a 3x3 system, Gaussian elimination, partial pivoting */
static void solve3(const double* Ain, const double* bin, double* x)
{
    double A[9], b[3];
    memcpy(A, Ain, sizeof A);
    memcpy(b, bin, sizeof b);
    for (int c = 0; c < 3; ++c) {
        int piv = c;
        for (int r = c + 1; r < 3; ++r)
            if (fabs(A[3 * r + c]) > fabs(A[3 * piv + c])) piv = r;
        if (piv != c) {
            for (int k = 0; k < 3; ++k) {
                double t = A[3 * c + k];
                A[3 * c + k] = A[3 * piv + k];
                A[3 * piv + k] = t;
            }
            double t = b[c];
            b[c] = b[piv];
            b[piv] = t;
        }
        for (int r = c + 1; r < 3; ++r) {
            double f = A[3 * r + c] / A[3 * c + c];
            for (int k = c; k < 3; ++k) A[3 * r + k] -= f * A[3 * c + k];
            b[r] -= f * b[c];
        }
    }
    for (int r = 2; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < 3; ++k) s -= A[3 * r + k] * x[k];
        x[r] = s / A[3 * r + r];
    }
}

/* ------------------------------------------------------------------ */
/* per-snake context                                                    */
/* ------------------------------------------------------------------ */

typedef struct {
    int B, M, S, nj, ground, fixed_root, linear;
    double m, L, R, g, h;
    double Ib[3];               /* principal inertia in the body frame */
    double a_s, a_b, a_t;       /* joint compliance = per-length value * L */
    double mu, relax;
    /* wheel carriage: bodies 0..B-1 are the segments, B + 2i + k the wheels
     * of segment i; NB bodies in all */
    int wheels, NB;
    double mw, rw, dw, hw;      /* wheel mass, radius, lateral offset, drop */
    double Iwh[3];              /* wheel inertia in its frame (axle e_y) */
    const double* anchor;       /* [2B*6] per wheel: contact point at the
                                 * start of the substep (world) and its arm
                                 * in the wheel frame */
} snake_ctx;

static void make_ctx(const orc_batch* b, int s, snake_ctx* c)
{
    c->M = b->n_modules[s];
    c->S = b->segs[s];
    c->B = c->M * c->S;
    c->nj = c->B - 1;
    c->ground = (b->flags & ORC_FLAG_NO_GROUND) ? 0 : 1;
    c->fixed_root = (b->flags & ORC_FLAG_FIXED_ROOT) ? 1 : 0;
    c->linear = (b->flags & ORC_FLAG_LINEARISED) ? 1 : 0;
    c->m = b->mass;
    c->L = b->length;
    c->R = b->radius;
    c->g = b->gravity;
    c->h = b->dt / b->substeps;
    /* solid cylinder of radius R and length L, axis along body e_x */
    c->Ib[0] = 0.5 * c->m * c->R * c->R;
    c->Ib[1] = c->m * (3.0 * c->R * c->R + c->L * c->L) / 12.0;
    c->Ib[2] = c->Ib[1];
    c->a_s = b->alpha_s[s] * c->L;
    c->a_b = b->alpha_b[s] * c->L;
    c->a_t = b->alpha_t[s] * c->L;
    c->mu = b->mu[s];
    c->relax = b->relax;
    c->wheels = (b->flags & ORC_FLAG_WHEELS) ? 1 : 0;
    c->NB = c->wheels ? 3 * c->B : c->B;
    /* a thin disc: axial inertia m r^2 / 2, diametral m r^2 / 4 */
    c->mw = c->m / 8.0;
    c->rw = 0.5 * c->R;
    c->dw = c->R;
    c->hw = 0.5 * c->R;
    c->Iwh[0] = 0.25 * c->mw * c->rw * c->rw;
    c->Iwh[1] = 0.5 * c->mw * c->rw * c->rw;
    c->Iwh[2] = c->Iwh[0];
    c->anchor = NULL;
}

static int is_fixed(const snake_ctx* c, int i) { return c->fixed_root && i == 0; }

static double inv_mass(const snake_ctx* c, int i)
{
    if (is_fixed(c, i)) return 0.0;
    return i >= c->B ? 1.0 / c->mw : 1.0 / c->m;
}

/* principal inertia of body i in its own frame */
static const double* body_inertia(const snake_ctx* c, int i) { return i >= c->B ? c->Iwh : c->Ib; }

/* world inverse inertia R diag(1/I) R^T (zero for a fixed body) */
static void inv_inertia_world(const snake_ctx* c, int i, const double* q, double* Iinv)
{
    if (is_fixed(c, i)) {
        memset(Iinv, 0, 9 * sizeof(double));
        return;
    }
    double R[9], RT[9], D[9] = {0}, T[9];
    q_to_matrix(q, R);
    m3_transpose(R, RT);
    for (int k = 0; k < 3; ++k) D[4 * k] = 1.0 / body_inertia(c, i)[k];
    m3_mul(R, D, T);
    m3_mul(T, RT, Iinv);
}

static void inertia_world(const snake_ctx* c, int i, const double* q, double* Iw)
{
    double R[9], RT[9], D[9] = {0}, T[9];
    q_to_matrix(q, R);
    m3_transpose(R, RT);
    for (int k = 0; k < 3; ++k) D[4 * k] = body_inertia(c, i)[k];
    m3_mul(R, D, T);
    m3_mul(T, RT, Iw);
}

/* number of blocks touching body i: two per joint on each side, one contact */
static int body_degree(int i, int B, int ground)
{
    int d = ground ? 1 : 0;
    if (i > 0) d += 2;
    if (i < B - 1) d += 2;
    return d;
}

/* ------------------------------------------------------------------ */
/* constraint blocks                                                    */
/* ------------------------------------------------------------------ */

enum { BLK_STRETCH = 0, BLK_BEND = 1, BLK_CONTACT = 2, BLK_HINGE = 3, BLK_AXLE = 4, BLK_WHEEL = 5 };

/* number of blocks touching body i of a wheel carriage: two per joint on
 * each side and two per wheel for a segment; hinge position, hinge axis and
 * contact for a wheel */
static int carriage_degree(const snake_ctx* c, int i)
{
    if (i >= c->B) return 2 + c->ground;
    return (i > 0 ? 2 : 0) + (i < c->B - 1 ? 2 : 0) + 4;
}

static int degree(const snake_ctx* c, int i)
{
    return c->wheels ? carriage_degree(c, i) : body_degree(i, c->B, c->ground);
}

typedef struct {
    int type, a, b;         /* b < 0 for a contact */
    double C[3];            /* constraint value at the current iterate */
    double Ja[18];          /* 3x6 row-major: d C / d (x_a, theta_a) */
    double Jb[18];          /* 3x6: d C / d (x_b, theta_b) */
    double comp[3];         /* alpha~ = compliance / h^2 per row */
    double scale;           /* relax / block degree */
} block_t;

/* Stretch: the end point of body a must coincide with the start point of
 * body b.  Same form as the rigid attachment c = x + R(q) r - x_p, here with
 * both points carried by rigid bodies: r_a = +L/2 e_x, r_b = -L/2 e_x. */
static void eval_stretch(const snake_ctx* c, const double* xa, const double* qa, const double* xb,
                         const double* qb, block_t* k)
{
    double ex[3] = {1.0, 0.0, 0.0}, Ra[9], Rb[9], ra[3], rb[3], Sa[9], Sb[9];
    q_to_matrix(qa, Ra);
    q_to_matrix(qb, Rb);
    m3_vec(Ra, ex, ra);
    m3_vec(Rb, ex, rb);
    for (int d = 0; d < 3; ++d) {
        ra[d] *= 0.5 * c->L;
        rb[d] *= -0.5 * c->L;
    }
    for (int d = 0; d < 3; ++d) k->C[d] = (xa[d] + ra[d]) - (xb[d] + rb[d]);
    /* a world rotation dtheta moves an attached offset r by dtheta x r = -[r]x dtheta */
    skew3(ra, Sa);
    skew3(rb, Sb);
    for (int r = 0; r < 3; ++r)
        for (int col = 0; col < 3; ++col) {
            double id = (r == col) ? 1.0 : 0.0;
            k->Ja[6 * r + col] = id;
            k->Ja[6 * r + 3 + col] = -Sa[3 * r + col];
            k->Jb[6 * r + col] = -id;
            k->Jb[6 * r + 3 + col] = Sb[3 * r + col];
        }
    double a = c->a_s / (c->h * c->h);
    k->comp[0] = k->comp[1] = k->comp[2] = a;
}

/* Bend-twist: relative rotation of body b in the frame of body a, measured
 * against the rest rotation q0 = rotation by theta0 about the body z axis.
 * e = conj(q0) conj(qa) qb (sign chosen so e_w >= 0), C = 2 e_xyz: rows are
 * twist (about x), bend about y, bend about z. */
static void eval_bend(const snake_ctx* c, const double* qa, const double* qb, double theta0,
                      block_t* k)
{
    double q0[4] = {cos(0.5 * theta0), 0.0, 0.0, sin(0.5 * theta0)};
    double q0c[4], qac[4], t[4], e[4];
    q_conj(q0, q0c);
    q_conj(qa, qac);
    q_mul(q0c, qac, t);
    q_mul(t, qb, e);
    if (e[0] < 0.0)
        for (int d = 0; d < 4; ++d) e[d] = -e[d];
    for (int d = 0; d < 3; ++d) k->C[d] = 2.0 * e[1 + d];
    /* d C = G F^T (dtheta_b - dtheta_a), G = e_w I - [e_xyz]x, F = R(qa q0) */
    double G[9], Se[9], F[9], FT[9], A[9], qaq0[4];
    skew3(e + 1, Se);
    for (int d = 0; d < 9; ++d) G[d] = -Se[d];
    G[0] += e[0];
    G[4] += e[0];
    G[8] += e[0];
    q_mul(qa, q0, qaq0);
    q_to_matrix(qaq0, F);
    m3_transpose(F, FT);
    m3_mul(G, FT, A);
    for (int r = 0; r < 3; ++r)
        for (int col = 0; col < 3; ++col) {
            k->Ja[6 * r + col] = 0.0;
            k->Jb[6 * r + col] = 0.0;
            k->Ja[6 * r + 3 + col] = -A[3 * r + col];
            k->Jb[6 * r + 3 + col] = A[3 * r + col];
        }
    double hh = c->h * c->h;
    k->comp[0] = c->a_t / hh;
    k->comp[1] = c->a_b / hh;
    k->comp[2] = c->a_b / hh;
}

/* Contact with the ground plane z = 0 of a sphere of radius R at the body
 * centre: C_n = z - R >= 0.  Friction rows measure the tangential slip of the
 * centre since the start of the substep (static friction keeps it at 0). */
static void eval_contact(const snake_ctx* c, const double* x, const double* xp, block_t* k)
{
    k->C[0] = x[2] - c->R;
    k->C[1] = x[0] - xp[0];
    k->C[2] = x[1] - xp[1];
    memset(k->Ja, 0, sizeof k->Ja);
    memset(k->Jb, 0, sizeof k->Jb);
    k->Ja[0 * 6 + 2] = 1.0;
    k->Ja[1 * 6 + 0] = 1.0;
    k->Ja[2 * 6 + 1] = 1.0;
    k->comp[0] = k->comp[1] = k->comp[2] = 0.0;
}

/* Hinge position (wheel side k): the wheel centre coincides with the point
 * r_h = (0, +-dw, -hw) of its segment, the attachment form of
 * eq. rigid_to_particle with the wheel centre as the attached point. */
static void eval_hinge(const snake_ctx* c, int k_side, const double* xa, const double* qa, const double* xw,
                       block_t* k)
{
    double Ra[9], rh[3] = {0.0, k_side == 0 ? c->dw : -c->dw, -c->hw}, ra[3], Sa[9];
    q_to_matrix(qa, Ra);
    m3_vec(Ra, rh, ra);
    for (int d = 0; d < 3; ++d) k->C[d] = (xa[d] + ra[d]) - xw[d];
    skew3(ra, Sa);
    for (int r = 0; r < 3; ++r)
        for (int col = 0; col < 3; ++col) {
            double id = (r == col) ? 1.0 : 0.0;
            k->Ja[6 * r + col] = id;
            k->Ja[6 * r + 3 + col] = -Sa[3 * r + col];
            k->Jb[6 * r + col] = -id;
            k->Jb[6 * r + 3 + col] = 0.0;
        }
    k->comp[0] = k->comp[1] = k->comp[2] = 0.0;
}

/* Hinge axis: the relative rotation of the wheel in its segment's frame is
 * a turn about the common y axis.  With e = conj(qa) qw (e_w >= 0) that is
 * e_x = e_z = 0: the twist and z-bend rows of the bend-twist form at rest
 * angle 0, rigid; the y row (the wheel's spin) is free and left at zero. */
static void eval_axle(const snake_ctx* c, const double* qa, const double* qw, block_t* k)
{
    eval_bend(c, qa, qw, 0.0, k);
    k->C[1] = 0.0;
    for (int col = 0; col < 6; ++col) {
        k->Ja[6 + col] = 0.0;
        k->Jb[6 + col] = 0.0;
    }
    k->comp[0] = k->comp[1] = k->comp[2] = 0.0;
}

/* Contact point of a wheel (disc of radius rw, axle a = R(q) e_y) with the
 * ground plane z = 0: the rim point lowest in z, x + r with
 * r = -rw (e_z - a_z a) / |e_z - a_z a| (r = 0 for a disc lying flat). */
static void wheel_low_point(const snake_ctx* c, const double* q, double* r)
{
    double R[9];
    q_to_matrix(q, R);
    double a[3] = {R[1], R[4], R[7]};
    double u[3] = {-a[2] * a[0], -a[2] * a[1], 1.0 - a[2] * a[2]};
    double n = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (int d = 0; d < 3; ++d) r[d] = n > 0.0 ? -c->rw * u[d] / n : 0.0;
}

/* Wheel contact (the non-interpenetration form of section "Rigid Body
 * Joints and Contact" with the ground plane): C_n = z of the wheel's lowest
 * rim point >= 0, Jacobian (e_z, r x e_z).  Friction rows measure the
 * tangential slip of the wheel's material point that was the contact point
 * at the start of the substep (world point p0, arm s0 in the wheel frame):
 * C_t = x + R(q) s0 - p0 along x and y, Jacobian (e_t, (R s0) x e_t), so a
 * wheel rolls without slip at the cost of its spin inertia only and slides
 * sideways against the full friction cone. */
static void eval_wheel_contact(const snake_ctx* c, const double* x, const double* q, const double* anc,
                               block_t* k)
{
    double r[3], R[9], s[3];
    wheel_low_point(c, q, r);
    q_to_matrix(q, R);
    m3_vec(R, anc + 3, s);
    memset(k->Ja, 0, sizeof k->Ja);
    memset(k->Jb, 0, sizeof k->Jb);
    k->C[0] = x[2] + r[2];
    k->C[1] = x[0] + s[0] - anc[0];
    k->C[2] = x[1] + s[1] - anc[1];
    /* (r x e_z), (s x e_x), (s x e_y) */
    k->Ja[0 * 6 + 2] = 1.0;
    k->Ja[0 * 6 + 3] = r[1];
    k->Ja[0 * 6 + 4] = -r[0];
    k->Ja[1 * 6 + 0] = 1.0;
    k->Ja[1 * 6 + 4] = s[2];
    k->Ja[1 * 6 + 5] = -s[1];
    k->Ja[2 * 6 + 1] = 1.0;
    k->Ja[2 * 6 + 3] = -s[2];
    k->Ja[2 * 6 + 5] = s[0];
    k->comp[0] = k->comp[1] = k->comp[2] = 0.0;
}

/* anchors of the wheels' friction rows from the start-of-substep pose */
static void wheel_anchors(const snake_ctx* c, const double* xp, const double* qp, double* anc)
{
    for (int wi = 0; wi < 2 * c->B; ++wi) {
        const double* x = xp + 3 * (c->B + wi);
        const double* q = qp + 4 * (c->B + wi);
        double r[3], R[9], RT[9];
        wheel_low_point(c, q, r);
        q_to_matrix(q, R);
        m3_transpose(R, RT);
        for (int d = 0; d < 3; ++d) anc[6 * wi + d] = x[d] + r[d];
        m3_vec(RT, r, anc + 6 * wi + 3);
    }
}

/* rest angle of joint j: intra-module joints follow their module's
 * pressure difference, joints between modules are straight */
static double rest_angle(const orc_batch* b, const snake_ctx* c, const double* p, int j)
{
    if ((j + 1) % c->S == 0) return 0.0;
    int m = j / c->S;
    return b->kappa_max * (p[2 * m] - p[2 * m + 1]) * c->L;
}

/* K += J W J^T for one body (J is 3x6, W = diag(w I, Iinv)) */
static void add_jwjt(const double* J, double w, const double* Iinv, double* K)
{
    for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s) {
            double acc = 0.0;
            for (int d = 0; d < 3; ++d) acc += J[6 * r + d] * w * J[6 * s + d];
            for (int d = 0; d < 3; ++d)
                for (int e = 0; e < 3; ++e) acc += J[6 * r + 3 + d] * Iinv[3 * d + e] * J[6 * s + 3 + e];
            K[3 * r + s] += acc;
        }
}

/* (dx, dth) += (w J_x^T l, Iinv J_th^T l) */
static void add_jt(const double* J, double w, const double* Iinv, const double* l, double* dx,
                   double* dth)
{
    double jx[3], jt[3], it[3];
    for (int d = 0; d < 3; ++d) {
        jx[d] = J[d] * l[0] + J[6 + d] * l[1] + J[12 + d] * l[2];
        jt[d] = J[3 + d] * l[0] + J[9 + d] * l[1] + J[15 + d] * l[2];
    }
    m3_vec(Iinv, jt, it);
    for (int d = 0; d < 3; ++d) {
        dx[d] += w * jx[d];
        dth[d] += it[d];
    }
}

/* Evaluate every block of the snake at configuration (x, q).
 * Block order: (stretch_j, bend_j) for j = 0..B-2, then contact_i. */
static void eval_blocks(const orc_batch* b, const snake_ctx* c, const double* x, const double* q,
                        const double* xp, const double* theta0, block_t* blk)
{
    int n = 0;
    for (int j = 0; j < c->nj; ++j) {
        block_t* ks = &blk[n++];
        block_t* kb = &blk[n++];
        ks->type = BLK_STRETCH;
        kb->type = BLK_BEND;
        ks->a = kb->a = j;
        ks->b = kb->b = j + 1;
        eval_stretch(c, x + 3 * j, q + 4 * j, x + 3 * (j + 1), q + 4 * (j + 1), ks);
        eval_bend(c, q + 4 * j, q + 4 * (j + 1), theta0[j], kb);
        int d = degree(c, j);
        int d1 = degree(c, j + 1);
        ks->scale = kb->scale = c->relax / (double)(d > d1 ? d : d1);
    }
    if (c->wheels) {
        for (int i = 0; i < c->B; ++i)
            for (int s = 0; s < 2; ++s) {
                int wb = c->B + 2 * i + s;
                int dd = degree(c, i) > degree(c, wb) ? degree(c, i) : degree(c, wb);
                block_t* kh = &blk[n++];
                block_t* ka = &blk[n++];
                kh->type = BLK_HINGE;
                ka->type = BLK_AXLE;
                kh->a = ka->a = i;
                kh->b = ka->b = wb;
                eval_hinge(c, s, x + 3 * i, q + 4 * i, x + 3 * wb, kh);
                eval_axle(c, q + 4 * i, q + 4 * wb, ka);
                kh->scale = ka->scale = c->relax / (double)dd;
                if (c->ground) {
                    block_t* kc = &blk[n++];
                    kc->type = BLK_WHEEL;
                    kc->a = wb;
                    kc->b = -1;
                    eval_wheel_contact(c, x + 3 * wb, q + 4 * wb, c->anchor + 6 * (2 * i + s), kc);
                    kc->scale = c->relax / (double)degree(c, wb);
                }
            }
        return;
    }
    if (c->ground)
        for (int i = 0; i < c->B; ++i) {
            block_t* k = &blk[n++];
            k->type = BLK_CONTACT;
            k->a = i;
            k->b = -1;
            eval_contact(c, x + 3 * i, xp + 3 * i, k);
            k->scale = c->relax / (double)body_degree(i, c->B, c->ground);
        }
    (void)b;
}

/* blocks of one wheel: hinge position, hinge axis, contact (if ground) */
static int wheel_blocks(const snake_ctx* c) { return 2 + c->ground; }

static int n_blocks(const snake_ctx* c)
{
    if (c->wheels) return 2 * c->nj + 2 * c->B * wheel_blocks(c);
    return 2 * c->nj + (c->ground ? c->B : 0);
}

/* lambda of block k inside the state arrays (for a wheel carriage lam_c
 * holds the wheels' multipliers, 9 per wheel) */
static double* block_lambda(const snake_ctx* c, double* lam_j, double* lam_c, const block_t* k, int idx)
{
    if (k->type == BLK_CONTACT) return lam_c + 3 * k->a;
    if (k->type == BLK_HINGE) return lam_c + 9 * (k->b - c->B);
    if (k->type == BLK_AXLE) return lam_c + 9 * (k->b - c->B) + 3;
    if (k->type == BLK_WHEEL) return lam_c + 9 * (k->a - c->B) + 6;
    return lam_j + 6 * (idx / 2) + 3 * (idx % 2);
}

/* multipliers of the contact-side array: 3 per body, or 9 per wheel */
static size_t contact_lambdas(const snake_ctx* c) { return (size_t)(c->wheels ? 18 * c->B : 3 * c->B); }

/* Gather the increments dl[block] onto body i in the fixed order
 * stretch_{i-1}, bend_{i-1}, stretch_i, bend_i, contact_i. */
static void gather_body(const snake_ctx* c, int i, const block_t* blk, const double* dl, double w,
                        const double* Iinv, double* dx, double* dth)
{
    dx[0] = dx[1] = dx[2] = 0.0;
    dth[0] = dth[1] = dth[2] = 0.0;
    if (c->wheels && i >= c->B) {
        /* a wheel: hinge position, hinge axis, contact */
        int wi = i - c->B;
        int k = 2 * c->nj + wheel_blocks(c) * wi;
        add_jt(blk[k].Jb, w, Iinv, dl + 3 * k, dx, dth);
        add_jt(blk[k + 1].Jb, w, Iinv, dl + 3 * (k + 1), dx, dth);
        if (c->ground) add_jt(blk[k + 2].Ja, w, Iinv, dl + 3 * (k + 2), dx, dth);
        return;
    }
    if (i > 0) {
        int k = 2 * (i - 1);
        add_jt(blk[k].Jb, w, Iinv, dl + 3 * k, dx, dth);
        add_jt(blk[k + 1].Jb, w, Iinv, dl + 3 * (k + 1), dx, dth);
    }
    if (i < c->B - 1) {
        int k = 2 * i;
        add_jt(blk[k].Ja, w, Iinv, dl + 3 * k, dx, dth);
        add_jt(blk[k + 1].Ja, w, Iinv, dl + 3 * (k + 1), dx, dth);
    }
    if (c->wheels) {
        /* then its wheels' hinge position and axis, side 0 then side 1 */
        for (int s = 0; s < 2; ++s) {
            int k = 2 * c->nj + wheel_blocks(c) * (2 * i + s);
            add_jt(blk[k].Ja, w, Iinv, dl + 3 * k, dx, dth);
            add_jt(blk[k + 1].Ja, w, Iinv, dl + 3 * (k + 1), dx, dth);
        }
    } else if (c->ground) {
        int k = 2 * c->nj + i;
        add_jt(blk[k].Ja, w, Iinv, dl + 3 * k, dx, dth);
    }
}

/* ------------------------------------------------------------------ */
/* one substep of one snake                                             */
/* ------------------------------------------------------------------ */

typedef struct {
    block_t* blk;       /* [n_blocks] */
    block_t* blk0;      /* [n_blocks] frozen copy (linearised mode) */
    double* dl;         /* [n_blocks*3] applied increments */
    double* xp;         /* [B*3] positions at the start of the substep */
    double* qp;         /* [B*4] */
    double* xt;         /* [B*3] predicted (after warm start) */
    double* qt;         /* [B*4] */
    double* acc;        /* [B*6] linearised accumulated displacement */
    double* Iinv;       /* [B*9] */
    double* theta0;     /* [B] */
    double* lz_j;       /* zero multipliers for the fallback's comparison */
    double* lz_c;
    double* xs;         /* [B*3] predicted state kept for the fallback's probes */
    double* qs;         /* [B*4] */
    double* l0_j;       /* lambda0 kept for the fallback's probes */
    double* l0_c;
    double* xz;         /* [B*3] the zero start's iterate K, kept for a fallback */
    double* qz;         /* [B*4] */
    /* Newton solver: per block a 3x3 compliance, per row the right-hand
     * side, the preconditioner's diagonal and the inner solve's vectors */
    double* nE;         /* [n_blocks*9] */
    double* nP;         /* [n_blocks*9] projector onto the free rows */
    double* nd;         /* [n_blocks*3] fixed increments */
    double* nrhs;       /* [n_blocks*3] */
    double* ndiag;
    double* nx;         /* the increment of the multipliers */
    double* nz;
    double* np;
    double* nAp;
    double* nAz;
    double* nMq;
    double* nu;         /* [B*6] W J^T v per body */
    double* kx;         /* [B*6] the kept (best) Newton iterate: x or the
                         * linearised displacement */
    double* kq;         /* [B*4] */
    double* kl_j;       /* [B*6] */
    double* kl_c;       /* [B*3] */
    double* anc;        /* [2B*6] wheel friction anchors */
} scratch_t;

static void scratch_alloc(scratch_t* w, const snake_ctx* c)
{
    int nb = n_blocks(c) + 1;
    int B = c->NB;
    size_t nlc = contact_lambdas(c);
    w->anc = (double*)calloc((size_t)c->B * 12, sizeof(double));
    w->blk = (block_t*)calloc((size_t)nb, sizeof(block_t));
    w->blk0 = (block_t*)calloc((size_t)nb, sizeof(block_t));
    w->dl = (double*)calloc((size_t)nb * 3, sizeof(double));
    w->xp = (double*)calloc((size_t)B * 3, sizeof(double));
    w->qp = (double*)calloc((size_t)B * 4, sizeof(double));
    w->xt = (double*)calloc((size_t)B * 3, sizeof(double));
    w->qt = (double*)calloc((size_t)B * 4, sizeof(double));
    w->acc = (double*)calloc((size_t)B * 6, sizeof(double));
    w->Iinv = (double*)calloc((size_t)B * 9, sizeof(double));
    w->theta0 = (double*)calloc((size_t)B, sizeof(double));
    w->lz_j = (double*)calloc((size_t)B * 6, sizeof(double));
    w->lz_c = (double*)calloc(nlc, sizeof(double));
    w->xs = (double*)calloc((size_t)B * 3, sizeof(double));
    w->qs = (double*)calloc((size_t)B * 4, sizeof(double));
    w->l0_j = (double*)calloc((size_t)B * 6, sizeof(double));
    w->l0_c = (double*)calloc(nlc, sizeof(double));
    w->xz = (double*)calloc((size_t)B * 3, sizeof(double));
    w->qz = (double*)calloc((size_t)B * 4, sizeof(double));
    size_t r3 = (size_t)(n_blocks(c) + 1) * 3;
    w->nE = (double*)calloc(r3 * 3, sizeof(double));
    w->nP = (double*)calloc(r3 * 3, sizeof(double));
    w->nd = (double*)calloc(r3, sizeof(double));
    w->nrhs = (double*)calloc(r3, sizeof(double));
    w->ndiag = (double*)calloc(r3, sizeof(double));
    w->nx = (double*)calloc(r3, sizeof(double));
    w->nz = (double*)calloc(r3, sizeof(double));
    w->np = (double*)calloc(r3, sizeof(double));
    w->nAp = (double*)calloc(r3, sizeof(double));
    w->nAz = (double*)calloc(r3, sizeof(double));
    w->nMq = (double*)calloc(r3, sizeof(double));
    w->nu = (double*)calloc((size_t)B * 6, sizeof(double));
    w->kx = (double*)calloc((size_t)B * 6, sizeof(double));
    w->kq = (double*)calloc((size_t)B * 4, sizeof(double));
    w->kl_j = (double*)calloc((size_t)B * 6, sizeof(double));
    w->kl_c = (double*)calloc(nlc, sizeof(double));
}

static void scratch_free(scratch_t* w)
{
    free(w->anc);
    free(w->blk);
    free(w->blk0);
    free(w->dl);
    free(w->xp);
    free(w->qp);
    free(w->xt);
    free(w->qt);
    free(w->acc);
    free(w->Iinv);
    free(w->theta0);
    free(w->lz_j);
    free(w->lz_c);
    free(w->xs);
    free(w->qs);
    free(w->l0_j);
    free(w->l0_c);
    free(w->xz);
    free(w->qz);
    free(w->nE);
    free(w->nP);
    free(w->nd);
    free(w->nrhs);
    free(w->ndiag);
    free(w->nx);
    free(w->nz);
    free(w->np);
    free(w->nAp);
    free(w->nAz);
    free(w->nMq);
    free(w->nu);
    free(w->kx);
    free(w->kq);
    free(w->kl_j);
    free(w->kl_c);
}

/* Predicted positions of a first-order implicit step: gravity on the linear
 * velocity, gyroscopic torque -w x (I w) on the angular velocity, then a
 * position-level step of length h. */
static void predict(const snake_ctx* c, double* x, double* q, double* v, double* w)
{
    for (int i = 0; i < c->NB; ++i) {
        if (is_fixed(c, i)) {
            v[3 * i] = v[3 * i + 1] = v[3 * i + 2] = 0.0;
            w[3 * i] = w[3 * i + 1] = w[3 * i + 2] = 0.0;
            continue;
        }
        v[3 * i + 2] -= c->h * c->g;
        for (int d = 0; d < 3; ++d) x[3 * i + d] += c->h * v[3 * i + d];
        double Iw[9], Iinv[9], Lw[3], tq[3], dw[3];
        inertia_world(c, i, q + 4 * i, Iw);
        inv_inertia_world(c, i, q + 4 * i, Iinv);
        m3_vec(Iw, w + 3 * i, Lw);
        cross3(w + 3 * i, Lw, tq);
        for (int d = 0; d < 3; ++d) tq[d] = -tq[d];
        m3_vec(Iinv, tq, dw);
        for (int d = 0; d < 3; ++d) w[3 * i + d] += c->h * dw[d];
        double dth[3] = {c->h * w[3 * i], c->h * w[3 * i + 1], c->h * w[3 * i + 2]};
        q_apply_rotvec(q + 4 * i, dth);
    }
}

/* Local solves of every evaluated block (increments into W->dl, scaled) and
 * the residual of the iterate they were evaluated at.  Reads lambda only. */
static double local_solves(const snake_ctx* c, scratch_t* W, double* lam_j, double* lam_c)
{
    int nb = n_blocks(c);
    double r;
    r = 0.0;
    for (int n = 0; n < nb; ++n) {
        block_t* kb = &W->blk[n];
        double* l = block_lambda(c, lam_j, lam_c, kb, n);
        double* dl = W->dl + 3 * n;
        if (kb->type == BLK_CONTACT) {
            int i = kb->a;
            double cn = kb->C[0];
            double rc = (l[0] > 0.0) ? fabs(cn) : (cn < 0.0 ? -cn : 0.0);
            rc /= c->L;
            if (rc > r || rc != rc) r = rc;
            double wi = inv_mass(c, i);
            if (wi == 0.0) {
                dl[0] = dl[1] = dl[2] = 0.0;
                continue;
            }
            /* normal: projected increment; tangential: trial increment
             * projected onto the Coulomb disc of radius mu * lambda_n */
            double ln = l[0] + kb->scale * (-cn / wi);
            if (ln < 0.0) ln = 0.0;
            double lt0 = l[1] + kb->scale * (-kb->C[1] / wi);
            double lt1 = l[2] + kb->scale * (-kb->C[2] / wi);
            double cap = c->mu * ln;
            double nt = sqrt(lt0 * lt0 + lt1 * lt1);
            if (ln <= 0.0) {
                lt0 = lt1 = 0.0;
            } else if (nt > cap) {
                lt0 *= cap / nt;
                lt1 *= cap / nt;
            }
            dl[0] = ln - l[0];
            dl[1] = lt0 - l[1];
            dl[2] = lt1 - l[2];
        } else if (kb->type == BLK_WHEEL) {
            /* the contact rule above with the wheel's own effective masses:
             * K = J W J^T of the block, the normal row by K_nn, the
             * tangential pair by its 2x2 block, then the Coulomb disc */
            double cn = kb->C[0];
            double rc = (l[0] > 0.0) ? fabs(cn) : (cn < 0.0 ? -cn : 0.0);
            rc /= c->L;
            if (rc > r || rc != rc) r = rc;
            double K[9] = {0};
            add_jwjt(kb->Ja, inv_mass(c, kb->a), W->Iinv + 9 * kb->a, K);
            double ln = l[0] + kb->scale * (-cn / K[0]);
            if (ln < 0.0) ln = 0.0;
            double det = K[4] * K[8] - K[5] * K[7];
            double y0 = (K[8] * kb->C[1] - K[5] * kb->C[2]) / det;
            double y1 = (K[4] * kb->C[2] - K[7] * kb->C[1]) / det;
            double lt0 = l[1] - kb->scale * y0;
            double lt1 = l[2] - kb->scale * y1;
            double cap = c->mu * ln;
            double nt = sqrt(lt0 * lt0 + lt1 * lt1);
            if (ln <= 0.0) {
                lt0 = lt1 = 0.0;
            } else if (nt > cap) {
                lt0 *= cap / nt;
                lt1 *= cap / nt;
            }
            dl[0] = ln - l[0];
            dl[1] = lt0 - l[1];
            dl[2] = lt1 - l[2];
        } else if (kb->type == BLK_AXLE) {
            /* the two rigid rows (x, z) solved together; the spin row
             * carries nothing */
            double K[9] = {0};
            add_jwjt(kb->Ja, inv_mass(c, kb->a), W->Iinv + 9 * kb->a, K);
            add_jwjt(kb->Jb, inv_mass(c, kb->b), W->Iinv + 9 * kb->b, K);
            double r0 = kb->C[0], r2 = kb->C[2];
            double rb = fabs(r0) > fabs(r2) ? fabs(r0) : fabs(r2);
            if (r0 != r0 || r2 != r2) rb = r0 + r2;
            if (rb > r || rb != rb) r = rb;
            double det = K[0] * K[8] - K[2] * K[6];
            double d0 = (K[8] * r0 - K[2] * r2) / det;
            double d2 = (K[0] * r2 - K[6] * r0) / det;
            dl[0] = -kb->scale * d0;
            dl[1] = 0.0;
            dl[2] = -kb->scale * d2;
        } else {
            double rhs[3], K[9] = {0}, Iinva[9], Iinvb[9], dlam[3];
            for (int d = 0; d < 3; ++d) rhs[d] = kb->C[d] + kb->comp[d] * l[d];
            double rb = 0.0;
            for (int d = 0; d < 3; ++d) {
                double t = fabs(rhs[d]);
                if (t > rb || t != t) rb = t;
            }
            if (kb->type == BLK_STRETCH || kb->type == BLK_HINGE) rb /= c->L;
            if (rb > r || rb != rb) r = rb;
            memcpy(Iinva, W->Iinv + 9 * kb->a, sizeof Iinva);
            memcpy(Iinvb, W->Iinv + 9 * kb->b, sizeof Iinvb);
            add_jwjt(kb->Ja, inv_mass(c, kb->a), Iinva, K);
            add_jwjt(kb->Jb, inv_mass(c, kb->b), Iinvb, K);
            for (int d = 0; d < 3; ++d) K[4 * d] += kb->comp[d];
            solve3(K, rhs, dlam);
            for (int d = 0; d < 3; ++d) dl[d] = -kb->scale * dlam[d];
        }
    }
    return r;
}

/* residual of configuration (x, q) with multipliers lambda, nothing applied */
static double residual_at(const orc_batch* b, const snake_ctx* c, scratch_t* W, const double* x,
                          const double* q, double* lam_j, double* lam_c)
{
    eval_blocks(b, c, x, q, W->xp, W->theta0, W->blk);
    for (int i = 0; i < c->NB; ++i) inv_inertia_world(c, i, q + 4 * i, W->Iinv + 9 * i);
    return local_solves(c, W, lam_j, lam_c);
}

/* x <- x + W J(x)^T lambda: the bodies take the displacement of the
 * multipliers currently in lam_j / lam_c (the warm start). */
static void apply_start(const orc_batch* b, const snake_ctx* c, scratch_t* W, double* x, double* q,
                        double* lam_j, double* lam_c)
{
    int nb = n_blocks(c);
    eval_blocks(b, c, x, q, W->xp, W->theta0, W->blk);
    for (int k = 0; k < nb; ++k) {
        double* l = block_lambda(c, lam_j, lam_c, &W->blk[k], k);
        for (int d = 0; d < 3; ++d) W->dl[3 * k + d] = l[d];
    }
    for (int i = 0; i < c->NB; ++i) inv_inertia_world(c, i, q + 4 * i, W->Iinv + 9 * i);
    for (int i = 0; i < c->NB; ++i) {
        double dx[3], dth[3];
        gather_body(c, i, W->blk, W->dl, inv_mass(c, i), W->Iinv + 9 * i, dx, dth);
        for (int d = 0; d < 3; ++d) x[3 * i + d] += dx[d];
        if (!is_fixed(c, i)) q_apply_rotvec(q + 4 * i, dth);
    }
}

/* Linearised mode: the blocks frozen at the start of the solve (blk0),
 * their values moved by J times the accumulated displacement. */
static void linear_blocks(const snake_ctx* c, scratch_t* W)
{
    int nb = n_blocks(c);
    memcpy(W->blk, W->blk0, sizeof(block_t) * (size_t)nb);
    for (int n = 0; n < nb; ++n) {
        block_t* kb = &W->blk[n];
        const double* da = W->acc + 6 * kb->a;
        for (int row = 0; row < 3; ++row) {
            double s = 0.0;
            for (int d = 0; d < 6; ++d) s += kb->Ja[6 * row + d] * da[d];
            if (kb->b >= 0) {
                const double* db = W->acc + 6 * kb->b;
                for (int d = 0; d < 6; ++d) s += kb->Jb[6 * row + d] * db[d];
            }
            kb->C[row] += s;
        }
    }
}

/* Block-Jacobi iterations from iterate k0 of the current (x, q, lambda):
 * evaluate, stop at the first iterate k with residual <= tol or k >= kmax
 * (probe: exactly at k = kmax, no convergence status), else apply.
 * Returns the index of the final iterate; *res is its residual. */
static int jacobi(const orc_batch* b, const snake_ctx* c, scratch_t* W, double* x, double* q, double* lam_j,
                  double* lam_c, int k0, int kmax, double tol, int probe, double* res, int* status)
{
    int nb = n_blocks(c);
    int B = c->NB;
    if (c->linear) {
        memcpy(W->xt, x, sizeof(double) * 3 * (size_t)B);
        memcpy(W->qt, q, sizeof(double) * 4 * (size_t)B);
        memset(W->acc, 0, sizeof(double) * 6 * (size_t)B);
        eval_blocks(b, c, x, q, W->xp, W->theta0, W->blk0);
        for (int i = 0; i < B; ++i) inv_inertia_world(c, i, q + 4 * i, W->Iinv + 9 * i);
    }

    int k = k0;
    double r = 0.0;
    for (;; ++k) {
        /* evaluate every block at the current iterate */
        if (c->linear) {
            linear_blocks(c, W);
        } else {
            eval_blocks(b, c, x, q, W->xp, W->theta0, W->blk);
            for (int i = 0; i < B; ++i) inv_inertia_world(c, i, q + 4 * i, W->Iinv + 9 * i);
        }

        r = local_solves(c, W, lam_j, lam_c);
        if (!isfinite(r)) {
            *status |= ORC_STATUS_NONFINITE;
            break;
        }
        int stop = probe ? (k >= kmax) : (tol > 0.0) ? (r <= tol || k >= kmax) : (k >= kmax);
        if (stop) {
            if (!probe && tol > 0.0 && r > tol) *status |= ORC_STATUS_NOT_CONVERGED;
            break;
        }

        /* apply: lambda += dl, bodies += W J^T dl in the fixed gather order */
        for (int n = 0; n < nb; ++n) {
            double* l = block_lambda(c, lam_j, lam_c, &W->blk[n], n);
            for (int d = 0; d < 3; ++d) l[d] += W->dl[3 * n + d];
        }
        for (int i = 0; i < B; ++i) {
            double dx[3], dth[3];
            gather_body(c, i, W->blk, W->dl, inv_mass(c, i), W->Iinv + 9 * i, dx, dth);
            if (c->linear) {
                for (int d = 0; d < 3; ++d) {
                    W->acc[6 * i + d] += dx[d];
                    W->acc[6 * i + 3 + d] += dth[d];
                }
            } else {
                for (int d = 0; d < 3; ++d) x[3 * i + d] += dx[d];
                if (!is_fixed(c, i)) q_apply_rotvec(q + 4 * i, dth);
            }
        }
    }

    if (c->linear) {
        for (int i = 0; i < B; ++i) {
            for (int d = 0; d < 3; ++d) x[3 * i + d] = W->xt[3 * i + d] + W->acc[6 * i + d];
            memcpy(q + 4 * i, W->qt + 4 * i, 4 * sizeof(double));
            if (!is_fixed(c, i)) q_apply_rotvec(q + 4 * i, W->acc + 6 * i + 3);
        }
    }
    *res = r;
    return k;
}

/* ------------------------------------------------------------------ */
/* the paper's scheme: Newton iterations with a preconditioned          */
/* conjugate-residual solve of eq. schur_system                         */
/* ------------------------------------------------------------------ */

/* Threshold below which the derivative of a contact row's reformulation
 * with respect to the constraint value counts as zero. */
#define NEWTON_EPS 1e-6
/* Scale of the friction natural map's trial, in units of the body mass:
 * every positive scale has the same roots, but the scale decides how the
 * semismooth iterates behave.  One body mass lets the contacts of the short
 * batch cycle between stick and slip at a few iterations; large scales make
 * full solves cycle; ten masses is the measured compromise (swept in the
 * tests). */
#define FRICTION_TRIAL_DEFAULT 10.0
static double FRICTION_TRIAL = FRICTION_TRIAL_DEFAULT;

/* Set the friction trial scale (the reading's sweep); returns the previous
 * value.  Not thread-safe against a running solve. */
double orc_set_friction_trial(double scale)
{
    double old = FRICTION_TRIAL;
    FRICTION_TRIAL = scale;
    return old;
}

/* Rows of contact block k at multipliers l (normal, tangential x, y) for
 * eq. schur_system.  Each row is a semismooth Newton step on F(C, l) = 0,
 * dF = F_C J W J^T dl + F_l dl.  Where F_C > 0 the row is divided by it:
 * compliance E = F_l / F_C, right-hand side -F / F_C, and it joins the
 * inner solve ("free").  Where F_C = 0 the row involves its multiplier
 * alone and fixes its increment ("fixed"); the inner solve then runs on
 * the free rows with the fixed increments moved to the right-hand side.
 *   normal: the Fischer-Burmeister function phi(a, b) = a + b - sqrt(a^2+b^2)
 *     of a = C_n and b = w l_n (both lengths); phi = 0 iff a >= 0, b >= 0,
 *     a b = 0 (the contact complementarity).  At (0, 0) the gradient is
 *     taken along the diagonal.  Fixed when d phi / d a <= NEWTON_EPS,
 *     which happens only for a > 0: the row is then phi(a, b) = 0 in b
 *     alone, whose root is b = 0, taken directly (dl = -l_n).
 *   tangential: the natural map F = l_t - proj(l_t - m C_t) onto the
 *     Coulomb disc of radius mu max(l_n, 0) (radius frozen at the current
 *     iterate), m = FRICTION_TRIAL times the body mass.  Inside the disc
 *     (stick) both rows are C_t = 0 (E = 0).
 *     Outside (slip, s = radius / |y| < 1, y the trial) the row along
 *     y^ = y / |y| is fixed (dl = radius - l.y^), the row across it free
 *     with E = (1 - s) / (m s).  A zero radius fixes both (dl = -l_t).
 * Out: E (3x3), rhs (3), the projector P onto the free rows (3x3) and the
 * fixed increment d (3, zero on free rows).  A body of infinite mass
 * keeps its contact multipliers: every row fixed with d = 0. */
static void contact_newton_rows(const snake_ctx* c, const block_t* k, const double* l, double w,
                                double* E, double* rhs, double* P, double* d)
{
    memset(E, 0, 9 * sizeof(double));
    memset(P, 0, 9 * sizeof(double));
    rhs[0] = rhs[1] = rhs[2] = 0.0;
    d[0] = d[1] = d[2] = 0.0;
    if (w == 0.0) return;
    double a = k->C[0], bb = w * l[0];
    double rr = sqrt(a * a + bb * bb);
    double fa, fb;
    if (rr > 0.0) {
        fa = 1.0 - a / rr;
        fb = 1.0 - bb / rr;
    } else {
        fa = fb = 1.0 - sqrt(0.5);
    }
    /* a + b - r without cancellation when a + b > 0: (a + b)^2 - r^2 = 2ab */
    double phi = (a + bb > 0.0) ? 2.0 * a * bb / (a + bb + rr) : a + bb - rr;
    if (fa > NEWTON_EPS) {
        P[0] = 1.0;
        E[0] = w * fb / fa;
        rhs[0] = -phi / fa;
    } else {
        /* here a > 0, so the row's root is b = 0 */
        d[0] = -l[0];
    }

    double m = FRICTION_TRIAL / w;
    double y0 = l[1] - m * k->C[1], y1 = l[2] - m * k->C[2];
    double cap = c->mu * (l[0] > 0.0 ? l[0] : 0.0);
    double ny = sqrt(y0 * y0 + y1 * y1);
    if (cap > 0.0 && ny <= cap) {
        P[4] = P[8] = 1.0;
        rhs[1] = -k->C[1];
        rhs[2] = -k->C[2];
        return;
    }
    if (!(cap > 0.0)) {
        d[1] = -l[1];
        d[2] = -l[2];
        return;
    }
    double s = cap / ny;
    double u0 = y0 / ny, u1 = y1 / ny;       /* along the trial */
    double v0 = -u1, v1 = u0;                /* across it */
    double fpar = l[1] * u0 + l[2] * u1 - cap;
    double fper = l[1] * v0 + l[2] * v1;
    double eper = (1.0 - s) / (m * s), bper = -fper / (m * s);
    d[1] = -fpar * u0;
    d[2] = -fpar * u1;
    P[4] = v0 * v0;
    P[5] = P[7] = v0 * v1;
    P[8] = v1 * v1;
    E[4] = eper * v0 * v0;
    E[5] = E[7] = eper * v0 * v1;
    E[8] = eper * v1 * v1;
    rhs[1] = bper * v0;
    rhs[2] = bper * v1;
}

/* J W J^T entry (r, r) of one block's row r on one body */
static double row_jwjt(const double* J, int r, double w, const double* Iinv)
{
    double acc = 0.0;
    for (int d = 0; d < 3; ++d) acc += J[6 * r + d] * w * J[6 * r + d];
    for (int d = 0; d < 3; ++d)
        for (int e = 0; e < 3; ++e) acc += J[6 * r + 3 + d] * Iinv[3 * d + e] * J[6 * r + 3 + e];
    return acc;
}

/* Right-hand side, compliance, free-row projector, fixed increments and
 * preconditioner diagonal of eq. schur_system at the evaluated blocks:
 * joint rows are free with E = alpha~, rhs = -(C + alpha~ l); contact rows
 * as above. */
static void newton_rows(const snake_ctx* c, scratch_t* W, double* lam_j, double* lam_c)
{
    int nb = n_blocks(c);
    for (int n = 0; n < nb; ++n) {
        block_t* kb = &W->blk[n];
        double* l = block_lambda(c, lam_j, lam_c, kb, n);
        double* E = W->nE + 9 * n;
        double* P = W->nP + 9 * n;
        double* rhs = W->nrhs + 3 * n;
        double* d = W->nd + 3 * n;
        if (kb->type == BLK_CONTACT) {
            contact_newton_rows(c, kb, l, inv_mass(c, kb->a), E, rhs, P, d);
        } else {
            memset(E, 0, 9 * sizeof(double));
            memset(P, 0, 9 * sizeof(double));
            for (int r = 0; r < 3; ++r) {
                E[4 * r] = kb->comp[r];
                P[4 * r] = 1.0;
                rhs[r] = -(kb->C[r] + kb->comp[r] * l[r]);
                d[r] = 0.0;
            }
        }
        for (int r = 0; r < 3; ++r) {
            double dg = row_jwjt(kb->Ja, r, inv_mass(c, kb->a), W->Iinv + 9 * kb->a);
            if (kb->b >= 0) dg += row_jwjt(kb->Jb, r, inv_mass(c, kb->b), W->Iinv + 9 * kb->b);
            /* zero only on the rows of a body of infinite mass, which are
             * fixed (projected out); 1 keeps the division finite there */
            double v = dg + E[4 * r];
            W->ndiag[3 * n + r] = v > 0.0 ? v : 1.0;
        }
    }
}

/* y = [J W J^T + E] v, matrix-free: per body u = W J^T v (the gather of
 * the Jacobi update), then per block J_a u_a + J_b u_b + E v. */
static void schur_apply(const snake_ctx* c, scratch_t* W, const double* v, double* y)
{
    int nb = n_blocks(c);
    for (int i = 0; i < c->B; ++i)
        gather_body(c, i, W->blk, v, inv_mass(c, i), W->Iinv + 9 * i, W->nu + 6 * i, W->nu + 6 * i + 3);
    for (int n = 0; n < nb; ++n) {
        const block_t* kb = &W->blk[n];
        const double* ua = W->nu + 6 * kb->a;
        const double* E = W->nE + 9 * n;
        for (int r = 0; r < 3; ++r) {
            double s = 0.0;
            for (int d = 0; d < 6; ++d) s += kb->Ja[6 * r + d] * ua[d];
            if (kb->b >= 0) {
                const double* ub = W->nu + 6 * kb->b;
                for (int d = 0; d < 6; ++d) s += kb->Jb[6 * r + d] * ub[d];
            }
            for (int e = 0; e < 3; ++e) s += E[3 * r + e] * v[3 * n + e];
            y[3 * n + r] = s;
        }
    }
}

/* v <- P v block by block (in place) */
static void project_free(const snake_ctx* c, const scratch_t* W, double* v)
{
    int nb = n_blocks(c);
    for (int n = 0; n < nb; ++n) {
        const double* P = W->nP + 9 * n;
        double t[3];
        for (int r = 0; r < 3; ++r) t[r] = P[3 * r] * v[3 * n] + P[3 * r + 1] * v[3 * n + 1] + P[3 * r + 2] * v[3 * n + 2];
        for (int r = 0; r < 3; ++r) v[3 * n + r] = t[r];
    }
}

/* out = P D^-1 P v (the diagonal preconditioner on the free rows) */
static void precondition(const snake_ctx* c, const scratch_t* W, const double* v, double* out)
{
    int n3 = 3 * n_blocks(c);
    memcpy(out, v, sizeof(double) * (size_t)n3);
    project_free(c, W, out);
    for (int k = 0; k < n3; ++k) out[k] /= W->ndiag[k];
    project_free(c, W, out);
}

/* Natural-map residual of the Coulomb friction rows at the evaluated
 * contact blocks, |l_t - proj(l_t - m C_t)| w / L (a length over the
 * segment length, as the normal rows' measure), maximum over bodies. */
static double friction_residual(const snake_ctx* c, scratch_t* W, double* lam_c)
{
    double r = 0.0;
    if (!c->ground) return r;
    for (int i = 0; i < c->B; ++i) {
        double w = inv_mass(c, i);
        if (w == 0.0) continue;
        const block_t* k = &W->blk[2 * c->nj + i];
        const double* l = lam_c + 3 * i;
        double m = 1.0 / w;
        double y0 = l[1] - m * k->C[1], y1 = l[2] - m * k->C[2];
        double cap = c->mu * (l[0] > 0.0 ? l[0] : 0.0);
        double ny = sqrt(y0 * y0 + y1 * y1);
        if (ny > cap) {
            double f = ny > 0.0 ? cap / ny : 0.0;
            y0 *= f;
            y1 *= f;
        }
        double e0 = l[1] - y0, e1 = l[2] - y1;
        double t = sqrt(e0 * e0 + e1 * e1) * w / c->L;
        if (t > r || t != t) r = t;
    }
    return r;
}

static double vdot(const double* a, const double* b, int n)
{
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += a[k] * b[k];
    return s;
}

/* Preconditioned conjugate residual (Saad, "Iterative Methods for Sparse
 * Linear Systems", the conjugate residual method with a preconditioner M)
 * on the free rows: operator P A P, right-hand side P (rhs - A d),
 * M^-1 = P D^-1 P with D the diagonal of A, from x = 0, exactly n_it
 * iterations unless (z, Az) or (Ap, M^-1 Ap) stops being positive.
 * With z = M^-1 r:
 *   alpha = (z, Az) / (Ap, M^-1 Ap),  x += alpha p,  z -= alpha M^-1 Ap,
 *   beta = (z', Az') / (z, Az),  p = z' + beta p,  Ap = Az' + beta Ap,
 * one product with A per iteration (none after the last).  The increment
 * x + d is left in nx. */
static void pcr_solve(const snake_ctx* c, scratch_t* W, int n_it)
{
    int n3 = 3 * n_blocks(c);
    /* right-hand side of the free rows: rhs - A d, projected */
    schur_apply(c, W, W->nd, W->nAz);
    for (int k = 0; k < n3; ++k) W->nAp[k] = W->nrhs[k] - W->nAz[k];
    project_free(c, W, W->nAp);
    precondition(c, W, W->nAp, W->nz);
    for (int k = 0; k < n3; ++k) {
        W->nx[k] = 0.0;
        W->np[k] = W->nz[k];
    }
    schur_apply(c, W, W->nz, W->nAz);
    project_free(c, W, W->nAz);
    memcpy(W->nAp, W->nAz, sizeof(double) * (size_t)n3);
    double rho = vdot(W->nz, W->nAz, n3);
    for (int it = 0; it < n_it; ++it) {
        if (!(rho > 0.0)) break;
        precondition(c, W, W->nAp, W->nMq);
        double den = vdot(W->nAp, W->nMq, n3);
        if (!(den > 0.0)) break;
        double alpha = rho / den;
        for (int k = 0; k < n3; ++k) {
            W->nx[k] += alpha * W->np[k];
            W->nz[k] -= alpha * W->nMq[k];
        }
        if (it == n_it - 1) break;
        schur_apply(c, W, W->nz, W->nAz);
        project_free(c, W, W->nAz);
        double rho1 = vdot(W->nz, W->nAz, n3);
        double beta = rho1 / rho;
        rho = rho1;
        for (int k = 0; k < n3; ++k) {
            W->np[k] = W->nz[k] + beta * W->np[k];
            W->nAp[k] = W->nAz[k] + beta * W->nAp[k];
        }
    }
    for (int k = 0; k < n3; ++k) W->nx[k] += W->nd[k];
}

/* Newton iterations on the compliant system from the current (x, q,
 * lambda): at each iterate evaluate the blocks and the residual (the
 * block-Jacobi measure, and the friction rows' natural map, which the
 * Jacobi local solve resolves at every iterate but a Newton step need
 * not), stop if it is <= tol (tol > 0) or after n_newton
 * solves, else solve eq. schur_system for the multiplier increment with
 * n_pcr inner iterations and apply lambda += dl, x += W J^T dl (rotations
 * as in the Jacobi update; in linearised mode into the accumulated
 * displacement, as there).  With newton_keep_best the substep ends at the
 * evaluated iterate with the smallest residual (the earliest of equals),
 * which a fixed budget otherwise leaves to chance where the iterates cycle.
 * Returns the inner iterations run. */
static int newton_pcr(const orc_batch* b, const snake_ctx* c, scratch_t* W, double* x, double* q,
                      double* lam_j, double* lam_c, int n_newton, int n_pcr, double tol, double* res,
                      int* status)
{
    int nb = n_blocks(c);
    int B = c->B;
    int its = 0;
    double r = 0.0;
    double best = INFINITY;
    size_t nj6 = sizeof(double) * 6 * (size_t)(c->nj > 0 ? c->nj : 1);
    size_t nc3 = sizeof(double) * 3 * (size_t)B;
    if (c->linear) {
        memcpy(W->xt, x, sizeof(double) * 3 * (size_t)B);
        memcpy(W->qt, q, sizeof(double) * 4 * (size_t)B);
        memset(W->acc, 0, sizeof(double) * 6 * (size_t)B);
        eval_blocks(b, c, x, q, W->xp, W->theta0, W->blk0);
        for (int i = 0; i < B; ++i) inv_inertia_world(c, i, q + 4 * i, W->Iinv + 9 * i);
    }
    for (int k = 0;; ++k) {
        if (c->linear) {
            linear_blocks(c, W);
            r = local_solves(c, W, lam_j, lam_c);
        } else {
            r = residual_at(b, c, W, x, q, lam_j, lam_c);
        }
        double rf = friction_residual(c, W, lam_c);
        if (rf > r || rf != rf) r = rf;
        if (b->newton_keep_best && r < best) {
            best = r;
            if (c->linear) {
                memcpy(W->kx, W->acc, sizeof(double) * 6 * (size_t)B);
            } else {
                memcpy(W->kx, x, sizeof(double) * 3 * (size_t)B);
                memcpy(W->kq, q, sizeof(double) * 4 * (size_t)B);
            }
            memcpy(W->kl_j, lam_j, nj6);
            memcpy(W->kl_c, lam_c, nc3);
        }
        if (!isfinite(r)) {
            *status |= ORC_STATUS_NONFINITE;
            break;
        }
        if ((tol > 0.0 && r <= tol) || k >= n_newton) {
            if (tol > 0.0 && r > tol) *status |= ORC_STATUS_NOT_CONVERGED;
            break;
        }
        newton_rows(c, W, lam_j, lam_c);
        pcr_solve(c, W, n_pcr);
        its += n_pcr;
        for (int n = 0; n < nb; ++n) {
            double* l = block_lambda(c, lam_j, lam_c, &W->blk[n], n);
            for (int d = 0; d < 3; ++d) l[d] += W->nx[3 * n + d];
        }
        for (int i = 0; i < B; ++i) {
            double dx[3], dth[3];
            gather_body(c, i, W->blk, W->nx, inv_mass(c, i), W->Iinv + 9 * i, dx, dth);
            if (c->linear) {
                for (int d = 0; d < 3; ++d) {
                    W->acc[6 * i + d] += dx[d];
                    W->acc[6 * i + 3 + d] += dth[d];
                }
            } else {
                for (int d = 0; d < 3; ++d) x[3 * i + d] += dx[d];
                if (!is_fixed(c, i)) q_apply_rotvec(q + 4 * i, dth);
            }
        }
    }
    /* with keep_best, end at the best evaluated iterate instead */
    if (b->newton_keep_best && !(r <= best) && isfinite(best)) {
        r = best;
        if (c->linear) {
            memcpy(W->acc, W->kx, sizeof(double) * 6 * (size_t)B);
        } else {
            memcpy(x, W->kx, sizeof(double) * 3 * (size_t)B);
            memcpy(q, W->kq, sizeof(double) * 4 * (size_t)B);
        }
        memcpy(lam_j, W->kl_j, nj6);
        memcpy(lam_c, W->kl_c, nc3);
        /* no status change: an iterate at or below tol ends the loop
         * itself, so the best one here is above tol whenever tol > 0 */
    }
    if (c->linear) {
        for (int i = 0; i < B; ++i) {
            for (int d = 0; d < 3; ++d) x[3 * i + d] = W->xt[3 * i + d] + W->acc[6 * i + d];
            memcpy(q + 4 * i, W->qt + 4 * i, 4 * sizeof(double));
            if (!is_fixed(c, i)) q_apply_rotvec(q + 4 * i, W->acc + 6 * i + 3);
        }
    }
    *res = r;
    return its;
}

/* Greedy colouring of one snake's blocks in block order (stretch_j, bend_j
 * for every joint, then the contacts): each block takes the smallest colour
 * not taken by an earlier block sharing a body.  Returns the colour count. */
static int block_colours(const snake_ctx* c, const block_t* blk, int* colour)
{
    int nb = n_blocks(c), ncol = 0;
    for (int k = 0; k < nb; ++k) {
        int col = 0;
        for (;;) {
            int clash = 0;
            for (int e = 0; e < k && !clash; ++e) {
                int share = blk[e].a == blk[k].a || (blk[k].b >= 0 && blk[e].a == blk[k].b) ||
                            (blk[e].b >= 0 && (blk[e].b == blk[k].a || blk[e].b == blk[k].b));
                if (share && colour[e] == col) clash = 1;
            }
            if (!clash) break;
            ++col;
        }
        colour[k] = col;
        if (col + 1 > ncol) ncol = col + 1;
    }
    return ncol;
}

/* Block Gauss-Seidel sweeps from the current (x, q, lambda), the blocks
 * visited colour by colour (blocks of one colour share no body, so their
 * order within the colour does not matter): at iterate k evaluate every
 * block and the residual (the block-Jacobi measure), stop as the Jacobi
 * iteration does, else for each colour evaluate every block at the current
 * state, take the local solutions of that colour's blocks scaled by relax
 * (no averaging: a body takes one of them per colour) and apply them to
 * the multipliers and the bodies at once.  Returns the sweeps run. */
static int gauss_seidel(const orc_batch* b, const snake_ctx* c, scratch_t* W, double* x, double* q,
                        double* lam_j, double* lam_c, int kmax, double tol, double* res, int* status)
{
    int nb = n_blocks(c);
    int B = c->B;
    int* colour = (int*)calloc((size_t)nb + 1, sizeof(int));
    eval_blocks(b, c, x, q, W->xp, W->theta0, W->blk);
    int ncol = block_colours(c, W->blk, colour);
    if (c->linear) {
        memcpy(W->xt, x, sizeof(double) * 3 * (size_t)B);
        memcpy(W->qt, q, sizeof(double) * 4 * (size_t)B);
        memset(W->acc, 0, sizeof(double) * 6 * (size_t)B);
        eval_blocks(b, c, x, q, W->xp, W->theta0, W->blk0);
        for (int i = 0; i < B; ++i) inv_inertia_world(c, i, q + 4 * i, W->Iinv + 9 * i);
    }
    int k = 0;
    double r = 0.0;
    for (;; ++k) {
        if (c->linear) {
            linear_blocks(c, W);
            r = local_solves(c, W, lam_j, lam_c);
        } else {
            r = residual_at(b, c, W, x, q, lam_j, lam_c);
        }
        if (!isfinite(r)) {
            *status |= ORC_STATUS_NONFINITE;
            break;
        }
        int stop = (tol > 0.0) ? (r <= tol || k >= kmax) : (k >= kmax);
        if (stop) {
            if (tol > 0.0 && r > tol) *status |= ORC_STATUS_NOT_CONVERGED;
            break;
        }
        for (int col = 0; col < ncol; ++col) {
            if (c->linear) {
                linear_blocks(c, W);
            } else {
                eval_blocks(b, c, x, q, W->xp, W->theta0, W->blk);
                for (int i = 0; i < B; ++i) inv_inertia_world(c, i, q + 4 * i, W->Iinv + 9 * i);
            }
            for (int n = 0; n < nb; ++n) W->blk[n].scale = c->relax;
            local_solves(c, W, lam_j, lam_c);
            for (int n = 0; n < nb; ++n) {
                double* l = block_lambda(c, lam_j, lam_c, &W->blk[n], n);
                if (colour[n] != col) {
                    W->dl[3 * n] = W->dl[3 * n + 1] = W->dl[3 * n + 2] = 0.0;
                    continue;
                }
                for (int d = 0; d < 3; ++d) l[d] += W->dl[3 * n + d];
            }
            for (int i = 0; i < B; ++i) {
                double dx[3], dth[3];
                gather_body(c, i, W->blk, W->dl, inv_mass(c, i), W->Iinv + 9 * i, dx, dth);
                if (c->linear) {
                    for (int d = 0; d < 3; ++d) {
                        W->acc[6 * i + d] += dx[d];
                        W->acc[6 * i + 3 + d] += dth[d];
                    }
                } else {
                    for (int d = 0; d < 3; ++d) x[3 * i + d] += dx[d];
                    if (!is_fixed(c, i)) q_apply_rotvec(q + 4 * i, dth);
                }
            }
        }
    }
    if (c->linear) {
        for (int i = 0; i < B; ++i) {
            for (int d = 0; d < 3; ++d) x[3 * i + d] = W->xt[3 * i + d] + W->acc[6 * i + d];
            memcpy(q + 4 * i, W->qt + 4 * i, 4 * sizeof(double));
            if (!is_fixed(c, i)) q_apply_rotvec(q + 4 * i, W->acc + 6 * i + 3);
        }
    }
    free(colour);
    *res = r;
    return k;
}

/* Solve of one substep from the predicted (x, q): block-Jacobi, or with
 * the Newton solver selected the Newton iterations above (from zero
 * multipliers, or from the previous substep's with the bodies moved by
 * W J^T lambda0 as for Jacobi), or with Gauss-Seidel selected its sweeps
 * from zero.  Returns the number of (inner) iterations run; *res is the
 * residual of the final iterate.
 *
 * Multiplier initialisation: zero, or lambda0 = the current lambda with
 * x <- x~ + W J(x~)^T lambda0.  With the fallback, a given lambda0 is kept
 * only if, after fallback_k iterations, its residual is not larger than the
 * zero start's after as many; fallback_k = 0 compares the starts themselves.
 * For fallback_k > 0 the zero start runs first (fallback_k iterations), then
 * the given start (fallback_k iterations); the solve continues from the
 * winner's iterate fallback_k, and the loser's fallback_k iterations count
 * on top of the total. */
static int solve_substep(const orc_batch* b, const snake_ctx* c, scratch_t* W, double* x, double* q,
                         double* lam_j, double* lam_c, int warm, int kmax, double tol, double* res,
                         int* status)
{
    int B = c->NB;
    size_t nj6 = sizeof(double) * 6 * (size_t)(c->nj > 0 ? c->nj : 1);
    size_t nc3 = sizeof(double) * contact_lambdas(c);
    int fallback = (warm == ORC_WARM_GIVEN && b->fallback);

    if (b->solver == ORC_SOLVER_NEWTON) {
        if (warm == ORC_WARM_PREV) {
            apply_start(b, c, W, x, q, lam_j, lam_c);
        } else {
            memset(lam_j, 0, nj6);
            memset(lam_c, 0, nc3);
        }
        return newton_pcr(b, c, W, x, q, lam_j, lam_c, b->newton_iters, b->pcr_iters, tol, res, status);
    }
    if (b->solver == ORC_SOLVER_GS) {
        memset(lam_j, 0, nj6);
        memset(lam_c, 0, nc3);
        return gauss_seidel(b, c, W, x, q, lam_j, lam_c, kmax, tol, res, status);
    }
    if (fallback && b->fallback_k > 0) {
        int K = b->fallback_k;
        double rz = 0.0, rw = 0.0;
        int st = 0;
        memcpy(W->xs, x, sizeof(double) * 3 * (size_t)B);
        memcpy(W->qs, q, sizeof(double) * 4 * (size_t)B);
        memcpy(W->l0_j, lam_j, nj6);
        memcpy(W->l0_c, lam_c, nc3);
        /* probe: zero start */
        memset(lam_j, 0, nj6);
        memset(lam_c, 0, nc3);
        jacobi(b, c, W, x, q, lam_j, lam_c, 0, K, 0.0, 1, &rz, &st);
        memcpy(W->xz, x, sizeof(double) * 3 * (size_t)B);
        memcpy(W->qz, q, sizeof(double) * 4 * (size_t)B);
        memcpy(W->lz_j, lam_j, nj6);
        memcpy(W->lz_c, lam_c, nc3);
        /* probe: given start */
        memcpy(x, W->xs, sizeof(double) * 3 * (size_t)B);
        memcpy(q, W->qs, sizeof(double) * 4 * (size_t)B);
        memcpy(lam_j, W->l0_j, nj6);
        memcpy(lam_c, W->l0_c, nc3);
        apply_start(b, c, W, x, q, lam_j, lam_c);
        st = 0;
        jacobi(b, c, W, x, q, lam_j, lam_c, 0, K, 0.0, 1, &rw, &st);
        /* keep the given start if it is finite and not farther than zero */
        if (isfinite(rw) && (!isfinite(rz) || rw <= rz)) {
            /* continue from the given start's iterate K; the zero probe's
             * K iterations count on top */
            return jacobi(b, c, W, x, q, lam_j, lam_c, K, kmax, tol, 0, res, status) + K;
        }
        /* continue from the zero start's iterate K; the given start's K
         * probe iterations count on top */
        memcpy(x, W->xz, sizeof(double) * 3 * (size_t)B);
        memcpy(q, W->qz, sizeof(double) * 4 * (size_t)B);
        memcpy(lam_j, W->lz_j, nj6);
        memcpy(lam_c, W->lz_c, nc3);
        *status |= ORC_STATUS_FELL_BACK;
        return jacobi(b, c, W, x, q, lam_j, lam_c, K, kmax, tol, 0, res, status) + K;
    }

    double r_zero = 0.0;
    if (fallback) {
        memcpy(W->xs, x, sizeof(double) * 3 * (size_t)B);
        memcpy(W->qs, q, sizeof(double) * 4 * (size_t)B);
        memset(W->lz_j, 0, nj6);
        memset(W->lz_c, 0, nc3);
        r_zero = residual_at(b, c, W, x, q, W->lz_j, W->lz_c);
    }
    if (warm != ORC_WARM_ZERO) {
        apply_start(b, c, W, x, q, lam_j, lam_c);
        if (fallback) {
            double r_nn = residual_at(b, c, W, x, q, lam_j, lam_c);
            if (!(r_nn <= r_zero)) {
                memcpy(x, W->xs, sizeof(double) * 3 * (size_t)B);
                memcpy(q, W->qs, sizeof(double) * 4 * (size_t)B);
                memset(lam_j, 0, sizeof(double) * 6 * (size_t)c->nj);
                memset(lam_c, 0, nc3);
                *status |= ORC_STATUS_FELL_BACK;
            }
        }
    } else {
        memset(lam_j, 0, sizeof(double) * 6 * (size_t)c->nj);
        memset(lam_c, 0, nc3);
    }
    return jacobi(b, c, W, x, q, lam_j, lam_c, 0, kmax, tol, 0, res, status);
}

/* velocities of the implicit step from the substep displacement */
static void finalize(const snake_ctx* c, const double* xp, const double* qp, const double* x,
                     const double* q, double* v, double* w)
{
    for (int i = 0; i < c->NB; ++i) {
        for (int d = 0; d < 3; ++d) v[3 * i + d] = (x[3 * i + d] - xp[3 * i + d]) / c->h;
        double qpc[4], dq[4];
        q_conj(qp + 4 * i, qpc);
        q_mul(q + 4 * i, qpc, dq);
        double sg = dq[0] >= 0.0 ? 1.0 : -1.0;
        for (int d = 0; d < 3; ++d) w[3 * i + d] = 2.0 / c->h * sg * dq[1 + d];
    }
}

/* ------------------------------------------------------------------ */
/* chamber pressure and command                                         */
/* ------------------------------------------------------------------ */

/* first-order lag toward the target over h, exact for a held target */
static double lag_update(double p, double u, double h, double tau_inf, double tau_def)
{
    double tau = (u > p) ? tau_inf : tau_def;
    return u + (p - u) * exp(-h / tau);
}

/* the paper's latency law, one application per step, pressures in psi:
 * inflating (target above pressure): p += p_s k_i ((u - p)/p_s)^2;
 * deflating: p -= min(k_d p, T_p), not going below the target */
static double paper_update(const orc_batch* b, double p_frac, double u_frac)
{
    double p = p_frac * b->amp_psi;
    double u = u_frac * b->amp_psi;
    if (u > p) {
        double dp = (u - p) / b->p_s;
        p = p + b->p_s * dp * dp * b->k_i;
    } else if (u < p) {
        double cut = p * b->k_d;
        if (cut > b->T_p) cut = b->T_p;
        p = p - cut;
        if (p < u) p = u;
    }
    return p / b->amp_psi;
}

void orc_offsets(const orc_batch* b, int64_t* body_off, int64_t* joint_off, int64_t* module_off,
                 int64_t* block_off)
{
    int ground = (b->flags & ORC_FLAG_NO_GROUND) ? 0 : 1;
    body_off[0] = joint_off[0] = module_off[0] = block_off[0] = 0;
    for (int s = 0; s < b->n_snakes; ++s) {
        int64_t B = (int64_t)b->n_modules[s] * b->segs[s];
        body_off[s + 1] = body_off[s] + B;
        joint_off[s + 1] = joint_off[s] + (B - 1);
        module_off[s + 1] = module_off[s] + b->n_modules[s];
        block_off[s + 1] = block_off[s] + 2 * (B - 1) + (ground ? B : 0);
    }
}

/* serpenoid command of module m at time t:
 * clamp(sin(2 pi f t + alpha m + phase0) + offset, -1, 1) */
static double serpenoid(const orc_batch* b, int s, int m, double t)
{
    const double two_pi = 6.283185307179586476925286766559;
    double a = sin(two_pi * b->freq[s] * t + b->ctrl_alpha * m + b->phase0[s]) + b->ctrl_offset;
    if (a > 1.0) a = 1.0;
    if (a < -1.0) a = -1.0;
    return a;
}

/* piecewise-constant schedule: value of the piece that holds step n */
static double schedule(const orc_batch* b, int64_t gm, int64_t n)
{
    int32_t a = b->sched_off[gm], e = b->sched_off[gm + 1];
    int64_t start = 0;
    for (int32_t k = a; k < e; ++k) {
        if (n < start + b->sched_steps[k]) return b->sched_val[k];
        start += b->sched_steps[k];
    }
    return e > a ? b->sched_val[e - 1] : 0.0;
}

static void offsets_of(const orc_batch* b, int s, int64_t* bo, int64_t* jo, int64_t* mo)
{
    int64_t B = 0, J = 0, M = 0;
    for (int k = 0; k < s; ++k) {
        int64_t nb = (int64_t)b->n_modules[k] * b->segs[k];
        B += nb;
        J += nb - 1;
        M += b->n_modules[k];
    }
    *bo = B;
    *jo = J;
    *mo = M;
}

/* commands of the M modules of snake s (first module index mo) for its
 * current step n: the value for the end of the step, t = (n+1) dt */
static void snake_commands(const orc_batch* b, int s, int64_t mo, int64_t n, double* cmd)
{
    double t = (double)(n + 1) * b->dt;
    for (int m = 0; m < b->n_modules[s]; ++m) {
        if (b->controller == ORC_CTRL_SERPENOID)
            cmd[m] = serpenoid(b, s, m, t);
        else if (b->controller == ORC_CTRL_SCHEDULE)
            cmd[m] = schedule(b, mo + m, n);
    }
}

void orc_commands(const orc_batch* b, orc_state* st, int32_t s0, int32_t s1)
{
    int64_t bo, jo, mo;
    offsets_of(b, s0, &bo, &jo, &mo);
    for (int s = s0; s < s1; ++s) {
        snake_commands(b, s, mo, st->step[s], st->cmd + mo);
        mo += b->n_modules[s];
    }
}

void orc_init_state(const orc_batch* b, orc_state* st)
{
    int64_t bo = 0, jo = 0, mo = 0;
    for (int s = 0; s < b->n_snakes; ++s) {
        snake_ctx c;
        make_ctx(b, s, &c);
        for (int i = 0; i < c.B; ++i) {
            double* x = st->x + 3 * (bo + i);
            double* q = st->q + 4 * (bo + i);
            x[0] = (i + 0.5) * c.L;
            x[1] = 0.0;
            x[2] = c.R;
            q[0] = 1.0;
            q[1] = q[2] = q[3] = 0.0;
            for (int d = 0; d < 3; ++d) {
                st->v[3 * (bo + i) + d] = 0.0;
                st->w[3 * (bo + i) + d] = 0.0;
                st->lam_c[3 * (bo + i) + d] = 0.0;
            }
        }
        if (c.wheels && st->wx)
            for (int wi = 0; wi < 2 * c.B; ++wi) {
                int i = wi / 2;
                double* x = st->wx + 3 * (2 * bo + wi);
                double* q = st->wq + 4 * (2 * bo + wi);
                x[0] = (i + 0.5) * c.L;
                x[1] = (wi % 2 == 0) ? c.dw : -c.dw;
                x[2] = c.R - c.hw;
                q[0] = 1.0;
                q[1] = q[2] = q[3] = 0.0;
                for (int d = 0; d < 3; ++d) {
                    st->wv[3 * (2 * bo + wi) + d] = 0.0;
                    st->ww[3 * (2 * bo + wi) + d] = 0.0;
                }
                for (int d = 0; d < 9; ++d) st->lam_w[9 * (2 * bo + wi) + d] = 0.0;
            }
        for (int j = 0; j < 6 * (c.B - 1); ++j) st->lam_j[6 * jo + j] = 0.0;
        for (int m = 0; m < c.M; ++m) {
            st->p[2 * (mo + m)] = st->p[2 * (mo + m) + 1] = 0.0;
            st->cmd[mo + m] = 0.0;
        }
        st->residual[s] = 0.0;
        st->iters[s] = 0;
        st->status[s] = 0;
        st->iters_total[s] = 0;
        st->step[s] = 0;
        bo += c.B;
        jo += c.B - 1;
        mo += c.M;
    }
}

/* a wheel carriage's bodies in one array: segments, then wheels */
static double* join_bodies(const double* seg, const double* whl, int B, int k)
{
    double* o = (double*)malloc(sizeof(double) * (size_t)(3 * B * k));
    memcpy(o, seg, sizeof(double) * (size_t)(B * k));
    memcpy(o + (size_t)B * k, whl, sizeof(double) * (size_t)(2 * B * k));
    return o;
}

static void split_bodies(double* o, double* seg, double* whl, int B, int k)
{
    memcpy(seg, o, sizeof(double) * (size_t)(B * k));
    memcpy(whl, o + (size_t)B * k, sizeof(double) * (size_t)(2 * B * k));
    free(o);
}

int orc_run(const orc_batch* b, orc_state* st, int32_t s0, int32_t s1, int32_t n_steps)
{
    if ((b->flags & ORC_FLAG_WHEELS) &&
        (b->solver != ORC_SOLVER_JACOBI || b->warm != ORC_WARM_ZERO || !st->wx || !st->lam_w))
        return -1;
    int64_t bo, jo, mo;
    offsets_of(b, s0, &bo, &jo, &mo);
    for (int s = s0; s < s1; ++s) {
        snake_ctx c;
        make_ctx(b, s, &c);
        scratch_t W;
        scratch_alloc(&W, &c);
        double* x = st->x + 3 * bo;
        double* q = st->q + 4 * bo;
        double* v = st->v + 3 * bo;
        double* w = st->w + 3 * bo;
        double* p = st->p + 2 * mo;
        double* cmd = st->cmd + mo;
        double* lj = st->lam_j + 6 * jo;
        double* lc = st->lam_c + 3 * bo;
        if (c.wheels) {
            x = join_bodies(x, st->wx + 6 * bo, c.B, 3);
            q = join_bodies(q, st->wq + 8 * bo, c.B, 4);
            v = join_bodies(v, st->wv + 6 * bo, c.B, 3);
            w = join_bodies(w, st->ww + 6 * bo, c.B, 3);
            lc = st->lam_w + 18 * bo;
            c.anchor = W.anc;
        }
        for (int n = 0; n < n_steps; ++n) {
            snake_commands(b, s, mo, st->step[s], cmd);
            double rmax = 0.0;
            int it = 0, status = 0;
            if (b->law == ORC_LAW_PAPER)
                for (int m = 0; m < c.M; ++m) {
                    double a = cmd[m];
                    p[2 * m] = paper_update(b, p[2 * m], a > 0.0 ? a : 0.0);
                    p[2 * m + 1] = paper_update(b, p[2 * m + 1], a < 0.0 ? -a : 0.0);
                }
            for (int sub = 0; sub < b->substeps; ++sub) {
                if (b->law == ORC_LAW_LAG)
                    for (int m = 0; m < c.M; ++m) {
                        double a = cmd[m];
                        p[2 * m] = lag_update(p[2 * m], a > 0.0 ? a : 0.0, c.h, b->tau_inf, b->tau_def);
                        p[2 * m + 1] =
                            lag_update(p[2 * m + 1], a < 0.0 ? -a : 0.0, c.h, b->tau_inf, b->tau_def);
                    }
                for (int j = 0; j < c.nj; ++j) W.theta0[j] = rest_angle(b, &c, p, j);
                memcpy(W.xp, x, sizeof(double) * 3 * (size_t)c.NB);
                memcpy(W.qp, q, sizeof(double) * 4 * (size_t)c.NB);
                if (c.wheels) wheel_anchors(&c, W.xp, W.qp, W.anc);
                predict(&c, x, q, v, w);
                double r;
                it += solve_substep(b, &c, &W, x, q, lj, lc, b->warm, b->iters, b->tol, &r, &status);
                if (r > rmax || r != r) rmax = r;
                finalize(&c, W.xp, W.qp, x, q, v, w);
            }
            st->residual[s] = rmax;
            st->iters[s] = it;
            st->status[s] = status;
            st->iters_total[s] += it;
            st->step[s] += 1;
        }
        if (c.wheels) {
            split_bodies(x, st->x + 3 * bo, st->wx + 6 * bo, c.B, 3);
            split_bodies(q, st->q + 4 * bo, st->wq + 8 * bo, c.B, 4);
            split_bodies(v, st->v + 3 * bo, st->wv + 6 * bo, c.B, 3);
            split_bodies(w, st->w + 3 * bo, st->ww + 6 * bo, c.B, 3);
        }
        scratch_free(&W);
        bo += c.B;
        jo += c.B - 1;
        mo += c.M;
    }
    return 0;
}

void orc_predict_snake(const orc_batch* b, int32_t snake, double* x, double* q, double* v, double* w,
                       double h)
{
    snake_ctx c;
    make_ctx(b, snake, &c);
    c.h = h;
    predict(&c, x, q, v, w);
}

static int assemble(const orc_batch* b, snake_ctx c, const double* x, const double* q, const double* xp,
                    const double* qp, const double* p, double* C, double* J, double* W, double* comp)
{
    int nb = n_blocks(&c);
    int B = c.NB;
    int ncol = 6 * B;
    block_t* blk = (block_t*)calloc((size_t)nb + 1, sizeof(block_t));
    double* th = (double*)calloc((size_t)B, sizeof(double));
    double* anc = (double*)calloc((size_t)c.B * 12 + 1, sizeof(double));
    for (int j = 0; j < c.nj; ++j) th[j] = rest_angle(b, &c, p, j);
    if (c.wheels) {
        wheel_anchors(&c, xp, qp, anc);
        c.anchor = anc;
    }
    eval_blocks(b, &c, x, q, xp, th, blk);
    int rows = 3 * nb;
    memset(J, 0, sizeof(double) * (size_t)rows * (size_t)ncol);
    memset(W, 0, sizeof(double) * (size_t)ncol * (size_t)ncol);
    for (int n = 0; n < nb; ++n)
        for (int r = 0; r < 3; ++r) {
            int row = 3 * n + r;
            C[row] = blk[n].C[r];
            comp[row] = blk[n].comp[r];
            for (int d = 0; d < 6; ++d) {
                J[(size_t)row * ncol + 6 * blk[n].a + d] = blk[n].Ja[6 * r + d];
                if (blk[n].b >= 0) J[(size_t)row * ncol + 6 * blk[n].b + d] = blk[n].Jb[6 * r + d];
            }
        }
    for (int i = 0; i < B; ++i) {
        double Iinv[9];
        inv_inertia_world(&c, i, q + 4 * i, Iinv);
        double wi = inv_mass(&c, i);
        for (int d = 0; d < 3; ++d) {
            W[(size_t)(6 * i + d) * ncol + 6 * i + d] = wi;
            for (int e = 0; e < 3; ++e) W[(size_t)(6 * i + 3 + d) * ncol + 6 * i + 3 + e] = Iinv[3 * d + e];
        }
    }
    free(blk);
    free(th);
    free(anc);
    return rows;
}

int orc_assemble(const orc_batch* b, int32_t snake, const double* x, const double* q,
                 const double* xp, const double* p, double* C, double* J, double* W, double* comp)
{
    snake_ctx c;
    make_ctx(b, snake, &c);
    c.wheels = 0;
    c.NB = c.B;
    return assemble(b, c, x, q, xp, NULL, p, C, J, W, comp);
}

int orc_assemble_wheels(const orc_batch* b, int32_t snake, const double* x, const double* q,
                        const double* xp, const double* qp, const double* p, double* C, double* J,
                        double* W, double* comp)
{
    snake_ctx c;
    make_ctx(b, snake, &c);
    if (!c.wheels) return -1;
    return assemble(b, c, x, q, xp, qp, p, C, J, W, comp);
}

/* ------------------------------------------------------------------ */
/* split substep and the warm-start network's inputs and targets        */
/* ------------------------------------------------------------------ */

/* First half of substep `sub` of snake `snake`: command effects on the
 * chamber pressures (the paper law at sub 0, the lag every substep) and the
 * prediction.  x and q keep the start of the substep; v, w become the
 * predicted velocities and q_pred the predicted orientation. */
void orc_pre_substep(const orc_batch* b, int32_t snake, int32_t sub, const double* x, const double* q,
                     double* v, double* w, double* p, const double* cmd, double* q_pred)
{
    if (b->flags & ORC_FLAG_WHEELS) return;   /* the split substep is the plain chain's */
    snake_ctx c;
    make_ctx(b, snake, &c);
    if (b->law == ORC_LAW_PAPER && sub == 0)
        for (int m = 0; m < c.M; ++m) {
            p[2 * m] = paper_update(b, p[2 * m], cmd[m] > 0.0 ? cmd[m] : 0.0);
            p[2 * m + 1] = paper_update(b, p[2 * m + 1], cmd[m] < 0.0 ? -cmd[m] : 0.0);
        }
    if (b->law == ORC_LAW_LAG)
        for (int m = 0; m < c.M; ++m) {
            double a = cmd[m];
            p[2 * m] = lag_update(p[2 * m], a > 0.0 ? a : 0.0, c.h, b->tau_inf, b->tau_def);
            p[2 * m + 1] = lag_update(p[2 * m + 1], a < 0.0 ? -a : 0.0, c.h, b->tau_inf, b->tau_def);
        }
    double* xt = (double*)malloc(sizeof(double) * 3 * (size_t)c.B);
    memcpy(xt, x, sizeof(double) * 3 * (size_t)c.B);
    memcpy(q_pred, q, sizeof(double) * 4 * (size_t)c.B);
    predict(&c, xt, q_pred, v, w);
    free(xt);
}

/* Second half: multiplier initialisation (the batch's warm mode; GIVEN
 * takes lam_j / lam_c as lambda0), iterations, velocities.  x, q are the
 * start of the substep and become its end. */
void orc_solve_substep(const orc_batch* b, int32_t snake, double* x, double* q, const double* q_pred,
                       double* v, double* w, const double* p, double* lam_j, double* lam_c,
                       double* residual, int32_t* iters, int32_t* status)
{
    if (b->flags & ORC_FLAG_WHEELS) return;   /* the split substep is the plain chain's */
    snake_ctx c;
    make_ctx(b, snake, &c);
    scratch_t W;
    scratch_alloc(&W, &c);
    for (int j = 0; j < c.nj; ++j) W.theta0[j] = rest_angle(b, &c, p, j);
    memcpy(W.xp, x, sizeof(double) * 3 * (size_t)c.B);
    memcpy(W.qp, q, sizeof(double) * 4 * (size_t)c.B);
    for (int i = 0; i < c.B; ++i) {
        if (!is_fixed(&c, i))
            for (int d = 0; d < 3; ++d) x[3 * i + d] += c.h * v[3 * i + d];
    }
    memcpy(q, q_pred, sizeof(double) * 4 * (size_t)c.B);
    double r = 0.0;
    int st = 0;
    int it = solve_substep(b, &c, &W, x, q, lam_j, lam_c, b->warm, b->iters, b->tol, &r, &st);
    finalize(&c, W.xp, W.qp, x, q, v, w);
    *residual = r;
    *iters = it;
    *status = st;
    scratch_free(&W);
}

static void rot_conj(const double* q, const double* v, double* o)
{
    double qc[4], R[9];
    q_conj(q, qc);
    q_to_matrix(qc, R);
    m3_vec(R, v, o);
}

/* Inputs of the network for the joints of one snake, two rows per joint
 * (stretch, then bend-twist), at the predicted state: x start positions,
 * v / w predicted velocities, q_pred predicted orientations.  Vectors are
 * expressed in the predicted axes of the joint's first body. */
void orc_features(const orc_batch* b, int32_t snake, const double* x, const double* v, const double* w,
                  const double* q_pred, const double* p, const double* cmd, const double* lam_j,
                  const double* lam_c, double* feat)
{
    snake_ctx c;
    make_ctx(b, snake, &c);
    const double ref = c.m * 9.81 * c.h * c.h, refb = ref * c.L;
    const double ex[3] = {1.0, 0.0, 0.0}, ez[3] = {0.0, 0.0, 1.0};
    for (int j = 0; j < c.nj; ++j) {
        const int a = j, bb = j + 1;
        const double* qa = q_pred + 4 * a;
        const double* qb = q_pred + 4 * bb;
        double Ra[9], Rb[9], ra[3], rb[3], xa[3], xb[3];
        q_to_matrix(qa, Ra);
        q_to_matrix(qb, Rb);
        m3_vec(Ra, ex, ra);
        m3_vec(Rb, ex, rb);
        for (int d = 0; d < 3; ++d) {
            ra[d] *= 0.5 * c.L;
            rb[d] *= -0.5 * c.L;
            xa[d] = x[3 * a + d] + c.h * v[3 * a + d];
            xb[d] = x[3 * bb + d] + c.h * v[3 * bb + d];
        }
        double f[32], t[3], u[3];
        for (int d = 0; d < 3; ++d) t[d] = ((xa[d] + ra[d]) - (xb[d] + rb[d])) / c.L;
        rot_conj(qa, t, f);
        /* bend-twist value at the predicted state */
        double th0 = rest_angle(b, &c, p, j);
        double q0[4] = {cos(0.5 * th0), 0.0, 0.0, sin(0.5 * th0)}, q0c[4], qac[4], tt[4], e[4];
        q_conj(q0, q0c);
        q_conj(qa, qac);
        q_mul(q0c, qac, tt);
        q_mul(tt, qb, e);
        if (e[0] < 0.0)
            for (int d = 0; d < 4; ++d) e[d] = -e[d];
        for (int d = 0; d < 3; ++d) f[3 + d] = 2.0 * e[1 + d];
        /* velocity of the A end point relative to the B start point, times h/L */
        double wa_r[3], wb_r[3];
        cross3(w + 3 * a, ra, wa_r);
        cross3(w + 3 * bb, rb, wb_r);
        for (int d = 0; d < 3; ++d)
            t[d] = ((v[3 * a + d] + wa_r[d]) - (v[3 * bb + d] + wb_r[d])) * c.h / c.L;
        rot_conj(qa, t, f + 6);
        for (int d = 0; d < 3; ++d) t[d] = (w[3 * bb + d] - w[3 * a + d]) * c.h;
        rot_conj(qa, t, f + 9);
        rot_conj(qa, ez, f + 12);
        const int m = j / c.S;
        f[15] = p[2 * m];
        f[16] = p[2 * m + 1];
        f[17] = cmd[m];
        f[18] = th0;
        double hh = c.h * c.h;
        f[22] = log10(fmax(c.a_s / hh, 1e-30));
        f[23] = log10(fmax(c.a_b / hh, 1e-30));
        f[24] = log10(fmax(c.a_t / hh, 1e-30));
        f[25] = c.mu;
        f[26] = lam_c[3 * a] / ref;
        f[27] = lam_c[3 * bb] / ref;
        f[28] = (xa[2] - c.R) / c.L;
        f[29] = (xb[2] - c.R) / c.L;
        f[31] = c.B > 1 ? (double)j / (double)(c.B - 1) : 0.0;
        for (int d = 0; d < 3; ++d) t[d] = lam_j[6 * j + d] / ref;
        rot_conj(qa, t, u);
        f[19] = u[0];
        f[20] = u[1];
        f[21] = u[2];
        f[30] = 0.0;
        memcpy(feat + 64 * j, f, sizeof f);
        for (int d = 0; d < 3; ++d) f[19 + d] = lam_j[6 * j + 3 + d] / refb;
        f[30] = 1.0;
        memcpy(feat + 64 * j + 32, f, sizeof f);
    }
}

/* Network targets from final multipliers: stretch in the predicted axes of
 * the joint's first body over m g h^2, bend-twist over m g h^2 L. */
void orc_targets(const orc_batch* b, int32_t snake, const double* q_pred, const double* lam_j, double* tgt)
{
    snake_ctx c;
    make_ctx(b, snake, &c);
    const double ref = c.m * 9.81 * c.h * c.h, refb = ref * c.L;
    for (int j = 0; j < c.nj; ++j) {
        double t[3];
        for (int d = 0; d < 3; ++d) t[d] = lam_j[6 * j + d] / ref;
        rot_conj(q_pred + 4 * j, t, tgt + 6 * j);
        for (int d = 0; d < 3; ++d) tgt[6 * j + 3 + d] = lam_j[6 * j + 3 + d] / refb;
    }
}

/* ------------------------------------------------------------------ */
/* index work                                                           */
/* ------------------------------------------------------------------ */

static const int32_t* g_sort_B;

static int cmp_work(const void* pa, const void* pb)
{
    int32_t a = *(const int32_t*)pa, b = *(const int32_t*)pb;
    if (g_sort_B[a] != g_sort_B[b]) return g_sort_B[a] > g_sort_B[b] ? -1 : 1;
    return (a > b) - (a < b);
}

void orc_index(const orc_batch* b, int32_t* blk_type, int32_t* blk_a, int32_t* blk_b,
               int32_t* blk_color, int32_t* body_degree_out, int32_t* bucket, int32_t* order)
{
    int ground = (b->flags & ORC_FLAG_NO_GROUND) ? 0 : 1;
    int64_t n = 0, bo = 0;
    int64_t nbody = 0;
    for (int s = 0; s < b->n_snakes; ++s) nbody += (int64_t)b->n_modules[s] * b->segs[s];
    /* colours already taken by coloured blocks on each body (at most 5) */
    int32_t* used = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nbody * 5 + 1));
    int32_t* nused = (int32_t*)calloc((size_t)nbody + 1, sizeof(int32_t));
    int32_t* Bs = (int32_t*)malloc(sizeof(int32_t) * (size_t)(b->n_snakes + 1));
    for (int s = 0; s < b->n_snakes; ++s) {
        int B = b->n_modules[s] * b->segs[s];
        Bs[s] = B;
        for (int j = 0; j < B - 1; ++j)
            for (int t = 0; t < 2; ++t) {
                blk_type[n] = t;
                blk_a[n] = (int32_t)(bo + j);
                blk_b[n] = (int32_t)(bo + j + 1);
                ++n;
            }
        if (ground)
            for (int i = 0; i < B; ++i) {
                blk_type[n] = 2;
                blk_a[n] = (int32_t)(bo + i);
                blk_b[n] = -1;
                ++n;
            }
        for (int i = 0; i < B; ++i) body_degree_out[bo + i] = body_degree(i, B, ground);
        int bk = 0;
        while ((1 << bk) < B) ++bk;
        bucket[s] = bk;
        bo += B;
    }
    /* sequential greedy colouring in block-list order: the smallest colour
     * not already taken by an earlier block that shares a body */
    for (int64_t k = 0; k < n; ++k) {
        int32_t bodies[2] = {blk_a[k], blk_b[k]};
        int col = 0;
        for (;;) {
            int clash = 0;
            for (int e = 0; e < 2 && !clash; ++e) {
                if (bodies[e] < 0) continue;
                for (int u = 0; u < nused[bodies[e]]; ++u)
                    if (used[5 * bodies[e] + u] == col) {
                        clash = 1;
                        break;
                    }
            }
            if (!clash) break;
            ++col;
        }
        blk_color[k] = col;
        for (int e = 0; e < 2; ++e)
            if (bodies[e] >= 0) used[5 * bodies[e] + nused[bodies[e]]++] = col;
    }
    /* work order: cost (bodies) descending, snake id ascending */
    for (int s = 0; s < b->n_snakes; ++s) order[s] = s;
    g_sort_B = Bs;
    qsort(order, (size_t)b->n_snakes, sizeof(int32_t), cmp_work);
    g_sort_B = NULL;
    free(used);
    free(nused);
    free(Bs);
}
