/*
 * FP64 oracle of the full-resolution soft link (sections "Particles",
 * "Tetrahedral Finite-Elements" and "Soft robotic snake model").
 * TEST INFRASTRUCTURE ONLY, like the rest of this folder; shares nothing
 * with the GPU library.
 *
 * A snake is n_links soft links joined end to end by rigid frames (n_links
 * + 1 of them).  A link is a tetrahedral particle mesh (section "Particles":
 * lumped masses, each particle a share of its elements' mass; section
 * "Soft robotic snake model": a radially symmetric mesh in cross-sections
 * along the link), held by
 *   - corotational constant-strain tetrahedra with the element compliance
 *     E_tetra (section "Tetrahedral Finite-Elements");
 *   - distance constraints along the link between the particles of
 *     neighbouring cross-sections and from each section's centre to its
 *     ring: the inextensible centre layer (the particles in the plane
 *     between the chambers) and the radial reinforcement are the paper's
 *     non-deformable constraints, given one small compliance
 *     (rigid_compliance, also on the attachments): with zero compliance
 *     the straight parallel lines of these rows between two frames repeat
 *     one another and the compliant system is singular;
 *   - actuation: the axial distance constraints of the commanded chamber
 *     take the rest length r eps(p), eps(p) = 1 + P / Y (eq. expansion),
 *     and only that chamber's constraints act ("only one chamber on the
 *     link is active at a time");
 *   - attachments of the end sections' particles to the frames
 *     (eq. rigid_to_particle);
 *   - ground contact of every particle with Coulomb friction (the contact
 *     and friction cone of section "Simulator").
 * Time stepping is the chain solver's: chamber pressures by a first-order
 * lag per substep, prediction, then block-Jacobi iterations on the compliant
 * system (linearisation eq. schur_system): every block takes its local
 * solution  -(K + E/h^2)^-1 (C + E/h^2 lambda)  at the current iterate
 * (K = J W J^T), scaled by relax / (the largest number of blocks on one of
 * its bodies), and the bodies gather W J^T (scaled increment) in the fixed
 * block order: tetrahedra, distance constraints, attachments (each link in
 * turn), then contacts.  The rotation of a tetrahedron's polar
 * decomposition is taken at the current iterate and held in its Jacobian.
 * Every quantity is double.
 *
 * Layout: array-of-structures; particles p = (snake * n_links + link) *
 * per_link + local, local = section * (ring + 1) + slot (slot 0 the centre,
 * slot 1 + k ring particle k at angle 2 pi k / ring); frames f = snake *
 * (n_links + 1) + junction.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int fem_tet_rest(const double* X, double* Dm_inv, double* volume);
int fem_tet_eval(const double* Dm_inv, const double* x, double* R, int rot_in, double* C, double* J);
void fem_tet_compliance(double V, double Y, double nu, double* E);
double fem_expansion(double p, double Y);
double fem_dist_eval(const double* xi, const double* xj, double r, double p, double Y, double* J);
void fem_attach_eval(const double* x, const double* q, const double* r, const double* xp, double* C, double* J);

#define LNK_FIXED_FRAME0 1
#define LNK_NO_GROUND 2
#define LNK_LINEARISED 8

#define LNK_CENTRE 0    /* inextensible centre layer (rigid)        */
#define LNK_RADIAL 1    /* radial reinforcement (rigid)             */
#define LNK_CHAMBER0 2  /* actuation, chamber 0 (side +y)           */
#define LNK_CHAMBER1 3  /* actuation, chamber 1 (side -y)           */

#define LNK_STATUS_NONFINITE 1
#define LNK_STATUS_NOT_CONVERGED 2

typedef struct {
    int32_t n_snakes, n_links;
    int32_t sections, ring, n_tets;   /* mesh of one link */
    const double* X;                  /* [per_link][3] rest positions, link frame, x along the link */
    const int32_t* tets;              /* [n_tets][4] positively oriented */
    const double* mu;                 /* [n_snakes] */
    double link_length, radius;       /* the mesh spans x in [0, link_length]; the axis rests at z = radius */
    double young, poisson, density, p_max;
    double frame_mass, frame_length;  /* frame: solid cylinder along x of radius `radius` */
    double gravity, dt;
    int32_t substeps, iters;
    double tol, relax, tau_inf, tau_def;
    double rigid_compliance;          /* m/N of the distance and attachment rows */
    int32_t flags;
} lnk_batch;

typedef struct {
    double *x, *v;             /* particles [P][3] */
    double *fx, *fq, *fv, *fw; /* frames [F][3], [F][4] (w,x,y,z), [F][3], [F][3] */
    double *p;                 /* [snakes*links][2] chamber pressures, fraction of full */
    double* cmd;               /* [snakes*links] signed command in [-1, 1] */
    double* lam_tet;           /* [T][6] */
    double* lam_dist;          /* [D] */
    double* lam_att;           /* [A][3] */
    double* lam_c;             /* [P][3] normal, tangential x, y */
    double* residual;          /* [snakes] */
    int32_t *iters, *status;   /* [snakes] */
} lnk_state;

/* ---------------------------------------------------------------- topology */

static int per_link(const lnk_batch* b) { return b->sections * (b->ring + 1); }

/* kind of the axial edge of ring slot `slot` (0 centre, 1 + k ring particle k):
 * the centre and the ring particles in the plane y = 0 belong to the
 * inextensible layer, those with y > 0 to chamber 0, y < 0 to chamber 1;
 * decided on the integer angle index (ring a multiple of 4). */
static int axial_kind(int ring, int slot)
{
    if (slot == 0) return LNK_CENTRE;
    int k = slot - 1, q = ring / 4;
    if (k == q || k == 3 * q) return LNK_CENTRE;
    return (k < q || k > 3 * q) ? LNK_CHAMBER0 : LNK_CHAMBER1;
}

int lnk_dist_per_link(const lnk_batch* b) { return (b->sections - 1) * (b->ring + 1) + (b->sections - 2) * b->ring; }
int lnk_att_per_link(const lnk_batch* b) { return 2 * (b->ring + 1); }

/* Distance constraints of one link in their fixed order (local particle
 * indices): the axial edges gap by gap, slot by slot; then the radial
 * spokes section by section, ring particle by ring particle.  The two end
 * sections carry no spokes: their particles are attached to a rigid frame,
 * which already holds their distances (rigid spokes there would repeat
 * those rows and leave the compliant system singular). */
void lnk_link_dists(const lnk_batch* b, int32_t* pi, int32_t* pj, int32_t* kind, double* rest)
{
    const int n = b->ring + 1;
    int c = 0;
    for (int g = 0; g + 1 < b->sections; ++g)
        for (int s = 0; s < n; ++s, ++c) {
            pi[c] = g * n + s;
            pj[c] = (g + 1) * n + s;
            kind[c] = axial_kind(b->ring, s);
        }
    for (int g = 1; g + 1 < b->sections; ++g)
        for (int k = 0; k < b->ring; ++k, ++c) {
            pi[c] = g * n;
            pj[c] = g * n + 1 + k;
            kind[c] = LNK_RADIAL;
        }
    for (int i = 0; i < c; ++i) {
        const double* a = b->X + 3 * pi[i];
        const double* d = b->X + 3 * pj[i];
        rest[i] = sqrt((a[0] - d[0]) * (a[0] - d[0]) + (a[1] - d[1]) * (a[1] - d[1]) + (a[2] - d[2]) * (a[2] - d[2]));
    }
}

/* Attachments of one link: section 0's particles to frame `link`, the last
 * section's to frame `link + 1` (frame offsets 0 and 1 in `side`). */
void lnk_link_atts(const lnk_batch* b, int32_t* part, int32_t* side)
{
    const int n = b->ring + 1;
    for (int s = 0; s < n; ++s) {
        part[s] = s;
        side[s] = 0;
        part[n + s] = (b->sections - 1) * n + s;
        side[n + s] = 1;
    }
}

/* Lumped particle masses of one link: each particle a quarter of the mass
 * of every element it belongs to (elements in order).  Returns -1 for a
 * degenerate element. */
int lnk_link_masses(const lnk_batch* b, double* m)
{
    const int P = per_link(b);
    for (int i = 0; i < P; ++i) m[i] = 0.0;
    for (int t = 0; t < b->n_tets; ++t) {
        double X[12], Di[9], V;
        for (int k = 0; k < 4; ++k)
            for (int c = 0; c < 3; ++c) X[3 * k + c] = b->X[3 * b->tets[4 * t + k] + c];
        if (fem_tet_rest(X, Di, &V) != 0) return -1;
        for (int k = 0; k < 4; ++k) m[b->tets[4 * t + k]] += 0.25 * b->density * V;
    }
    return 0;
}

/* Structural degree of every particle and frame of one snake: the number
 * of blocks touching it (both chambers' actuation counted; contact counted
 * with ground). */
static void degrees(const lnk_batch* b, const int32_t* di, const int32_t* dj, const int32_t* ap,
                    const int32_t* as, int* dp, int* df)
{
    const int P = per_link(b), L = b->n_links, ND = lnk_dist_per_link(b), NA = lnk_att_per_link(b);
    const int ground = (b->flags & LNK_NO_GROUND) ? 0 : 1;
    for (int i = 0; i < L * P; ++i) dp[i] = ground;
    for (int f = 0; f <= L; ++f) df[f] = 0;
    for (int l = 0; l < L; ++l) {
        for (int t = 0; t < b->n_tets; ++t)
            for (int k = 0; k < 4; ++k) dp[l * P + b->tets[4 * t + k]] += 1;
        for (int d = 0; d < ND; ++d) {
            dp[l * P + di[d]] += 1;
            dp[l * P + dj[d]] += 1;
        }
        for (int a = 0; a < NA; ++a) {
            dp[l * P + ap[a]] += 1;
            df[l + as[a]] += 1;
        }
    }
}

/* Index work of one snake for the bit-exact comparison: particle and frame
 * degrees and the distance constraints' particle pairs and kinds (snake-local). */
void lnk_index(const lnk_batch* b, int32_t* deg_p, int32_t* deg_f, int32_t* dpi, int32_t* dpj, int32_t* dkind)
{
    const int P = per_link(b), ND = lnk_dist_per_link(b), NA = lnk_att_per_link(b);
    int32_t* di = malloc(sizeof(int32_t) * ND);
    int32_t* dj = malloc(sizeof(int32_t) * ND);
    int32_t* dk = malloc(sizeof(int32_t) * ND);
    double* dr = malloc(sizeof(double) * ND);
    int32_t* ap = malloc(sizeof(int32_t) * NA);
    int32_t* as = malloc(sizeof(int32_t) * NA);
    lnk_link_dists(b, di, dj, dk, dr);
    lnk_link_atts(b, ap, as);
    int* dp = malloc(sizeof(int) * b->n_links * P);
    int* df = malloc(sizeof(int) * (b->n_links + 1));
    degrees(b, di, dj, ap, as, dp, df);
    for (int i = 0; i < b->n_links * P; ++i) deg_p[i] = dp[i];
    for (int f = 0; f <= b->n_links; ++f) deg_f[f] = df[f];
    for (int l = 0; l < b->n_links; ++l)
        for (int d = 0; d < ND; ++d) {
            dpi[l * ND + d] = l * P + di[d];
            dpj[l * ND + d] = l * P + dj[d];
            dkind[l * ND + d] = dk[d];
        }
    free(di), free(dj), free(dk), free(dr), free(ap), free(as), free(dp), free(df);
}

/* ---------------------------------------------------------------- rigid frame helpers */

static void q_mul(const double* a, const double* b, double* o)
{
    o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    o[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    o[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

static void q_normalize(double* q)
{
    double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; ++k) q[k] /= n;
}

/* q <- normalize(q + 1/2 [0, th] (x) q) */
static void q_turn(double* q, const double* th)
{
    const double e[4] = {0.0, th[0], th[1], th[2]};
    double d[4];
    q_mul(e, q, d);
    for (int k = 0; k < 4; ++k) q[k] += 0.5 * d[k];
    q_normalize(q);
}

static void q_matrix(const double* q, double* R)
{
    const double w = q[0], a = q[1], b = q[2], c = q[3];
    R[0] = 1 - 2 * (b * b + c * c), R[1] = 2 * (a * b - w * c), R[2] = 2 * (a * c + w * b);
    R[3] = 2 * (a * b + w * c), R[4] = 1 - 2 * (a * a + c * c), R[5] = 2 * (b * c - w * a);
    R[6] = 2 * (a * c - w * b), R[7] = 2 * (b * c + w * a), R[8] = 1 - 2 * (a * a + b * b);
}

/* world inverse inertia R diag(1/I) R^T of a frame (solid cylinder along body x) */
static void frame_inv_inertia(const lnk_batch* b, const double* q, double* Iinv)
{
    const double m = b->frame_mass, R = b->radius, L = b->frame_length;
    const double d[3] = {2.0 / (m * R * R), 12.0 / (m * (3 * R * R + L * L)), 12.0 / (m * (3 * R * R + L * L))};
    double Rm[9];
    q_matrix(q, Rm);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += Rm[3 * i + k] * d[k] * Rm[3 * j + k];
            Iinv[3 * i + j] = s;
        }
}

static void frame_inertia(const lnk_batch* b, const double* q, double* I)
{
    const double m = b->frame_mass, R = b->radius, L = b->frame_length;
    const double d[3] = {0.5 * m * R * R, m * (3 * R * R + L * L) / 12.0, m * (3 * R * R + L * L) / 12.0};
    double Rm[9];
    q_matrix(q, Rm);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += Rm[3 * i + k] * d[k] * Rm[3 * j + k];
            I[3 * i + j] = s;
        }
}

/* solve the n x n system A x = r (A row-major, overwritten) by Gaussian
 * elimination with partial pivoting */
static void solve_n(int n, double* A, double* r, double* x)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int i = c + 1; i < n; ++i)
            if (fabs(A[n * i + c]) > fabs(A[n * piv + c])) piv = i;
        if (piv != c) {
            for (int k = 0; k < n; ++k) {
                double t = A[n * c + k];
                A[n * c + k] = A[n * piv + k];
                A[n * piv + k] = t;
            }
            double t = r[c];
            r[c] = r[piv];
            r[piv] = t;
        }
        for (int i = c + 1; i < n; ++i) {
            double f = A[n * i + c] / A[n * c + c];
            for (int k = c; k < n; ++k) A[n * i + k] -= f * A[n * c + k];
            r[i] -= f * r[c];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = r[i];
        for (int k = i + 1; k < n; ++k) s -= A[n * i + k] * x[k];
        x[i] = s / A[n * i + i];
    }
}

/* ---------------------------------------------------------------- one snake */

typedef struct {
    const lnk_batch* b;
    int P, F, T, D, A, NP;          /* per snake: particles, frames, tets, dists, atts */
    int P1, ND1, NA1;               /* per link */
    int ground, fixed0, linear;
    double h, Lref;
    /* per link, local */
    int32_t *di, *dj, *dk, *ap, *as;
    double *drest, *mass1;
    double *Dm_inv, *vol;           /* per mesh tet */
    int *dp, *df;                   /* snake degrees */
} ctx_t;

static void ctx_init(const lnk_batch* b, ctx_t* c)
{
    memset(c, 0, sizeof *c);
    c->b = b;
    c->P1 = per_link(b);
    c->ND1 = lnk_dist_per_link(b);
    c->NA1 = lnk_att_per_link(b);
    c->P = b->n_links * c->P1;
    c->F = b->n_links + 1;
    c->T = b->n_links * b->n_tets;
    c->D = b->n_links * c->ND1;
    c->A = b->n_links * c->NA1;
    c->ground = (b->flags & LNK_NO_GROUND) ? 0 : 1;
    c->fixed0 = (b->flags & LNK_FIXED_FRAME0) ? 1 : 0;
    c->linear = (b->flags & LNK_LINEARISED) ? 1 : 0;
    c->h = b->dt / b->substeps;
    c->Lref = b->link_length / (b->sections - 1);
    c->di = malloc(sizeof(int32_t) * c->ND1);
    c->dj = malloc(sizeof(int32_t) * c->ND1);
    c->dk = malloc(sizeof(int32_t) * c->ND1);
    c->drest = malloc(sizeof(double) * c->ND1);
    c->ap = malloc(sizeof(int32_t) * c->NA1);
    c->as = malloc(sizeof(int32_t) * c->NA1);
    c->mass1 = malloc(sizeof(double) * c->P1);
    c->Dm_inv = malloc(sizeof(double) * 9 * b->n_tets);
    c->vol = malloc(sizeof(double) * b->n_tets);
    c->dp = malloc(sizeof(int) * c->P);
    c->df = malloc(sizeof(int) * c->F);
    lnk_link_dists(b, c->di, c->dj, c->dk, c->drest);
    lnk_link_atts(b, c->ap, c->as);
    lnk_link_masses(b, c->mass1);
    for (int t = 0; t < b->n_tets; ++t) {
        double X[12];
        for (int k = 0; k < 4; ++k)
            for (int q = 0; q < 3; ++q) X[3 * k + q] = b->X[3 * b->tets[4 * t + k] + q];
        fem_tet_rest(X, c->Dm_inv + 9 * t, c->vol + t);
    }
    degrees(b, c->di, c->dj, c->ap, c->as, c->dp, c->df);
}

static void ctx_free(ctx_t* c)
{
    free(c->di), free(c->dj), free(c->dk), free(c->drest), free(c->ap), free(c->as);
    free(c->mass1), free(c->Dm_inv), free(c->vol), free(c->dp), free(c->df);
}

static double pmass(const ctx_t* c, int i) { return c->mass1[i % c->P1]; }
static int frame_fixed(const ctx_t* c, int f) { return c->fixed0 && f == 0; }

/* rest position of particle i (snake-local) and frame f in the world */
void lnk_rest_particle(const lnk_batch* b, int i, double* x)
{
    const int P1 = per_link(b), l = i / P1, k = i % P1;
    x[0] = b->X[3 * k] + l * b->link_length;
    x[1] = b->X[3 * k + 1];
    x[2] = b->X[3 * k + 2] + b->radius;
}

static void rest_frame(const lnk_batch* b, int f, double* x)
{
    x[0] = f * b->link_length;
    x[1] = 0.0;
    x[2] = b->radius;
}

/* attachment point of attachment a (link-local index) in its frame's body
 * frame: the particle's rest position relative to the frame's */
static void att_point(const ctx_t* c, int l, int a, double* r)
{
    double xp[3], xf[3];
    lnk_rest_particle(c->b, l * c->P1 + c->ap[a], xp);
    rest_frame(c->b, l + c->as[a], xf);
    for (int k = 0; k < 3; ++k) r[k] = xp[k] - xf[k];
}

/* The snake's working set for one substep.  Body iterate: particles x, frames
 * (fx, fq); in linearised mode the accumulated displacement (particles 3,
 * frames 6) from the predicted state with every block's value and Jacobian
 * frozen there. */
typedef struct {
    double *x, *xp;       /* particles: iterate, start of substep */
    double *fx, *fq, *fxp, *fqp;
    double *xt, *fxt, *fqt; /* predicted state (linearised mode) */
    double *acc, *facc;   /* linearised displacements */
    double *C0, *J0, *R0; /* frozen values / Jacobians (linearised) */
    double *dl_tet, *dl_dist, *dl_att, *dl_c; /* scaled increments of the iteration */
    double *imp_tet;      /* [T][12] impulses J^T dl per vertex */
    double *imp_att;      /* [A][9] (frame force, frame torque, particle force) */
    double *imp_dist;     /* [D][3] force on particle i (j takes the negative) */
} work_t;

/* Evaluate every block at the current iterate and return the snake
 * residual; with `apply` also compute the scaled increments and impulses. */
static double eval_blocks(const ctx_t* c, const lnk_state* st, int s, work_t* w, const double* cmd_l,
                          const double* p_l, int apply)
{
    const lnk_batch* b = c->b;
    const double h2 = c->h * c->h;
    double res = 0.0;
    double E[36];
    /* tetrahedra */
    for (int l = 0; l < b->n_links; ++l)
        for (int t = 0; t < b->n_tets; ++t) {
            const int T = l * b->n_tets + t, g = s * c->T + T;
            const int32_t* v = b->tets + 4 * t;
            double xv[12], C[6], J[72], R[9];
            for (int k = 0; k < 4; ++k)
                for (int q = 0; q < 3; ++q) xv[3 * k + q] = w->x[3 * (l * c->P1 + v[k]) + q];
            if (c->linear) {
                memcpy(J, w->J0 + 72 * (size_t)T, sizeof J);
                for (int r = 0; r < 6; ++r) {
                    double sacc = w->C0[6 * (size_t)T + r];
                    for (int k = 0; k < 4; ++k)
                        for (int q = 0; q < 3; ++q) sacc += J[12 * r + 3 * k + q] * w->acc[3 * (l * c->P1 + v[k]) + q];
                    C[r] = sacc;
                }
            } else if (fem_tet_eval(c->Dm_inv + 9 * t, xv, R, 0, C, J) != 0) {
                return INFINITY;
            }
            fem_tet_compliance(c->vol[t], b->young, b->poisson, E);
            const double* lam = st->lam_tet + 6 * (size_t)g;
            double K[36], rhs[6], dl[6];
            for (int r = 0; r < 6; ++r) {
                double a = C[r];
                for (int q = 0; q < 6; ++q) a += E[6 * r + q] / h2 * lam[q];
                rhs[r] = -a;
                res = fmax(res, fabs(a));
                for (int q = 0; q < 6; ++q) {
                    double sacc = E[6 * r + q] / h2;
                    for (int k = 0; k < 4; ++k) {
                        const double wi = 1.0 / pmass(c, v[k]);
                        for (int z = 0; z < 3; ++z) sacc += J[12 * r + 3 * k + z] * wi * J[12 * q + 3 * k + z];
                    }
                    K[6 * r + q] = sacc;
                }
            }
            if (!apply) continue;
            solve_n(6, K, rhs, dl);
            int dmax = 0;
            for (int k = 0; k < 4; ++k) dmax = c->dp[l * c->P1 + v[k]] > dmax ? c->dp[l * c->P1 + v[k]] : dmax;
            const double sc = b->relax / dmax;
            for (int r = 0; r < 6; ++r) w->dl_tet[6 * T + r] = sc * dl[r];
            for (int k = 0; k < 4; ++k)
                for (int z = 0; z < 3; ++z) {
                    double sacc = 0.0;
                    for (int r = 0; r < 6; ++r) sacc += J[12 * r + 3 * k + z] * w->dl_tet[6 * T + r];
                    w->imp_tet[12 * (size_t)T + 3 * k + z] = sacc;
                }
        }
    /* distance constraints */
    for (int l = 0; l < b->n_links; ++l) {
        const double u0 = cmd_l[l] > 0.0 ? cmd_l[l] : 0.0, u1 = cmd_l[l] < 0.0 ? -cmd_l[l] : 0.0;
        for (int d = 0; d < c->ND1; ++d) {
            const int D = l * c->ND1 + d;
            const int i = l * c->P1 + c->di[d], j = l * c->P1 + c->dj[d];
            const int kind = c->dk[d];
            double Jd[6], Cd, rest = c->drest[d], press = 0.0;
            w->dl_dist[D] = 0.0;
            for (int z = 0; z < 3; ++z) w->imp_dist[3 * D + z] = 0.0;
            if ((kind == LNK_CHAMBER0 && !(u0 > 0.0)) || (kind == LNK_CHAMBER1 && !(u1 > 0.0))) continue;
            if (kind == LNK_CHAMBER0) press = p_l[2 * l] * b->p_max;
            if (kind == LNK_CHAMBER1) press = p_l[2 * l + 1] * b->p_max;
            if (c->linear) {
                memcpy(Jd, w->J0 + 72 * (size_t)c->T + 6 * (size_t)D, sizeof Jd);
                Cd = w->C0[6 * (size_t)c->T + D];
                for (int z = 0; z < 3; ++z) Cd += Jd[z] * w->acc[3 * i + z] + Jd[3 + z] * w->acc[3 * j + z];
            } else {
                Cd = fem_dist_eval(w->x + 3 * i, w->x + 3 * j, rest, press, b->young, Jd);
            }
            const double at = b->rigid_compliance / h2, ld = st->lam_dist[(size_t)s * c->D + D];
            res = fmax(res, fabs(Cd + at * ld) / c->Lref);
            if (!apply) continue;
            const double K = 1.0 / pmass(c, i) + 1.0 / pmass(c, j) + at;
            const int dmax = c->dp[i] > c->dp[j] ? c->dp[i] : c->dp[j];
            const double dl = b->relax / dmax * (-(Cd + at * ld) / K);
            w->dl_dist[D] = dl;
            for (int z = 0; z < 3; ++z) w->imp_dist[3 * D + z] = Jd[z] * dl;
        }
    }
    /* attachments */
    for (int l = 0; l < b->n_links; ++l)
        for (int a = 0; a < c->NA1; ++a) {
            const int A = l * c->NA1 + a, i = l * c->P1 + c->ap[a], f = l + c->as[a];
            const int g = s * c->A + A;
            double r[3], Ca[3], Ja[27];
            att_point(c, l, a, r);
            if (c->linear) {
                memcpy(Ja, w->J0 + 72 * (size_t)c->T + 6 * (size_t)c->D + 27 * (size_t)A, sizeof Ja);
                for (int q = 0; q < 3; ++q) {
                    double sacc = w->C0[6 * (size_t)c->T + c->D + 3 * A + q];
                    for (int z = 0; z < 3; ++z)
                        sacc += Ja[9 * q + z] * w->facc[6 * f + z] + Ja[9 * q + 3 + z] * w->facc[6 * f + 3 + z] +
                                Ja[9 * q + 6 + z] * w->acc[3 * i + z];
                    Ca[q] = sacc;
                }
            } else {
                fem_attach_eval(w->fx + 3 * f, w->fq + 4 * f, r, w->x + 3 * i, Ca, Ja);
            }
            const double at = b->rigid_compliance / h2;
            const double* la = st->lam_att + 3 * (size_t)g;
            for (int q = 0; q < 3; ++q) res = fmax(res, fabs(Ca[q] + at * la[q]) / c->Lref);
            if (!apply) continue;
            double K[9], Iinv[9], rhs[3], dl[3];
            const double wf = frame_fixed(c, f) ? 0.0 : 1.0 / b->frame_mass;
            if (frame_fixed(c, f))
                memset(Iinv, 0, sizeof Iinv);
            else
                frame_inv_inertia(b, c->linear ? w->fqt + 4 * f : w->fq + 4 * f, Iinv);
            const double wp = 1.0 / pmass(c, i);
            for (int q = 0; q < 3; ++q) {
                rhs[q] = -(Ca[q] + at * la[q]);
                for (int e = 0; e < 3; ++e) {
                    double sacc = q == e ? at : 0.0;
                    for (int z = 0; z < 3; ++z) {
                        sacc += Ja[9 * q + z] * wf * Ja[9 * e + z];
                        sacc += Ja[9 * q + 6 + z] * wp * Ja[9 * e + 6 + z];
                        for (int y = 0; y < 3; ++y) sacc += Ja[9 * q + 3 + z] * Iinv[3 * z + y] * Ja[9 * e + 3 + y];
                    }
                    K[3 * q + e] = sacc;
                }
            }
            solve_n(3, K, rhs, dl);
            const int dmax = c->dp[i] > c->df[f] ? c->dp[i] : c->df[f];
            const double sc = b->relax / dmax;
            for (int q = 0; q < 3; ++q) w->dl_att[3 * A + q] = sc * dl[q];
            for (int z = 0; z < 9; ++z) {
                double sacc = 0.0;
                for (int q = 0; q < 3; ++q) sacc += Ja[9 * q + z] * w->dl_att[3 * A + q];
                w->imp_att[9 * A + z] = sacc;
            }
        }
    /* contacts */
    if (c->ground)
        for (int i = 0; i < c->P; ++i) {
            const int g = s * c->P + i;
            const double m = pmass(c, i);
            const double* lc = st->lam_c + 3 * (size_t)g;
            double z = w->x[3 * i + 2], ux = w->x[3 * i] - w->xp[3 * i], uy = w->x[3 * i + 1] - w->xp[3 * i + 1];
            if (c->linear) {
                z = w->xt[3 * i + 2] + w->acc[3 * i + 2];
                ux = w->xt[3 * i] + w->acc[3 * i] - w->xp[3 * i];
                uy = w->xt[3 * i + 1] + w->acc[3 * i + 1] - w->xp[3 * i + 1];
            }
            res = fmax(res, (lc[0] > 0.0 ? fabs(z) : fmax(-z, 0.0)) / c->Lref);
            if (!apply) continue;
            const double sc = b->relax / c->dp[i];
            const double ln = fmax(0.0, lc[0] + sc * (-m * z));
            double tx = lc[1] + sc * (-m * ux), ty = lc[2] + sc * (-m * uy);
            const double cap = b->mu[s] * ln, nt = sqrt(tx * tx + ty * ty);
            if (!(ln > 0.0)) {
                tx = ty = 0.0;
            } else if (nt > cap) {
                tx *= cap / nt;
                ty *= cap / nt;
            }
            w->dl_c[3 * i] = ln - lc[0];
            w->dl_c[3 * i + 1] = tx - lc[1];
            w->dl_c[3 * i + 2] = ty - lc[2];
        }
    return res;
}

/* apply the scaled increments: multipliers, then every body gathers in the
 * fixed block order */
static void apply_blocks(const ctx_t* c, lnk_state* st, int s, work_t* w)
{
    const lnk_batch* b = c->b;
    for (int T = 0; T < c->T; ++T)
        for (int r = 0; r < 6; ++r) st->lam_tet[6 * ((size_t)s * c->T + T) + r] += w->dl_tet[6 * T + r];
    for (int D = 0; D < c->D; ++D) st->lam_dist[(size_t)s * c->D + D] += w->dl_dist[D];
    for (int A = 0; A < c->A; ++A)
        for (int q = 0; q < 3; ++q) st->lam_att[3 * ((size_t)s * c->A + A) + q] += w->dl_att[3 * A + q];
    if (c->ground)
        for (int i = 0; i < c->P; ++i)
            for (int q = 0; q < 3; ++q) st->lam_c[3 * ((size_t)s * c->P + i) + q] += w->dl_c[3 * i + q];

    double* fp = calloc(3 * (size_t)c->P, sizeof(double));
    double* ff = calloc(6 * (size_t)c->F, sizeof(double));
    for (int l = 0; l < b->n_links; ++l)
        for (int t = 0; t < b->n_tets; ++t)
            for (int k = 0; k < 4; ++k)
                for (int z = 0; z < 3; ++z)
                    fp[3 * (l * c->P1 + b->tets[4 * t + k]) + z] += w->imp_tet[12 * (size_t)(l * b->n_tets + t) + 3 * k + z];
    for (int l = 0; l < b->n_links; ++l)
        for (int d = 0; d < c->ND1; ++d) {
            const int D = l * c->ND1 + d;
            for (int z = 0; z < 3; ++z) {
                fp[3 * (l * c->P1 + c->di[d]) + z] += w->imp_dist[3 * D + z];
                fp[3 * (l * c->P1 + c->dj[d]) + z] -= w->imp_dist[3 * D + z];
            }
        }
    for (int l = 0; l < b->n_links; ++l)
        for (int a = 0; a < c->NA1; ++a) {
            const int A = l * c->NA1 + a, i = l * c->P1 + c->ap[a], f = l + c->as[a];
            for (int z = 0; z < 6; ++z) ff[6 * f + z] += w->imp_att[9 * A + z];
            for (int z = 0; z < 3; ++z) fp[3 * i + z] += w->imp_att[9 * A + 6 + z];
        }
    if (c->ground)
        for (int i = 0; i < c->P; ++i) {
            fp[3 * i] += w->dl_c[3 * i + 1];
            fp[3 * i + 1] += w->dl_c[3 * i + 2];
            fp[3 * i + 2] += w->dl_c[3 * i];
        }
    for (int i = 0; i < c->P; ++i) {
        const double wi = 1.0 / pmass(c, i);
        for (int z = 0; z < 3; ++z) {
            if (c->linear)
                w->acc[3 * i + z] += wi * fp[3 * i + z];
            else
                w->x[3 * i + z] += wi * fp[3 * i + z];
        }
    }
    for (int f = 0; f < c->F; ++f) {
        if (frame_fixed(c, f)) continue;
        double Iinv[9], th[3];
        frame_inv_inertia(b, c->linear ? w->fqt + 4 * f : w->fq + 4 * f, Iinv);
        for (int r = 0; r < 3; ++r)
            th[r] = Iinv[3 * r] * ff[6 * f + 3] + Iinv[3 * r + 1] * ff[6 * f + 4] + Iinv[3 * r + 2] * ff[6 * f + 5];
        for (int z = 0; z < 3; ++z) {
            if (c->linear) {
                w->facc[6 * f + z] += ff[6 * f + z] / b->frame_mass;
                w->facc[6 * f + 3 + z] += th[z];
            } else {
                w->fx[3 * f + z] += ff[6 * f + z] / b->frame_mass;
            }
        }
        if (!c->linear) q_turn(w->fq + 4 * f, th);
    }
    free(fp);
    free(ff);
}

/* freeze every block's value and Jacobian at the predicted state (linearised mode) */
static void freeze(const ctx_t* c, const double* cmd_l, const double* p_l, work_t* w)
{
    const lnk_batch* b = c->b;
    for (int l = 0; l < b->n_links; ++l)
        for (int t = 0; t < b->n_tets; ++t) {
            const int T = l * b->n_tets + t;
            double xv[12], R[9];
            for (int k = 0; k < 4; ++k)
                for (int q = 0; q < 3; ++q) xv[3 * k + q] = w->xt[3 * (l * c->P1 + b->tets[4 * t + k]) + q];
            fem_tet_eval(c->Dm_inv + 9 * t, xv, R, 0, w->C0 + 6 * (size_t)T, w->J0 + 72 * (size_t)T);
        }
    for (int l = 0; l < b->n_links; ++l) {
        for (int d = 0; d < c->ND1; ++d) {
            const int D = l * c->ND1 + d, i = l * c->P1 + c->di[d], j = l * c->P1 + c->dj[d];
            double press = 0.0;
            if (c->dk[d] == LNK_CHAMBER0) press = p_l[2 * l] * b->p_max;
            if (c->dk[d] == LNK_CHAMBER1) press = p_l[2 * l + 1] * b->p_max;
            (void)cmd_l;
            w->C0[6 * (size_t)c->T + D] = fem_dist_eval(w->xt + 3 * i, w->xt + 3 * j, c->drest[d], press, b->young,
                                                      w->J0 + 72 * (size_t)c->T + 6 * (size_t)D);
        }
        for (int a = 0; a < c->NA1; ++a) {
            const int A = l * c->NA1 + a, i = l * c->P1 + c->ap[a], f = l + c->as[a];
            double r[3];
            att_point(c, l, a, r);
            fem_attach_eval(w->fxt + 3 * f, w->fqt + 4 * f, r, w->xt + 3 * i, w->C0 + 6 * (size_t)c->T + c->D + 3 * A,
                            w->J0 + 72 * (size_t)c->T + 6 * (size_t)c->D + 27 * (size_t)A);
        }
    }
}

static void work_alloc(const ctx_t* c, work_t* w)
{
    memset(w, 0, sizeof *w);
    w->x = calloc(3 * (size_t)c->P, sizeof(double));
    w->xp = calloc(3 * (size_t)c->P, sizeof(double));
    w->xt = calloc(3 * (size_t)c->P, sizeof(double));
    w->acc = calloc(3 * (size_t)c->P, sizeof(double));
    w->fx = calloc(3 * (size_t)c->F, sizeof(double));
    w->fq = calloc(4 * (size_t)c->F, sizeof(double));
    w->fxp = calloc(3 * (size_t)c->F, sizeof(double));
    w->fqp = calloc(4 * (size_t)c->F, sizeof(double));
    w->fxt = calloc(3 * (size_t)c->F, sizeof(double));
    w->fqt = calloc(4 * (size_t)c->F, sizeof(double));
    w->facc = calloc(6 * (size_t)c->F, sizeof(double));
    w->dl_tet = calloc(6 * (size_t)c->T, sizeof(double));
    w->dl_dist = calloc((size_t)c->D, sizeof(double));
    w->dl_att = calloc(3 * (size_t)c->A, sizeof(double));
    w->dl_c = calloc(3 * (size_t)c->P, sizeof(double));
    w->imp_tet = calloc(12 * (size_t)c->T, sizeof(double));
    w->imp_att = calloc(9 * (size_t)c->A, sizeof(double));
    w->imp_dist = calloc(3 * (size_t)c->D, sizeof(double));
    if (c->linear) {
        const size_t rows = 6 * (size_t)c->T + c->D + 3 * (size_t)c->A;
        w->C0 = calloc(rows, sizeof(double));
        w->J0 = calloc(72 * (size_t)c->T + 6 * (size_t)c->D + 27 * (size_t)c->A, sizeof(double));
    }
}

static void work_free(work_t* w)
{
    double* all[] = {w->x, w->xp, w->xt, w->acc, w->fx, w->fq, w->fxp, w->fqp, w->fxt, w->fqt, w->facc,
                     w->dl_tet, w->dl_dist, w->dl_att, w->dl_c, w->imp_tet, w->imp_att, w->imp_dist, w->C0, w->J0};
    for (size_t k = 0; k < sizeof all / sizeof all[0]; ++k) free(all[k]);
}

/* One substep of snake s: pressures, prediction, iterations, velocities. */
static void substep(const ctx_t* c, lnk_state* st, int s, work_t* w)
{
    const lnk_batch* b = c->b;
    const double h = c->h;
    const int L = b->n_links;
    double* cmd_l = st->cmd + (size_t)s * L;
    double* p_l = st->p + 2 * (size_t)s * L;
    /* chamber pressures: first-order lag toward the commanded chamber */
    const double lag_in = exp(-h / b->tau_inf), lag_de = exp(-h / b->tau_def);
    for (int l = 0; l < L; ++l) {
        const double u[2] = {cmd_l[l] > 0.0 ? cmd_l[l] : 0.0, cmd_l[l] < 0.0 ? -cmd_l[l] : 0.0};
        for (int k = 0; k < 2; ++k) {
            double* p = p_l + 2 * l + k;
            *p = u[k] + (*p - u[k]) * (u[k] > *p ? lag_in : lag_de);
        }
    }
    /* prediction */
    for (int i = 0; i < c->P; ++i) {
        double* x = st->x + 3 * ((size_t)s * c->P + i);
        double* v = st->v + 3 * ((size_t)s * c->P + i);
        for (int z = 0; z < 3; ++z) w->xp[3 * i + z] = x[z];
        v[2] -= h * b->gravity;
        for (int z = 0; z < 3; ++z) w->x[3 * i + z] = x[z] + h * v[z];
    }
    for (int f = 0; f < c->F; ++f) {
        const size_t g = (size_t)s * c->F + f;
        double *x = st->fx + 3 * g, *q = st->fq + 4 * g, *v = st->fv + 3 * g, *om = st->fw + 3 * g;
        memcpy(w->fxp + 3 * f, x, 3 * sizeof(double));
        memcpy(w->fqp + 4 * f, q, 4 * sizeof(double));
        memcpy(w->fx + 3 * f, x, 3 * sizeof(double));
        memcpy(w->fq + 4 * f, q, 4 * sizeof(double));
        if (frame_fixed(c, f)) {
            for (int z = 0; z < 3; ++z) v[z] = om[z] = 0.0;
            continue;
        }
        v[2] -= h * b->gravity;
        for (int z = 0; z < 3; ++z) w->fx[3 * f + z] = x[z] + h * v[z];
        double I[9], Iinv[9], Iw[3], tq[3], dw[3];
        frame_inertia(b, q, I);
        frame_inv_inertia(b, q, Iinv);
        for (int r = 0; r < 3; ++r) Iw[r] = I[3 * r] * om[0] + I[3 * r + 1] * om[1] + I[3 * r + 2] * om[2];
        tq[0] = -(om[1] * Iw[2] - om[2] * Iw[1]);
        tq[1] = -(om[2] * Iw[0] - om[0] * Iw[2]);
        tq[2] = -(om[0] * Iw[1] - om[1] * Iw[0]);
        for (int r = 0; r < 3; ++r) dw[r] = Iinv[3 * r] * tq[0] + Iinv[3 * r + 1] * tq[1] + Iinv[3 * r + 2] * tq[2];
        for (int z = 0; z < 3; ++z) om[z] += h * dw[z];
        const double th[3] = {h * om[0], h * om[1], h * om[2]};
        q_turn(w->fq + 4 * f, th);
    }
    /* zero multipliers */
    memset(st->lam_tet + 6 * (size_t)s * c->T, 0, 6 * (size_t)c->T * sizeof(double));
    memset(st->lam_dist + (size_t)s * c->D, 0, (size_t)c->D * sizeof(double));
    memset(st->lam_att + 3 * (size_t)s * c->A, 0, 3 * (size_t)c->A * sizeof(double));
    memset(st->lam_c + 3 * (size_t)s * c->P, 0, 3 * (size_t)c->P * sizeof(double));
    if (c->linear) {
        memcpy(w->xt, w->x, 3 * (size_t)c->P * sizeof(double));
        memcpy(w->fxt, w->fx, 3 * (size_t)c->F * sizeof(double));
        memcpy(w->fqt, w->fq, 4 * (size_t)c->F * sizeof(double));
        memset(w->acc, 0, 3 * (size_t)c->P * sizeof(double));
        memset(w->facc, 0, 6 * (size_t)c->F * sizeof(double));
        freeze(c, cmd_l, p_l, w);
    }
    /* iterations: evaluate iterate k (residual r^k); stop, or apply */
    int k = 0;
    double r = 0.0;
    for (;;) {
        r = eval_blocks(c, st, s, w, cmd_l, p_l, 1);
        const int bad = !(r < INFINITY);
        if (bad || (b->tol > 0.0 ? (r <= b->tol || k >= b->iters) : k >= b->iters)) {
            if (bad) st->status[s] |= LNK_STATUS_NONFINITE;
            else if (b->tol > 0.0 && r > b->tol) st->status[s] |= LNK_STATUS_NOT_CONVERGED;
            break;
        }
        apply_blocks(c, st, s, w);
        ++k;
    }
    st->iters[s] += k;
    st->residual[s] = fmax(st->residual[s], r);
    if (c->linear) {
        for (int i = 0; i < 3 * c->P; ++i) w->x[i] = w->xt[i] + w->acc[i];
        for (int f = 0; f < c->F; ++f) {
            for (int z = 0; z < 3; ++z) w->fx[3 * f + z] = w->fxt[3 * f + z] + w->facc[6 * f + z];
            memcpy(w->fq + 4 * f, w->fqt + 4 * f, 4 * sizeof(double));
            q_turn(w->fq + 4 * f, w->facc + 6 * f + 3);
        }
    }
    /* velocities of the implicit step */
    for (int i = 0; i < c->P; ++i) {
        const size_t g = (size_t)s * c->P + i;
        for (int z = 0; z < 3; ++z) {
            st->v[3 * g + z] = (w->x[3 * i + z] - w->xp[3 * i + z]) / h;
            st->x[3 * g + z] = w->x[3 * i + z];
        }
    }
    for (int f = 0; f < c->F; ++f) {
        const size_t g = (size_t)s * c->F + f;
        if (frame_fixed(c, f)) continue;
        double qc[4] = {w->fqp[4 * f], -w->fqp[4 * f + 1], -w->fqp[4 * f + 2], -w->fqp[4 * f + 3]}, dq[4];
        q_mul(w->fq + 4 * f, qc, dq);
        const double sg = dq[0] >= 0.0 ? 2.0 / h : -2.0 / h;
        for (int z = 0; z < 3; ++z) {
            st->fv[3 * g + z] = (w->fx[3 * f + z] - w->fxp[3 * f + z]) / h;
            st->fw[3 * g + z] = sg * dq[1 + z];
            st->fx[3 * g + z] = w->fx[3 * f + z];
        }
        memcpy(st->fq + 4 * g, w->fq + 4 * f, 4 * sizeof(double));
    }
}

/* ---------------------------------------------------------------- entry points */

void lnk_sizes(const lnk_batch* b, int32_t* out)
{
    out[0] = per_link(b) * b->n_links;          /* particles per snake */
    out[1] = b->n_links + 1;                    /* frames per snake */
    out[2] = b->n_tets * b->n_links;            /* tetrahedra per snake */
    out[3] = lnk_dist_per_link(b) * b->n_links; /* distance constraints per snake */
    out[4] = lnk_att_per_link(b) * b->n_links;  /* attachments per snake */
}

/* Rest state: links end to end along +x, axis at height `radius`, frames
 * at the junctions, everything at rest, zero pressure and multipliers. */
void lnk_init_state(const lnk_batch* b, lnk_state* st)
{
    int32_t sz[5];
    lnk_sizes(b, sz);
    for (int s = 0; s < b->n_snakes; ++s) {
        for (int i = 0; i < sz[0]; ++i) {
            lnk_rest_particle(b, i, st->x + 3 * ((size_t)s * sz[0] + i));
            for (int z = 0; z < 3; ++z) st->v[3 * ((size_t)s * sz[0] + i) + z] = 0.0;
        }
        for (int f = 0; f < sz[1]; ++f) {
            const size_t g = (size_t)s * sz[1] + f;
            rest_frame(b, f, st->fx + 3 * g);
            st->fq[4 * g] = 1.0;
            st->fq[4 * g + 1] = st->fq[4 * g + 2] = st->fq[4 * g + 3] = 0.0;
            for (int z = 0; z < 3; ++z) st->fv[3 * g + z] = st->fw[3 * g + z] = 0.0;
        }
        for (int l = 0; l < b->n_links; ++l) {
            st->p[2 * ((size_t)s * b->n_links + l)] = st->p[2 * ((size_t)s * b->n_links + l) + 1] = 0.0;
            st->cmd[(size_t)s * b->n_links + l] = 0.0;
        }
    }
    memset(st->lam_tet, 0, 6 * (size_t)b->n_snakes * sz[2] * sizeof(double));
    memset(st->lam_dist, 0, (size_t)b->n_snakes * sz[3] * sizeof(double));
    memset(st->lam_att, 0, 3 * (size_t)b->n_snakes * sz[4] * sizeof(double));
    memset(st->lam_c, 0, 3 * (size_t)b->n_snakes * sz[0] * sizeof(double));
}

/* Advance snakes [s0, s1) by n_steps steps with their held commands.
 * residual/iters/status describe the last step (max / sum over substeps). */
int lnk_run(const lnk_batch* b, lnk_state* st, int s0, int s1, int n_steps)
{
    ctx_t c;
    ctx_init(b, &c);
    work_t w;
    work_alloc(&c, &w);
    for (int s = s0; s < s1; ++s)
        for (int n = 0; n < n_steps; ++n) {
            st->residual[s] = 0.0;
            st->iters[s] = 0;
            st->status[s] = 0;
            for (int sub = 0; sub < b->substeps; ++sub) substep(&c, st, s, &w);
        }
    work_free(&w);
    ctx_free(&c);
    return 0;
}

/* Assembled compliant system of snake s at the given state (particles x,
 * frames fx, fq), every block active (both chambers' actuation rows at the
 * given pressures), contacts left out.  Rows: tetrahedra (6 each), distance
 * constraints, attachments (3 each); columns: particles (3 each), then
 * frames (x 3, rotation 3).  Outputs C[m], J[m][n] and the inverse mass
 * matrix W[n][n]; E[m][m] the compliance blocks divided by h^2.  Returns m. */
int lnk_assemble(const lnk_batch* b, const double* x, const double* fx, const double* fq, const double* p_l,
                 double* Cout, double* Jout, double* Wout, double* Eout)
{
    ctx_t c;
    ctx_init(b, &c);
    const int n = 3 * c.P + 6 * c.F, m = 6 * c.T + c.D + 3 * c.A;
    const double h2 = c.h * c.h;
    memset(Jout, 0, sizeof(double) * (size_t)m * n);
    memset(Wout, 0, sizeof(double) * (size_t)n * n);
    memset(Eout, 0, sizeof(double) * (size_t)m * m);
    int row = 0;
    for (int l = 0; l < b->n_links; ++l)
        for (int t = 0; t < b->n_tets; ++t, row += 6) {
            double xv[12], R[9], J[72], E[36];
            for (int k = 0; k < 4; ++k)
                for (int q = 0; q < 3; ++q) xv[3 * k + q] = x[3 * (l * c.P1 + b->tets[4 * t + k]) + q];
            fem_tet_eval(c.Dm_inv + 9 * t, xv, R, 0, Cout + row, J);
            for (int r = 0; r < 6; ++r)
                for (int k = 0; k < 4; ++k)
                    for (int q = 0; q < 3; ++q)
                        Jout[(size_t)(row + r) * n + 3 * (l * c.P1 + b->tets[4 * t + k]) + q] = J[12 * r + 3 * k + q];
            fem_tet_compliance(c.vol[t], b->young, b->poisson, E);
            for (int r = 0; r < 6; ++r)
                for (int q = 0; q < 6; ++q) Eout[(size_t)(row + r) * m + row + q] = E[6 * r + q] / h2;
        }
    for (int l = 0; l < b->n_links; ++l)
        for (int d = 0; d < c.ND1; ++d, ++row) {
            const int i = l * c.P1 + c.di[d], j = l * c.P1 + c.dj[d];
            double Jd[6], press = 0.0;
            if (c.dk[d] == LNK_CHAMBER0) press = p_l[2 * l] * b->p_max;
            if (c.dk[d] == LNK_CHAMBER1) press = p_l[2 * l + 1] * b->p_max;
            Cout[row] = fem_dist_eval(x + 3 * i, x + 3 * j, c.drest[d], press, b->young, Jd);
            Eout[(size_t)row * m + row] = b->rigid_compliance / h2;
            for (int q = 0; q < 3; ++q) {
                Jout[(size_t)row * n + 3 * i + q] = Jd[q];
                Jout[(size_t)row * n + 3 * j + q] = Jd[3 + q];
            }
        }
    for (int l = 0; l < b->n_links; ++l)
        for (int a = 0; a < c.NA1; ++a, row += 3) {
            const int i = l * c.P1 + c.ap[a], f = l + c.as[a];
            double r[3], Ja[27];
            att_point(&c, l, a, r);
            fem_attach_eval(fx + 3 * f, fq + 4 * f, r, x + 3 * i, Cout + row, Ja);
            for (int q = 0; q < 3; ++q) Eout[(size_t)(row + q) * m + row + q] = b->rigid_compliance / h2;
            for (int q = 0; q < 3; ++q)
                for (int z = 0; z < 3; ++z) {
                    Jout[(size_t)(row + q) * n + 3 * c.P + 6 * f + z] = Ja[9 * q + z];
                    Jout[(size_t)(row + q) * n + 3 * c.P + 6 * f + 3 + z] = Ja[9 * q + 3 + z];
                    Jout[(size_t)(row + q) * n + 3 * i + z] = Ja[9 * q + 6 + z];
                }
        }
    for (int i = 0; i < c.P; ++i)
        for (int q = 0; q < 3; ++q) Wout[(size_t)(3 * i + q) * n + 3 * i + q] = 1.0 / pmass(&c, i);
    for (int f = 0; f < c.F; ++f) {
        if (frame_fixed(&c, f)) continue;
        double Iinv[9];
        frame_inv_inertia(b, fq + 4 * f, Iinv);
        const int o = 3 * c.P + 6 * f;
        for (int q = 0; q < 3; ++q) {
            Wout[(size_t)(o + q) * n + o + q] = 1.0 / b->frame_mass;
            for (int z = 0; z < 3; ++z) Wout[(size_t)(o + 3 + q) * n + o + 3 + z] = Iinv[3 * q + z];
        }
    }
    ctx_free(&c);
    return m;
}

/* Per-snake prediction (the stage every substep starts with) on copies:
 * particles x, v and frames fx, fq, fv, fw are advanced in place by h. */
void lnk_predict(const lnk_batch* b, double* x, double* v, double* fx, double* fq, double* fv, double* fw)
{
    ctx_t c;
    ctx_init(b, &c);
    const double h = c.h;
    for (int i = 0; i < c.P; ++i) {
        v[3 * i + 2] -= h * b->gravity;
        for (int z = 0; z < 3; ++z) x[3 * i + z] += h * v[3 * i + z];
    }
    for (int f = 0; f < c.F; ++f) {
        if (frame_fixed(&c, f)) continue;
        double I[9], Iinv[9], Iw[3], tq[3], dw[3];
        double *q = fq + 4 * f, *om = fw + 3 * f;
        fv[3 * f + 2] -= h * b->gravity;
        for (int z = 0; z < 3; ++z) fx[3 * f + z] += h * fv[3 * f + z];
        frame_inertia(b, q, I);
        frame_inv_inertia(b, q, Iinv);
        for (int r = 0; r < 3; ++r) Iw[r] = I[3 * r] * om[0] + I[3 * r + 1] * om[1] + I[3 * r + 2] * om[2];
        tq[0] = -(om[1] * Iw[2] - om[2] * Iw[1]);
        tq[1] = -(om[2] * Iw[0] - om[0] * Iw[2]);
        tq[2] = -(om[0] * Iw[1] - om[1] * Iw[0]);
        for (int r = 0; r < 3; ++r) dw[r] = Iinv[3 * r] * tq[0] + Iinv[3 * r + 1] * tq[1] + Iinv[3 * r + 2] * tq[2];
        for (int z = 0; z < 3; ++z) om[z] += h * dw[z];
        const double th[3] = {h * om[0], h * om[1], h * om[2]};
        q_turn(q, th);
    }
    ctx_free(&c);
}
