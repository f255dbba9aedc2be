/*
 * FP64 oracle pieces of the full-resolution link (particles and tetrahedral
 * finite elements).  TEST INFRASTRUCTURE ONLY, like the rest of this
 * folder; shares nothing with the GPU library.
 *
 *   - the constant-strain tetrahedron of section "Tetrahedral
 *     Finite-Elements": deformation gradient F = Ds Dm^-1 from the edge
 *     matrices of the current and rest shapes, rotation R of the polar
 *     decomposition F = R S, corotational strain eps = sym(R^T F) - I in
 *     Voigt order (xx, yy, zz, yz, xz, xy; tensor shear components), and
 *     its Jacobian with R held fixed (the rotation frozen within an
 *     iteration);
 *   - the element compliance E_tetra = M / (V Y) of the same section;
 *   - the actuation distance constraint |x_i - x_j| - r eps(p) with the
 *     strain eps(p) = 1 + p / Y of eq. expansion (section "Actuation
 *     Constraints"), and its Jacobian;
 *   - the attachment of a particle to a point of a rigid body,
 *     eq. rigid_to_particle, and its Jacobian.
 * Every quantity is double.
 */
#include <math.h>
#include <string.h>

static double det3(const double* A)
{
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* inverse of a 3x3 (row-major) by the adjugate; returns the determinant */
static double inv3(const double* A, double* B)
{
    double d = det3(A);
    B[0] = (A[4] * A[8] - A[5] * A[7]) / d;
    B[1] = (A[2] * A[7] - A[1] * A[8]) / d;
    B[2] = (A[1] * A[5] - A[2] * A[4]) / d;
    B[3] = (A[5] * A[6] - A[3] * A[8]) / d;
    B[4] = (A[0] * A[8] - A[2] * A[6]) / d;
    B[5] = (A[2] * A[3] - A[0] * A[5]) / d;
    B[6] = (A[3] * A[7] - A[4] * A[6]) / d;
    B[7] = (A[1] * A[6] - A[0] * A[7]) / d;
    B[8] = (A[0] * A[4] - A[1] * A[3]) / d;
    return d;
}

/* edge matrix: column k = x_{k+1} - x_0 */
static void edges(const double* x, double* D)
{
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) D[3 * r + k] = x[3 * (k + 1) + r] - x[r];
}

/* Rest state of a tetrahedron (vertices X[4][3]): Dm^-1 and the volume
 * |det Dm| / 6.  Returns 0, or -1 for a degenerate element. */
int fem_tet_rest(const double* X, double* Dm_inv, double* volume)
{
    double Dm[9];
    edges(X, Dm);
    double d = det3(Dm);
    if (!(fabs(d) > 0.0)) return -1;
    inv3(Dm, Dm_inv);
    *volume = fabs(d) / 6.0;
    return 0;
}

/* Rotation of the polar decomposition of F (det F > 0) by the Newton
 * iteration R <- (R + R^-T) / 2 from R = F (Higham), to round-off. */
int fem_polar(const double* F, double* R)
{
    double A[9], B[9];
    memcpy(A, F, sizeof A);
    if (!(det3(A) > 0.0)) return -1;
    for (int it = 0; it < 100; ++it) {
        inv3(A, B);
        double diff = 0.0;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double v = 0.5 * (A[3 * r + c] + B[3 * c + r]);
                diff = fmax(diff, fabs(v - A[3 * r + c]));
                A[3 * r + c] = v;
            }
        if (diff <= 1e-15) break;
    }
    memcpy(R, A, sizeof A);
    return 0;
}

/* Corotational strain of the tetrahedron with current vertices x[4][3]:
 * C[6] = (eps_xx, eps_yy, eps_zz, eps_yz, eps_xz, eps_xy) of
 * eps = (R^T F + F^T R) / 2 - I, and J[6][12] = d C / d x (vertex-major,
 * x_0 .. x_3) with R held fixed.  R[9] is used as given when rot_in is
 * nonzero, else taken from the polar decomposition of F and returned in R.
 * Returns 0, or -1 for an inverted element. */
int fem_tet_eval(const double* Dm_inv, const double* x, double* R, int rot_in, double* C, double* J)
{
    double Ds[9], F[9];
    edges(x, Ds);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += Ds[3 * r + k] * Dm_inv[3 * k + c];
            F[3 * r + c] = s;
        }
    if (!rot_in && fem_polar(F, R) != 0) return -1;
    double S[9];   /* R^T F */
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int i = 0; i < 3; ++i) s += R[3 * i + a] * F[3 * i + b];
            S[3 * a + b] = s;
        }
    static const int va[6] = {0, 1, 2, 1, 0, 0}, vb[6] = {0, 1, 2, 2, 2, 1};
    for (int v = 0; v < 6; ++v) {
        int a = va[v], b = vb[v];
        C[v] = 0.5 * (S[3 * a + b] + S[3 * b + a]) - (a == b ? 1.0 : 0.0);
    }
    /* d F_ib / d (x_m)_c = delta_ic g_m[b], g_m = row m-1 of Dm^-1 (m >= 1),
     * g_0 = -(sum of the rows); so d (R^T F)_ab / d (x_m)_c = R_ca g_m[b] */
    double g[4][3];
    for (int b = 0; b < 3; ++b) {
        g[0][b] = -(Dm_inv[b] + Dm_inv[3 + b] + Dm_inv[6 + b]);
        for (int m = 1; m < 4; ++m) g[m][b] = Dm_inv[3 * (m - 1) + b];
    }
    for (int v = 0; v < 6; ++v) {
        int a = va[v], b = vb[v];
        for (int m = 0; m < 4; ++m)
            for (int c = 0; c < 3; ++c)
                J[12 * v + 3 * m + c] = 0.5 * (R[3 * c + a] * g[m][b] + R[3 * c + b] * g[m][a]);
    }
    return 0;
}

/* E_tetra = M / (V Y): M has 1 on the normal diagonal, -nu off it, 1 + nu
 * on the shear diagonal (E[6][6], row-major). */
void fem_tet_compliance(double V, double Y, double nu, double* E)
{
    memset(E, 0, 36 * sizeof(double));
    double s = 1.0 / (V * Y);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) E[6 * r + c] = (r == c ? 1.0 : -nu) * s;
    for (int r = 3; r < 6; ++r) E[7 * r] = (1.0 + nu) * s;
}

/* eq. expansion: strain of a chamber at pressure p, eps(p) = 1 + p / Y */
double fem_expansion(double p, double Y) { return 1.0 + p / Y; }

/* Actuation distance constraint between particles xi, xj at rest length r
 * and pressure p: C = |xi - xj| - r eps(p); J[6] = (n, -n), n the unit
 * direction from xj to xi.  Returns C. */
double fem_dist_eval(const double* xi, const double* xj, double r, double p, double Y, double* J)
{
    double d[3] = {xi[0] - xj[0], xi[1] - xj[1], xi[2] - xj[2]};
    double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int k = 0; k < 3; ++k) {
        double n = L > 0.0 ? d[k] / L : 0.0;
        J[k] = n;
        J[3 + k] = -n;
    }
    return L - r * fem_expansion(p, Y);
}

/* Attachment of particle xp to the point r (body frame) of a rigid body
 * (centre x, unit quaternion q = (w, x, y, z)), eq. rigid_to_particle:
 * C = x + R(q) r - xp (3 rows); J[3][9] = d C / d (x, theta, xp) with theta
 * a world rotation vector: (I, -[R r]x, -I). */
void fem_attach_eval(const double* x, const double* q, const double* r, const double* xp, double* C, double* J)
{
    const double w = q[0], a = q[1], b = q[2], c = q[3];
    const double R[9] = {1 - 2 * (b * b + c * c), 2 * (a * b - w * c), 2 * (a * c + w * b),
                         2 * (a * b + w * c), 1 - 2 * (a * a + c * c), 2 * (b * c - w * a),
                         2 * (a * c - w * b), 2 * (b * c + w * a), 1 - 2 * (a * a + b * b)};
    double u[3];
    for (int i = 0; i < 3; ++i) u[i] = R[3 * i] * r[0] + R[3 * i + 1] * r[1] + R[3 * i + 2] * r[2];
    for (int i = 0; i < 3; ++i) C[i] = x[i] + u[i] - xp[i];
    /* rows of -[u]x: d (theta x u) = -u x d theta */
    const double S[9] = {0, u[2], -u[1], -u[2], 0, u[0], u[1], -u[0], 0};
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) {
            J[9 * i + k] = i == k ? 1.0 : 0.0;
            J[9 * i + 3 + k] = S[3 * i + k];
            J[9 * i + 6 + k] = i == k ? -1.0 : 0.0;
        }
}
