/*
 * FP64 CPU oracle of the warm-start network: a 32 -> 64 -> 64 -> 3
 * perceptron with exact-erf GELU after the two hidden layers, inputs
 * standardised by per-feature mean and standard deviation, mean-squared
 * error loss, and one Adam step.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check); shares no code with the GPU
 * library.  Plain loops in double precision.
 *
 * Parameter vector (6467 doubles): W1[64][32], b1[64], W2[64][64], b2[64],
 * W3[3][64], b3[3]; W[o][i] multiplies input i into output o.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define NI 32
#define NH 64
#define NO 3
#define P_W1 0
#define P_B1 (P_W1 + NH * NI)
#define P_W2 (P_B1 + NH)
#define P_B2 (P_W2 + NH * NH)
#define P_W3 (P_B2 + NH)
#define P_B3 (P_W3 + NO * NH)
#define P_COUNT (P_B3 + NO)

int mlo_param_count(void) { return P_COUNT; }

static double gelu(double z) { return 0.5 * z * (1.0 + erf(z / sqrt(2.0))); }

/* derivative of z Phi(z): Phi(z) + z phi(z) */
static double gelu_grad(double z)
{
    const double inv_sqrt_2pi = 0.39894228040143267794;
    return 0.5 * (1.0 + erf(z / sqrt(2.0))) + z * inv_sqrt_2pi * exp(-0.5 * z * z);
}

/* per-feature mean and standard deviation (population, plus 1e-12 inside the root) */
void mlo_norm_stats(const double* x, int64_t n, double* mean, double* stdv)
{
    for (int i = 0; i < NI; ++i) {
        double s = 0.0;
        for (int64_t r = 0; r < n; ++r) s += x[r * NI + i];
        mean[i] = s / (double)n;
    }
    for (int i = 0; i < NI; ++i) {
        double s = 0.0;
        for (int64_t r = 0; r < n; ++r) {
            double d = x[r * NI + i] - mean[i];
            s += d * d;
        }
        stdv[i] = sqrt(s / (double)n + 1e-12);
    }
}

/* forward pass of one sample; keeps pre-activations for the backward pass */
static void forward1(const double* p, const double* mean, const double* stdv, const double* x,
                     double* xn, double* z1, double* h1, double* z2, double* h2, double* y)
{
    for (int i = 0; i < NI; ++i) xn[i] = (x[i] - mean[i]) / stdv[i];
    for (int o = 0; o < NH; ++o) {
        double s = p[P_B1 + o];
        for (int i = 0; i < NI; ++i) s += p[P_W1 + o * NI + i] * xn[i];
        z1[o] = s;
        h1[o] = gelu(s);
    }
    for (int o = 0; o < NH; ++o) {
        double s = p[P_B2 + o];
        for (int i = 0; i < NH; ++i) s += p[P_W2 + o * NH + i] * h1[i];
        z2[o] = s;
        h2[o] = gelu(s);
    }
    for (int o = 0; o < NO; ++o) {
        double s = p[P_B3 + o];
        for (int i = 0; i < NH; ++i) s += p[P_W3 + o * NH + i] * h2[i];
        y[o] = s;
    }
}

void mlo_forward(const double* p, const double* mean, const double* stdv, const double* x, int64_t n,
                 double* y)
{
    double xn[NI], z1[NH], h1[NH], z2[NH], h2[NH];
    for (int64_t r = 0; r < n; ++r) forward1(p, mean, stdv, x + r * NI, xn, z1, h1, z2, h2, y + r * NO);
}

/* loss = mean over samples and outputs of (y - t)^2; grad = d loss / d p */
double mlo_loss_grad(const double* p, const double* mean, const double* stdv, const double* x,
                     const double* t, int64_t n, double* grad)
{
    double xn[NI], z1[NH], h1[NH], z2[NH], h2[NH], y[NO], dy[NO], dz2[NH], dz1[NH];
    double loss = 0.0;
    const double scale = 1.0 / ((double)n * NO);
    if (grad) memset(grad, 0, sizeof(double) * P_COUNT);
    for (int64_t r = 0; r < n; ++r) {
        forward1(p, mean, stdv, x + r * NI, xn, z1, h1, z2, h2, y);
        for (int o = 0; o < NO; ++o) {
            double e = y[o] - t[r * NO + o];
            loss += e * e * scale;
            dy[o] = 2.0 * e * scale;
        }
        if (!grad) continue;
        for (int o = 0; o < NO; ++o) {
            grad[P_B3 + o] += dy[o];
            for (int i = 0; i < NH; ++i) grad[P_W3 + o * NH + i] += dy[o] * h2[i];
        }
        for (int i = 0; i < NH; ++i) {
            double s = 0.0;
            for (int o = 0; o < NO; ++o) s += p[P_W3 + o * NH + i] * dy[o];
            dz2[i] = s * gelu_grad(z2[i]);
        }
        for (int o = 0; o < NH; ++o) {
            grad[P_B2 + o] += dz2[o];
            for (int i = 0; i < NH; ++i) grad[P_W2 + o * NH + i] += dz2[o] * h1[i];
        }
        for (int i = 0; i < NH; ++i) {
            double s = 0.0;
            for (int o = 0; o < NH; ++o) s += p[P_W2 + o * NH + i] * dz2[o];
            dz1[i] = s * gelu_grad(z1[i]);
        }
        for (int o = 0; o < NH; ++o) {
            grad[P_B1 + o] += dz1[o];
            for (int i = 0; i < NI; ++i) grad[P_W1 + o * NI + i] += dz1[o] * xn[i];
        }
    }
    return loss;
}

/* Scale of the rounding error of each gradient entry when the products of
 * the backward pass take operands rounded to a short mantissa: every entry
 * is a sum over samples of (delta * activation) products, so its error is
 * bounded by a small multiple of the unit roundoff times
 *   A = sum over samples of |delta| * |activation|,
 * with |delta| carried backward through the absolute values of the weights
 * and of the activation derivatives (no cancellation inside a dot product
 * can hide an operand's error).  A has the layout of the gradient. */
void mlo_grad_abs(const double* p, const double* mean, const double* stdv, const double* x,
                  const double* t, int64_t n, double* A)
{
    double xn[NI], z1[NH], h1[NH], z2[NH], h2[NH], y[NO], dy[NO], dz2[NH], dz1[NH];
    const double scale = 1.0 / ((double)n * NO);
    memset(A, 0, sizeof(double) * P_COUNT);
    for (int64_t r = 0; r < n; ++r) {
        forward1(p, mean, stdv, x + r * NI, xn, z1, h1, z2, h2, y);
        for (int o = 0; o < NO; ++o) dy[o] = fabs(2.0 * (y[o] - t[r * NO + o]) * scale);
        for (int o = 0; o < NO; ++o) {
            A[P_B3 + o] += dy[o];
            for (int i = 0; i < NH; ++i) A[P_W3 + o * NH + i] += dy[o] * fabs(h2[i]);
        }
        for (int i = 0; i < NH; ++i) {
            double s = 0.0;
            for (int o = 0; o < NO; ++o) s += fabs(p[P_W3 + o * NH + i]) * dy[o];
            dz2[i] = s * fabs(gelu_grad(z2[i]));
        }
        for (int o = 0; o < NH; ++o) {
            A[P_B2 + o] += dz2[o];
            for (int i = 0; i < NH; ++i) A[P_W2 + o * NH + i] += dz2[o] * fabs(h1[i]);
        }
        for (int i = 0; i < NH; ++i) {
            double s = 0.0;
            for (int o = 0; o < NH; ++o) s += fabs(p[P_W2 + o * NH + i]) * dz2[o];
            dz1[i] = s * fabs(gelu_grad(z1[i]));
        }
        for (int o = 0; o < NH; ++o) {
            A[P_B1 + o] += dz1[o];
            for (int i = 0; i < NI; ++i) A[P_W1 + o * NI + i] += dz1[o] * fabs(xn[i]);
        }
    }
}

/* Adam (Kingma and Ba): m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
 * p <- p - lr * m/(1-b1^t) / (sqrt(v/(1-b2^t)) + eps); t counts from 1 */
void mlo_adam(double* p, double* m, double* v, const double* g, int n, int t, double lr, double b1,
              double b2, double eps)
{
    for (int k = 0; k < n; ++k) {
        m[k] = b1 * m[k] + (1.0 - b1) * g[k];
        v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k];
        double mh = m[k] / (1.0 - pow(b1, t));
        double vh = v[k] / (1.0 - pow(b2, t));
        p[k] -= lr * mh / (sqrt(vh) + eps);
    }
}
