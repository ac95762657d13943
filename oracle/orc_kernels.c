/*
 * Oracle: product-weight SI and DSI kernels (test infrastructure only).
 */
#include <math.h>
#include <stddef.h>

#include "orc.h"

/* FP64 value of a 64-digit coordinate: u * 2^-64 rounded to nearest (the C
 * conversion of uint64 to double rounds to nearest-even; scaling by 2^-64 is
 * exact). */
static double unit_value(uint64_t u) { return (double)u * 0x1p-64; }

/* Digit t (t = 1..64, weight 2^-t) of a coordinate word. */
static int digit(uint64_t u, int t) { return (int)((u >> (64 - t)) & 1u); }

/* Bernoulli numbers B_0..B_6 (textbook values). */
static const double bernoulli_number[7] = {1.0, -0.5, 1.0 / 6.0, 0.0, -1.0 / 30.0, 0.0,
                                           1.0 / 42.0};

static double binomial(int n, int k)
{
    double c = 1.0;
    for (int i = 1; i <= k; ++i) c = c * (double)(n - k + i) / (double)i;
    return c;
}

/* Bernoulli polynomial B_N(x) = sum_k binom(N,k) B_k x^(N-k). */
static double bernoulli_poly(int N, double x)
{
    double s = 0.0;
    for (int k = 0; k <= N; ++k) s += binomial(N, k) * bernoulli_number[k] * pow(x, N - k);
    return s;
}

/* Sec. 5.2: one-dimensional SI factor
 *   K_alpha(x, x') = (2 pi)^(2 alpha) / ((-1)^(alpha+1) (2 alpha)!) B_{2 alpha}((x - x') mod 1)
 * with delta = (u - u') mod 2^64 the fixed-point difference.  alpha in 1..3. */
double orc_si_factor(int alpha, uint64_t delta)
{
    const double x = unit_value(delta);
    double fact = 1.0;
    for (int i = 2; i <= 2 * alpha; ++i) fact *= (double)i;
    const double sign = (alpha % 2 == 1) ? 1.0 : -1.0; /* (-1)^(alpha+1) */
    const double coef = pow(2.0 * M_PI, 2 * alpha) / (sign * fact);
    return coef * bernoulli_poly(2 * alpha, x);
}

/* Sec. 5.3, Theorem 1 (base 2): closed forms of the DSI factors.
 *   beta(x) = -floor(log2 x) = index of the first nonzero digit of x,
 *   t_nu(x) = 2^(-nu beta(x)); both 0 at x = 0.
 * The theorem's "-1+-" is read as "-1-" (its proof in Appendix B gives that
 * sign).  delta = u XOR u' is the digitwise difference (Sec. 5.3).
 *
 * alpha = 1 is not printed in the paper (it is deferred to the literature);
 * this oracle uses the reading K_1(x) = 1 - 3 t_1(x), K_1(0) = 1, the DSI
 * kernel with Walsh coefficients 2^(-2 a_1 - 1) (a_1 = leading bit of k).
 * PARITY UNPINNED against the paper: pinned only by its own Walsh series. */
double orc_dsi_factor(int alpha, uint64_t delta)
{
    int beta = 0;
    for (int t = 1; t <= 64; ++t)
        if (digit(delta, t)) { beta = t; break; }
    const double x = unit_value(delta);
    const double b = (double)beta;
    const double t1 = beta ? ldexp(1.0, -beta) : 0.0;
    const double t2 = beta ? ldexp(1.0, -2 * beta) : 0.0;
    const double t3 = beta ? ldexp(1.0, -3 * beta) : 0.0;
    switch (alpha) {
    case 1:
        return 1.0 - 3.0 * t1;
    case 2:
        return -1.0 - b * x + 2.5 * (1.0 - t1);
    case 3:
        return -1.0 + b * x * x - 5.0 * (1.0 - t1) * x + (43.0 / 18.0) * (1.0 - t2);
    case 4: {
        /* sum_{a>=0} wal_{2^a}(x) / 2^{3a}, wal_{2^a}(x) = (-1)^{digit a+1};
         * digits beyond the 64th are zero, so the tail is sum_{a>=64} 8^-a. */
        double series = 0.0;
        for (int a = 0; a < 64; ++a)
            series += (digit(delta, a + 1) ? -1.0 : 1.0) * ldexp(1.0, -3 * a);
        series += ldexp(1.0, -192) * 8.0 / 7.0;
        return -1.0 - (2.0 / 3.0) * b * x * x * x + 5.0 * (1.0 - t1) * x * x
               - (43.0 / 9.0) * (1.0 - t2) * x + (701.0 / 294.0) * (1.0 - t3)
               + b * (series / 48.0 - 1.0 / 42.0);
    }
    default:
        return NAN;
    }
}

/* First column of the product-weight Gram matrix, eq. (K_SI_prod) and its
 * DSI analogue in Sec. 5.3:  k1_i = zeta prod_j (1 + gamma_j K_{alpha_j}(x_ij (-) x0_j)).
 * pts: [R][n][d]; x0: [R][d] (the anchor point); k1: [R][n]. */
int orc_kernel_column(int kind, int R, int d, int64_t n, const uint64_t *pts,
                      const uint64_t *x0, const int *alpha, const double *gamma,
                      double zeta, double *k1)
{
    for (int j = 0; j < d; ++j) {
        if (kind == ORC_LATTICE && (alpha[j] < 1 || alpha[j] > 3)) return -1;
        if (kind == ORC_DNET && (alpha[j] < 1 || alpha[j] > 4)) return -1;
    }
    for (int r = 0; r < R; ++r)
        for (int64_t i = 0; i < n; ++i) {
            double prod = zeta;
            for (int j = 0; j < d; ++j) {
                const uint64_t u = pts[((size_t)r * n + i) * d + j];
                const uint64_t u0 = x0[(size_t)r * d + j];
                const double f = (kind == ORC_LATTICE) ? orc_si_factor(alpha[j], u - u0)
                                                       : orc_dsi_factor(alpha[j], u ^ u0);
                prod *= 1.0 + gamma[j] * f;
            }
            k1[(size_t)r * n + i] = prod;
        }
    return 0;
}
