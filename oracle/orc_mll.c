/*
 * Oracle: Gaussian-process log marginal likelihood and its gradient in the
 * kernel parameters, through the diagonalisation of Sec. 5.4 (test
 * infrastructure only).
 *
 * The paper motivates fitting the kernel's hyperparameters by maximising the
 * marginal likelihood (Sec. 3) but prints no formula for it; the standard GP
 * objective is used, written in the eigenbasis K = V diag(lambda) V^H / n of
 * Sec. 5.4 (V unitary up to sqrt(n), so y^T (K + s2 I)^-1 y and the log
 * determinant become sums over k):
 *   L = -1/2 sum_k |yt_k|^2 / (lambda_k + s2) - 1/2 sum_k log(lambda_k + s2)
 *       - (n / 2) log(2 pi),                    yt = FT(y) (orthonormal).
 * Its derivative in lambda_k (yt does not depend on the kernel) is
 *   g_k = 1/2 |yt_k|^2 / (lambda_k + s2)^2 - 1/2 / (lambda_k + s2),
 * and dL/d log s2 = s2 sum_k g_k.  Since lambda = sqrt(n) FT(k1) is linear in
 * the first column k1, dL/dk1 is the adjoint of that map applied to g, and the
 * chain rule through k1_i = zeta prod_j (1 + gamma_j K_j(delta_ij)) gives the
 * gradient in log gamma_j and log zeta.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>

#include "orc.h"

/* L[r], g[r][n], dlogs2[r] for one response y[r][n] per replication. */
int orc_mll(int kind, int R, int m, const double *lam, double sigma2, const double *y,
            double *L, double *g, double *dlogs2)
{
    if (m < 0 || m > 26 || R < 0 || !(sigma2 >= 0.0)) return -1;
    const int64_t n = (int64_t)1 << m;
    const int lat = kind == ORC_LATTICE;
    /* yt = FT(y): complex for the lattice (FFTBR), real for the net (FWHT) */
    double *in = malloc(sizeof(double) * (size_t)n * (lat ? 2 : 1));
    double *yt = malloc(sizeof(double) * (size_t)n * (lat ? 2 : 1));
    if (!in || !yt) {
        free(in);
        free(yt);
        return -2;
    }
    int rc = 0;
    for (int r = 0; r < R && rc == 0; ++r) {
        const double *yr = y + (size_t)r * n;
        const double *lr = lam + (size_t)r * n;
        for (int64_t i = 0; i < n; ++i) {
            if (lat) {
                in[2 * i] = yr[i];
                in[2 * i + 1] = 0.0;
            } else {
                in[i] = yr[i];
            }
        }
        rc = orc_transform(kind, 1, 1, m, in, yt);
        double quad = 0.0, logdet = 0.0, gsum = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            const double p = lat ? yt[2 * k] * yt[2 * k] + yt[2 * k + 1] * yt[2 * k + 1]
                                 : yt[k] * yt[k];
            const double s = lr[k] + sigma2;
            quad += p / s;
            logdet += log(s);
            const double gk = 0.5 * p / (s * s) - 0.5 / s;
            g[(size_t)r * n + k] = gk;
            gsum += gk;
        }
        L[r] = -0.5 * quad - 0.5 * logdet - 0.5 * (double)n * log(2.0 * M_PI);
        dlogs2[r] = sigma2 * gsum;
    }
    free(in);
    free(yt);
    return rc;
}

/* a = dL/dk1 from g = dL/dlambda, the adjoint of lambda = sqrt(n) FT(k1):
 *   net:      lambda = H k1 with H symmetric, so a = H g = sqrt(n) FWHT(g);
 *   lattice:  lambda_k = Re sum_j k1_j W^{k R(j)}, so
 *             a_j = Re sum_k g_k W^{k R(j)} = Re sum_k g_k W^{-k R(j)}
 *             = Re (sqrt(n) IFFTBR(g))_j  (g real, the cosine is even). */
int orc_mll_adjoint(int kind, int R, int m, const double *g, double *a)
{
    if (m < 0 || m > 26 || R < 0) return -1;
    const int64_t n = (int64_t)1 << m;
    const double rn = sqrt((double)n);
    const int lat = kind == ORC_LATTICE;
    double *in = malloc(sizeof(double) * (size_t)n * (lat ? 2 : 1));
    double *out = malloc(sizeof(double) * (size_t)n * (lat ? 2 : 1));
    if (!in || !out) {
        free(in);
        free(out);
        return -2;
    }
    int rc = 0;
    for (int r = 0; r < R && rc == 0; ++r) {
        const double *gr = g + (size_t)r * n;
        for (int64_t k = 0; k < n; ++k) {
            if (lat) {
                in[2 * k] = gr[k];
                in[2 * k + 1] = 0.0;
            } else {
                in[k] = gr[k];
            }
        }
        rc = orc_transform(kind, lat ? -1 : 1, 1, m, in, out);
        for (int64_t j = 0; j < n; ++j) a[(size_t)r * n + j] = rn * (lat ? out[2 * j] : out[j]);
    }
    free(in);
    free(out);
    return rc;
}

/* Gradient of sum_i a_i k1_i in (log gamma_1..d, log zeta):
 *   d k1_i / d log gamma_j = zeta gamma_j K_j(delta_ij) prod_{l != j} (1 + gamma_l K_l(delta_il)),
 *   d k1_i / d log zeta    = k1_i.
 * The product over l != j is formed from prefix and suffix products, never
 * by dividing k1_i by (1 + gamma_j K_j), which can be exactly zero.
 * pts: [R][n][d]; x0: [R][d]; a: [R][n]; grad: [R][d + 1]. */
int orc_kernel_grad(int kind, int R, int d, int64_t n, const uint64_t *pts, const uint64_t *x0,
                    const int *alpha, const double *gamma, double zeta, const double *a,
                    double *grad)
{
    for (int j = 0; j < d; ++j) {
        if (kind == ORC_LATTICE && (alpha[j] < 1 || alpha[j] > 3)) return -1;
        if (kind == ORC_DNET && (alpha[j] < 1 || alpha[j] > 4)) return -1;
    }
    double *t = malloc(sizeof(double) * (size_t)(d + 1)); /* gamma_j K_j */
    double *pre = malloc(sizeof(double) * (size_t)(d + 1)); /* prod_{l < j} f_l */
    if (!t || !pre) {
        free(t);
        free(pre);
        return -2;
    }
    for (int r = 0; r < R; ++r) {
        double *gr = grad + (size_t)r * (d + 1);
        for (int j = 0; j <= d; ++j) gr[j] = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            const double ai = a[(size_t)r * n + i];
            double p = 1.0;
            for (int j = 0; j < d; ++j) {
                const uint64_t u = pts[((size_t)r * n + i) * d + j];
                const uint64_t u0 = x0[(size_t)r * d + j];
                const double K = (kind == ORC_LATTICE) ? orc_si_factor(alpha[j], u - u0)
                                                       : orc_dsi_factor(alpha[j], u ^ u0);
                t[j] = gamma[j] * K;
                pre[j] = p;
                p *= 1.0 + t[j];
            }
            double suf = 1.0;
            for (int j = d - 1; j >= 0; --j) {
                gr[j] += ai * zeta * t[j] * pre[j] * suf;
                suf *= 1.0 + t[j];
            }
            gr[d] += ai * zeta * p;
        }
    }
    free(t);
    free(pre);
    return 0;
}
