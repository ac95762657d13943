/*
 * Oracle: the whole marginal-likelihood gradient step in long double (test
 * infrastructure only).  It follows the FP64 oracle's steps (the first
 * column, lambda = sqrt(n) FT(k1), yt = FT(y), L and g = dL/dlambda, the
 * adjoint a = dL/dk1, the chain rule through the product kernel; see
 * orc_mll.c and orc_kernels.c) with every intermediate held in long double,
 * and exists only to measure the FP64 oracle's own rounding error on a
 * given input: tests gate a GPU result against the FP64 oracle by a
 * multiple of that error.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>

#include "orc.h"

long double orc_si_factor_ld(int alpha, uint64_t delta);
long double orc_dsi_factor_ld(int alpha, uint64_t delta);
void orc_fwht_ldr(int64_t n, long double *x);
void orc_fftbr_ldr(int64_t n, long double complex *x);
void orc_ifftbr_ldr(int64_t n, long double complex *x);

/* pts [R][n][d], x0 [R][d], y [R][n] -> L [R], grad [R][d + 2] in
 * (log gamma_1..d, log zeta, log sigma2), rounded to double at the end. */
int orc_mll_grad_ld(int kind, int R, int d, int m, const uint64_t *pts, const uint64_t *x0,
                    const int *alpha, const double *gamma, double zeta, double sigma2,
                    const double *y, double *L, double *grad)
{
    if (m < 0 || m > 26 || R < 0 || d < 1 || !(sigma2 >= 0.0)) return -1;
    for (int j = 0; j < d; ++j) {
        if (kind == ORC_LATTICE && (alpha[j] < 1 || alpha[j] > 3)) return -1;
        if (kind == ORC_DNET && (alpha[j] < 1 || alpha[j] > 4)) return -1;
    }
    const int64_t n = (int64_t)1 << m;
    const int lat = kind == ORC_LATTICE;
    const long double rn = sqrtl((long double)n), s2 = sigma2, z = zeta;
    long double *k1 = malloc(sizeof(long double) * (size_t)n);
    long double *lam = malloc(sizeof(long double) * (size_t)n);
    long double *g = malloc(sizeof(long double) * (size_t)n);
    long double *a = malloc(sizeof(long double) * (size_t)n);
    long double *wr = malloc(sizeof(long double) * (size_t)n);
    long double complex *wc = malloc(sizeof(long double complex) * (size_t)n);
    long double *t = malloc(sizeof(long double) * (size_t)(d + 1));
    long double *pre = malloc(sizeof(long double) * (size_t)(d + 1));
    long double *gr = malloc(sizeof(long double) * (size_t)(d + 2));
    int rc = 0;
    if (!k1 || !lam || !g || !a || !wr || !wc || !t || !pre || !gr) rc = -2;
    for (int r = 0; r < R && rc == 0; ++r) {
        /* first column, eq. (K_SI_prod) and its DSI analogue */
        for (int64_t i = 0; i < n; ++i) {
            long double prod = z;
            for (int j = 0; j < d; ++j) {
                const uint64_t u = pts[((size_t)r * n + i) * d + j];
                const uint64_t u0 = x0[(size_t)r * d + j];
                const long double f = lat ? orc_si_factor_ld(alpha[j], u - u0)
                                          : orc_dsi_factor_ld(alpha[j], u ^ u0);
                prod *= 1 + (long double)gamma[j] * f;
            }
            k1[i] = prod;
        }
        /* lambda = sqrt(n) FT(k1) (real part for the lattice) */
        if (lat) {
            for (int64_t i = 0; i < n; ++i) wc[i] = k1[i];
            orc_fftbr_ldr(n, wc);
            for (int64_t k = 0; k < n; ++k) lam[k] = rn * creall(wc[k]);
        } else {
            for (int64_t i = 0; i < n; ++i) wr[i] = k1[i];
            orc_fwht_ldr(n, wr);
            for (int64_t k = 0; k < n; ++k) lam[k] = rn * wr[k];
        }
        /* yt = FT(y), L, g = dL/dlambda, dL/dlog s2 = s2 sum g */
        long double quad = 0, logdet = 0, gsum = 0;
        if (lat) {
            for (int64_t i = 0; i < n; ++i) wc[i] = y[(size_t)r * n + i];
            orc_fftbr_ldr(n, wc);
        } else {
            for (int64_t i = 0; i < n; ++i) wr[i] = y[(size_t)r * n + i];
            orc_fwht_ldr(n, wr);
        }
        for (int64_t k = 0; k < n; ++k) {
            const long double p = lat ? creall(wc[k]) * creall(wc[k]) + cimagl(wc[k]) * cimagl(wc[k])
                                      : wr[k] * wr[k];
            const long double s = lam[k] + s2;
            quad += p / s;
            logdet += logl(s);
            g[k] = p / (2 * s * s) - 1 / (2 * s);
            gsum += g[k];
        }
        L[r] = (double)(-quad / 2 - logdet / 2 -
                        (long double)n / 2 * logl(2 * 3.14159265358979323846264338327950288L));
        /* a = dL/dk1: net H g = sqrt(n) FWHT(g); lattice Re sqrt(n) IFFTBR(g) */
        if (lat) {
            for (int64_t k = 0; k < n; ++k) wc[k] = g[k];
            orc_ifftbr_ldr(n, wc);
            for (int64_t j = 0; j < n; ++j) a[j] = rn * creall(wc[j]);
        } else {
            for (int64_t k = 0; k < n; ++k) wr[k] = g[k];
            orc_fwht_ldr(n, wr);
            for (int64_t j = 0; j < n; ++j) a[j] = rn * wr[j];
        }
        /* chain rule through the product kernel, prefix / suffix products */
        for (int j = 0; j < d + 2; ++j) gr[j] = 0;
        for (int64_t i = 0; i < n; ++i) {
            long double p = 1;
            for (int j = 0; j < d; ++j) {
                const uint64_t u = pts[((size_t)r * n + i) * d + j];
                const uint64_t u0 = x0[(size_t)r * d + j];
                const long double K = lat ? orc_si_factor_ld(alpha[j], u - u0)
                                          : orc_dsi_factor_ld(alpha[j], u ^ u0);
                t[j] = (long double)gamma[j] * K;
                pre[j] = p;
                p *= 1 + t[j];
            }
            long double suf = 1;
            for (int j = d - 1; j >= 0; --j) {
                gr[j] += a[i] * z * t[j] * pre[j] * suf;
                suf *= 1 + t[j];
            }
            gr[d] += a[i] * z * p;
        }
        gr[d + 1] = s2 * gsum;
        for (int j = 0; j < d + 2; ++j) grad[(size_t)r * (d + 2) + j] = (double)gr[j];
    }
    free(k1);
    free(lam);
    free(g);
    free(a);
    free(wr);
    free(wc);
    free(t);
    free(pre);
    free(gr);
    return rc;
}
