/*
 * Oracle: fast transforms and structured Gram algebra of Sec. 5 (test
 * infrastructure only).  The arithmetic lives in orc_algebra.inc, compiled
 * here in double and in long double.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>

#include "orc.h"

/* ---- FP64 instantiation ---- */
#define REAL double
#define CPLX double complex
#define FN(name) dbl_##name
#define RCOS cos
#define RSIN sin
#define RLOG log
#define RSQRT sqrt
#define PI_R 3.14159265358979323846264338327950288
#define CREAL creal
#define CIMAG cimag
#define CONJ conj
#include "orc_algebra.inc"
#undef REAL
#undef CPLX
#undef FN
#undef RCOS
#undef RSIN
#undef RLOG
#undef RSQRT
#undef PI_R
#undef CREAL
#undef CIMAG
#undef CONJ

/* ---- long double instantiation (error reference) ---- */
#define REAL long double
#define CPLX long double complex
#define FN(name) ldb_##name
#define RCOS cosl
#define RSIN sinl
#define RLOG logl
#define RSQRT sqrtl
#define PI_R 3.14159265358979323846264338327950288L
#define CREAL creall
#define CIMAG cimagl
#define CONJ conjl
#include "orc_algebra.inc"

void orc_fwht(int64_t n, double *x) { dbl_fwht(n, x); }
void orc_fftbr(int64_t n, double *xc) { dbl_fftbr(n, (double complex *)xc); }
void orc_ifftbr(int64_t n, double *xc) { dbl_ifftbr(n, (double complex *)xc); }

int orc_transform(int kind, int dir, int B, int m, const double *in, double *out)
{
    return dbl_transform_impl(kind, dir, B, m, in, out);
}
int orc_transform_ld(int kind, int dir, int B, int m, const double *in, double *out)
{
    return ldb_transform_impl(kind, dir, B, m, in, out);
}
int orc_eig(int kind, int R, int m, const double *k1, double *lam, double *max_imag)
{
    return dbl_eig_impl(kind, R, m, k1, lam, max_imag);
}
int orc_eig_ld(int kind, int R, int m, const double *k1, double *lam)
{
    return ldb_eig_impl(kind, R, m, k1, lam, 0);
}
int orc_solve(int kind, int R, int nrhs, int m, const double *lam, double sigma2,
              const double *y, double *c)
{
    return dbl_apply_impl(kind, R, nrhs, m, lam, sigma2, y, c, 0);
}
int orc_solve_ld(int kind, int R, int nrhs, int m, const double *lam, double sigma2,
                 const double *y, double *c)
{
    return ldb_apply_impl(kind, R, nrhs, m, lam, sigma2, y, c, 0);
}
int orc_matvec(int kind, int R, int nrhs, int m, const double *lam, const double *y,
               double *out)
{
    return dbl_apply_impl(kind, R, nrhs, m, lam, 0.0, y, out, 1);
}
int orc_matvec_ld(int kind, int R, int nrhs, int m, const double *lam, const double *y,
                  double *out)
{
    return ldb_apply_impl(kind, R, nrhs, m, lam, 0.0, y, out, 1);
}
int orc_logdet(int R, int m, const double *lam, double sigma2, double *out)
{
    return dbl_logdet_impl(R, m, lam, sigma2, out);
}
int orc_logdet_ld(int R, int m, const double *lam, double sigma2, double *out)
{
    return ldb_logdet_impl(R, m, lam, sigma2, out);
}

/* Sec. 5.4, transform update (eq. (ft_next_parts) and the two listings):
 *   y~_{m+1} = 2^-1/2 [ y~_m + w (.) y~_new ; y~_m - w (.) y~_new ],
 * y~_new = FFTBR_m(y_new) with w_k = exp(-pi i k / n) (lattice), or
 * y~_new = FWHT_m(y_new) with w = 1 (net).  Lattice spectra are complex
 * (interleaved); y_new is real. */
int orc_update_double(int kind, int B, int m, const double *yt_old, const double *y_new,
                      double *yt_full)
{
    const int64_t n = (int64_t)1 << m;
    const double h = 1.0 / sqrt(2.0);
    if (kind == ORC_LATTICE) {
        double complex *w = (double complex *)malloc(sizeof(double complex) * (size_t)n);
        if (!w) return -2;
        for (int b = 0; b < B; ++b) {
            for (int64_t i = 0; i < n; ++i) w[i] = y_new[(size_t)b * n + i];
            dbl_fftbr(n, w);
            const double *old = yt_old + (size_t)b * 2 * n;
            double *full = yt_full + (size_t)b * 4 * n;
            for (int64_t k = 0; k < n; ++k) {
                const double ang = -M_PI * (double)k / (double)n;
                const double complex om = cos(ang) + sin(ang) * I;
                const double complex a = old[2 * k] + old[2 * k + 1] * I;
                const double complex top = (a + om * w[k]) * h, bot = (a - om * w[k]) * h;
                full[2 * k] = creal(top);
                full[2 * k + 1] = cimag(top);
                full[2 * (n + k)] = creal(bot);
                full[2 * (n + k) + 1] = cimag(bot);
            }
        }
        free(w);
    } else {
        double *w = (double *)malloc(sizeof(double) * (size_t)n);
        if (!w) return -2;
        for (int b = 0; b < B; ++b) {
            for (int64_t i = 0; i < n; ++i) w[i] = y_new[(size_t)b * n + i];
            dbl_fwht(n, w);
            const double *old = yt_old + (size_t)b * n;
            double *full = yt_full + (size_t)b * 2 * n;
            for (int64_t k = 0; k < n; ++k) {
                full[k] = (old[k] + w[k]) * h;
                full[n + k] = (old[k] - w[k]) * h;
            }
        }
        free(w);
    }
    return 0;
}

/* Eigenvalue update when n doubles: with lambda_hat = sqrt(n) FT_m(k1_new)
 * (k1_new = first-column entries of the points n..2n-1),
 *   lambda_{m+1} = [ lambda_m + w (.) lambda_hat ; lambda_m - w (.) lambda_hat ],
 * real part taken for the lattice (the exact result is real). */
int orc_eig_update_double(int kind, int R, int m, const double *lam_old,
                          const double *k1_new, double *lam_full)
{
    const int64_t n = (int64_t)1 << m;
    const double sn = sqrt((double)n);
    if (kind == ORC_LATTICE) {
        double complex *w = (double complex *)malloc(sizeof(double complex) * (size_t)n);
        if (!w) return -2;
        for (int r = 0; r < R; ++r) {
            for (int64_t i = 0; i < n; ++i) w[i] = k1_new[(size_t)r * n + i];
            dbl_fftbr(n, w);
            for (int64_t k = 0; k < n; ++k) {
                const double ang = -M_PI * (double)k / (double)n;
                const double complex om = cos(ang) + sin(ang) * I;
                const double part = creal(om * w[k]) * sn;
                lam_full[(size_t)r * 2 * n + k] = lam_old[(size_t)r * n + k] + part;
                lam_full[(size_t)r * 2 * n + n + k] = lam_old[(size_t)r * n + k] - part;
            }
        }
        free(w);
    } else {
        double *w = (double *)malloc(sizeof(double) * (size_t)n);
        if (!w) return -2;
        for (int r = 0; r < R; ++r) {
            for (int64_t i = 0; i < n; ++i) w[i] = k1_new[(size_t)r * n + i];
            dbl_fwht(n, w);
            for (int64_t k = 0; k < n; ++k) {
                lam_full[(size_t)r * 2 * n + k] = lam_old[(size_t)r * n + k] + sn * w[k];
                lam_full[(size_t)r * 2 * n + n + k] = lam_old[(size_t)r * n + k] - sn * w[k];
            }
        }
        free(w);
    }
    return 0;
}

/* Long-double transforms on long-double data, for the extended-precision
 * twin of the likelihood path (orc_mll_ld.c). */
void orc_fwht_ldr(int64_t n, long double *x) { ldb_fwht(n, x); }
void orc_fftbr_ldr(int64_t n, long double complex *x) { ldb_fftbr(n, x); }
void orc_ifftbr_ldr(int64_t n, long double complex *x) { ldb_ifftbr(n, x); }
