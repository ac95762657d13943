/*
 * Oracle: product-weight SI and DSI kernels (test infrastructure only).  The
 * one-dimensional factors live in orc_kernels.inc, compiled here in double
 * (the oracle) and in long double (its error reference).
 */
#include <math.h>
#include <stddef.h>

#include "orc.h"

/* Digit t (t = 1..64, weight 2^-t) of a coordinate word. */
static int digit(uint64_t u, int t) { return (int)((u >> (64 - t)) & 1u); }

/* ---- FP64 instantiation ---- */
#define REAL double
#define FN(name) dbl_##name
#define RPOW pow
#define RLDEXP ldexp
#define PI_R 3.14159265358979323846264338327950288
#include "orc_kernels.inc"
#undef REAL
#undef FN
#undef RPOW
#undef RLDEXP
#undef PI_R

/* ---- long double instantiation (error reference) ---- */
#define REAL long double
#define FN(name) ldb_##name
#define RPOW powl
#define RLDEXP ldexpl
#define PI_R 3.14159265358979323846264338327950288L
#include "orc_kernels.inc"

double orc_si_factor(int alpha, uint64_t delta) { return dbl_si_factor(alpha, delta); }
double orc_dsi_factor(int alpha, uint64_t delta) { return dbl_dsi_factor(alpha, delta); }
long double orc_si_factor_ld(int alpha, uint64_t delta) { return ldb_si_factor(alpha, delta); }
long double orc_dsi_factor_ld(int alpha, uint64_t delta) { return ldb_dsi_factor(alpha, delta); }

/* Threads the OpenMP loops may use (1 unless built with -fopenmp). */
#ifdef _OPENMP
#include <omp.h>
int orc_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int t) { omp_set_num_threads(t > 0 ? t : 1); }
#else
int orc_threads(void) { return 1; }
void orc_set_threads(int t) { (void)t; }
#endif

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
    /* every entry is independent (OpenMP in the CPU-baseline build only) */
#pragma omp parallel for collapse(2) schedule(static)
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
