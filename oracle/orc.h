/*
 * Oracle for the fast kernel-method path: plain, slow, obviously correct CPU
 * code in FP64 (and an 80-bit long-double twin of the transforms used only
 * to measure the FP64 oracle's own rounding error).
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header,
 * table or constant with the GPU library, and neither side includes or
 * links the other.
 *
 * Parity status of each function (what pins it) is listed in the Python
 * wrapper's module docstring; the DSI order-1 factor is "parity unpinned"
 * against the paper (it is a stated reading, pinned only by its own Walsh
 * series).
 *
 * Conventions: a coordinate is a uint64 u holding the first 64 base-2 digits
 * of x in [0,1), digit t (weight 2^-t, t = 1..64) at bit 64 - t; its FP64
 * value is u * 2^-64 rounded to nearest.
 */
#ifndef LDK_ORACLE_ORC_H
#define LDK_ORACLE_ORC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_LATTICE = 0, ORC_DNET = 1 };
enum { ORC_NATURAL = 0, ORC_LINEAR = 1, ORC_GRAY = 2 };

/* Sec. 4.2 */
int orc_lattice_points(int R, int d, int m, int order, int64_t n_min, int64_t n_max,
                       const uint64_t *g, const uint64_t *shift, uint64_t *out);
/* Sec. 4.3 (b = 2): LMS, digital shift, natural or Gray order */
int orc_dnet_points(int R, int d, int m_max, int order, int64_t n_min, int64_t n_max,
                    const uint64_t *C, const uint64_t *S, const uint64_t *shift,
                    uint64_t *out);
int orc_lms(int d, int m, const uint64_t *C, const uint64_t *S, uint64_t *Ct);
uint64_t orc_gray(uint64_t i);

/* Point sets without FWHT structure (orc_bpoints.c): digital sequences in a
 * prime base (Faure: one base b, C_j = Pascal^(j-1); Halton, Sec. 4.4: the
 * j-th prime, C_j = I) with optional LMS, digit permutations and digital
 * shift, as FP64 coordinates [R][n][d]; and nested uniform scrambling of a
 * base-2 net (Sec. 4.3) as point words [R][n][d].
 * lms: uint8 [R][d][53][53] (row t, column k); perm: uint8 [R][d][53][256];
 * shift: uint8 [R][d][53]; seed: uint64 [R][d]. */
enum { ORC_HALTON = 2, ORC_FAURE = 3 };
enum { ORC_BR_LMS = 1, ORC_BR_DP = 2, ORC_BR_DS = 4 };
int orc_bdigits(int b);
int orc_nth_prime(int j);
int orc_bpoints(int kind, int R, int d, int base, int flags, int64_t n_min, int64_t n_max,
                const uint8_t *lms, const uint8_t *perm, const uint8_t *shift, double *out);
uint64_t orc_mix64(uint64_t z);
int orc_nus_points(int R, int d, int m, int64_t n_min, int64_t n_max, const uint64_t *C,
                   const uint64_t *seed, uint64_t *out);

/* Sec. 5.2 (Bernoulli SI factor) and Sec. 5.3 / Theorem 1 (DSI factor) */
double orc_si_factor(int alpha, uint64_t delta);
double orc_dsi_factor(int alpha, uint64_t delta);
int orc_kernel_column(int kind, int R, int d, int64_t n, const uint64_t *pts,
                      const uint64_t *x0, const int *alpha, const double *gamma,
                      double zeta, double *k1);

/* Figure 3 transforms, orthonormal, in place. Complex = interleaved (re, im). */
void orc_fwht(int64_t n, double *x);
void orc_fftbr(int64_t n, double *xc);
void orc_ifftbr(int64_t n, double *xc);

/* Sec. 5.4 fast Gram algebra, batched over rows.  All arrays double.
 * kind selects FFTBR (lattice, complex spectra) or FWHT (net, real). */
int orc_transform(int kind, int dir, int B, int m, const double *in, double *out);
int orc_eig(int kind, int R, int m, const double *k1, double *lam, double *max_imag);
int orc_solve(int kind, int R, int nrhs, int m, const double *lam, double sigma2,
              const double *y, double *c);
int orc_matvec(int kind, int R, int nrhs, int m, const double *lam, const double *y,
               double *out);
int orc_logdet(int R, int m, const double *lam, double sigma2, double *out);
int orc_update_double(int kind, int B, int m, const double *yt_old, const double *y_new,
                      double *yt_full);
int orc_eig_update_double(int kind, int R, int m, const double *lam_old,
                          const double *k1_new, double *lam_full);

/* Gaussian-process log marginal likelihood in the eigenbasis of Sec. 5.4 and
 * its gradient (one response per replication; y: [R][n], g: [R][n]). */
int orc_mll(int kind, int R, int m, const double *lam, double sigma2, const double *y,
            double *L, double *g, double *dlogs2);
int orc_mll_adjoint(int kind, int R, int m, const double *g, double *a);
int orc_kernel_grad(int kind, int R, int d, int64_t n, const uint64_t *pts, const uint64_t *x0,
                    const int *alpha, const double *gamma, double zeta, const double *a,
                    double *grad);

/* Long-double twins (inputs/outputs double, arithmetic in long double). */
int orc_eig_ld(int kind, int R, int m, const double *k1, double *lam);
int orc_solve_ld(int kind, int R, int nrhs, int m, const double *lam, double sigma2,
                 const double *y, double *c);
int orc_matvec_ld(int kind, int R, int nrhs, int m, const double *lam, const double *y,
                  double *out);
int orc_logdet_ld(int R, int m, const double *lam, double sigma2, double *out);
int orc_transform_ld(int kind, int dir, int B, int m, const double *in, double *out);
/* The whole likelihood-gradient step in long double (error reference):
 * pts [R][n][d], x0 [R][d], y [R][n] -> L [R], grad [R][d + 2]. */
int orc_mll_grad_ld(int kind, int R, int d, int m, const uint64_t *pts, const uint64_t *x0,
                    const int *alpha, const double *gamma, double zeta, double sigma2,
                    const double *y, double *L, double *grad);

#ifdef __cplusplus
}
#endif
#endif
