/*
 * ldk.h -- C ABI of the MI355X (gfx950) fast kernel-method library.
 *
 * Fast Gram-matrix algebra on randomized low-discrepancy point sets, after
 * "QMCPy: randomized low-discrepancy sequences, quasi-Monte Carlo, and fast
 * kernel methods" (arXiv 2502.14256):
 *   - randomized rank-1 lattices and base-2 digital nets as exact 64-digit
 *     words (Sec. 4.2, 4.3);
 *   - the first column of product-weight shift-invariant (SI, lattice) or
 *     digitally-shift-invariant (DSI, net) Gram matrices (Sec. 5.2, 5.3,
 *     Theorem 1);
 *   - eigenvalues, matvec, solve and log-det through FFTBR/IFFTBR (lattice)
 *     or the FWHT (net), and the transform update that doubles n (Sec. 5.4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every data pointer is a DEVICE pointer owned by the caller (HIP device
 *    memory on the current device).  Struct arguments themselves live in
 *    host memory.  The library never allocates or frees caller memory.
 *  - Calls validate their arguments on the host, then enqueue kernels on
 *    `stream` and return without synchronising; outputs are valid once the
 *    stream has reached that point.  An invalid call enqueues nothing.
 *  - Return value: LDK_OK (0) or a negative ldk_status.  After LDK_EDEVICE
 *    the HIP error of the failing call is available from ldk_last_hip_error()
 *    (per host thread).  No C++ exception crosses this boundary.
 *  - Sizes: transforms act on n = 2^m entries, 0 <= m <= LDK_MAX_M (the
 *    update entry points need m + 1 <= LDK_MAX_M).  Arrays are contiguous and
 *    row-major; batch dimensions come first.
 *  - A coordinate is a uint64 word u holding the first 64 base-2 digits of
 *    x in [0,1): digit t (weight 2^-t, t = 1..64) is bit 64 - t.  Floating
 *    kernels use x = u * 2^-64 rounded to nearest.
 *  - Real data are double (LDK_F64) or float (LDK_F32) as selected by
 *    `dtype`; complex data are interleaved (re, im) pairs of that type.
 *  - Eigenvalues are always FP64 (double): the small ones carry an absolute
 *    rounding error of about u ||k1|| and decide lambda + sigma^2, so they are
 *    never held in FP32.  `dtype` selects the storage and transform
 *    arithmetic of the per-solve data (k1, y, c, transformed responses); the
 *    nugget sigma^2 is added, and divided by, in FP64.
 *  - Calls are reentrant.  Twiddle tables are built once per device by
 *    ldk_init() (called implicitly by the first entry point that needs it;
 *    call it explicitly before capturing calls into a HIP graph).
 */
#ifndef LDK_H
#define LDK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque stream handle: pass a hipStream_t (or 0 for the null stream). */
typedef void *ldk_stream;

#define LDK_MAX_M 26 /* largest transform length log2(n) (eig, solve, ...) */
#define LDK_MAX_D 4096 /* largest supported dimension */

typedef enum {
    LDK_OK = 0,
    LDK_EINVAL = -1,  /* bad argument (nothing enqueued) */
    LDK_ENOTSUP = -2, /* valid but unsupported combination */
    LDK_EDEVICE = -3, /* a HIP call failed; see ldk_last_hip_error() */
    LDK_ENOTSPD = -4, /* some lambda_k + sigma^2 <= 0 (checked entry points) */
    LDK_ETOOBIG = -5  /* input exceeds the fixed scratch of an allocation-free entry point */
} ldk_status;

/* Size of the fixed device scratch of ldk_solve_noalloc (per GPU, held
 * until the process ends). */
#define LDK_NOALLOC_SCRATCH_BYTES (16u << 20)

typedef enum { LDK_LATTICE = 0, LDK_DNET_B2 = 1 } ldk_kind;
typedef enum { LDK_NATURAL = 0, LDK_LINEAR = 1, LDK_GRAY = 2 } ldk_order;
typedef enum { LDK_F64 = 0, LDK_F32 = 1 } ldk_dtype;

/* A randomized low-discrepancy point set (host struct, device arrays).
 *  kind  LDK_LATTICE: rank-1 lattice sequence z_i = v(i) g mod 1 (Sec. 4.2,
 *        van der Corput v of Sec. 4.1), shifted x_i = (z_i + Delta) mod 1.
 *        order NATURAL (radical inverse, extensible) or LINEAR (fixed
 *        n = 2^m_max: z_i = i g / n mod 1).
 *        gen = g[d] (uint64; only g mod 2^64 matters).
 *  kind  LDK_DNET_B2: base-2 digital net z_ij = F(C_j D(i) mod 2) (Sec. 4.3),
 *        with linear matrix scrambling Ct_j = S_j C_j mod 2 and digital shift
 *        x_ij = z_ij XOR Delta_j.  order NATURAL or GRAY (point i uses the
 *        digit vector of i XOR (i >> 1); Table 1).
 *        gen = C[d][m_max]: one word per column k, row t at bit 63 - t.
 *        lms = S[R][d][64]: one word per row t, entry (t, s) at bit 63 - s,
 *        or NULL for no scrambling.
 *  shift = Delta[R][d] (digital shift digits, or the 64-bit fixed-point
 *        lattice shift), or NULL for none.
 *  R     number of independent randomizations (replications), >= 1.
 *  m_max points exist for indices 0 <= i < 2^m_max (nets, linear lattices);
 *        natural-order lattices accept any i < 2^62.
 *  flags 0, or LDK_GEN_PER_REPLICATION (nets only): gen holds the columns of
 *        every replication, C[R][d][m_max] (for instance the interlaced,
 *        scrambled columns of a higher-order net from ldk_interlace, with
 *        lms = NULL). */
#define LDK_GEN_PER_REPLICATION 1
typedef struct {
    int32_t kind;
    int32_t order;
    int32_t R;
    int32_t d;
    int32_t m_max;
    int32_t flags;
    const uint64_t *gen;
    const uint64_t *lms;
    const uint64_t *shift;
} ldk_pointset;

/* Product-weight kernel  K(x, x') = zeta prod_j (1 + gamma_j K_{alpha_j}(x_j (-) x'_j)).
 *  kind  LDK_LATTICE: SI factor (Sec. 5.2, eq. K_SI_prod)
 *        K_a(x) = (2 pi)^{2a} / ((-1)^{a+1} (2a)!) B_{2a}(x), x = (u - u') mod 1,
 *        alpha_j in {1, 2, 3}.
 *  kind  LDK_DNET_B2: DSI factor (Sec. 5.3, Theorem 1), x = u XOR u',
 *        alpha_j in {1, 2, 3, 4}; alpha = 1 is the order-1 kernel
 *        K_1(x) = 1 - 3 * 2^{-beta(x)} (a reading: the paper defers its form
 *        to the literature).
 *  alpha = HOST int32[d] (orders are configuration: validated on the host,
 *  an order outside the range above gives LDK_EINVAL, and uniform orders get
 *  specialised kernels); gamma = device double[d]; zeta > 0. */
typedef struct {
    int32_t kind;
    int32_t d;
    const int32_t *alpha;
    const double *gamma;
    double zeta;
} ldk_kernel;

/* Build the per-device twiddle tables (once per device; thread safe).
 * Synchronous.  Returns LDK_OK or LDK_EDEVICE. */
int ldk_init(void);

/* Tuned plan parameters.  The transform passes of ldk_transform, ldk_eig,
 * ldk_solve, ldk_matvec and ldk_fit use a tile of 2^log_tile elements per
 * workgroup and in-register butterfly groups of radix r (2, 4 or 8); the
 * defaults (2^11 complex FP64 elements, 2^12 otherwise; radix 8) can be
 * replaced per (kind, working dtype, log2 n, number of rows) by a table
 * that the project's tuner (paper_2502_14256_amd/tune.py) writes after
 * timing the candidates on the device.  File format: one entry per line,
 *     kind dtype m rows_log2 log_tile log2_radix [engine]
 * (kind and dtype as the enums below; '#' starts a comment line).  The
 * optional engine field selects the Walsh-Hadamard passes of FP32
 * digital-net solves and matvecs: 0 (the default) the FP32 butterflies, 1
 * the split-FP16 matrix-core passes of ldk_fwht_split16 (allowed only for
 * kind LDK_DNET_B2, dtype LDK_F32 and m >= 12; normwise error of order 1e-7
 * per transform, like the butterflies; the eigenvalues stay FP64).  For a
 * call with `rows` rows (R * nrhs for solves) the entry with the largest
 * rows_log2 <= floor(log2 rows) applies.  ldk_init_tuned(path) builds the
 * twiddle tables (as ldk_init) and replaces the table; path = NULL clears it.
 * Returns LDK_EINVAL, leaving the table unchanged, when the file cannot be
 * read or names a plan the pass kernels cannot run.  Results of a call
 * depend on the plan (the rounding order of the passes), within the
 * tolerances the tests state; workspace sizes (ldk_workspace_bytes) cover
 * every plan the table may select.  Not to be called while other threads
 * enqueue transform calls. */
int ldk_init_tuned(const char *path);

/* The plan a call of (kind, dtype, log2 n = m, rows) would use: *log_tile,
 * *radix (2, 4 or 8), *passes (HBM round trips of one transform) and
 * *engine (0 butterflies, 1 split-FP16 matrix cores).  Any output pointer
 * may be NULL. */
int ldk_plan_info(int kind, int dtype, int m, int64_t rows, int *log_tile, int *radix,
                  int *passes, int *engine);

/* Points i = n_min .. n_max-1 of every replication (Sec. 4.2, 4.3).
 * out = uint64[R][n_max - n_min][d].  Requires 0 <= n_min <= n_max and, for
 * nets and linear lattices, n_max <= 2^m_max. */
int ldk_gen_points(const ldk_pointset *ps, int64_t n_min, int64_t n_max, uint64_t *out,
                   ldk_stream stream);

/* Generating columns of a higher-order base-2 digital net by digital
 * interlacing (Sec. 4.3, digital interlacing for higher-order nets, and
 * higher-order LMS: scramble the alpha d source matrices, then interlace).
 * src: a base-2 net of alpha d dimensions, gen = C[alpha d][m_max] (shared,
 * flags = 0), lms = S[R][alpha d][64] or NULL; its shift and order are not
 * used.  Output, for replication r, dimension j < d, column k < m_max:
 *   digit t of cols[r][j][k] (bit 63 - t, t < 64) =
 *   digit floor(t / alpha) of column k of S_s C_s, s = alpha j + (t mod alpha)
 * (0-based j and s: row t of the interlaced matrix is row floor(t / alpha) of
 * source matrix alpha j + (t mod alpha); 64 digits are kept, so the top
 * 64 / alpha digits of each source column enter).  cols = uint64[R][d][m_max]
 * device, for a net with flags = LDK_GEN_PER_REPLICATION, lms = NULL and a
 * d-dimensional shift of its own.  alpha in 1..4; src->d must be a multiple
 * of alpha.  alpha = 1 gives each replication's scrambled columns S_j C_j:
 * with them (and the same shift) the net yields the same points as the LMS
 * net, and the kernels that regenerate points skip the scrambling. */
int ldk_interlace(const ldk_pointset *src, int alpha, uint64_t *cols, ldk_stream stream);

/* First Gram column k1_i = K(x_i, x_0) for i = n_min .. n_max-1 (Sec. 5.4:
 * only the first column is stored).  Points come from `pts` =
 * uint64[R][n_max - n_min][d] with anchor rows x0 = uint64[R][d] (x0 may be
 * NULL when n_min == 0: row 0 of pts is then the anchor), or, when pts is
 * NULL, are regenerated on the fly from `ps` with the anchor at index 0.
 * ps must be given in both cases (it supplies R, d and kind).
 * k->kind must equal ps->kind.  out = dtype[R][n_max - n_min]. */
int ldk_kernel_column(const ldk_kernel *k, const ldk_pointset *ps, const uint64_t *pts,
                      const uint64_t *x0, int64_t n_min, int64_t n_max, int dtype,
                      void *out, ldk_stream stream);

/* Points and first Gram column in one call: the outputs of
 *   ldk_gen_points(ps, n_min, n_max, pts) and
 *   ldk_kernel_column(k, ps, NULL, NULL, n_min, n_max, dtype, k1),
 * bit for bit (Sec. 4.2, 4.3 and 5.4), with the same arguments, layouts and
 * restrictions.  The column regenerates the points in registers and does
 * not read pts, so the two run as one launch, the column's arithmetic
 * beside the point words' stores.  pts and k1 must not overlap. */
int ldk_points_column(const ldk_kernel *k, const ldk_pointset *ps, int64_t n_min, int64_t n_max,
                      uint64_t *pts, int dtype, void *k1, ldk_stream stream);

/* Orthonormal transform of B rows of length n = 2^m (Figure 3, Sec. 5.2-5.3).
 *  LDK_LATTICE: complex rows; dir = +1 FFTBR  y_k = n^-1/2 sum_j x_j W^{k R_m(j)},
 *               dir = -1 IFFTBR (its inverse), W = exp(-2 pi i / n).
 *  LDK_DNET_B2: real rows; FWHT  y_k = n^-1/2 sum_j (-1)^{popcount(j & k)} x_j
 *               (dir ignored: the FWHT is its own inverse).
 * in and out may alias exactly (in place).  ws: workspace of
 * ldk_workspace_bytes(LDK_OP_TRANSFORM, ...) bytes (may be NULL if 0). */
int ldk_transform(int kind, int dir, int B, int m, int dtype, const void *in, void *out,
                  void *ws, ldk_stream stream);

/* Eigenvalues lambda = sqrt(n) conj(V_m) k1 (Sec. 5.4): sqrt(n) FFTBR(k1)
 * (lattice; real since K is real symmetric) or sqrt(n) FWHT(k1) (net).
 * k1 = real dtype[R][n]; lam = double[R][n], natural frequency / Walsh
 * order.  The transform runs in FP64 for either input dtype; lattice
 * lam_k = Re sqrt(n) FFTBR(k1)_k.
 * ws: ldk_workspace_bytes(LDK_OP_EIG, ...) bytes (lattice with n > 2^12 only). */
int ldk_eig(int kind, int R, int m, int dtype, const void *k1, double *lam, void *ws,
            ldk_stream stream);

/* Solve (K + sigma^2 I) c = y:  c = V (conj(V) y (/) (lambda + sigma^2)) (Sec. 5.4).
 * lam = double[R][n]; y, c = dtype[R][nrhs][n] (y and c may alias exactly;
 * right-hand side q of replication r uses row r of lam).  sigma2 >= 0; the
 * division is done in FP64.  Lattice: c is the real part of that product
 * (the whole of it when lambda_k = lambda_{n-k}, as for a real symmetric K);
 * for n >= 4 the real rows run as packed complex rows of n/2.
 * ws: ldk_workspace_bytes(LDK_OP_SOLVE, kind, R * nrhs, m, dtype) bytes
 * (lattice with n > 2^12 in FP64, n > 2^13 in FP32, only). */
int ldk_solve(int kind, int R, int nrhs, int m, int dtype, const double *lam, double sigma2,
              const void *y, void *c, void *ws, ldk_stream stream);

/* ldk_solve, checked: K + sigma^2 I = V (Lambda + sigma^2 I) conj(V) with V
 * unitary (Sec. 5.4) is positive definite exactly when every
 * lambda_k + sigma^2 > 0.  This variant first counts, on the device, the
 * eigenvalues of every row of lam that fail that test (NaN fails), waits for
 * the count (it SYNCHRONISES `stream`), and returns LDK_ENOTSPD without
 * enqueueing the solve when it is not zero; otherwise it enqueues exactly
 * what ldk_solve enqueues and returns.  Same arguments and layouts as
 * ldk_solve.  Checked calls on one device are serialised by the library
 * (they share one device counter). */
int ldk_solve_checked(int kind, int R, int nrhs, int m, int dtype, const double *lam,
                      double sigma2, const void *y, void *c, void *ws, ldk_stream stream);

/* ldk_solve without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The intermediate
 * rows that ldk_solve keeps in `ws` live instead in a fixed device array of
 * LDK_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends (its address is looked up once per device, by
 * ldk_init or by this call's first use on a device).  Returns LDK_ETOOBIG,
 * enqueueing nothing, when ldk_workspace_bytes(LDK_OP_SOLVE, kind, R * nrhs,
 * m, dtype) exceeds that size (for instance FP64 lattice rows with
 * R * nrhs * n > 2^22).  Otherwise the same arguments, results (bit for bit)
 * and stream semantics as ldk_solve.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (other streams, other host
 * threads) race and give wrong results; nothing in it needs clearing
 * between calls (every intermediate is written before it is read). */
int ldk_solve_noalloc(int kind, int R, int nrhs, int m, int dtype, const double *lam,
                      double sigma2, const void *y, void *c, ldk_stream stream);

/* Matvec K y = V (conj(V) y (.) lambda) (Sec. 5.4); layout as ldk_solve. */
int ldk_matvec(int kind, int R, int nrhs, int m, int dtype, const double *lam, const void *y,
               void *out, void *ws, ldk_stream stream);

/* log det(K + sigma^2 I) = sum_k log(lambda_k + sigma^2) (V unitary, Sec. 5.4),
 * accumulated in FP64 in a fixed order (bit-reproducible run to run).
 * lam = double[R][n]; out = device double[R]; a row with some
 * lambda_k + sigma^2 <= 0 yields NaN.  ws: ldk_workspace_bytes(LDK_OP_LOGDET). */
int ldk_logdet(int R, int m, const double *lam, double sigma2, double *out, void *ws,
               ldk_stream stream);

/* ldk_logdet, checked: returns LDK_ENOTSPD (and enqueues nothing more)
 * when some lambda_k + sigma^2 <= 0 or is NaN, instead of a NaN log-det;
 * SYNCHRONISES `stream` (see ldk_solve_checked).  Same arguments. */
int ldk_logdet_checked(int R, int m, const double *lam, double sigma2, double *out, void *ws,
                       ldk_stream stream);

/* The fit of Sec. 5.4 in one call: lam = eigenvalues of k1 (as ldk_eig),
 * c = (K + sigma^2 I)^-1 y (as ldk_solve, nrhs right-hand sides per
 * replication; nrhs may be 0) and, if logdet != NULL, logdet[r] (as
 * ldk_logdet).  Lattice rows in FP64 with n >= 4 share launches: the
 * column's and the right-hand sides' forward passes run as one launch, and
 * the pass that forms the eigenvalues also sums their logarithms per tile,
 * so the log-det costs one small reduction instead of a pass over lambda.
 * Other cases run the three entry points in turn.  lam and c equal the
 * separate calls bit for bit; the log-det to rounding (another fixed
 * summation order).
 * k1 = dtype[R][n]; y, c = dtype[R][nrhs][n]; lam = double[R][n];
 * logdet = device double[R].
 * ws: ldk_workspace_bytes(LDK_OP_FIT, kind, R * (nrhs + 1), m, dtype) bytes. */
int ldk_fit(int kind, int R, int nrhs, int m, int dtype, const void *k1, double sigma2,
            const void *y, double *lam, void *c, double *logdet, void *ws, ldk_stream stream);

/* Transform update when n doubles (Sec. 5.4, eq. ft_next_parts and its listings):
 *   yt_full = 2^-1/2 [ yt_old + w (.) FT_m(y_new) ; yt_old - w (.) FT_m(y_new) ],
 * w_k = exp(-pi i k / n) (lattice, FT = FFTBR) or 1 (net, FT = FWHT).
 * yt_old = [B][n] (complex for lattice, real for net), y_new = real [B][n],
 * yt_full = [B][2n] (complex for lattice, real for net).
 * Equals FT_{m+1} of the concatenation [y_old ; y_new]. */
int ldk_update_double(int kind, int B, int m, int dtype, const void *yt_old,
                      const void *y_new, void *yt_full, void *ws, ldk_stream stream);

/* Eigenvalue update when n doubles:  with lh = sqrt(n) FT_m(k1_new),
 *   lam_full = [ lam_old + Re(w (.) lh) ; lam_old - Re(w (.) lh) ],
 * k1_new = first-column entries of points n .. 2n-1 (dtype [R][n]);
 * lam_old = double[R][n]; lam_full = double[R][2n].  FP64 arithmetic.
 * ws: ldk_workspace_bytes(LDK_OP_EIG_UPDATE_DOUBLE, ...) bytes (lattice). */
int ldk_eig_update_double(int kind, int R, int m, int dtype, const double *lam_old,
                          const void *k1_new, double *lam_full, void *ws, ldk_stream stream);

/* Gaussian-process log marginal likelihood in the eigenbasis (Sec. 5.4; the
 * paper motivates fitting kernel parameters by it in Sec. 3 but prints no
 * formula, so the standard GP objective is used).  One response per
 * replication, yt = FT(y) orthonormal:
 *   L[r]      = -1/2 sum_k |yt_k|^2 / (lambda_k + s2) - 1/2 sum_k log(lambda_k + s2)
 *               - (n/2) log(2 pi),
 *   g[r][k]   = dL/dlambda_k = 1/2 |yt_k|^2 / (lambda_k + s2)^2 - 1/2 / (lambda_k + s2),
 *   dlogs2[r] = dL/dlog s2 = s2 sum_k g[r][k]   (dlogs2 may be NULL).
 * lam = double[R][n] (ldk_eig); y = dtype[R][n]; L, dlogs2 = device double[R];
 * g = device double[R][n].  The transform of y runs in dtype, everything
 * after it (|yt|^2, g, the sums) in FP64, summed in a fixed order.  A row
 * with some lambda_k + s2 <= 0 gives L = NaN.
 * ws: ldk_workspace_bytes(LDK_OP_MLL, kind, R, m, dtype) bytes. */
int ldk_mll(int kind, int R, int m, int dtype, const double *lam, double sigma2, const void *y,
            double *L, double *g, double *dlogs2, void *ws, ldk_stream stream);

/* dL/dk1 from g = dL/dlambda: the adjoint of lambda = sqrt(n) FT(k1) (Sec. 5.4),
 *   net:     a = H g (unnormalised Walsh-Hadamard; H is symmetric),
 *   lattice: a_j = Re sum_k g_k W^{-k R_m(j)}, W = exp(-2 pi i / n).
 * g, a = device double[R][n] (may alias exactly).  FP64.
 * ws: ldk_workspace_bytes(LDK_OP_MLL_ADJOINT, kind, R, m, LDK_F64) bytes
 * (lattice with n > 2^12 only). */
int ldk_mll_adjoint(int kind, int R, int m, const double *g, double *a, void *ws,
                    ldk_stream stream);

/* Gradient of sum_i a_i k1_i in the kernel parameters (chain rule through
 * the product kernel of ldk_kernel_column; with a = dL/dk1 it gives the
 * marginal-likelihood gradient):
 *   grad[r][j] = sum_i a_ri zeta t_ij prod_{l != j} (1 + t_il),  t_ij = gamma_j K_j,
 *                (d k1_i / d log gamma_j), j < d;
 *   grad[r][d] = sum_i a_ri k1_ri  (d k1_i / d log zeta).
 * Points, anchors, window and kernel as for ldk_kernel_column (the same
 * restrictions apply); dtype = precision of the factor evaluation (the
 * products of the other factors are formed without dividing by a factor
 * that is exactly zero); the sums are FP64, in a fixed order.
 * k1 (optional, may be NULL): the column ldk_kernel_column returned for the
 * same arguments and dtype; the factors are formed bit for bit as there, so
 * the product of the other factors is k1_i / f_ij and one sweep over the
 * dimensions replaces two (tiles holding a zero k1_i take the two sweeps).
 * a = device double[R][n_max - n_min]; grad = device double[R][d + 1].
 * ws: ldk_kernel_grad_workspace_bytes(R, d, n_min, n_max, pts != NULL). */
int ldk_kernel_grad(const ldk_kernel *k, const ldk_pointset *ps, const uint64_t *pts,
                    const uint64_t *x0, int64_t n_min, int64_t n_max, int dtype, const void *k1,
                    const double *a, double *grad, void *ws, ldk_stream stream);
size_t ldk_kernel_grad_workspace_bytes(int R, int d, int64_t n_min, int64_t n_max,
                                       int points_given);

/* Squared worst-case error of nw cubature rules sum_i w_i f(x_i) per
 * replication, over the unit ball of the RKHS of the product kernel of
 * ldk_kernel_column (Sec. 3.2):
 *   e2[r][q] = int int K - 2 sum_i w_rqi kappa_i + w_rq^T K_r w_rq
 *            = zeta - 2 zeta sum_i w_rqi + sum_k lambda_rk |wt_k|^2,
 * with kappa_i = int K(u, x_i) du.  Every factor 1 + gamma_j K_alpha of the
 * kernel integrates to one over [0, 1) (K_alpha has mean zero), so kappa_i
 * and the double integral both equal zeta; wt = FT(w_rq) orthonormal
 * (Sec. 5.4), so the quadratic form costs one transform.
 * lam = double[R][n] (ldk_eig); w = dtype[R][nw][n] in the point order of
 * lam; e2 = device double[R][nw].  The transform of w runs in dtype (sum_i
 * w_i is its zero frequency), the weighted sums in FP64 in a fixed order.
 * e2 is a difference of terms of size zeta: its error is absolute, of
 * order (m + 2) u (zeta + 2 zeta sum_i |w_i| + sum_k |lambda_k| |wt_k|^2),
 * u the unit roundoff of dtype.
 * R * nw <= 65535.  ws: ldk_workspace_bytes(LDK_OP_WCE, kind, R * nw, m, dtype). */
int ldk_wce(int kind, int R, int nw, int m, int dtype, const double *lam, double zeta,
            const void *w, double *e2, void *ws, ldk_stream stream);

/* Fields of one replication's ldk_bayes_cubature result. */
enum {
    LDK_BC_MEAN = 0,   /* posterior mean of int f */
    LDK_BC_VAR = 1,    /* posterior variance of int f per unit GP scale */
    LDK_BC_SCALE = 2,  /* maximum-likelihood GP scale */
    LDK_BC_HALF = 3,   /* credible-interval half width */
    LDK_BC_WEIGHT = 4, /* the (equal) optimal cubature weights */
    LDK_BC_WCE2 = 5,   /* squared worst-case error of those weights */
    LDK_BC_FIELDS = 6
};

/* Bayesian cubature (named in Secs. 1.1 and 1.3; the paper prints no
 * formula, so the standard Gaussian conditioning is used): f ~ GP(0, s K)
 * with the kernel of ldk_kernel_column, observed as y_i = f(x_i) + e_i,
 * e_i ~ N(0, s sigma2), and the integral I = int f.  With kappa_i = zeta (see ldk_wce) and the
 * constant vector an eigenvector of K with eigenvalue lambda_0 = sum_i k1_i
 * (the points form a group under the shift or the digital sum):
 *   WEIGHT = (K + sigma2 I)^{-1} kappa, every entry zeta / (lambda_0 + sigma2)
 *            (the optimal weights of Sec. 3.2 at sigma2 = 0),
 *   MEAN   = kappa^T (K + sigma2 I)^{-1} y = WEIGHT sum_i y_i,
 *   VAR    = zeta - kappa^T (K + sigma2 I)^{-1} kappa
 *          = zeta (lambda_0 + sigma2 - n zeta) / (lambda_0 + sigma2),
 *   SCALE  = y^T (K + sigma2 I)^{-1} y / n = sum_k |yt_k|^2 / (lambda_k + sigma2) / n
 *            (maximum likelihood for s; yt = FT(y) orthonormal),
 *   HALF   = z sqrt(SCALE max(VAR, 0))  (z: the normal quantile of the
 *            credible level, e.g. 2.5758 for 99 %),
 *   WCE2   = zeta - 2 n zeta WEIGHT + n WEIGHT^2 lambda_0 (equals VAR at
 *            sigma2 = 0).
 * lam = double[R][n] (ldk_eig); y = dtype[R][n]; out = device
 * double[R][LDK_BC_FIELDS].  The transform of y runs in dtype (sum_i y_i is
 * its zero frequency), the rest in FP64.  VAR and WCE2 carry the absolute
 * rounding of lambda_0 (about (m + 1) u sum_i |k1_i| / n relative to zeta).
 * A replication with some lambda_k + sigma2 <= 0 gets SCALE = HALF = NaN.
 * ws: ldk_workspace_bytes(LDK_OP_BAYES_CUBATURE, kind, R, m, dtype) bytes. */
int ldk_bayes_cubature(int kind, int R, int m, int dtype, const double *lam, double sigma2,
                       double zeta, const void *y, double z, double *out, void *ws,
                       ldk_stream stream);

/* ---------------------------------------------------------------------
 * Batched fit of an instance table (Sec. 6 runs many randomizations and
 * right-hand sides together, vectorised over them).  An instance is one
 * randomized point set -- a shifted rank-1 lattice or an (LMS-scrambled,)
 * digitally shifted base-2 net, over the table's one generating vector or
 * matrix per kind -- with n = 2^m points and nrhs responses; its fit is the
 * first column, the eigenvalues, every solve (K + sigma^2 I) c = y and the
 * log-det (as ldk_kernel_column followed by ldk_fit).
 *
 * The plan groups instances by (kind, m, nrhs, scrambled): the instances of
 * a group are the replications of one point set, so each group is one
 * first-column launch and one fit, and groups are shared out over
 * desc->streams streams (1..8; forked from and joined back to the caller's
 * stream through events; default priority).  Data live in five
 * caller-owned device arenas whose sizes the plan gives
 * (ldk_plan_arena_bytes): responses Y and solutions C (dtype), eigenvalues
 * LAM and log-dets LOGDET (double), and the workspace WS (the groups'
 * shifts, scrambles and scrambled columns, first columns and fit
 * workspaces).  Instance i's rows start at ldk_plan_instance_offset(i, ...)
 * elements into Y / C ([nrhs][n]), LAM ([n]), LOGDET ([1]) and, for K1
 * (its first column, dtype [n]), into WS.  Plans allocate no device
 * memory; creation and binding are not for hot loops (binding gathers the
 * instances' shifts and scrambles with device copies and forms each net
 * replication's scrambled columns once, on `stream`). */
typedef struct {
    int32_t d;            /* dimensions of every instance */
    int32_t m_max;        /* net generating columns per dimension; every m <= m_max */
    int32_t dtype;        /* LDK_F64 or LDK_F32 (first columns, y, c) */
    int32_t streams;      /* 1..8 */
    double sigma2;        /* nugget of every solve */
    const uint64_t *lattice_gen;  /* device g[d] (when the table has lattices) */
    const uint64_t *net_gen;      /* device C[d][m_max] (when it has nets) */
    ldk_kernel lattice_kernel;    /* SI kernel (kind LDK_LATTICE) */
    ldk_kernel net_kernel;        /* DSI kernel (kind LDK_DNET_B2) */
} ldk_batch_desc;

typedef struct {
    int32_t kind;   /* LDK_LATTICE or LDK_DNET_B2 */
    int32_t m;      /* n = 2^m, m <= m_max */
    int32_t nrhs;   /* >= 1 */
    int32_t reserved;
    const uint64_t *shift;  /* device [d] (read by ldk_plan_bind) */
    const uint64_t *lms;    /* device [d][64] or NULL (nets only; read by ldk_plan_bind) */
} ldk_instance;

enum {
    LDK_ARENA_Y = 0,
    LDK_ARENA_C = 1,
    LDK_ARENA_LAM = 2,
    LDK_ARENA_LOGDET = 3,
    LDK_ARENA_WS = 4,
    LDK_ARENA_COUNT = 5,
    LDK_ARENA_K1 = 5 /* instance offsets only: the first column, in WS */
};

typedef struct ldk_plan_s *ldk_plan;

/* Validates the table and lays out the arenas (host work only).
 * LDK_EINVAL for a bad description or instance; LDK_ENOTSUP for a group of
 * more than 65535 instances. */
int ldk_plan_create(const ldk_batch_desc *desc, int n_inst, const ldk_instance *inst,
                    ldk_plan *out);
/* Arena size in bytes (0 for a bad argument). */
size_t ldk_plan_arena_bytes(ldk_plan p, int which);
/* Instance i's first element in arena `which` (elements of the arena's type). */
int ldk_plan_instance_offset(ldk_plan p, int i, int which, size_t *offset);
/* Binds the arenas (logdet may be NULL) and enqueues the one-time gathers on
 * `stream`; drops a graph captured for an earlier binding. */
int ldk_plan_bind(ldk_plan p, void *y, void *c, double *lam, double *logdet, void *ws,
                  ldk_stream stream);
/* Enqueues the whole table on `stream` (replays the captured graph when
 * there is one).  Outputs are valid once the stream reaches this point. */
int ldk_batch_launch(ldk_plan p, ldk_stream stream);
/* Captures the table's launch sequence on `stream` (not the null stream)
 * as one HIP graph kept by the plan; later ldk_batch_launch calls replay
 * it.  Nothing runs during the capture. */
int ldk_batch_capture(ldk_plan p, ldk_stream stream);
/* Number of groups, and kernel nodes of the captured graph (-1 before a
 * capture). */
int ldk_plan_stats(ldk_plan p, int *groups, int *kernel_nodes);
/* Frees the plan's host memory, streams, events and graph. */
int ldk_plan_destroy(ldk_plan p);

/* Test integrands of the RQMC estimate, functions of s = sum_j c_j x_j:
 *   LDK_GENZ_CORNER_PEAK  (1 + s)^-(d+1)   (the Genz corner peak, the
 *                                           integrand of the paper's RQMC
 *                                           example in Sec. 6)
 *   LDK_GENZ_OSCILLATORY  cos(2 pi u + s)  (the Genz oscillatory). */
enum { LDK_GENZ_CORNER_PEAK = 0, LDK_GENZ_OSCILLATORY = 1 };

/* Fields of ldk_rqmc's stats output. */
enum { LDK_RQMC_MEAN = 0, LDK_RQMC_STD = 1, LDK_RQMC_HALF = 2, LDK_RQMC_FIELDS = 3 };

/* RQMC estimate of int_[0,1]^d f over the R randomizations of a point set
 * (eq. RQMC and the Student-t interval stated with it):
 *   mu_r[r] = (1/n) sum_{i<n} f(x_ri)            (points 0 .. n-1 of
 *                                                 replication r, as
 *                                                 ldk_gen_points makes them)
 *   stats[LDK_RQMC_MEAN] = mu = (1/R) sum_r mu_r
 *   stats[LDK_RQMC_STD]  = sigma = sqrt(sum_r (mu_r - mu)^2 / (R - 1))
 *                          (NaN when R = 1)
 *   stats[LDK_RQMC_HALF] = t sigma / sqrt(R), t = the Student-t quantile
 *                          t_{R-1, tau/2} of the 100(1 - tau)% interval
 *                          mu +- HALF, passed in by the caller.
 * The points are regenerated inside the kernel (never written to memory).
 * A coordinate word u is split into its exact high and low 32-bit halves,
 * x_j = hi 2^-32 + lo 2^-64, and s = sum_j c_j x_j is formed as
 * 2^-32 sum_j c_j hi_j + 2^-64 sum_j c_j lo_j (each half's products summed
 * in FP64, no coordinate rounded to 53 bits first), so |s - s_exact| is
 * below about 2 d u sum_j |c_j x_j| (u = 2^-53); the corner peak's power is
 * taken by binary powering of its integer exponent.  Every sum over points
 * is FP64 in a fixed order.  ps: any point set ldk_gen_points accepts
 * (shifted lattice, LMS + digitally shifted net, per-replication columns
 * with or without scrambles); 1 <= n <= the limit of ldk_gen_points.  A
 * natural-order lattice with n so large that the dispatch would exceed
 * 2^32 work items along x (n above about 2^35) gives LDK_ENOTSUP.  integrand: LDK_GENZ_*; coef =
 * device double[d] (c_j); u: the oscillatory phase (ignored by the corner
 * peak).  mu_r = device double[R]; stats = device double[LDK_RQMC_FIELDS].
 * ws: ldk_rqmc_workspace_bytes(ps, n) bytes (the tile sums and, for an LMS
 * net, every replication's scrambled columns, formed once per call). */
int ldk_rqmc(const ldk_pointset *ps, int64_t n, int integrand, const double *coef, double u,
             double t, double *mu_r, double *stats, void *ws, ldk_stream stream);
size_t ldk_rqmc_workspace_bytes(const ldk_pointset *ps, int64_t n);

/* Point sets without the fast-transform structure; they feed QMC means only
 * (the RQMC estimate over given coordinates, ldk_rqmc_points).
 *
 *  kind LDK_HALTON (Sec. 4.4): dimension j (from 0) has the (j+1)-th prime
 *        b_j as its base and the identity generating matrix: the radical
 *        inverse of i; 1 <= d <= 54 (bases below 256).
 *  kind LDK_FAURE (Sec. 4.3, a digital sequence in prime base b): one
 *        prime base b with d <= b <= 251; dimension j uses C = P^j mod b, P
 *        the upper-triangular Pascal matrix (entries binom(k, t) j^(k-t)).
 *     Digits: the base-b digits a_k of i give z_t = sum_k C[t][k] a_k mod b
 *     (digit t weighs b^-(t+1)); then, each when its flag is set and in this
 *     order: LDK_BR_LMS z <- S z mod b (S lower triangular, nonzero
 *     diagonal), LDK_BR_DP z_t <- pi_t(z_t) (a permutation of the digit
 *     values per position), LDK_BR_DS z_t <- z_t + delta_t mod b.  T digits
 *     are kept, the largest T with b^T <= 2^53, and the coordinate is the
 *     integer sum_t z_t b^(T-1-t) divided by b^T, rounded once to FP64.
 *     Scrambles (device, uint8, for every replication r and dimension j; only
 *     the first T rows and the first b values of each row are read):
 *       lms   [R][d][53][53]  S[t][k] at [r][j][t][k];
 *       perm  [R][d][53][256] pi_t(v) at [r][j][t][v];
 *       shift [R][d][53]      delta_t at [r][j][t].
 *  kind LDK_DNET_NUS (Sec. 4.3, nested uniform scrambling of a base-2 net):
 *        gen = device uint64 [d][m] generating columns (as for LDK_DNET_B2,
 *        digit t at bit 64 - t), 0 <= m <= 32; seed = device uint64 [R][d].
 *        Point word z = C_j i, then digit t = 1..64 is flipped when the top
 *        bit of mix64(key XOR seed_rj) is set, key = 2^(t-1) + the digits
 *        above t as an integer; mix64 is the SplitMix64 finaliser
 *        (Steele, Lea and Flood 2014; Stafford's Mix13 constants).  The
 *        coordinate is the word times 2^-64 rounded to the nearest double.
 *        flags, base, lms, perm and shift are ignored.
 * R <= 65535 replications; indices below 2^32. */
typedef enum { LDK_HALTON = 2, LDK_FAURE = 3, LDK_DNET_NUS = 4 } ldk_bkind;
#define LDK_BDIGITS_MAX 53
#define LDK_BR_LMS 1
#define LDK_BR_DP 2
#define LDK_BR_DS 4
typedef struct {
    int32_t kind;
    int32_t R;
    int32_t d;
    int32_t base;  /* LDK_FAURE */
    int32_t flags; /* LDK_HALTON, LDK_FAURE: OR of LDK_BR_* */
    int32_t m;     /* LDK_DNET_NUS */
    const uint8_t *lms;
    const uint8_t *perm;
    const uint8_t *shift;
    const uint64_t *gen;  /* LDK_DNET_NUS */
    const uint64_t *seed; /* LDK_DNET_NUS */
} ldk_bpointset;

/* Coordinates of points i = n_min .. n_max-1 of every replication: out =
 * device double [R][n_max - n_min][d], d fastest.  ws:
 * ldk_bpoints_workspace_bytes(ps) bytes (the Faure matrices, formed on every
 * call; 0 for the other kinds).  LDK_EINVAL for an invalid set or a missing
 * scramble its flags ask for; LDK_ENOTSUP for n_max > 2^32. */
int ldk_gen_bpoints(const ldk_bpointset *ps, int64_t n_min, int64_t n_max, double *out, void *ws,
                    ldk_stream stream);
size_t ldk_bpoints_workspace_bytes(const ldk_bpointset *ps);

/* eq. RQMC over given points: x = device double [R][n][d] (any of the point
 * sets above, or any coordinates), 1 <= d <= 128, with the integrands,
 * outputs and interval of ldk_rqmc.  ws: ldk_rqmc_points_workspace_bytes(R,
 * n) bytes. */
int ldk_rqmc_points(int R, int64_t n, int d, const double *x, int integrand, const double *coef,
                    double u, double t, double *mu_r, double *stats, void *ws, ldk_stream stream);
size_t ldk_rqmc_points_workspace_bytes(int R, int64_t n);

/* Orthonormal Walsh-Hadamard transform of B FP32 rows of n = 2^m (Sec. 5.3,
 * the recursion of H_m) on the matrix cores: each radix-16 stage is two
 * accumulating FP16 matrix instructions H_16 X_lo + H_16 X_hi with FP32
 * sums, where X_hi + X_lo is a two-term FP16 split of the (power-of-two scaled) FP32
 * data, redone before every stage (about 22 significant bits per stage;
 * normwise error of order 1e-6 against the exact transform).  Same result
 * as ldk_transform(LDK_DNET_B2, ..., LDK_F32, ...) up to that rounding.
 * in, out = device float[B][n]; may alias exactly.  No workspace. */
int ldk_fwht_split16(int B, int m, const float *in, float *out, ldk_stream stream);

/* Quantiles of the interval statistics (host functions, no device work):
 * the standard normal quantile z_p (the credible level of
 * ldk_bayes_cubature: z = z_{(1 + level)/2}) and the Student-t quantile
 * t_{dof, p} (eq. RQMC's interval uses t = t_{R-1, 1 - tau/2}).
 * Normal: start from the rational approximation 26.2.23 of Abramowitz and
 * Stegun, then Halley steps on Phi(x) - p (Phi through erfc, tail-side
 * residuals); relative error about 1e-15.  Student t: closed forms for
 * dof 1 and 2; otherwise the Cornish-Fisher start (Abramowitz and Stegun
 * 26.7.5) and Newton steps on the upper tail (1/2) I_{dof/(dof+t^2)}(dof/2, 1/2),
 * the regularised incomplete beta function by its continued fraction.
 * ldk_normal_quantile returns NaN unless 0 < p < 1; ldk_student_t_quantile
 * returns LDK_EINVAL unless 0 < p < 1, dof >= 1 and out != NULL. */
double ldk_normal_quantile(double p);
int ldk_student_t_quantile(double p, int dof, double *out);

typedef enum {
    LDK_OP_TRANSFORM = 0,
    LDK_OP_EIG = 1,
    LDK_OP_SOLVE = 2,
    LDK_OP_MATVEC = 3,
    LDK_OP_LOGDET = 4,
    LDK_OP_UPDATE_DOUBLE = 5,
    LDK_OP_EIG_UPDATE_DOUBLE = 6,
    LDK_OP_MLL = 7,
    LDK_OP_MLL_ADJOINT = 8,
    LDK_OP_FIT = 9,
    LDK_OP_WCE = 10,
    LDK_OP_BAYES_CUBATURE = 11
} ldk_op;

/* Workspace bytes needed by `op` for B rows (or R * nrhs rows) of 2^m. */
size_t ldk_workspace_bytes(int op, int kind, int64_t B, int m, int dtype);

/* Human-readable status string (static storage). */
const char *ldk_strerror(int status);

/* hipError_t of the last failing HIP call on this host thread (0 if none). */
int ldk_last_hip_error(void);

/* Library version, "major.minor.patch". */
const char *ldk_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LDK_H */
