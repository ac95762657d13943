// Pass-based FWHT / FFTBR / IFFTBR engine for gfx950.
//
// A length-2^m transform is split over the bits of the element index: a
// "row" pass transforms the low a0 bits (contiguous tiles), then "column"
// passes transform higher bit groups (tiles of 2^a strided rows x W
// contiguous columns).  Inside a pass, a workgroup holds its tile in LDS and
// every thread keeps E = 16 elements in registers; radix-2^g stages run in
// registers and bit groups are exchanged through LDS.
//
// FFTBR (Sec. 5.2: decimation-in-time FFT without the input bit reversal)
// factors over the index bits: transform the low bits first; before the
// group of bits [s, s+g) apply the twiddle W_{2^{s+g}}^{k R_g(c)}, where k is
// the (already transformed, natural-order) low index and c the group digit,
// then transform the group.  IFFTBR runs the same steps backwards with
// conjugate twiddles.  The FWHT is the same schedule without twiddles
// (H_m is the Kronecker power of H_1).  All passes are unnormalised; the
// caller folds n^-1/2 or 1/n into one multiply.
#pragma once

#include "common.hpp"

namespace ldk {

// PM_POWER, PM_ADJ and PM_QFORM exist only in the real-input lattice top pass.
enum PassMode {
    PM_FWD = 0,
    PM_INV = 1,
    PM_SOLVE = 2,
    PM_MATVEC = 3,
    PM_POWER = 4,
    PM_ADJ = 5,
    PM_QFORM = 6
};

struct PassGeom {
    int b0;    // index bit where this pass's axis starts
    int a;     // axis bits (tile rows 2^a)
    int logW;  // tile width (contiguous columns) log2, logW <= b0
    int logE;  // registers per thread log2 (g), logE <= a
};

struct Plan {
    int m;
    int P;  // number of passes (0 when m == 0)
    PassGeom pass[4];
};

// log_tile: log2 of the elements per workgroup tile (LDS budget); loge_max:
// log2 of the largest register group (the butterfly radix of the in-register
// stages).  The plan depends on m and these two only, so for given
// parameters results do not depend on the batch size.
Plan make_plan(int m, int log_tile, int loge_max = 3);
int log_tile_for(int kind, int dtype);
// Whether every pass of a plan fits the pass kernels (threads per
// workgroup, register groups per axis).
bool plan_ok(const Plan &pl);

// Plan parameters of the eigenvalue, solve, matvec, fit and transform
// paths.  Defaults: log_tile_for(kind, dtype) and radix 8.  A table written
// by the tuner (ldk_init_tuned) may replace them per (kind, working dtype,
// log2 n, rows): the entry with the largest rows_log2 <= log2(rows) applies.
// engine: the FWHT of FP32 digital-net solves and matvecs (m >= 12):
// 0 = the FP32 butterfly passes, 1 = the split-FP16 matrix-core passes.
struct PlanParams {
    int log_tile;
    int loge_max;
    int engine;
};
enum { ENGINE_BUTTERFLY = 0, ENGINE_SPLIT16 = 1 };
PlanParams plan_params(int kind, int dtype, int m, int64_t rows);
// Every parameter set plan_params may return for (kind, dtype, m), whatever
// the rows (workspace sizes are the largest over them).  Returns the count.
int plan_candidates(int kind, int dtype, int m, PlanParams *out, int cap);
// Loads (path) or clears (nullptr) the tuned-parameter table.
int load_tune_table(const char *path);

struct PassArgs {
    const void *src;
    void *dst;
    int64_t src_row;  // elements between consecutive batch rows in src
    int64_t dst_row;  // elements between consecutive batch rows in dst
    int64_t rows;     // batch rows
    int m;
    PassGeom g;
    const double *lam;  // eigenvalues [rows / nrhs][2^m] (solve / matvec), FP64
    int nrhs;
    int global_tw;    // apply the inter-pass FFT twiddle (column passes)
    int64_t half;     // packed real IO: offset of the imaginary half (N), elements
    double sigma2;
    double scale;     // solve: scale / (lambda + sigma2); matvec: scale * lambda;
                      // fwd / inv: multiplies the stored values
    // PM_INV only, optional: blocks 0 .. ld_rows-1 also add up ld_count
    // log-det partial sums per row (ld_part[r][ld_count]) into ld_out[r].
    const double *ld_part;
    double *ld_out;
    int64_t ld_rows;
    int64_t ld_count;
    // PM_QFORM only: weights lambda_k (1) or 1 / (lambda_k + sigma2) (0)
    int qform_lam;
    // Real-input lattice top pass, PM_SOLVE / PM_MATVEC, optional: the
    // filter's per-frequency coefficients (p, q) as working-type complex
    // pairs [rows / nrhs][N] (launch_filter_coef); NULL forms them from lam
    // in the pass itself.
    const void *coef;
    // PIO_COMBINE only: the old half's transform [rows][2^m]; the store
    // writes (old + w) / sqrt 2 at k and (old - w) / sqrt 2 at 2^m + k of
    // dst rows of 2^(m+1), w the pass output (times W_{2^(m+1)}^k, lattice).
    // With combine_real: FP64 rows old +- Re w, unnormalised (eigenvalues).
    const void *old;
    int combine_real;
};

// Global IO of a pass (lattice only; nets are always real):
enum PassIo {
    PIO_SAME = 0,    // complex rows
    PIO_REAL = 1,    // real rows: load as (x, 0) / store the real part
    PIO_PACKED = 2,  // real rows of 2N carrying a complex row of N: z_e = y_e + i y_{e+N}
    PIO_POWER = 3,   // store only: FP64 rows receiving |x|^2 (forward passes)
    PIO_COMBINE = 4, // store only: the n -> 2n update's butterfly with a.old (forward)
};

// kind: LDK_LATTICE (complex FFTBR) or LDK_DNET_B2 (real FWHT).
// dtype: working precision of the pass.
// ld, st: PassIo of the source and destination rows.
// src_f32: src holds floats widened to the FP64 working type (PM_FWD only).
int launch_pass(int kind, int dtype, int mode, int ld, int st, const PassArgs &a, hipStream_t s,
                bool src_f32 = false);

// Real-input lattice top pass (see realfft.hip): forward transform of the
// packed half-length row's top bit group, untangling of the real spectrum,
// and either the eigenvalues (mode PM_FWD) or the filter by 1/(lambda+s2)
// (PM_SOLVE) / lambda (PM_MATVEC) followed by the inverse top group.
// lam_out receives the eigenvalues for PM_FWD and the power spectrum |Y|^2
// for PM_POWER (FP64 rows of 2N).  PM_ADJ reads a real spectrum from a.lam
// and runs only the inverse half.  With one pass (b0 = 0) the source and
// destination rows are packed real rows.
// ld_part (PM_FWD only, may be NULL): per-tile sums of log(lambda + a.sigma2),
// [rows][tiles per row], for a log-det finished by one reduction kernel.
int launch_real_top(int dtype, int mode, const PassArgs &a, double *lam_out, hipStream_t s,
                    bool src_f32 = false, double *ld_part = nullptr);

// The real-input lattice solve's (PM_SOLVE) or matvec's (PM_MATVEC) filter
// coefficients, one (p, q) pair per frequency k < N = 2^mp of each of the
// lam_rows eigenvalue rows [lam_rows][2N], into coef (dtype complex pairs
// [lam_rows][N]); scale as the top pass's.
int launch_filter_coef(int dtype, int mode, int mp, int64_t lam_rows, const double *lam,
                       double sigma2, double scale, void *coef, hipStream_t s);

// The fused fit's top passes (FP64 lattice, one right-hand side per column
// row): aK's tiles give the eigenvalues (lam_out, and the log-det partial
// sums when ld_part is set), aY's tiles the filtered solve by
// aY.scale / (lambda + aY.sigma2), in one launch.  Same geometry for both;
// the geometry's logE is 2 or 3 and 2^(a + logW - logE) a multiple of 64, at
// most 256.
// The whole fit of a one-pass FP64 net, one workgroup per replication:
// eigenvalue pass aE, then the solve passes aS (nrhs >= 1), then the
// log-det.  LDK_ENOTSUP when the geometry is not one pass shared by both.
int launch_fit_net_one(const PassArgs &aE, const PassArgs &aS, double *logdet, hipStream_t s);
int launch_fit_top(const PassArgs &aK, const PassArgs &aY, double *lam_out, double *ld_part,
                   hipStream_t s);
// Whether launch_fit_top takes geometry g.
bool fit_top_supported(const PassGeom &g);

// Two jobs of the same pass kind in one launch (blocks of job 0, then job 1).
int launch_pass2(int kind, int dtype, int mode, int ld, int st, const PassArgs &a0,
                 const PassArgs &a1, hipStream_t s);

// Solve (PM_SOLVE) or matvec (PM_MATVEC) of FP32 digital-net rows on the
// matrix-core FWHT (fwht_mfma.hip): rows = R nrhs rows of n = 2^m, m >= 12
// (LDK_ENOTSUP below); lam = FP64 [R][n]; c may alias y; no workspace (the
// intermediate lives in c).
int fwht16_apply(int mode, int m, int64_t rows, int nrhs, const double *lam, double sigma2,
                 const float *y, float *c, hipStream_t s);

// |H y|^2 (unnormalised) of FP32 digital-net rows, FP64 into pw [rows][n],
// on the matrix-core FWHT; m >= 12; tmp = FP32 [rows][n] for the passes
// before the last (unused when m = 12).
int fwht16_power(int m, int64_t rows, const float *y, float *tmp, double *pw, hipStream_t s);

// Sum of log(s) over a thread's values in product form: s = m 2^e with m in
// [1/2, 1); the mantissas multiply and the exponents add, with one log at
// the end (k mantissas keep the product above 2^-k, so no underflow for the
// few dozen values a thread takes).  NaN when some s <= 0 or is NaN.  About
// three instructions per value instead of a logarithm each.
struct LogProd {
    double mant = 1.0;
    int exp = 0;
    bool bad = false;
    __device__ __forceinline__ void add(double s)
    {
        int e;
        const double m = frexp(s, &e);
        mant *= m;
        exp += e;
        bad |= !(s > 0.0);
    }
    __device__ __forceinline__ double value() const
    {
        return bad ? __builtin_nan("") : log(mant) + (double)exp * 0.69314718055994530942;
    }
};

// LDS of one workgroup on gfx950 (the fused fit's top pass takes up to this).
constexpr size_t LDS_PER_GROUP = 163840;

// Workspace bytes of LDK_OP_MLL / LDK_OP_MLL_ADJOINT (mll.hip).
size_t mll_ws_bytes(int op, int kind, int64_t R, int m, int dtype);
// Workspace bytes of LDK_OP_WCE / LDK_OP_BAYES_CUBATURE for B rows (mll.hip).
size_t cub_ws_bytes(int kind, int64_t B, int m, int dtype);

}  // namespace ldk
