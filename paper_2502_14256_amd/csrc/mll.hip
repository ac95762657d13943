// Gaussian-process log marginal likelihood in the eigenbasis of Sec. 5.4 and
// the adjoint that carries its gradient back to the first Gram column.
//
// With yt = FT(y) orthonormal (V unitary up to sqrt(n)),
//   L   = -1/2 sum_k |yt_k|^2 / (lambda_k + s2) - 1/2 sum_k log(lambda_k + s2)
//         - (n/2) log(2 pi),
//   g_k = dL/dlambda_k = 1/2 |yt_k|^2 / (lambda_k + s2)^2 - 1/2 / (lambda_k + s2),
//   dL/dlog s2 = s2 sum_k g_k.
// |yt_k|^2 comes straight out of the last transform pass (power-spectrum
// store, FP64), so yt itself is never written.  Since lambda = sqrt(n) FT(k1)
// is linear in k1, dL/dk1 = a is the adjoint map applied to g: H g for the
// net (H symmetric) and Re sum_k g_k W^{-k R(j)} for the lattice.
//
// Kernel cubature (Sec. 3.2) uses the same power spectrum.
// For the product kernels of ldk_kernel_column every factor 1 + gamma K_alpha
// integrates to one over [0, 1) (K_alpha has mean zero), so
// kappa_i = int K(u, x_i) du = zeta and int int K = zeta; then
//   e2(w) = zeta - 2 zeta sum_i w_i + sum_k lambda_k |wt_k|^2   (wt = FT(w)).
// The points form a group under the shift (lattice) or the digital sum
// (net), so the constant vector is an eigenvector of K with eigenvalue
// lambda_0 = sum_i k1_i, and (K + s2 I)^{-1} kappa = zeta / (lambda_0 + s2) 1:
// the optimal weights are equal and the Bayesian-cubature posterior of the
// integral needs only lambda_0, sum_i y_i and y^T (K + s2 I)^{-1} y.
#include "transform.hpp"

namespace ldk {

namespace {
constexpr int MLL_THREADS = 256;
constexpr int MLL_ITEMS = 8;
constexpr int MLL_CHUNK = MLL_THREADS * MLL_ITEMS;

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
size_t esz(int dtype) { return dtype == LDK_F64 ? 8 : 4; }

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block sum of three values (fixed order: lanes, then waves).
__device__ __forceinline__ void block_sum3(double (&v)[3], double (*red)[3])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = wave_sum(v[c]);
    if (lane == 0)
        for (int c = 0; c < 3; ++c) red[wave][c] = v[c];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w][c];
            v[c] = s;
        }
}

// p (in g) -> g; partial sums of p/n/(lambda+s2), log(lambda+s2), g per chunk.
__global__ __launch_bounds__(MLL_THREADS) void k_mll_terms(const double *__restrict__ lam,
                                                           double *__restrict__ g, int64_t n,
                                                           double sigma2, double inv_n, int chunks,
                                                           double *__restrict__ part)
{
    __shared__ double red[MLL_THREADS / 64][3];
    const int r = blockIdx.y, ch = blockIdx.x;
    const double *lr = lam + (size_t)r * n;
    double *gr = g + (size_t)r * n;
    double acc[3] = {0.0, 0.0, 0.0};
    LogProd lsum;  // sum of log(lambda + s2)
    const int64_t lo = (int64_t)ch * MLL_CHUNK;
#pragma unroll
    for (int it = 0; it < MLL_ITEMS; ++it) {
        const int64_t k = lo + threadIdx.x + (int64_t)it * MLL_THREADS;
        if (k < n) {
            const double s = lr[k] + sigma2;
            const double p = gr[k] * inv_n;
            const double is = 1.0 / s;
            const double q = p * is;
            acc[0] += q;
            lsum.add(s);
            const double gk = 0.5 * (q - 1.0) * is;  // 1/2 p/s^2 - 1/2 /s
            acc[2] += gk;
            gr[k] = gk;
        }
    }
    acc[1] = lsum.value();
    block_sum3(acc, red);
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) part[((size_t)r * chunks + ch) * 3 + c] = acc[c];
}

__global__ __launch_bounds__(MLL_THREADS) void k_mll_final(const double *__restrict__ part,
                                                           int chunks, int64_t n, double sigma2,
                                                           double *__restrict__ L,
                                                           double *__restrict__ dlogs2)
{
    __shared__ double red[MLL_THREADS / 64][3];
    const int r = blockIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int c = threadIdx.x; c < chunks; c += MLL_THREADS)
        for (int q = 0; q < 3; ++q) acc[q] += part[((size_t)r * chunks + c) * 3 + q];
    block_sum3(acc, red);
    if (threadIdx.x == 0) {
        const double log2pi = 1.8378770664093454835606594728112353;
        L[r] = -0.5 * acc[0] - 0.5 * acc[1] - 0.5 * (double)n * log2pi;
        if (dlogs2) dlogs2[r] = sigma2 * acc[2];
    }
}

// y^2 into FP64 (n = 1: the transform is the identity).
template <typename R>
__global__ void k_square(const R *__restrict__ y, double *__restrict__ out, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = (double)y[i] * (double)y[i];
}

__global__ void k_copy_f64(const double *__restrict__ x, double *__restrict__ out, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = x[i];
}

bool real_lattice(int kind, int m) { return kind == LDK_LATTICE && m >= 2; }

// Transform scratch of the power spectrum / adjoint (bytes), 0 for one pass.
size_t power_tmp_bytes(int kind, int64_t R, int m, int dtype)
{
    if (real_lattice(kind, m)) {
        const Plan pl = make_plan(m - 1, log_tile_for(LDK_LATTICE, dtype));
        return pl.P > 1 ? (size_t)R * ((size_t)1 << (m - 1)) * 2 * esz(dtype) : 0;
    }
    const Plan pl = make_plan(m, log_tile_for(LDK_DNET_B2, dtype));
    return pl.P > 1 ? (size_t)R * ((size_t)1 << m) * esz(dtype) : 0;
}

int chunks_of(int m) { return (int)((((int64_t)1 << m) + MLL_CHUNK - 1) / MLL_CHUNK); }

// p[r][k] = |FT(y_r)_k|^2 (unnormalised transform), FP64, into `pw`.
int power_spectrum(int kind, int R, int m, int dtype, const void *y, double *pw, void *tmp,
                   hipStream_t s)
{
    const int64_t n = (int64_t)1 << m;
    if (m == 0) {
        const int64_t cnt = (int64_t)R;
        const unsigned blocks = (unsigned)((cnt + 255) / 256);
        if (dtype == LDK_F64)
            hipLaunchKernelGGL(k_square<double>, dim3(blocks), dim3(256), 0, s, (const double *)y, pw, cnt);
        else
            hipLaunchKernelGGL(k_square<float>, dim3(blocks), dim3(256), 0, s, (const float *)y, pw, cnt);
        LDK_LAUNCH_CHECK();
        return LDK_OK;
    }
    PassArgs a{};
    a.rows = R;
    a.nrhs = 1;
    a.scale = 1.0;
    if (real_lattice(kind, m)) {
        // packed half-length complex rows; the real top pass writes |Y_k|^2
        const int mp = m - 1;
        const int64_t N = n / 2;
        const Plan pl = make_plan(mp, log_tile_for(LDK_LATTICE, dtype));
        a.m = mp;
        a.half = N;
        for (int p = 0; p < pl.P - 1; ++p) {
            a.src = p == 0 ? y : tmp;
            a.src_row = p == 0 ? n : N;
            a.dst = tmp;
            a.dst_row = N;
            a.g = pl.pass[p];
            a.global_tw = p > 0;
            const int st = launch_pass(LDK_LATTICE, dtype, PM_FWD, p == 0 ? PIO_PACKED : PIO_SAME,
                                       PIO_SAME, a, s);
            if (st) return st;
        }
        a.src = pl.P == 1 ? y : tmp;
        a.src_row = pl.P == 1 ? n : N;
        a.g = pl.pass[pl.P - 1];
        a.global_tw = pl.P > 1;
        return launch_real_top(dtype, PM_POWER, a, pw, s);
    }
    // FWHT (nets; for n = 2 the lattice FFTBR is the same 2-point butterfly)
    if (kind == LDK_DNET_B2 && dtype == LDK_F32 && m >= 12 &&
        plan_params(kind, dtype, m, R).engine == ENGINE_SPLIT16)
        return fwht16_power(m, R, static_cast<const float *>(y), static_cast<float *>(tmp), pw, s);
    const Plan pl = make_plan(m, log_tile_for(LDK_DNET_B2, dtype));
    a.m = m;
    for (int p = 0; p < pl.P; ++p) {
        const bool last = p == pl.P - 1;
        a.src = p == 0 ? y : tmp;
        a.src_row = n;
        a.dst = last ? (void *)pw : tmp;
        a.dst_row = n;
        a.g = pl.pass[p];
        const int st = launch_pass(LDK_DNET_B2, dtype, PM_FWD, PIO_SAME, last ? PIO_POWER : PIO_SAME,
                                   a, s);
        if (st) return st;
    }
    return LDK_OK;
}

// Per-row outputs from q = sum_k w_k |W_k|^2 (unnormalised spectrum; w_k =
// lambda_k for the worst-case error, 1 / (lambda_k + s2) for the posterior)
// and s1 = sum_i of the row.
template <bool BC>
__device__ __forceinline__ void cub_row_out(int row, double q, double s1, int64_t n,
                                                 const double *__restrict__ lam, double sigma2,
                                                 double zeta, double z, double *__restrict__ out)
{
    const double nd = (double)n;
    if constexpr (!BC) {
        // zeta - 2 zeta sum w + w^T K w
        out[row] = fma(-2.0 * zeta, s1, zeta) + q / nd;
    } else {
        const double l0 = lam[(size_t)row * n];
        const double s = l0 + sigma2;
        const double t = s - nd * zeta;  // lambda_0 + s2 - n zeta
        const double wgt = zeta / s;
        const double var = zeta * t / s;
        const double scale = q / (nd * nd);
        double *o = out + (size_t)row * LDK_BC_FIELDS;
        o[LDK_BC_MEAN] = wgt * s1;
        o[LDK_BC_VAR] = var;
        o[LDK_BC_SCALE] = scale;
        const double sv = scale * var;  // NaN stays NaN; rounding below zero gives 0
        o[LDK_BC_HALF] = z * sqrt(sv < 0.0 ? 0.0 : sv);
        o[LDK_BC_WEIGHT] = wgt;
        // zeta - 2 n zeta wgt + n wgt^2 lambda_0 = zeta (t^2 + n zeta (t - s2)) / s^2
        o[LDK_BC_WCE2] = zeta * fma(t, t, nd * zeta * (t - sigma2)) / (s * s);
    }
}

// Cubature partial sums per (row, chunk), rows = R * nw, lambda row = row / nw:
//   BC = false: [0] sum_k lambda_k p_k,        [1] sum_i w_i
//   BC = true:  [0] sum_k p_k / (lambda_k + s2) (NaN when some
//               lambda_k + s2 <= 0),           [1] sum_i y_i
template <typename R, bool BC>
__global__ __launch_bounds__(MLL_THREADS) void k_cub_terms(const double *__restrict__ lam,
                                                           const double *__restrict__ pw,
                                                           const R *__restrict__ w, int64_t n,
                                                           int nw, double sigma2, int chunks,
                                                           double *__restrict__ part)
{
    __shared__ double red[MLL_THREADS / 64][3];
    const int row = blockIdx.y, ch = blockIdx.x;
    const double *lr = lam + (size_t)(row / nw) * n;
    const double *pr = pw + (size_t)row * n;
    const R *wr = w + (size_t)row * n;
    double acc[3] = {0.0, 0.0, 0.0};
    const int64_t lo = (int64_t)ch * MLL_CHUNK;
#pragma unroll
    for (int it = 0; it < MLL_ITEMS; ++it) {
        const int64_t k = lo + threadIdx.x + (int64_t)it * MLL_THREADS;
        if (k < n) {
            const double p = pr[k];
            if constexpr (BC) {
                const double s = lr[k] + sigma2;
                acc[0] += s > 0.0 ? p / s : __builtin_nan("");
            } else {
                acc[0] = fma(lr[k], p, acc[0]);
            }
            acc[1] += (double)wr[k];
        }
    }
    block_sum3(acc, red);
    if (threadIdx.x == 0)
        for (int c = 0; c < 2; ++c) part[((size_t)row * chunks + ch) * 2 + c] = acc[c];
}

// Per row: e2 (BC = false) or the posterior fields (BC = true).
template <bool BC>
__global__ __launch_bounds__(MLL_THREADS) void k_cub_final(const double *__restrict__ part,
                                                           int chunks, int64_t n,
                                                           const double *__restrict__ lam,
                                                           double sigma2, double zeta, double z,
                                                           double *__restrict__ out)
{
    __shared__ double red[MLL_THREADS / 64][3];
    const int row = blockIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int c = threadIdx.x; c < chunks; c += MLL_THREADS)
        for (int q = 0; q < 2; ++q) acc[q] += part[((size_t)row * chunks + c) * 2 + q];
    block_sum3(acc, red);
    if (threadIdx.x != 0) return;
    cub_row_out<BC>(row, acc[0], acc[1], n, lam, sigma2, zeta, z, out);
}

// The fused lattice path: the top pass left the weighted sum of |W_k|^2 per
// tile (qpart[row][tiles]) and the row sums W_0 (y0[row]).
template <bool BC>
__global__ __launch_bounds__(MLL_THREADS) void k_cub_final_q(const double *__restrict__ qpart,
                                                             int tiles,
                                                             const double *__restrict__ y0,
                                                             int64_t n,
                                                             const double *__restrict__ lam,
                                                             double sigma2, double zeta, double z,
                                                             double *__restrict__ out)
{
    __shared__ double red[MLL_THREADS / 64][3];
    const int row = blockIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int c = threadIdx.x; c < tiles; c += MLL_THREADS) acc[0] += qpart[(size_t)row * tiles + c];
    block_sum3(acc, red);
    if (threadIdx.x != 0) return;
    cub_row_out<BC>(row, acc[0], y0[row], n, lam, sigma2, zeta, z, out);
}

}  // namespace

// Workspace of the likelihood ops (LDK_OP_MLL, LDK_OP_MLL_ADJOINT).
size_t mll_ws_bytes(int op, int kind, int64_t R, int m, int dtype)
{
    if (op == LDK_OP_MLL)
        return align256((size_t)R * chunks_of(m) * 3 * sizeof(double)) +
               power_tmp_bytes(kind, R, m, dtype);
    // adjoint: FP64; the FWHT runs in place in the output
    return real_lattice(kind, m) ? power_tmp_bytes(kind, R, m, LDK_F64) : 0;
}

// Workspace of the cubature ops for B transformed rows: partial sums, the
// power spectrum, the transform scratch.
size_t cub_ws_bytes(int kind, int64_t B, int m, int dtype)
{
    return align256((size_t)B * chunks_of(m) * 2 * sizeof(double)) +
           align256((size_t)B * ((size_t)1 << m) * sizeof(double)) +
           power_tmp_bytes(kind, B, m, dtype);
}

}  // namespace ldk

using namespace ldk;

extern "C" int ldk_mll(int kind, int R, int m, int dtype, const double *lam, double sigma2,
                       const void *y, double *L, double *g, double *dlogs2, void *ws,
                       ldk_stream stream)
{
    if ((kind != LDK_LATTICE && kind != LDK_DNET_B2) || (dtype != LDK_F64 && dtype != LDK_F32))
        return LDK_EINVAL;
    if (m < 0 || m > TW_MAX_LOG || R < 0 || R > 65535 || !(sigma2 >= 0.0 && sigma2 <= 1.0e300))
        return LDK_EINVAL;
    if (R == 0) return LDK_OK;
    if (!lam || !y || !L || !g || !ws) return LDK_EINVAL;
    int st = ensure_init();
    if (st) return st;
    hipStream_t s = as_stream(stream);
    const int64_t n = (int64_t)1 << m;
    const int chunks = chunks_of(m);
    double *part = static_cast<double *>(ws);
    void *tmp = static_cast<unsigned char *>(ws) + align256((size_t)R * chunks * 3 * sizeof(double));
    st = power_spectrum(kind, R, m, dtype, y, g, tmp, s);
    if (st) return st;
    hipLaunchKernelGGL(k_mll_terms, dim3(chunks, R), dim3(MLL_THREADS), 0, s, lam, g, n, sigma2,
                       1.0 / (double)n, chunks, part);
    LDK_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_mll_final, dim3(R), dim3(MLL_THREADS), 0, s, (const double *)part, chunks,
                       n, sigma2, L, dlogs2);
    LDK_LAUNCH_CHECK();
    return LDK_OK;
}

extern "C" int ldk_mll_adjoint(int kind, int R, int m, const double *g, double *a, void *ws,
                               ldk_stream stream)
{
    if ((kind != LDK_LATTICE && kind != LDK_DNET_B2) || m < 0 || m > TW_MAX_LOG || R < 0 ||
        R > 65535)
        return LDK_EINVAL;
    if (R == 0) return LDK_OK;
    if (!g || !a) return LDK_EINVAL;
    const size_t need = mll_ws_bytes(LDK_OP_MLL_ADJOINT, kind, R, m, LDK_F64);
    if (need && !ws) return LDK_EINVAL;
    int st = ensure_init();
    if (st) return st;
    hipStream_t s = as_stream(stream);
    const int64_t n = (int64_t)1 << m;
    if (m == 0) {
        const unsigned blocks = (unsigned)((R + 255) / 256);
        hipLaunchKernelGGL(k_copy_f64, dim3(blocks), dim3(256), 0, s, g, a, (int64_t)R);
        LDK_LAUNCH_CHECK();
        return LDK_OK;
    }
    PassArgs p{};
    p.rows = R;
    p.nrhs = 1;
    if (real_lattice(kind, m)) {
        // inverse half of the packed real transform, FP64: top pass from g,
        // then the inverse column and row passes
        const int mp = m - 1;
        const int64_t N = n / 2;
        const Plan pl = make_plan(mp, log_tile_for(LDK_LATTICE, LDK_F64));
        p.m = mp;
        p.half = N;
        p.lam = g;
        p.scale = 2.0;  // sum_k C_k W^{-k R(j)} with C = (g_k + g_{n-k}) / 2
        p.dst = pl.P == 1 ? (void *)a : ws;
        p.dst_row = pl.P == 1 ? n : N;
        p.g = pl.pass[pl.P - 1];
        p.global_tw = pl.P > 1;
        st = launch_real_top(LDK_F64, PM_ADJ, p, nullptr, s);
        if (st) return st;
        for (int q = pl.P - 2; q >= 0; --q) {
            PassArgs b = p;
            b.lam = nullptr;
            b.scale = 1.0;
            b.src = ws;
            b.src_row = N;
            b.dst = q == 0 ? (void *)a : ws;
            b.dst_row = q == 0 ? n : N;
            b.g = pl.pass[q];
            b.global_tw = q > 0;
            st = launch_pass(LDK_LATTICE, LDK_F64, PM_INV, PIO_SAME, q == 0 ? PIO_PACKED : PIO_SAME, b,
                             s);
            if (st) return st;
        }
        return LDK_OK;
    }
    // unnormalised FWHT (H symmetric; for n = 2 also the lattice case)
    const Plan pl = make_plan(m, log_tile_for(LDK_DNET_B2, LDK_F64));
    p.m = m;
    p.scale = 1.0;
    for (int q = 0; q < pl.P; ++q) {
        p.src = q == 0 ? (const void *)g : (const void *)a;
        p.src_row = n;
        p.dst = a;
        p.dst_row = n;
        p.g = pl.pass[q];
        st = launch_pass(LDK_DNET_B2, LDK_F64, PM_FWD, PIO_SAME, PIO_SAME, p, s);
        if (st) return st;
    }
    return LDK_OK;
}

namespace {

template <bool BC>
int cubature(int kind, int R, int nw, int m, int dtype, const double *lam, double sigma2,
             double zeta, const void *w, double z, double *out, void *ws, hipStream_t s)
{
    const int64_t n = (int64_t)1 << m;
    const int rows = R * nw;
    const int chunks = chunks_of(m);
    double *part = static_cast<double *>(ws);
    double *pw = reinterpret_cast<double *>(static_cast<unsigned char *>(ws) +
                                            align256((size_t)rows * chunks * 2 * sizeof(double)));
    void *tmp = reinterpret_cast<unsigned char *>(pw) + align256((size_t)rows * n * sizeof(double));
    if (real_lattice(kind, m)) {
        // packed half-length rows; the real top pass forms the weighted sums
        // itself (PM_QFORM), so the spectrum is never written.  Its tile sums
        // and the row sums use the partial-sum region of the workspace.
        const int mp = m - 1;
        const int64_t N = n / 2;
        const Plan pl = make_plan(mp, log_tile_for(LDK_LATTICE, dtype));
        const PassGeom top = pl.pass[pl.P - 1];
        const int64_t tiles = (int64_t)1 << (top.b0 - top.logW);
        if ((tiles + 1) > 2 * (int64_t)chunks) return LDK_ENOTSUP;  // region too small
        double *qpart = part;
        double *y0 = part + (size_t)rows * tiles;
        PassArgs a{};
        a.rows = rows;
        a.nrhs = nw;  // lambda row = row / nw
        a.m = mp;
        a.half = N;
        a.scale = 1.0;
        for (int p = 0; p < pl.P - 1; ++p) {
            a.src = p == 0 ? w : tmp;
            a.src_row = p == 0 ? n : N;
            a.dst = tmp;
            a.dst_row = N;
            a.g = pl.pass[p];
            a.global_tw = p > 0;
            const int st = launch_pass(LDK_LATTICE, dtype, PM_FWD, p == 0 ? PIO_PACKED : PIO_SAME,
                                       PIO_SAME, a, s);
            if (st) return st;
        }
        a.src = pl.P == 1 ? w : tmp;
        a.src_row = pl.P == 1 ? n : N;
        a.g = top;
        a.global_tw = pl.P > 1;
        a.lam = lam;
        a.sigma2 = sigma2;
        a.qform_lam = BC ? 0 : 1;
        int st = launch_real_top(dtype, PM_QFORM, a, y0, s, false, qpart);
        if (st) return st;
        hipLaunchKernelGGL(k_cub_final_q<BC>, dim3(rows), dim3(MLL_THREADS), 0, s,
                           (const double *)qpart, (int)tiles, (const double *)y0, n, lam, sigma2,
                           zeta, z, out);
        LDK_LAUNCH_CHECK();
        return LDK_OK;
    }
    int st = power_spectrum(kind, rows, m, dtype, w, pw, tmp, s);
    if (st) return st;
    if (dtype == LDK_F64)
        hipLaunchKernelGGL((k_cub_terms<double, BC>), dim3(chunks, rows), dim3(MLL_THREADS), 0, s,
                           lam, (const double *)pw, (const double *)w, n, nw, sigma2, chunks, part);
    else
        hipLaunchKernelGGL((k_cub_terms<float, BC>), dim3(chunks, rows), dim3(MLL_THREADS), 0, s,
                           lam, (const double *)pw, (const float *)w, n, nw, sigma2, chunks, part);
    LDK_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cub_final<BC>, dim3(rows), dim3(MLL_THREADS), 0, s, (const double *)part,
                       chunks, n, lam, sigma2, zeta, z, out);
    LDK_LAUNCH_CHECK();
    return LDK_OK;
}

bool finite_param(double v) { return v >= -1.0e300 && v <= 1.0e300; }

}  // namespace

extern "C" int ldk_wce(int kind, int R, int nw, int m, int dtype, const double *lam, double zeta,
                       const void *w, double *e2, void *ws, ldk_stream stream)
{
    if ((kind != LDK_LATTICE && kind != LDK_DNET_B2) || (dtype != LDK_F64 && dtype != LDK_F32))
        return LDK_EINVAL;
    if (m < 0 || m > TW_MAX_LOG || R < 0 || nw < 0 || !finite_param(zeta)) return LDK_EINVAL;
    if ((int64_t)R * nw > 65535) return LDK_EINVAL;
    if (R == 0 || nw == 0) return LDK_OK;
    if (!lam || !w || !e2 || !ws) return LDK_EINVAL;
    const int st = ensure_init();
    if (st) return st;
    return cubature<false>(kind, R, nw, m, dtype, lam, 0.0, zeta, w, 0.0, e2, ws,
                           as_stream(stream));
}

extern "C" int ldk_bayes_cubature(int kind, int R, int m, int dtype, const double *lam,
                                  double sigma2, double zeta, const void *y, double z,
                                  double *out, void *ws, ldk_stream stream)
{
    if ((kind != LDK_LATTICE && kind != LDK_DNET_B2) || (dtype != LDK_F64 && dtype != LDK_F32))
        return LDK_EINVAL;
    if (m < 0 || m > TW_MAX_LOG || R < 0 || R > 65535 || !(sigma2 >= 0.0 && sigma2 <= 1.0e300) ||
        !finite_param(zeta) || !(z >= 0.0 && z <= 1.0e300))
        return LDK_EINVAL;
    if (R == 0) return LDK_OK;
    if (!lam || !y || !out || !ws) return LDK_EINVAL;
    const int st = ensure_init();
    if (st) return st;
    return cubature<true>(kind, R, 1, m, dtype, lam, sigma2, zeta, y, z, out, ws,
                          as_stream(stream));
}
