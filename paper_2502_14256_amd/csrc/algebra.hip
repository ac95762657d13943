// Structured Gram algebra of Sec. 5.4 on top of the pass engine:
//   K = V Lambda conj(V),  lambda = sqrt(n) conj(V) k1,
//   K y = V (conj(V) y (.) lambda),  (K + s2 I)^-1 y = V (conj(V) y (/) (lambda + s2)),
//   log det(K + s2 I) = sum log(lambda + s2),
// with V = T_m / sqrt(n) (lattice, FFTBR / IFFTBR) or H_m / sqrt(n) (net, FWHT),
// and the update that doubles n (eq. ft_next_parts).
#include <cmath>

#include "transform.hpp"

namespace ldk {

namespace {

constexpr int LOGDET_THREADS = 256;
constexpr int LOGDET_CHUNK = 2048;  // eigenvalues per partial sum (one workgroup)

size_t esize(int dtype) { return dtype == LDK_F64 ? 8 : 4; }

bool valid_kind(int kind) { return kind == LDK_LATTICE || kind == LDK_DNET_B2; }
bool valid_dtype(int dtype) { return dtype == LDK_F64 || dtype == LDK_F32; }
bool valid_m(int m) { return m >= 0 && m <= TW_MAX_LOG; }

// Workspace for the complex intermediate of the lattice transforms.
size_t cplx_rows_bytes(int64_t rows, int m, int dtype) { return (size_t)rows * ((size_t)2 << m) * esize(dtype); }
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// The plan over mp index bits of a transform of length 2^m_key, with the
// parameters plan_params gives (kind, dtype, m_key, rows).
Plan tuned_plan(int kind, int dtype, int m_key, int mp, int64_t rows)
{
    const PlanParams p = plan_params(kind, dtype, m_key, rows);
    return make_plan(mp, p.log_tile, p.loge_max);
}

// Whether any plan that may be chosen for (kind, dtype, m_key) over mp bits
// has more than one pass (the workspace must then hold the intermediate).
bool any_multipass(int kind, int dtype, int m_key, int mp)
{
    PlanParams c[16];
    const int nc = plan_candidates(kind, dtype, m_key, c, 16);
    for (int i = 0; i < nc; ++i)
        if (make_plan(mp, c[i].log_tile, c[i].loge_max).P > 1) return true;
    return false;
}

// ---------------------------------------------------------------------------
// n = 1 (m = 0): every transform is the identity.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_scalar_apply(const double *lam, const R *y, R *c, int64_t rows, int nrhs,
                               double sigma2, int mode)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    const double l = lam[i / nrhs];
    const double v = (double)y[i];
    c[i] = (R)(mode == 0 ? v / (l + sigma2) : v * l);
}

// ---------------------------------------------------------------------------
// log det: fixed-order FP64 tree sums (deterministic run to run)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(LOGDET_THREADS) void k_logdet_partial(const double *lam, int64_t n,
                                                                   double sigma2, int chunks,
                                                                   double *partial)
{
    __shared__ double red[LOGDET_THREADS];
    const int r = blockIdx.y, ch = blockIdx.x, t = threadIdx.x;
    const double *row = lam + (int64_t)r * n;
    const int64_t lo = (int64_t)ch * LOGDET_CHUNK;
    const int64_t hi = lo + LOGDET_CHUNK < n ? lo + LOGDET_CHUNK : n;
    LogProd acc;
    static_assert(LOGDET_CHUNK % LOGDET_THREADS == 0, "whole items per thread");
    double lv[LOGDET_CHUNK / LOGDET_THREADS];
#pragma unroll
    for (int it = 0; it < LOGDET_CHUNK / LOGDET_THREADS; ++it) {  // loads first
        const int64_t k = lo + t + (int64_t)it * LOGDET_THREADS;
        lv[it] = k < hi ? row[k] : 0.0;
    }
#pragma unroll
    for (int it = 0; it < LOGDET_CHUNK / LOGDET_THREADS; ++it) {
        const int64_t k = lo + t + (int64_t)it * LOGDET_THREADS;
        if (k < hi) acc.add(lv[it] + sigma2);
    }
    red[t] = acc.value();
    __syncthreads();
    for (int w = LOGDET_THREADS / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) partial[(int64_t)r * chunks + ch] = red[0];
}

__global__ __launch_bounds__(LOGDET_THREADS) void k_logdet_final(const double *partial, int chunks,
                                                                 double *out)
{
    __shared__ double red[LOGDET_THREADS];
    const int r = blockIdx.x, t = threadIdx.x;
    double acc = 0.0;
    for (int c = t; c < chunks; c += LOGDET_THREADS) acc += partial[(int64_t)r * chunks + c];
    red[t] = acc;
    __syncthreads();
    for (int w = LOGDET_THREADS / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) out[r] = red[0];
}

// ---------------------------------------------------------------------------
// Update combine.  The size-n unnormalised transform U of the new half sits
// in the second half of each output row.
//   ytilde: full[k] = h (old[k] + c w_k U[k]), full[n+k] = h (old[k] - c w_k U[k])
//           with h = 2^-1/2, c = n^-1/2;
//   lambda: full[k] = old[k] + Re(w_k U[k]), full[n+k] = old[k] - Re(w_k U[k]).
// w_k = W_{2n}^k (lattice) or 1 (net).
// ---------------------------------------------------------------------------
template <typename R, bool CPLX, bool U_REAL>
__global__ void k_update_combine(const void *old_, void *full_, const void *u_, int64_t u_row,
                                 int64_t rows, int m, double c)
{
    const int64_t n = (int64_t)1 << m;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= rows * n) return;
    const int64_t row = gid >> m, k = gid & (n - 1);
    const R h = (R)0.70710678118654752440;
    if constexpr (CPLX) {
        const cplx<R> *old = static_cast<const cplx<R> *>(old_) + row * n;
        cplx<R> *full = static_cast<cplx<R> *>(full_) + row * 2 * n;
        cplx<R> uk;
        if constexpr (U_REAL)
            uk = {static_cast<const R *>(u_)[row * u_row + k], (R)0};
        else
            uk = static_cast<const cplx<R> *>(u_)[row * u_row + k];
        cplx<R> w = cmul(uk, tw_any<R>((uint64_t)k, m + 1));
        w = {w.re * (R)c, w.im * (R)c};
        const cplx<R> o = old[k];
        full[k] = {h * (o.re + w.re), h * (o.im + w.im)};
        full[n + k] = {h * (o.re - w.re), h * (o.im - w.im)};
    } else {
        const R *old = static_cast<const R *>(old_) + row * n;
        R *full = static_cast<R *>(full_) + row * 2 * n;
        const R *u = static_cast<const R *>(u_) + row * u_row;
        const R w = u[k] * (R)c;
        const R o = old[k];
        full[k] = h * (o + w);
        full[n + k] = h * (o - w);
    }
}

// n = 1 (FT_0 is the identity, w_0 = 1): lambda_full = [lambda_m + u; lambda_m - u]
// with u the new half's k1 (widened to FP64).
template <typename U_T>
__global__ void k_eig_update_combine(const double *old, double *full, const void *u_, int64_t u_row,
                                     int64_t rows, int m)
{
    const int64_t n = (int64_t)1 << m;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= rows * n) return;
    const int64_t row = gid >> m, k = gid & (n - 1);
    const double part = (double)static_cast<const U_T *>(u_)[row * u_row + k];
    const double o = old[row * n + k];
    full[row * 2 * n + k] = o + part;
    full[row * 2 * n + n + k] = o - part;
}

// n = 1 eigenvalues: lambda = k1 (widened to FP64).
template <typename R>
__global__ void k_widen(const R *in, double *out, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = (double)in[i];
}

unsigned blocks_for(int64_t work, int threads) { return (unsigned)((work + threads - 1) / threads); }

// Forward transform of `rows` rows through all passes: src (real or complex)
// -> dst.  dst_real keeps the real part at the last pass.  `scale` is applied
// at the last store.
int forward_all(int kind, int dtype, int m, int64_t rows, const void *src, int64_t src_row,
                bool src_real, void *dst, int64_t dst_row, bool dst_real, void *tmp,
                int64_t tmp_row, double scale, hipStream_t s, bool src_f32 = false)
{
    const Plan pl = tuned_plan(kind, dtype, m, m, rows);
    for (int p = 0; p < pl.P; ++p) {
        const bool first = p == 0, last = p == pl.P - 1;
        PassArgs a{};
        a.src = first ? src : tmp;
        a.src_row = first ? src_row : tmp_row;
        a.dst = last ? dst : tmp;
        a.dst_row = last ? dst_row : tmp_row;
        a.rows = rows;
        a.m = m;
        a.g = pl.pass[p];
        a.nrhs = 1;
        a.global_tw = p > 0;
        a.scale = last ? scale : 1.0;
        const int st = launch_pass(kind, dtype, PM_FWD, first && src_real ? PIO_REAL : PIO_SAME,
                                   last && dst_real ? PIO_REAL : PIO_SAME, a, s, first && src_f32);
        if (st) return st;
    }
    return LDK_OK;
}

// Solve / matvec through all passes: src (real rows) -> dst (real rows);
// complex intermediates (lattice, more than one pass) live in tmp.
int apply_all(int kind, int dtype, int mode, int m, int64_t rows, int nrhs, const double *lam,
              double sigma2, const void *src, void *dst, void *tmp, hipStream_t s)
{
    const Plan pl = tuned_plan(kind, dtype, m, m, rows);
    const int64_t n = (int64_t)1 << m;
    const bool lat = kind == LDK_LATTICE;
    void *work = (lat && pl.P > 1) ? tmp : dst;
    const double scale = 1.0 / (double)n;
    // forward passes below the top one
    for (int p = 0; p < pl.P - 1; ++p) {
        PassArgs a{};
        a.src = p == 0 ? src : work;
        a.dst = work;
        a.src_row = a.dst_row = n;
        a.rows = rows;
        a.m = m;
        a.g = pl.pass[p];
        a.nrhs = nrhs;
        a.global_tw = p > 0;
        a.scale = 1.0;
        const int st = launch_pass(kind, dtype, PM_FWD, lat && p == 0 ? PIO_REAL : PIO_SAME, PIO_SAME,
                                   a, s);
        if (st) return st;
    }
    {
        const int p = pl.P - 1;
        PassArgs a{};
        a.src = p == 0 ? src : work;
        a.dst = p == 0 ? dst : work;
        a.src_row = a.dst_row = n;
        a.rows = rows;
        a.m = m;
        a.g = pl.pass[p];
        a.lam = lam;
        a.nrhs = nrhs;
        a.global_tw = p > 0;
        a.sigma2 = sigma2;
        a.scale = scale;
        const int io = lat && p == 0 ? PIO_REAL : PIO_SAME;
        const int st = launch_pass(kind, dtype, mode, io, io, a, s);
        if (st) return st;
    }
    for (int p = pl.P - 2; p >= 0; --p) {
        PassArgs a{};
        a.src = work;
        a.dst = p == 0 ? dst : work;
        a.src_row = a.dst_row = n;
        a.rows = rows;
        a.m = m;
        a.g = pl.pass[p];
        a.nrhs = nrhs;
        a.global_tw = p > 0;
        a.scale = 1.0;
        const int st = launch_pass(kind, dtype, PM_INV, PIO_SAME, lat && p == 0 ? PIO_REAL : PIO_SAME,
                                   a, s);
        if (st) return st;
    }
    return LDK_OK;
}

// ---------------------------------------------------------------------------
// Real-input lattice transforms through the packed half-length FFTBR
// (realfft.hip): N = n/2 complex, plan over m - 1 bits, top pass special.
// ---------------------------------------------------------------------------
bool real_path(int kind, int m) { return kind == LDK_LATTICE && m >= 2; }

// lambda = Re FFTBR_n(k1) (unnormalised), FP64, from real k1 rows of n.
// With ld_part, the top pass also leaves each row's log-det partial sums
// there (*ld_count per row, at ld_part + row * *ld_count), sigma2 added.
int real_eig(int m, int64_t rows, const void *k1, bool k1_f32, double *lam, void *ws, hipStream_t s,
             double *ld_part = nullptr, double sigma2 = 0.0, int *ld_count = nullptr)
{
    const int mp = m - 1;
    const int64_t N = (int64_t)1 << mp;
    const Plan pl = tuned_plan(LDK_LATTICE, LDK_F64, m, mp, rows);
    PassArgs a{};
    a.rows = rows;
    a.m = mp;
    a.nrhs = 1;
    a.half = N;
    a.scale = 1.0;
    a.sigma2 = sigma2;
    const PassGeom &top = pl.pass[pl.P - 1];
    if (ld_count) *ld_count = 1 << (top.b0 - top.logW);
    if (pl.P == 1) {
        a.src = k1;
        a.src_row = 2 * N;
        a.g = pl.pass[0];
        return launch_real_top(LDK_F64, PM_FWD, a, lam, s, k1_f32, ld_part);
    }
    for (int p = 0; p < pl.P - 1; ++p) {
        a.src = p == 0 ? k1 : ws;
        a.src_row = p == 0 ? 2 * N : N;
        a.dst = ws;
        a.dst_row = N;
        a.g = pl.pass[p];
        a.global_tw = p > 0;
        const int st = launch_pass(LDK_LATTICE, LDK_F64, PM_FWD, p == 0 ? PIO_PACKED : PIO_SAME,
                                   PIO_SAME, a, s, p == 0 && k1_f32);
        if (st) return st;
    }
    a.src = ws;
    a.src_row = N;
    a.g = pl.pass[pl.P - 1];
    a.global_tw = 1;
    return launch_real_top(LDK_F64, PM_FWD, a, lam, s, false, ld_part);
}

// c = (K + s2 I)^-1 y (PM_SOLVE) or K y (PM_MATVEC) for real rows of n.
// With ld_out, the first inverse pass also sums each of ld_rows rows'
// ld_count log-det partials (left by real_eig) into ld_out when it has a full
// wave per tile; *ld_done says whether it did.
int real_apply(int dtype, int mode, int m, int64_t rows, int nrhs, const double *lam, double sigma2,
               const void *y, void *c, void *ws, hipStream_t s, const double *ld_part = nullptr,
               int ld_count = 0, double *ld_out = nullptr, int64_t ld_rows = 0, bool *ld_done = nullptr)
{
    if (ld_done) *ld_done = false;
    const int mp = m - 1;
    const int64_t N = (int64_t)1 << mp;
    const Plan pl = tuned_plan(LDK_LATTICE, dtype, m, mp, rows);
    PassArgs a{};
    a.rows = rows;
    a.m = mp;
    a.nrhs = nrhs;
    a.half = N;
    a.lam = lam;
    a.sigma2 = sigma2;
    if (pl.P == 1) {
        a.src = y;
        a.dst = c;
        a.src_row = a.dst_row = 2 * N;
        a.g = pl.pass[0];
        a.scale = 1.0 / (double)N;
        return launch_real_top(dtype, mode, a, nullptr, s);
    }
    for (int p = 0; p < pl.P - 1; ++p) {
        PassArgs b = a;
        b.src = p == 0 ? y : ws;
        b.src_row = p == 0 ? 2 * N : N;
        b.dst = ws;
        b.dst_row = N;
        b.g = pl.pass[p];
        b.global_tw = p > 0;
        b.scale = 1.0;
        const int st = launch_pass(LDK_LATTICE, dtype, PM_FWD, p == 0 ? PIO_PACKED : PIO_SAME,
                                   PIO_SAME, b, s);
        if (st) return st;
    }
    {
        PassArgs b = a;
        b.src = b.dst = ws;
        b.src_row = b.dst_row = N;
        b.g = pl.pass[pl.P - 1];
        b.global_tw = 1;
        b.scale = 1.0 / (double)N;
        if (nrhs >= 2) {
            // every eigenvalue row serves nrhs rows: form its filter once
            void *coef = static_cast<unsigned char *>(ws) + align256(cplx_rows_bytes(rows, mp, dtype));
            const int st = launch_filter_coef(dtype, mode, mp, rows / nrhs, lam, sigma2, b.scale,
                                              coef, s);
            if (st) return st;
            b.coef = coef;
        }
        const int st = launch_real_top(dtype, mode, b, nullptr, s);
        if (st) return st;
    }
    for (int p = pl.P - 2; p >= 0; --p) {
        PassArgs b = a;
        b.src = ws;
        b.src_row = N;
        b.dst = p == 0 ? c : ws;
        b.dst_row = p == 0 ? 2 * N : N;
        b.g = pl.pass[p];
        b.global_tw = p > 0;
        b.scale = 1.0;
        const int64_t tiles = b.rows << (mp - b.g.a - b.g.logW);
        if (ld_out && ld_done && !*ld_done && (b.g.a + b.g.logW - b.g.logE) >= 6 && tiles >= ld_rows) {
            b.ld_part = ld_part;
            b.ld_out = ld_out;
            b.ld_rows = ld_rows;
            b.ld_count = ld_count;
            *ld_done = true;
        }
        const int st = launch_pass(LDK_LATTICE, dtype, PM_INV, PIO_SAME,
                                   p == 0 ? PIO_PACKED : PIO_SAME, b, s);
        if (st) return st;
    }
    return LDK_OK;
}

// The fused fit (lattice, FP64, n >= 4): eigenvalues, every solve and the
// log-det share the tile passes of the half-length packed transforms.
bool fit_fused(int kind, int m, int dtype) { return kind == LDK_LATTICE && m >= 2 && dtype == LDK_F64; }


// Top-pass geometry of the fused fit: the plan's top pass, narrowed until
// the column and rhs tiles fit a workgroup's LDS together, with four
// elements per thread where the kernel takes it.  At one replication of
// n = 2^20 the plan's 4 + 4 columns fit (68 KiB, eight elements per thread:
// 49.7 us for the fit against 52.0 with 2 + 2 columns in 64 KiB and four
// elements per thread), so the tile rows are 64-byte runs.
PassGeom fit_top_geom(const Plan &pl)
{
    PassGeom g = pl.pass[pl.P - 1];
    while (g.b0 > 0 && g.logW > 1 &&
           2 * (((size_t)1 << (g.a + g.logW)) * 17 / 16) * 16 > LDS_PER_GROUP)
        --g.logW;
    PassGeom g4 = g;
    g4.logE = 2;
    return (g.logE == 3 && fit_top_supported(g4)) ? g4 : g;
}

// Fit workspace for B = R (nrhs + 1) rows: [log-det partials | column rows | rhs rows].
size_t fit_ws_bytes(int kind, int64_t B, int m, int dtype);

size_t ws_bytes(int op, int kind, int64_t B, int m, int dtype)
{
    if (op == LDK_OP_FIT) return fit_ws_bytes(kind, B, m, dtype);
    if (op == LDK_OP_MLL || op == LDK_OP_MLL_ADJOINT) return mll_ws_bytes(op, kind, B, m, dtype);
    if (op == LDK_OP_WCE || op == LDK_OP_BAYES_CUBATURE) return cub_ws_bytes(kind, B, m, dtype);
    if (m == 0) return op == LDK_OP_LOGDET ? (size_t)B * sizeof(double) : 0;
    const bool lat = kind == LDK_LATTICE;
    // sizes hold for every plan the tuned table may select (any rows)
    switch (op) {
    case LDK_OP_TRANSFORM: return 0;
    case LDK_OP_EIG: {
        // FP64 transform whatever the input dtype; real lattice rows of n run
        // as packed complex rows of n/2
        if (real_path(kind, m))
            return any_multipass(kind, LDK_F64, m, m - 1) ? cplx_rows_bytes(B, m - 1, LDK_F64) : 0;
        return (lat && any_multipass(kind, LDK_F64, m, m)) ? cplx_rows_bytes(B, m, LDK_F64) : 0;
    }
    case LDK_OP_SOLVE:
    case LDK_OP_MATVEC:
        // real lattice rows: the complex intermediate, then room for the
        // filter coefficients of up to B / 2 eigenvalue rows (formed when
        // every eigenvalue row serves two or more right-hand sides)
        if (real_path(kind, m))
            return any_multipass(kind, dtype, m, m - 1)
                       ? align256(cplx_rows_bytes(B, m - 1, dtype)) + cplx_rows_bytes(B / 2, m - 1, dtype)
                       : 0;
        return (lat && any_multipass(kind, dtype, m, m)) ? cplx_rows_bytes(B, m, dtype) : 0;
    case LDK_OP_LOGDET: {
        const int64_t n = (int64_t)1 << m;
        const int64_t chunks = (n + LOGDET_CHUNK - 1) / LOGDET_CHUNK;
        return (size_t)B * chunks * sizeof(double);
    }
    case LDK_OP_UPDATE_DOUBLE: return 0;
    case LDK_OP_EIG_UPDATE_DOUBLE: return lat ? cplx_rows_bytes(B, m, LDK_F64) : 0;
    default: return 0;
    }
}

size_t fit_ws_bytes(int kind, int64_t B, int m, int dtype)
{
    // eig, solve and log-det one after the other, sharing the workspace (the
    // path taken when the fused one does not apply, and for nrhs = 0)
    size_t w = ws_bytes(LDK_OP_EIG, kind, B, m, dtype);
    if (fit_fused(kind, m, dtype)) {
        PlanParams cand[16];
        const int nc = plan_candidates(LDK_LATTICE, LDK_F64, m, cand, 16);
        for (int i = 0; i < nc; ++i) {
            const Plan pl = make_plan(m - 1, cand[i].log_tile, cand[i].loge_max);
            const PassGeom top = fit_top_geom(pl);  // at least as many tiles as the plan's top
            const size_t cb = (size_t)1 << (top.b0 - top.logW);
            const size_t rows = pl.P > 1 ? (size_t)B * ((size_t)1 << (m - 1)) * 16 : 0;
            // + the solve filter's coefficients (nrhs >= 2: at most B / 3 rows)
            const size_t coef = pl.P > 1 ? align256(cplx_rows_bytes(B / 2, m - 1, LDK_F64)) : 0;
            const size_t f = align256((size_t)B * cb * sizeof(double)) + align256(rows) + coef;
            if (f > w) w = f;
        }
    }
    const size_t ws = ws_bytes(LDK_OP_SOLVE, kind, B, m, dtype);
    const size_t wl = ws_bytes(LDK_OP_LOGDET, kind, B, m, dtype);
    if (ws > w) w = ws;
    if (wl > w) w = wl;
    if (real_path(kind, m) && !fit_fused(kind, m, dtype)) {
        // the log-det partials of the eigenvalue pass, kept through the solve
        size_t cbmax = 1;
        PlanParams cand[16];
        const int nc = plan_candidates(LDK_LATTICE, LDK_F64, m, cand, 16);
        for (int i = 0; i < nc; ++i) {
            const Plan pl = make_plan(m - 1, cand[i].log_tile, cand[i].loge_max);
            const PassGeom &top = pl.pass[pl.P - 1];
            const size_t cb = (size_t)1 << (top.b0 - top.logW);
            if (cb > cbmax) cbmax = cb;
        }
        const size_t e = ws_bytes(LDK_OP_EIG, kind, B, m, dtype);
        const size_t f = align256((size_t)B * cbmax * sizeof(double)) + (e > ws ? e : ws);
        if (f > w) w = f;
    }
    return w;
}

}  // namespace

}  // namespace ldk

using namespace ldk;

extern "C" {

size_t ldk_workspace_bytes(int op, int kind, int64_t B, int m, int dtype)
{
    if (!valid_kind(kind) || !valid_dtype(dtype) || !valid_m(m) || B < 0) return 0;
    return ws_bytes(op, kind, B, m, dtype);
}

int ldk_transform(int kind, int dir, int B, int m, int dtype, const void *in, void *out, void *ws,
                  ldk_stream stream)
{
    (void)ws;
    if (!valid_kind(kind) || !valid_dtype(dtype) || !valid_m(m) || B < 0 || !in || !out)
        return LDK_EINVAL;
    if (kind == LDK_LATTICE && dir != 1 && dir != -1) return LDK_EINVAL;
    if (B == 0) return LDK_OK;
    int st = ensure_init();
    if (st) return st;
    hipStream_t s = as_stream(stream);
    const int64_t n = (int64_t)1 << m;
    const size_t row_bytes = (size_t)n * esize(dtype) * (kind == LDK_LATTICE ? 2 : 1);
    if (m == 0) {
        if (in != out) LDK_HIP_CHECK(hipMemcpyAsync(out, in, row_bytes * B, hipMemcpyDeviceToDevice, s));
        return LDK_OK;
    }
    const double scale = 1.0 / std::sqrt((double)n);
    if (kind == LDK_DNET_B2 || dir == 1)
        return forward_all(kind, dtype, m, B, in, n, false, out, n, false, out, n, scale, s);
    // inverse FFTBR: passes from the top down
    const Plan pl = tuned_plan(kind, dtype, m, m, B);
    for (int p = pl.P - 1; p >= 0; --p) {
        PassArgs a{};
        a.src = p == pl.P - 1 ? in : out;
        a.dst = out;
        a.src_row = a.dst_row = n;
        a.rows = B;
        a.m = m;
        a.g = pl.pass[p];
        a.nrhs = 1;
        a.global_tw = p > 0;
        a.scale = p == 0 ? scale : 1.0;
        st = launch_pass(kind, dtype, PM_INV, PIO_SAME, PIO_SAME, a, s);
        if (st) return st;
    }
    return LDK_OK;
}

int ldk_eig(int kind, int R, int m, int dtype, const void *k1, double *lam, void *ws,
            ldk_stream stream)
{
    if (!valid_kind(kind) || !valid_dtype(dtype) || !valid_m(m) || R < 0 || !k1 || !lam)
        return LDK_EINVAL;
    if (R == 0) return LDK_OK;
    if (ws_bytes(LDK_OP_EIG, kind, R, m, dtype) && !ws) return LDK_EINVAL;
    int st = ensure_init();
    if (st) return st;
    hipStream_t s = as_stream(stream);
    const int64_t n = (int64_t)1 << m;
    if (m == 0) {
        if (dtype == LDK_F64)
            hipLaunchKernelGGL(k_widen<double>, dim3(blocks_for(R, 256)), dim3(256), 0, s,
                               (const double *)k1, lam, (int64_t)R);
        else
            hipLaunchKernelGGL(k_widen<float>, dim3(blocks_for(R, 256)), dim3(256), 0, s,
                               (const float *)k1, lam, (int64_t)R);
        LDK_LAUNCH_CHECK();
        return LDK_OK;
    }
    const bool lat = kind == LDK_LATTICE;
    if (real_path(kind, m)) return real_eig(m, R, k1, dtype == LDK_F32, lam, ws, s);
    // lambda = sqrt(n) * orthonormal transform = unnormalised transform, in FP64
    return forward_all(kind, LDK_F64, m, R, k1, n, lat, lam, n, lat, lat ? ws : (void *)lam, n, 1.0,
                       s, dtype == LDK_F32);
}

static int apply_entry(int mode, int kind, int R, int nrhs, int m, int dtype, const double *lam,
                       double sigma2, const void *y, void *c, void *ws, ldk_stream stream)
{
    if (!valid_kind(kind) || !valid_dtype(dtype) || !valid_m(m) || R < 0 || nrhs < 0 || !lam ||
        !y || !c)
        return LDK_EINVAL;
    if (!(sigma2 >= 0.0)) return LDK_EINVAL;
    const int64_t rows = (int64_t)R * nrhs;
    if (rows == 0) return LDK_OK;
    if (ws_bytes(LDK_OP_SOLVE, kind, rows, m, dtype) && !ws) return LDK_EINVAL;
    int st = ensure_init();
    if (st) return st;
    hipStream_t s = as_stream(stream);
    if (m == 0) {
        if (dtype == LDK_F64)
            hipLaunchKernelGGL(k_scalar_apply<double>, dim3(blocks_for(rows, 256)), dim3(256), 0, s,
                               lam, (const double *)y, (double *)c, rows, nrhs,
                               sigma2, mode == PM_SOLVE ? 0 : 1);
        else
            hipLaunchKernelGGL(k_scalar_apply<float>, dim3(blocks_for(rows, 256)), dim3(256), 0, s,
                               lam, (const float *)y, (float *)c, rows, nrhs,
                               sigma2, mode == PM_SOLVE ? 0 : 1);
        LDK_LAUNCH_CHECK();
        return LDK_OK;
    }
    if (real_path(kind, m)) return real_apply(dtype, mode, m, rows, nrhs, lam, sigma2, y, c, ws, s);
    if (kind == LDK_DNET_B2 && dtype == LDK_F32 && m >= 12 &&
        plan_params(kind, dtype, m, rows).engine == ENGINE_SPLIT16)
        return fwht16_apply(mode, m, rows, nrhs, lam, sigma2, static_cast<const float *>(y),
                            static_cast<float *>(c), s);
    return apply_all(kind, dtype, mode, m, rows, nrhs, lam, sigma2, y, c, ws, s);
}

int ldk_solve(int kind, int R, int nrhs, int m, int dtype, const double *lam, double sigma2,
              const void *y, void *c, void *ws, ldk_stream stream)
{
    return apply_entry(PM_SOLVE, kind, R, nrhs, m, dtype, lam, sigma2, y, c, ws, stream);
}

int ldk_matvec(int kind, int R, int nrhs, int m, int dtype, const double *lam, const void *y,
               void *out, void *ws, ldk_stream stream)
{
    return apply_entry(PM_MATVEC, kind, R, nrhs, m, dtype, lam, 0.0, y, out, ws, stream);
}

int ldk_logdet(int R, int m, const double *lam, double sigma2, double *out, void *ws,
               ldk_stream stream)
{
    if (!valid_m(m) || R < 0 || R > 65535 || !lam || !out || !(sigma2 >= 0.0)) return LDK_EINVAL;
    if (R == 0) return LDK_OK;
    if (!ws) return LDK_EINVAL;
    hipStream_t s = as_stream(stream);
    const int64_t n = (int64_t)1 << m;
    const int chunks = (int)((n + LOGDET_CHUNK - 1) / LOGDET_CHUNK);
    double *partial = static_cast<double *>(ws);
    hipLaunchKernelGGL(k_logdet_partial, dim3(chunks, R), dim3(LOGDET_THREADS), 0, s, lam, n, sigma2,
                       chunks, partial);
    LDK_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_logdet_final, dim3(R), dim3(LOGDET_THREADS), 0, s, partial, chunks, out);
    LDK_LAUNCH_CHECK();
    return LDK_OK;
}

int ldk_fit(int kind, int R, int nrhs, int m, int dtype, const void *k1, double sigma2,
            const void *y, double *lam, void *c, double *logdet, void *ws, ldk_stream stream)
{
    if (!valid_kind(kind) || !valid_dtype(dtype) || !valid_m(m) || R < 0 || R > 65535 || nrhs < 0)
        return LDK_EINVAL;
    if (!(sigma2 >= 0.0)) return LDK_EINVAL;
    if (R == 0) return LDK_OK;
    if (!k1 || !lam || (nrhs > 0 && (!y || !c))) return LDK_EINVAL;
    const int64_t B = (int64_t)R * (nrhs + 1);
    if (fit_ws_bytes(kind, B, m, dtype) && !ws) return LDK_EINVAL;
    int st;
    if (kind == LDK_DNET_B2 && dtype == LDK_F64 && nrhs > 0 && m >= 1) {
        // a net whose eigenvalue and solve plans are both one pass: the
        // whole fit in one launch, with the separate calls' pass arguments
        const Plan pe = tuned_plan(LDK_DNET_B2, LDK_F64, m, m, R);
        const Plan pq = tuned_plan(LDK_DNET_B2, LDK_F64, m, m, (int64_t)R * nrhs);
        if (pe.P == 1 && pq.P == 1) {
            st = ensure_init();
            if (st) return st;
            const int64_t n = (int64_t)1 << m;
            PassArgs aE{}, aS{};
            aE.src = k1;
            aE.dst = lam;
            aE.src_row = aE.dst_row = n;
            aE.rows = R;
            aE.m = m;
            aE.g = pe.pass[0];
            aE.nrhs = 1;
            aE.scale = 1.0;
            aS.src = y;
            aS.dst = c;
            aS.src_row = aS.dst_row = n;
            aS.rows = (int64_t)R * nrhs;
            aS.m = m;
            aS.g = pq.pass[0];
            aS.lam = lam;
            aS.nrhs = nrhs;
            aS.sigma2 = sigma2;
            aS.scale = 1.0 / (double)n;
            st = launch_fit_net_one(aE, aS, logdet, as_stream(stream));
            if (st != LDK_ENOTSUP) return st;
        }
    }
    if (real_path(kind, m) && !fit_fused(kind, m, dtype) && nrhs > 0 && logdet) {
        // FP32 lattice: the eigenvalue pass leaves the log-det partials, the
        // solve's first inverse pass sums them (no separate log-det read of
        // lambda); the partials sit below the passes' own workspace
        st = ensure_init();
        if (st) return st;
        hipStream_t s = as_stream(stream);
        const Plan pe = tuned_plan(LDK_LATTICE, LDK_F64, m, m - 1, R);
        const PassGeom &top = pe.pass[pe.P - 1];
        double *partial = static_cast<double *>(ws);
        void *rest = static_cast<unsigned char *>(ws) +
                     align256((size_t)R * ((size_t)1 << (top.b0 - top.logW)) * sizeof(double));
        int cb = 0;
        st = real_eig(m, R, k1, dtype == LDK_F32, lam, rest, s, partial, sigma2, &cb);
        if (st) return st;
        bool done = false;
        st = real_apply(dtype, PM_SOLVE, m, (int64_t)R * nrhs, nrhs, lam, sigma2, y, c, rest, s, partial, cb,
                        logdet, R, &done);
        if (st) return st;
        if (!done) {
            hipLaunchKernelGGL(k_logdet_final, dim3(R), dim3(LOGDET_THREADS), 0, s, (const double *)partial,
                               cb, logdet);
            LDK_LAUNCH_CHECK();
        }
        return LDK_OK;
    }
    if (!fit_fused(kind, m, dtype) || nrhs == 0) {
        st = ldk_eig(kind, R, m, dtype, k1, lam, ws, stream);
        if (st) return st;
        if (nrhs > 0) {
            st = ldk_solve(kind, R, nrhs, m, dtype, lam, sigma2, y, c, ws, stream);
            if (st) return st;
        }
        return logdet ? ldk_logdet(R, m, lam, sigma2, logdet, ws, stream) : LDK_OK;
    }
    st = ensure_init();
    if (st) return st;
    hipStream_t s = as_stream(stream);
    const int mp = m - 1;
    const int64_t n = (int64_t)1 << m, N = n / 2;
    const Plan pl = tuned_plan(LDK_LATTICE, LDK_F64, m, mp, B);
    // one rhs per column: both top passes in one launch (narrower tiles)
    const PassGeom ftop = fit_top_geom(pl);
    const bool one_top = nrhs == 1 && fit_top_supported(ftop);
    const PassGeom top = one_top ? ftop : pl.pass[pl.P - 1];
    const int cb_count = 1 << (top.b0 - top.logW);
    unsigned char *w8 = static_cast<unsigned char *>(ws);
    double *partial = reinterpret_cast<double *>(w8);
    void *wsK = w8 + align256((size_t)B * cb_count * sizeof(double));
    void *wsY = static_cast<unsigned char *>(wsK) + (size_t)R * N * 16;
    PassArgs aK{}, aY{};
    aK.rows = R;
    aK.nrhs = 1;
    aY.rows = (int64_t)R * nrhs;
    aY.nrhs = nrhs;
    aK.m = aY.m = mp;
    aK.half = aY.half = N;
    aK.sigma2 = aY.sigma2 = sigma2;
    aK.scale = 1.0;
    aY.lam = lam;
    // forward passes below the top one: column and right-hand sides in one launch
    for (int p = 0; p < pl.P - 1; ++p) {
        PassArgs k0 = aK, y0 = aY;
        k0.src = p == 0 ? k1 : (const void *)wsK;
        y0.src = p == 0 ? y : (const void *)wsY;
        k0.src_row = y0.src_row = p == 0 ? n : N;
        k0.dst = wsK;
        y0.dst = wsY;
        k0.dst_row = y0.dst_row = N;
        k0.g = y0.g = pl.pass[p];
        k0.global_tw = y0.global_tw = p > 0;
        k0.scale = y0.scale = 1.0;
        y0.lam = nullptr;
        st = launch_pass2(LDK_LATTICE, LDK_F64, PM_FWD, p == 0 ? PIO_PACKED : PIO_SAME, PIO_SAME, k0,
                          y0, s);
        if (st) return st;
    }
    // top passes: eigenvalues (+ log-det partial sums), then the filtered solves
    const bool single = pl.P == 1;
    aK.src = single ? k1 : (const void *)wsK;
    aK.src_row = single ? n : N;
    aY.src = single ? y : (const void *)wsY;
    aY.dst = single ? c : wsY;
    aY.src_row = aY.dst_row = single ? n : N;
    aK.g = aY.g = top;
    aK.global_tw = aY.global_tw = !single;
    aY.scale = 1.0 / (double)N;
    if (one_top) {
        st = launch_fit_top(aK, aY, lam, logdet ? partial : nullptr, s);
        if (st) return st;
    } else {
        st = launch_real_top(LDK_F64, PM_FWD, aK, lam, s, false, logdet ? partial : nullptr);
        if (st) return st;
        if (!single && nrhs >= 2) {
            // the filter once per eigenvalue row, as ldk_solve forms it
            void *coef = w8 + align256((size_t)B * cb_count * sizeof(double)) +
                         align256((size_t)R * N * 16 + (size_t)R * nrhs * N * 16);
            st = launch_filter_coef(LDK_F64, PM_SOLVE, mp, R, lam, sigma2, aY.scale, coef, s);
            if (st) return st;
            aY.coef = coef;
        }
        st = launch_real_top(LDK_F64, PM_SOLVE, aY, nullptr, s);
        if (st) return st;
    }
    // inverse passes of the right-hand sides; the first one also finishes
    // the log-det when it has a full wave per tile
    bool ld_done = false;
    for (int p = pl.P - 2; p >= 0; --p) {
        PassArgs b = aY;
        b.lam = nullptr;
        b.src = wsY;
        b.src_row = N;
        b.dst = p == 0 ? c : wsY;
        b.dst_row = p == 0 ? n : N;
        b.g = pl.pass[p];
        b.global_tw = p > 0;
        b.scale = 1.0;
        const int64_t tiles = b.rows << (mp - b.g.a - b.g.logW);
        if (logdet && !ld_done && (b.g.a + b.g.logW - b.g.logE) >= 6 && tiles >= R) {
            b.ld_part = partial;
            b.ld_out = logdet;
            b.ld_rows = R;
            b.ld_count = cb_count;
            ld_done = true;
        }
        st = launch_pass(LDK_LATTICE, LDK_F64, PM_INV, PIO_SAME, p == 0 ? PIO_PACKED : PIO_SAME, b, s);
        if (st) return st;
    }
    if (logdet && !ld_done) {
        hipLaunchKernelGGL(k_logdet_final, dim3(R), dim3(LOGDET_THREADS), 0, s,
                           (const double *)partial, cb_count, logdet);
        LDK_LAUNCH_CHECK();
    }
    return LDK_OK;
}

int ldk_update_double(int kind, int B, int m, int dtype, const void *yt_old, const void *y_new,
                      void *yt_full, void *ws, ldk_stream stream)
{
    (void)ws;
    if (!valid_kind(kind) || !valid_dtype(dtype) || !valid_m(m) || m + 1 > TW_MAX_LOG || B < 0 ||
        !yt_old || !y_new || !yt_full)
        return LDK_EINVAL;
    if (B == 0) return LDK_OK;
    int st = ensure_init();
    if (st) return st;
    hipStream_t s = as_stream(stream);
    const int64_t n = (int64_t)1 << m;
    const bool lat = kind == LDK_LATTICE;
    const size_t eb = esize(dtype) * (lat ? 2 : 1);
    // U = unnormalised FT_m(y_new), written into the second half of each output row
    void *u = static_cast<unsigned char *>(yt_full) + n * eb;
    if (m == 0) {
        // FT_0 is the identity: combine directly with y_new
        if (lat) {
            if (dtype == LDK_F64)
                hipLaunchKernelGGL((k_update_combine<double, true, true>), dim3(blocks_for(B, 256)),
                                   dim3(256), 0, s, yt_old, yt_full, y_new, (int64_t)1, (int64_t)B, 0, 1.0);
            else
                hipLaunchKernelGGL((k_update_combine<float, true, true>), dim3(blocks_for(B, 256)),
                                   dim3(256), 0, s, yt_old, yt_full, y_new, (int64_t)1, (int64_t)B, 0, 1.0);
        } else {
            if (dtype == LDK_F64)
                hipLaunchKernelGGL((k_update_combine<double, false, true>), dim3(blocks_for(B, 256)),
                                   dim3(256), 0, s, yt_old, yt_full, y_new, (int64_t)1, (int64_t)B, 0, 1.0);
            else
                hipLaunchKernelGGL((k_update_combine<float, false, true>), dim3(blocks_for(B, 256)),
                                   dim3(256), 0, s, yt_old, yt_full, y_new, (int64_t)1, (int64_t)B, 0, 1.0);
        }
        LDK_LAUNCH_CHECK();
        return LDK_OK;
    }
    // the transform of the new half; intermediates of a multi-pass plan live
    // in the output rows' second halves (stride 2n), and the last pass meets
    // the old half's transform in its store (PIO_COMBINE) and writes both
    // halves of every output row
    const Plan pl = make_plan(m, log_tile_for(kind, dtype));
    for (int p = 0; p < pl.P; ++p) {
        const bool first = p == 0, last = p == pl.P - 1;
        PassArgs a{};
        a.src = first ? y_new : (const void *)u;
        a.src_row = first ? n : 2 * n;
        a.dst = last ? yt_full : u;
        a.dst_row = 2 * n;
        a.rows = B;
        a.m = m;
        a.g = pl.pass[p];
        a.nrhs = 1;
        a.global_tw = p > 0;
        a.scale = last ? 1.0 / std::sqrt((double)n) : 1.0;
        a.old = yt_old;
        st = launch_pass(kind, dtype, PM_FWD, first && lat ? PIO_REAL : PIO_SAME,
                         last ? PIO_COMBINE : PIO_SAME, a, s);
        if (st) return st;
    }
    return LDK_OK;
}

int ldk_eig_update_double(int kind, int R, int m, int dtype, const double *lam_old,
                          const void *k1_new, double *lam_full, void *ws, ldk_stream stream)
{
    if (!valid_kind(kind) || !valid_dtype(dtype) || !valid_m(m) || m + 1 > TW_MAX_LOG || R < 0 ||
        !lam_old || !k1_new || !lam_full)
        return LDK_EINVAL;
    if (R == 0) return LDK_OK;
    const bool lat = kind == LDK_LATTICE;
    if (ws_bytes(LDK_OP_EIG_UPDATE_DOUBLE, kind, R, m, dtype) && !ws) return LDK_EINVAL;
    int st = ensure_init();
    if (st) return st;
    hipStream_t s = as_stream(stream);
    const int64_t n = (int64_t)1 << m;
    const int64_t work = (int64_t)R * n;
    const dim3 grid(blocks_for(work, 256)), block(256);
    if (m == 0) {
        // FT_0 is the identity and w_0 = 1: the new half is k1_new itself
        if (dtype == LDK_F64)
            hipLaunchKernelGGL((k_eig_update_combine<double>), grid, block, 0, s, lam_old,
                               lam_full, k1_new, (int64_t)1, (int64_t)R, 0);
        else
            hipLaunchKernelGGL((k_eig_update_combine<float>), grid, block, 0, s, lam_old,
                               lam_full, k1_new, (int64_t)1, (int64_t)R, 0);
        LDK_LAUNCH_CHECK();
        return LDK_OK;
    }
    // FP64 transform of the new half (k1 widened when FP32); intermediates of
    // a multi-pass plan in the workspace (lattice, complex) or in the output
    // rows' second halves (net), and the last pass stores through the
    // doubling step lambda_m +- Re(w_k u_k) into both halves (PIO_COMBINE)
    const Plan pl = make_plan(m, log_tile_for(kind, LDK_F64));
    for (int p = 0; p < pl.P; ++p) {
        const bool first = p == 0, last = p == pl.P - 1;
        PassArgs a{};
        a.src = first ? k1_new : (lat ? (const void *)ws : (const void *)(lam_full + n));
        a.src_row = first ? n : (lat ? n : 2 * n);
        a.dst = last ? (void *)lam_full : (lat ? ws : (void *)(lam_full + n));
        a.dst_row = last ? 2 * n : (lat ? n : 2 * n);
        a.rows = R;
        a.m = m;
        a.g = pl.pass[p];
        a.nrhs = 1;
        a.global_tw = p > 0;
        a.scale = 1.0;
        a.old = lam_old;
        a.combine_real = 1;
        st = launch_pass(kind, LDK_F64, PM_FWD, first && lat ? PIO_REAL : PIO_SAME,
                         last ? PIO_COMBINE : PIO_SAME, a, s, first && dtype == LDK_F32);
        if (st) return st;
    }
    return LDK_OK;
}

}  // extern "C"
