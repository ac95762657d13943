// Pass kernels of the FWHT / FFTBR / IFFTBR engine (see transform.hpp).
#include <cstdio>
#include <mutex>
#include <type_traits>
#include <vector>

#include "passkit.hpp"

namespace ldk {

// Dynamic LDS of the pass kernels (tile + padding).
extern __shared__ unsigned char g_pass_lds[];

using namespace kit;

namespace {

// One pass over a tile: rows = 2^a along the axis, W = 2^logW columns.
// CA, CLW >= 0: a and logW fixed at compile time (they must equal a.g.a and
// a.g.logW); the index maps, group loops and twiddle choices then fold to
// constants.  REGLAM (real rows only): the E values a thread stores at tile
// positions t + Tn i go to regl[i] too (PM_FWD), or the filter takes its
// eigenvalues from regl[i] instead of a.lam (PM_SOLVE / PM_MATVEC) -- the
// same elements, when both passes have the same geometry.
template <typename T, int LOGE, int MODE, int LD, int ST, bool SRC_F32, int CA = -1, int CLW = -1,
          bool REGLAM = false>
__device__ __forceinline__ void pass_body(const PassArgs &a, int64_t bid, double *regl = nullptr)
{
    static_assert(!REGLAM || std::is_floating_point<T>::value, "eigenvalues in registers: real rows");
    using R = typename real_of<T>::type;
    constexpr int E = 1 << LOGE;
    constexpr bool FFT = !std::is_floating_point<T>::value;
    T *lds = reinterpret_cast<T *>(g_pass_lds);

    const int A = CA >= 0 ? CA : a.g.a, logW = CLW >= 0 ? CLW : a.g.logW, b0 = a.g.b0;
    const int S = 1 << (A + logW);
    const int Tn = S >> LOGE;  // threads
    const int t = threadIdx.x;

    // block -> (row, outer, column block)
    const int64_t tile = bid;
    const int64_t cb_count = (int64_t)1 << (b0 - logW);
    const int64_t outer_count = (int64_t)1 << (a.m - b0 - A);
    const int64_t cb = bid % cb_count;
    bid /= cb_count;
    const int64_t outer = bid % outer_count;
    const int64_t row = bid / outer_count;
    const int64_t base = outer * ((int64_t)1 << (b0 + A)) + (cb << logW);
    const int64_t rstride = (int64_t)1 << b0;

    // global index (within a row) of tile element q
    auto gidx = [&](int q) -> int64_t {
        return base + (int64_t)(q >> logW) * rstride + (q & ((1 << logW) - 1));
    };

    // groups over the axis bits: lowest group has rem bits, the rest LOGE bits
    const int G = (A + LOGE - 1) / LOGE;
    const int rem = A - LOGE * (G - 1);
    const int top_s = A - LOGE;  // axis bit where the top group starts

    T v[E];
    // ---- load (coalesced: q = t + Tn * i; the registers hold the top group)
#pragma unroll
    for (int i = 0; i < E; ++i)
        v[i] = load_elem<T, LD, SRC_F32>(a.src, row * a.src_row + gidx(t + Tn * i), a.half);
    // twiddle table reads issued right behind the data loads (one latency)
    GroupBases<T> gb{};
    PassTw<R> ptw{};
    if constexpr (FFT) {
        group_bases<R, LOGE>(gb, t, A, logW, Tn);
        if (a.global_tw)
            ptw = pass_tw_fetch<R, LOGE>(t, (uint64_t)((cb << logW) + (t & ((1 << logW) - 1))),
                                         logW, A, b0);
    }

    if constexpr (MODE != PM_INV) {
        if constexpr (FFT) {
            if (a.global_tw) pass_tw_apply<T, E, LOGE, false>(v, ptw);
        }
        if (G > 1) {
            lds_write(v, lds, t, LOGE, logW + top_s, Tn);
            __syncthreads();
            int s = 0;
            for (int gidx_ = 0; gidx_ < G - 1; ++gidx_) {
                const int gs = gidx_ == 0 ? rem : LOGE;
                lds_read(v, lds, t, gs, logW + s, Tn);
                if (gidx_ > 0) {
                    const auto gbase = pick_base(gidx_, gb.b1, gb.b2, gb.b3);
                    apply_group_twiddle<T, E, LOGE, false>(v, gbase);
                }
                reg_fwd<T, E, LOGE, false>(v, gs);
                lds_write(v, lds, t, gs, logW + s, Tn);
                __syncthreads();
                s += gs;
            }
            lds_read(v, lds, t, LOGE, logW + top_s, Tn);
            apply_group_twiddle<T, E, LOGE, false>(v, pick_base(G - 1, gb.b1, gb.b2, gb.b3));
        }
        reg_fwd<T, E, LOGE, false>(v, LOGE);
    }

    if constexpr (MODE == PM_SOLVE || MODE == PM_MATVEC) {
        const double *lam = a.lam + (row / a.nrhs) * ((int64_t)1 << a.m);
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const double l = REGLAM ? regl[i] : lam[gidx(t + Tn * i)];
            const double f = MODE == PM_SOLVE ? a.scale / (l + a.sigma2) : a.scale * l;
            v[i] = scl(v[i], (R)f);
        }
    }

    if constexpr (MODE != PM_FWD) {
        reg_inv<T, E, LOGE>(v, LOGE);
        if (G > 1) {
            apply_group_twiddle<T, E, LOGE, true>(v, pick_base(G - 1, gb.b1, gb.b2, gb.b3));
            if constexpr (MODE != PM_INV) __syncthreads();  // LDS reuse after the forward half
            lds_write(v, lds, t, LOGE, logW + top_s, Tn);
            __syncthreads();
            int s = top_s;
            for (int gi = G - 2; gi >= 0; --gi) {
                const int gs = gi == 0 ? rem : LOGE;
                s -= gs;
                lds_read(v, lds, t, gs, logW + s, Tn);
                reg_inv<T, E, LOGE>(v, gs);
                if (gi > 0) {
                    const auto gbase = pick_base(gi, gb.b1, gb.b2, gb.b3);
                    apply_group_twiddle<T, E, LOGE, true>(v, gbase);
                }
                lds_write(v, lds, t, gs, logW + s, Tn);
                __syncthreads();
            }
            lds_read(v, lds, t, LOGE, logW + top_s, Tn);
        }
        if constexpr (FFT) {
            if (a.global_tw) pass_tw_apply<T, E, LOGE, true>(v, ptw);
        }
    }

    // ---- store
    const R sc = (MODE == PM_FWD || MODE == PM_INV) ? (R)a.scale : (R)1;
#pragma unroll
    for (int i = 0; i < E; ++i) {
        T o = v[i];
        if (MODE == PM_FWD || MODE == PM_INV) o = scl(o, sc);
        if constexpr (REGLAM && MODE == PM_FWD) regl[i] = (double)o;
        if constexpr (ST == IO_COMBINE) {
            // the doubling update: the new half's transform o meets the old
            // half's at k (Sec. 5.4, eq. ft_next_parts)
            const int64_t n = (int64_t)1 << a.m;
            const int64_t k = gidx(t + Tn * i);
            const R h = (R)0.70710678118654752440;
            if constexpr (FFT) o = cmul(o, tw_any<R>((uint64_t)k, a.m + 1));
            if (a.combine_real) {
                // eigenvalue update: real FP64 rows, lambda_m +- Re(w)
                double part;
                if constexpr (FFT) part = (double)o.re;
                else part = (double)o;
                const double od = static_cast<const double *>(a.old)[row * n + k];
                double *full = static_cast<double *>(a.dst) + row * a.dst_row;
                full[k] = od + part;
                full[n + k] = od - part;
            } else {
                const T od = static_cast<const T *>(a.old)[row * n + k];
                T *full = static_cast<T *>(a.dst) + row * a.dst_row;
                full[k] = scl(add(od, o), h);
                full[n + k] = scl(sub(od, o), h);
            }
        } else {
            store_elem<T, ST>(a.dst, row * a.dst_row + gidx(t + Tn * i), o, a.half);
        }
    }

    if constexpr (MODE == PM_INV) {
        // the log-det of the fused fit: the first wave of tile r adds row r's
        // partial sums (written by the top pass that ran before this one)
        if (a.ld_out && tile < a.ld_rows && t < 64) {
            const double *p = a.ld_part + tile * a.ld_count;
            double acc = 0.0;
            for (int64_t c = t; c < a.ld_count; c += 64) acc += p[c];
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
            if (t == 0) a.ld_out[tile] = acc;
        }
    }
}

template <typename T, int LOGE, int MODE, int LD, int ST, bool SRC_F32, int CA = -1, int CLW = -1>
__global__ __launch_bounds__(CA >= 0 ? (1 << (CA + CLW - LOGE)) : 512) void k_pass(PassArgs a)
{
    pass_body<T, LOGE, MODE, LD, ST, SRC_F32, CA, CLW>(a, xcd_tile(blockIdx.x, gridDim.x));
}

// Two jobs in one grid: the first nb0 tiles (after the XCD order) are job 0.
template <typename T, int LOGE, int MODE, int LD, int ST, bool SRC_F32, int CA = -1, int CLW = -1>
__global__ __launch_bounds__(CA >= 0 ? (1 << (CA + CLW - LOGE)) : 512) void k_pass2(
    PassArgs a0, PassArgs a1, int64_t nb0)
{
    const int64_t b = xcd_tile(blockIdx.x, gridDim.x);
    if (b < nb0) pass_body<T, LOGE, MODE, LD, ST, SRC_F32, CA, CLW>(a0, b);
    else pass_body<T, LOGE, MODE, LD, ST, SRC_F32, CA, CLW>(a1, b - nb0);
}

// The passes of the plans at n = 2^20 get kernels with their geometry
// fixed at compile time: the lattice row passes (the packed half-length row
// in one contiguous tile: 11 axis bits in FP64, also the row pass of every
// FP64 lattice plan from n = 2^13; 12 in FP32), and the digital-net passes
// (FP64 and FP32: 12 row bits, and the top pass with the filter over 8 bits
// in 16-column tiles).
template <typename T>
constexpr int row_a()
{
    return std::is_same<T, cplx<double>>::value ? 11 : 12;
}
template <typename T, int LOGE, bool SRC_F32>
constexpr bool row_specialised()
{
    // float sources: the FP64 eigenvalue transform of an FP32 column
    return !std::is_floating_point<T>::value && LOGE == 3 &&
           (!SRC_F32 || std::is_same<T, cplx<double>>::value);
}
constexpr int NET_ROW_A = 12, NET_TOP_A = 8, NET_TOP_LOGW = 4;
template <typename T, int LOGE, bool SRC_F32>
constexpr bool net_specialised()
{
    return std::is_floating_point<T>::value && LOGE == 3 && !SRC_F32;
}

// The fit of a net whose transform is one pass (the whole row in one tile),
// FP64: workgroup r runs replication r's eigenvalue tile, then its
// right-hand sides' solve tiles, with the pass bodies and arguments of
// ldk_eig and ldk_solve (so lambda and c are theirs bit for bit; the solve
// takes the eigenvalues this workgroup has just computed from registers),
// then the log-det of the row: per-thread products of the values (LogProd,
// each thread's values in the order of ldk_logdet's partial loop) and a
// fixed-order tree.
template <int LOGE>
__global__ __launch_bounds__(512) void k_fit_net_one(PassArgs aE, PassArgs aS, double *logdet)
{
    const int64_t r = blockIdx.x;
    // thread t keeps the eigenvalues at positions t + T i of the row (the
    // tile is the whole row, and the solve tiles have the same geometry):
    // the solves and the log-det take them from registers, not back from
    // memory
    constexpr int E = 1 << LOGE;
    double lam_t[E];
    pass_body<double, LOGE, PM_FWD, IO_SAME, IO_SAME, false, -1, -1, true>(aE, r, lam_t);
    __syncthreads();  // the LDS is free for the solve tiles
    for (int q = 0; q < aS.nrhs; ++q) {
        pass_body<double, LOGE, PM_SOLVE, IO_SAME, IO_SAME, false, -1, -1, true>(
            aS, r * aS.nrhs + q, lam_t);
        __syncthreads();  // the LDS is free for the next tile
    }
    if (!logdet) return;
    const int t = threadIdx.x, T = blockDim.x;
    LogProd acc;
#pragma unroll
    for (int i = 0; i < E; ++i) acc.add(lam_t[i] + aS.sigma2);
    double *red = reinterpret_cast<double *>(g_pass_lds);
    red[t] = acc.value();
    __syncthreads();
    for (int w = T / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) logdet[r] = red[0];
}

template <typename T, int LOGE, int MODE, bool SRC_F32>
int launch_t(int ld, int st, const PassArgs &a, hipStream_t s)
{
    const int S = 1 << (a.g.a + a.g.logW);
    const int threads = S >> LOGE;
    const int64_t blocks = a.rows * ((int64_t)1 << (a.m - a.g.a - a.g.logW));
    if (blocks > 0x7fffffff || threads > 512 || threads < 1) return LDK_ENOTSUP;
    if ((a.g.a + LOGE - 1) / LOGE > MAX_GROUPS) return LDK_ENOTSUP;  // group twiddle bases
    const size_t lds = (size_t)(S + (S >> LDS_PAD_SHIFT)) * sizeof(T);
    const dim3 grid((unsigned)blocks), block(threads);
    if constexpr (net_specialised<T, LOGE, SRC_F32>() && (MODE == PM_FWD || MODE == PM_INV)) {
        if (ld == IO_SAME && st == IO_SAME && a.g.a == NET_ROW_A && a.g.logW == 0) {
            hipLaunchKernelGGL((k_pass<T, LOGE, MODE, IO_SAME, IO_SAME, SRC_F32, NET_ROW_A, 0>), grid,
                               block, lds, s, a);
            LDK_LAUNCH_CHECK();
            return LDK_OK;
        }
    }
    if constexpr (net_specialised<T, LOGE, SRC_F32>() && MODE == PM_SOLVE) {
        if (ld == IO_SAME && st == IO_SAME && a.g.a == NET_TOP_A && a.g.logW == NET_TOP_LOGW) {
            hipLaunchKernelGGL(
                (k_pass<T, LOGE, MODE, IO_SAME, IO_SAME, SRC_F32, NET_TOP_A, NET_TOP_LOGW>), grid,
                block, lds, s, a);
            LDK_LAUNCH_CHECK();
            return LDK_OK;
        }
    }
    if constexpr (row_specialised<T, LOGE, SRC_F32>() && (MODE == PM_FWD || MODE == PM_INV)) {
        constexpr int RA = row_a<T>();
        if (a.g.a == RA && a.g.logW == 0) {
            constexpr int LDs = MODE == PM_FWD ? IO_PACKED : IO_SAME;
            constexpr int STs = MODE == PM_FWD ? IO_SAME : IO_PACKED;
            if (ld == LDs && st == STs) {
                hipLaunchKernelGGL((k_pass<T, LOGE, MODE, LDs, STs, SRC_F32, RA, 0>), grid, block,
                                   lds, s, a);
                LDK_LAUNCH_CHECK();
                return LDK_OK;
            }
        }
    }
#define LDK_PASS(LD_, ST_) hipLaunchKernelGGL((k_pass<T, LOGE, MODE, LD_, ST_, SRC_F32>), grid, block, lds, s, a)
    if constexpr (std::is_floating_point<T>::value) {
        if (ld != IO_SAME) return LDK_ENOTSUP;
        if (st == IO_SAME) LDK_PASS(IO_SAME, IO_SAME);
        else if (MODE == PM_FWD && st == IO_POWER) LDK_PASS(IO_SAME, IO_POWER);
        else if (MODE == PM_FWD && st == IO_COMBINE) LDK_PASS(IO_SAME, IO_COMBINE);
        else return LDK_ENOTSUP;
    } else if constexpr (MODE == PM_FWD) {
        if (st == IO_COMBINE) {
            if (ld == IO_SAME) LDK_PASS(IO_SAME, IO_COMBINE);
            else if (ld == IO_REAL) LDK_PASS(IO_REAL, IO_COMBINE);
            else return LDK_ENOTSUP;
            LDK_LAUNCH_CHECK();
            return LDK_OK;
        }
        if (st == IO_PACKED || st == IO_POWER) return LDK_ENOTSUP;
        if (ld == IO_SAME && st == IO_SAME) LDK_PASS(IO_SAME, IO_SAME);
        else if (ld == IO_SAME) LDK_PASS(IO_SAME, IO_REAL);
        else if (ld == IO_REAL && st == IO_SAME) LDK_PASS(IO_REAL, IO_SAME);
        else if (ld == IO_REAL) LDK_PASS(IO_REAL, IO_REAL);
        else if (st == IO_SAME) LDK_PASS(IO_PACKED, IO_SAME);
        else return LDK_ENOTSUP;
    } else if constexpr (MODE == PM_INV) {
        if (ld != IO_SAME || st == IO_POWER || st == IO_COMBINE) return LDK_ENOTSUP;
        if (st == IO_SAME) LDK_PASS(IO_SAME, IO_SAME);
        else if (st == IO_REAL) LDK_PASS(IO_SAME, IO_REAL);
        else LDK_PASS(IO_SAME, IO_PACKED);
    } else {
        if (ld == IO_SAME && st == IO_SAME) LDK_PASS(IO_SAME, IO_SAME);
        else if (ld == IO_REAL && st == IO_REAL) LDK_PASS(IO_REAL, IO_REAL);
        else return LDK_ENOTSUP;
    }
#undef LDK_PASS
    LDK_LAUNCH_CHECK();
    return LDK_OK;
}

template <typename T, int MODE, bool SRC_F32>
int launch_e(int ld, int st, const PassArgs &a, hipStream_t s)
{
    switch (a.g.logE) {
    case 1: return launch_t<T, 1, MODE, SRC_F32>(ld, st, a, s);
    case 2: return launch_t<T, 2, MODE, SRC_F32>(ld, st, a, s);
    case 3: return launch_t<T, 3, MODE, SRC_F32>(ld, st, a, s);
    default: return LDK_ENOTSUP;
    }
}

template <typename T>
int launch_m(int mode, int ld, int st, const PassArgs &a, hipStream_t s)
{
    switch (mode) {
    case PM_FWD: return launch_e<T, PM_FWD, false>(ld, st, a, s);
    case PM_INV: return launch_e<T, PM_INV, false>(ld, st, a, s);
    case PM_SOLVE: return launch_e<T, PM_SOLVE, false>(ld, st, a, s);
    case PM_MATVEC: return launch_e<T, PM_MATVEC, false>(ld, st, a, s);
    default: return LDK_EINVAL;
    }
}

}  // namespace

Plan make_plan(int m, int log_tile, int loge_max)
{
    Plan p{};
    p.m = m;
    if (m == 0) return p;
    constexpr int LOG_THREADS = 9;  // at most 512 threads per workgroup
    const int LOGE_MAX = loge_max < 1 ? 1 : (loge_max > 3 ? 3 : loge_max);  // elements per thread
    // row pass: the low a0 bits; column passes: the rest, split evenly into
    // chunks of at most 8 bits (at least 4 where possible)
    int a0 = m < log_tile ? m : log_tile;
    int r = m - a0;
    if (r > 0 && r < 4) {
        a0 = m - 4;
        r = 4;
    }
    int logE0 = a0 < LOGE_MAX ? a0 : LOGE_MAX;
    if (a0 - logE0 > LOG_THREADS) logE0 = a0 - LOG_THREADS;
    p.pass[0] = PassGeom{0, a0, 0, logE0};
    p.P = 1;
    const int C = (r + 7) / 8;
    int b0 = a0;
    for (int c = 0; c < C; ++c) {
        const int a = r / C + (c < r % C ? 1 : 0);
        const int logE = a < LOGE_MAX ? a : LOGE_MAX;
        // tile 2^a rows x 2^logW columns: at most 2^log_tile elements,
        // at most 2^LOG_THREADS threads (2^(a + logW - logE)), at most 2^b0 columns
        int logW = log_tile - a;
        if (logW > LOG_THREADS + logE - a) logW = LOG_THREADS + logE - a;
        if (logW > b0) logW = b0;
        p.pass[p.P++] = PassGeom{b0, a, logW, logE};
        b0 += a;
    }
    return p;
}

int log_tile_for(int kind, int dtype) { return (kind == LDK_LATTICE && dtype == LDK_F64) ? 11 : 12; }

bool plan_ok(const Plan &pl)
{
    for (int p = 0; p < pl.P; ++p) {
        const PassGeom &g = pl.pass[p];
        const int lt = g.a + g.logW - g.logE;  // log2 threads
        if (g.logE < 1 || g.logE > 3 || lt < 0 || lt > 9) return false;
        if ((g.a + g.logE - 1) / g.logE > MAX_GROUPS) return false;
        if (g.logW > g.b0) return false;
    }
    return true;
}

namespace {
struct TuneEntry {
    int kind, dtype, m, rows_log2, log_tile, loge_max, engine;
};
std::mutex g_tune_mutex;
std::vector<TuneEntry> g_tune;

int floor_log2(int64_t v)
{
    int r = 0;
    while (v > 1) {
        v >>= 1;
        ++r;
    }
    return r;
}
}  // namespace

PlanParams plan_params(int kind, int dtype, int m, int64_t rows)
{
    PlanParams p{log_tile_for(kind, dtype), 3, ENGINE_BUTTERFLY};
    const int rl = floor_log2(rows < 1 ? 1 : rows);
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    int best = -1;
    for (const TuneEntry &e : g_tune)
        if (e.kind == kind && e.dtype == dtype && e.m == m && e.rows_log2 <= rl && e.rows_log2 > best) {
            best = e.rows_log2;
            p = PlanParams{e.log_tile, e.loge_max, e.engine};
        }
    return p;
}

int plan_candidates(int kind, int dtype, int m, PlanParams *out, int cap)
{
    int c = 0;
    if (c < cap) out[c++] = PlanParams{log_tile_for(kind, dtype), 3, ENGINE_BUTTERFLY};
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    for (const TuneEntry &e : g_tune)
        if (e.kind == kind && e.dtype == dtype && e.m == m && c < cap)
            out[c++] = PlanParams{e.log_tile, e.loge_max, e.engine};
    return c;
}

// Replaces the table (empty for path == nullptr); a file that does not parse
// or names a plan the pass kernels cannot run leaves the table unchanged.
int load_tune_table(const char *path)
{
    std::vector<TuneEntry> t;
    if (path) {
        FILE *f = std::fopen(path, "r");
        if (!f) return LDK_EINVAL;
        char line[256];
        int bad = 0;
        while (std::fgets(line, sizeof line, f)) {
            const char *q = line;
            while (*q == ' ' || *q == '\t') ++q;
            if (*q == '#' || *q == '\n' || *q == 0) continue;
            TuneEntry e{};
            // six fields, and an optional seventh: the engine (0 when absent)
            const int got = std::sscanf(q, "%d %d %d %d %d %d %d", &e.kind, &e.dtype, &e.m,
                                        &e.rows_log2, &e.log_tile, &e.loge_max, &e.engine);
            if (got != 6 && got != 7) {
                bad = 1;
                break;
            }
            if (got == 6) e.engine = ENGINE_BUTTERFLY;
            // the matrix-core passes: FP32 net rows of at least 2^12
            if (e.engine != ENGINE_BUTTERFLY &&
                (e.engine != ENGINE_SPLIT16 || e.kind != LDK_DNET_B2 || e.dtype != LDK_F32 || e.m < 12)) {
                bad = 1;
                break;
            }
            const bool ok_key = (e.kind == LDK_LATTICE || e.kind == LDK_DNET_B2) &&
                                (e.dtype == LDK_F64 || e.dtype == LDK_F32) && e.m >= 1 &&
                                e.m <= LDK_MAX_M && e.rows_log2 >= 0 && e.rows_log2 < 63;
            // LDS: the largest tile is 2^12 complex FP64 (68 KiB with padding)
            if (!ok_key || e.log_tile < 6 || e.log_tile > 12 || e.loge_max < 1 || e.loge_max > 3) {
                bad = 1;
                break;
            }
            // the plan it selects (real lattice rows run as complex rows of n/2)
            const int mp = (e.kind == LDK_LATTICE && e.m >= 2) ? e.m - 1 : e.m;
            const Plan pl = make_plan(mp, e.log_tile, e.loge_max);
            // the real-data top pass pairs mirror columns: at least 2 per tile
            const bool mirror_ok = !(e.kind == LDK_LATTICE && e.m >= 2 && pl.P > 1 &&
                                     pl.pass[pl.P - 1].logW < 1);
            if (!plan_ok(pl) || !mirror_ok) {
                bad = 1;
                break;
            }
            t.push_back(e);
        }
        std::fclose(f);
        if (bad) return LDK_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune.swap(t);
    return LDK_OK;
}

int launch_pass(int kind, int dtype, int mode, int ld, int st, const PassArgs &a, hipStream_t s,
                bool src_f32)
{
    if (src_f32) {
        // FP64 forward transform of float data (eigenvalues from an FP32 column)
        if (dtype != LDK_F64 || mode != PM_FWD) return LDK_EINVAL;
        if (kind == LDK_DNET_B2) return launch_e<double, PM_FWD, true>(IO_SAME, st, a, s);
        return launch_e<cplx<double>, PM_FWD, true>(ld, st, a, s);
    }
    if (kind == LDK_DNET_B2) {
        if (dtype == LDK_F64) return launch_m<double>(mode, ld, st, a, s);
        return launch_m<float>(mode, ld, st, a, s);
    }
    if (dtype == LDK_F64) return launch_m<cplx<double>>(mode, ld, st, a, s);
    return launch_m<cplx<float>>(mode, ld, st, a, s);
}

}  // namespace ldk

namespace ldk {

int launch_fit_net_one(const PassArgs &aE, const PassArgs &aS, double *logdet, hipStream_t s)
{
    const PassGeom &g = aE.g;
    const int S = 1 << (g.a + g.logW);
    if (g.a + g.logW != aE.m || g.b0 != 0 || aS.g.a != g.a || aS.g.logW != g.logW || aS.g.logE != g.logE ||
        aS.g.b0 != 0 || aS.m != aE.m)
        return LDK_ENOTSUP;  // not one pass, or the two plans differ
    const int threads = S >> g.logE;
    if (threads > 512 || threads < 1 || (threads & (threads - 1)) || aE.rows > 0x7fffffff)
        return LDK_ENOTSUP;
    const size_t lds = (size_t)(S + (S >> LDS_PAD_SHIFT)) * sizeof(double);
    const dim3 grid((unsigned)aE.rows), block(threads);
    switch (g.logE) {
    case 1:
        if ((g.a + 1 - 1) / 1 > MAX_GROUPS) return LDK_ENOTSUP;
        hipLaunchKernelGGL(k_fit_net_one<1>, grid, block, lds, s, aE, aS, logdet);
        break;
    case 2:
        if ((g.a + 2 - 1) / 2 > MAX_GROUPS) return LDK_ENOTSUP;
        hipLaunchKernelGGL(k_fit_net_one<2>, grid, block, lds, s, aE, aS, logdet);
        break;
    case 3:
        if ((g.a + 3 - 1) / 3 > MAX_GROUPS) return LDK_ENOTSUP;
        hipLaunchKernelGGL(k_fit_net_one<3>, grid, block, lds, s, aE, aS, logdet);
        break;
    default: return LDK_ENOTSUP;
    }
    LDK_LAUNCH_CHECK();
    return LDK_OK;
}

namespace {
template <typename T, int LOGE, int LD>
int launch_fwd2(const PassArgs &a0, const PassArgs &a1, hipStream_t s)
{
    const int S = 1 << (a0.g.a + a0.g.logW);
    const int threads = S >> LOGE;
    const int64_t per_row = (int64_t)1 << (a0.m - a0.g.a - a0.g.logW);
    const int64_t nb0 = a0.rows * per_row, nb1 = a1.rows * per_row;
    if (nb0 + nb1 > 0x7fffffff || threads > 512 || threads < 1) return LDK_ENOTSUP;
    if ((a0.g.a + LOGE - 1) / LOGE > MAX_GROUPS) return LDK_ENOTSUP;
    const size_t lds = (size_t)(S + (S >> LDS_PAD_SHIFT)) * sizeof(T);
    if constexpr (row_specialised<T, LOGE, false>() && LD == IO_PACKED) {
        constexpr int RA = row_a<T>();
        if (a0.g.a == RA && a0.g.logW == 0) {
            hipLaunchKernelGGL((k_pass2<T, LOGE, PM_FWD, LD, IO_SAME, false, RA, 0>),
                               dim3((unsigned)(nb0 + nb1)), dim3(threads), lds, s, a0, a1, nb0);
            LDK_LAUNCH_CHECK();
            return LDK_OK;
        }
    }
    hipLaunchKernelGGL((k_pass2<T, LOGE, PM_FWD, LD, IO_SAME, false>), dim3((unsigned)(nb0 + nb1)),
                       dim3(threads), lds, s, a0, a1, nb0);
    LDK_LAUNCH_CHECK();
    return LDK_OK;
}
template <typename T, int LD>
int launch_fwd2_e(const PassArgs &a0, const PassArgs &a1, hipStream_t s)
{
    switch (a0.g.logE) {
    case 1: return launch_fwd2<T, 1, LD>(a0, a1, s);
    case 2: return launch_fwd2<T, 2, LD>(a0, a1, s);
    case 3: return launch_fwd2<T, 3, LD>(a0, a1, s);
    default: return LDK_ENOTSUP;
    }
}
}  // namespace

int launch_pass2(int kind, int dtype, int mode, int ld, int st, const PassArgs &a0,
                 const PassArgs &a1, hipStream_t s)
{
    // forward FP64 passes only (the fused fit's column and right-hand sides)
    if (mode != PM_FWD || dtype != LDK_F64 || st != IO_SAME) return LDK_ENOTSUP;
    if (a0.m != a1.m || a0.g.b0 != a1.g.b0 || a0.g.a != a1.g.a || a0.g.logW != a1.g.logW ||
        a0.g.logE != a1.g.logE)
        return LDK_EINVAL;
    if (kind == LDK_LATTICE) {
        if (ld == IO_PACKED) return launch_fwd2_e<cplx<double>, IO_PACKED>(a0, a1, s);
        if (ld == IO_SAME) return launch_fwd2_e<cplx<double>, IO_SAME>(a0, a1, s);
        return LDK_ENOTSUP;
    }
    if (ld != IO_SAME) return LDK_ENOTSUP;
    return launch_fwd2_e<double, IO_SAME>(a0, a1, s);
}

}  // namespace ldk

extern "C" int ldk_init_tuned(const char *path)
{
    const int st = ldk::ensure_init();
    if (st) return st;
    return ldk::load_tune_table(path);
}

extern "C" int ldk_plan_info(int kind, int dtype, int m, int64_t rows, int *log_tile,
                             int *radix, int *passes, int *engine)
{
    if ((kind != LDK_LATTICE && kind != LDK_DNET_B2) || (dtype != LDK_F64 && dtype != LDK_F32) ||
        m < 0 || m > LDK_MAX_M || rows < 1)
        return LDK_EINVAL;
    const ldk::PlanParams p = ldk::plan_params(kind, dtype, m, rows);
    const int mp = (kind == LDK_LATTICE && m >= 2) ? m - 1 : m;
    const ldk::Plan pl = ldk::make_plan(mp, p.log_tile, p.loge_max);
    if (log_tile) *log_tile = p.log_tile;
    if (radix) *radix = 1 << p.loge_max;
    if (passes) *passes = pl.P;
    if (engine) *engine = p.engine;
    return LDK_OK;
}

