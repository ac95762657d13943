// RQMC estimate over the R randomizations of a point set (eq. RQMC):
//   mu_r = (1/n) sum_{i<n} f(x_ri),  mu = (1/R) sum_r mu_r,
//   sigma^2 = sum_r (mu_r - mu)^2 / (R - 1),  half width t sigma / sqrt(R),
// for two Genz test integrands of s = sum_j c_j x_j: the corner peak
// (1 + s)^-(d+1) (the integrand of the paper's RQMC example) and the
// oscillatory cos(2 pi u + s).  The points are regenerated in registers and
// never written: a block takes KC_THREADS IT consecutive indices of one
// replication (IT = 8 points per thread, or 2 when that leaves the grid
// short of the chip's 256 compute units), accumulates s over the dimensions
// with the same point
// recurrences as the regenerating kernel column (plus the randomization's
// shift), applies the integrand and sums in FP64 in a fixed order.
#include "kfactor.hpp"

namespace ldk {

namespace {

constexpr int RQ_FINAL_THREADS = 1024;

__device__ __forceinline__ double wave_sum64(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block sum (fixed order: lanes, then waves); the result is valid in thread 0.
template <int THREADS>
__device__ __forceinline__ double block_sum(double v, double *red)
{
    v = wave_sum64(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < THREADS / 64; ++w) s += red[w];
    return s;
}

// A 32-bit word to double as one conversion instruction (left to itself the
// optimiser may widen it into a 64-bit conversion sequence, or copy the
// source word first).
__device__ __forceinline__ double cvt_u32(uint32_t v)
{
    double r;
    asm("v_cvt_f64_u32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}

// s[l] += c_j x_j over every dimension for the lattice points
// i = tile0 + t + KC_THREADS l, l < IT, of replication r (tile0 a multiple of
// KC_THREADS IT, so the bits of tile0, t and l are disjoint).
//
// Natural order: brev(i) g = brev(tile0) g + (rev8(t) g) 2^56 + brev(256 l) g
// (mod 2^64).  The first term plus the shift is the same for the whole block
// and alone sets the low word; the other two only add to the high word.  So
// x = hi 2^-32 + lo 2^-64 with lo shared by the block, and sum_j c_j x_j is
// taken as (sum_j c_j hi_j) 2^-32 + (sum_j c_j lo_j) 2^-64: one add, one
// conversion and one multiply-add per point and dimension, the low-word
// terms summed once per thread.
//
// Linear order: the shift is added to the base word before the points are
// split into high and low halves.
template <int ORDER, int IT>
__device__ __forceinline__ void lattice_dot(const PointsetArgs &ps, const double *__restrict__ coef,
                                            int r, int64_t tile0, double (&s)[IT])
{
    static_assert(IT <= 8 && KC_LOG_THREADS == 8, "offset table assumes up to 8 x 256");
    constexpr uint32_t br3[8] = {0, 4, 2, 6, 1, 5, 3, 7};
    const int d = ps.d, m = ps.m_max;
    if constexpr (ORDER == LDK_NATURAL) {
        const uint64_t btile = brev64((uint64_t)tile0);
        const uint32_t t8 = __builtin_bitreverse32((uint32_t)threadIdx.x) >> 24;
        // sums in units of 2^-32 (high words) and 2^-64 (low words): the
        // powers of two are applied once at the end, exactly
        double s_lo = 0.0;
        for (int j = 0; j < d; ++j) {
            const uint64_t g = ps.gen[j];
            const uint64_t sh = ps.shift ? ps.shift[(size_t)r * d + j] : 0;
            const double c = coef[j];
            const uint64_t B = btile * g + sh;
            // rev8(t) g mod 2^8 in the top byte (a 24-bit multiply: only the
            // low 8 bits of the product are kept); one register word per
            // thread, to which each point adds a scalar offset
            uint32_t tg;
            asm("v_mul_u32_u24 %0, %1, %2" : "=v"(tg) : "s"((uint32_t)g), "v"(t8));
            const uint32_t h = opaque32((uint32_t)(B >> 32) + (tg << 24));
            const uint32_t Gh = (uint32_t)(g << 21);  // high word of brev(256) g = g 2^53
            s_lo = fma(c, (double)(uint32_t)B, s_lo);
#pragma unroll
            for (int l = 0; l < IT; ++l) s[l] = fma(c, (double)(h + br3[l] * Gh), s[l]);
        }
#pragma unroll
        for (int l = 0; l < IT; ++l) s[l] = fma(s_lo, 0x1p-32, s[l]) * 0x1p-32;
    } else {
        const uint64_t first = (uint64_t)tile0 + threadIdx.x;
        for (int j = 0; j < d; ++j) {
            const uint64_t g = ps.gen[j];
            const uint64_t sh = ps.shift ? ps.shift[(size_t)r * d + j] : 0;
            const double c = coef[j];
            const uint64_t base = (m == 0 ? 0 : ((first * g) << (64 - m))) + sh;
            const uint64_t G = m <= 8 ? 0 : ((g << 8) << (64 - m));
#pragma unroll
            for (int l = 0; l < IT; ++l) s[l] = fma(c, unit<double>(base + (uint64_t)l * G), s[l]);
        }
    }
}

// The same for net points: scrambled columns and XOR steps from the LDS
// tables of the regenerating column, the digital shift folded into the
// starting word.  The high and low words of a point are summed apart (no
// product of the two conversions per point).
template <int IT>
__device__ __forceinline__ void net_dot(const KcolArgs &a, NetLds &L, const double *__restrict__ coef,
                                        int r, int64_t tile0, double (&s)[IT])
{
    constexpr int sft = KC_LOG_THREADS;
    const int d = a.ps.d, t = threadIdx.x;
    const bool gray = a.ps.order == LDK_GRAY;
    const uint64_t code_tile = gray ? gray_code((uint64_t)tile0) : (uint64_t)tile0;
    const uint32_t code_t = gray ? (uint32_t)gray_code((uint64_t)t) : (uint32_t)t;
    // sums of c_j hi_j and c_j lo_j for x = hi 2^-32 + lo 2^-64, scaled by
    // the powers of two once at the end (exactly)
    double s_lo[IT];
#pragma unroll
    for (int l = 0; l < IT; ++l) s_lo[l] = 0.0;
    for (int jc = 0; jc < d; jc += KC_DIM_CHUNK) {
        const int DB = min(KC_DIM_CHUNK, d - jc);
        build_net_chunk(a, L, r, jc, DB, code_tile);
        for (int jj = 0; jj < DB; ++jj) {
            const int j = jc + jj;
            const uint64_t sh = a.ps.shift ? a.ps.shift[(size_t)r * d + j] : 0;
            const double c = coef[j];
            // the shift enters once: XOR steps commute with it
            uint64_t z = L.zb[jj] ^ L.nib[jj][0][code_t & 15] ^ L.nib[jj][1][(code_t >> 4) & 15] ^ sh;
#pragma unroll
            for (int l = 0; l < IT; ++l) {
                s[l] = fma(c, cvt_u32((uint32_t)(z >> 32)), s[l]);
                s_lo[l] = fma(c, cvt_u32((uint32_t)z), s_lo[l]);
                // past the last index of the net the step columns are zero
                // (such points are masked by the caller)
                const uint64_t nb = ((uint64_t)tile0 >> sft) + (uint64_t)l + 1;
                if (l + 1 < IT) z ^= L.step[jj][ctz64(nb)];
            }
        }
    }
#pragma unroll
    for (int l = 0; l < IT; ++l) s[l] = fma(s_lo[l], 0x1p-32, s[l]) * 0x1p-32;
}

// b^-e for an integer e >= 1 by binary powering (e is block-uniform): about
// log2 e squarings, popcount e products and one division, each rounded once,
// so a relative error of at most about (e + 1) u, far cheaper than pow.
__device__ __forceinline__ double inv_ipow(double b, int e)
{
    double r = 1.0;
    for (;;) {
        if (e & 1) r *= b;
        e >>= 1;
        if (!e) break;
        b *= b;
    }
    return 1.0 / r;
}

template <int F>
__device__ __forceinline__ double integrand(double s, int d, double phase)
{
    if constexpr (F == LDK_GENZ_CORNER_PEAK)
        return inv_ipow(1.0 + s, d + 1);
    else
        return cos(phase + s);
}

// One block per (tile of KC_THREADS IT indices, replication): partial sums of f.
template <int KIND, int ORDER, int F, int IT>
__global__ __launch_bounds__(KC_THREADS) void k_rqmc_tiles(KcolArgs a, const double *__restrict__ coef,
                                                           double phase, int64_t n,
                                                           double *__restrict__ part)
{
    __shared__ double red[KC_THREADS / 64];
    const int r = blockIdx.y;
    const int64_t tile0 = (int64_t)blockIdx.x * (KC_THREADS * IT);
    const int64_t first = tile0 + threadIdx.x;
    double s[IT];
#pragma unroll
    for (int l = 0; l < IT; ++l) s[l] = 0.0;
    if constexpr (KIND == LDK_DNET_B2) {
        __shared__ NetLds L;
        net_dot<IT>(a, L, coef, r, tile0, s);
    } else {
        lattice_dot<ORDER, IT>(a.ps, coef, r, tile0, s);
    }
    double acc = 0.0;
#pragma unroll
    for (int l = 0; l < IT; ++l)
        if (first + (int64_t)l * KC_THREADS < n) acc += integrand<F>(s[l], a.ps.d, phase);
    const double tot = block_sum<KC_THREADS>(acc, red);
    if (threadIdx.x == 0) part[(size_t)r * gridDim.x + blockIdx.x] = tot;
}

// One block: wave w forms mu_r for r = w, w + waves, ... from its tile
// sums (lanes stride over the tiles, then a fixed-order wave sum); after the
// barrier the block forms mu, sigma (R >= 2, else NaN) and t sigma / sqrt(R).
__global__ __launch_bounds__(RQ_FINAL_THREADS) void k_rqmc_final(const double *__restrict__ part,
                                                                 int tiles, int R, double n,
                                                                 double t,
                                                                 double *__restrict__ mu_r,
                                                                 double *__restrict__ stats)
{
    __shared__ double red[RQ_FINAL_THREADS / 64];
    __shared__ double mean_s;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int WAVES = RQ_FINAL_THREADS / 64;
    for (int r = wave; r < R; r += WAVES) {
        double acc = 0.0;
        for (int c = lane; c < tiles; c += 64) acc += part[(size_t)r * tiles + c];
        acc = wave_sum64(acc);
        if (lane == 0) mu_r[r] = acc / n;
    }
    __syncthreads();  // the block's own writes of mu_r are visible to it now
    double acc = 0.0;
    for (int r = threadIdx.x; r < R; r += RQ_FINAL_THREADS) acc += mu_r[r];
    const double tot = block_sum<RQ_FINAL_THREADS>(acc, red);
    if (threadIdx.x == 0) mean_s = tot / (double)R;
    __syncthreads();
    const double mu = mean_s;
    double sq = 0.0;
    for (int r = threadIdx.x; r < R; r += RQ_FINAL_THREADS) {
        const double e = mu_r[r] - mu;
        sq = fma(e, e, sq);
    }
    const double ss = block_sum<RQ_FINAL_THREADS>(sq, red);
    if (threadIdx.x == 0) {
        const double sigma = R > 1 ? sqrt(ss / (double)(R - 1)) : __builtin_nan("");
        stats[LDK_RQMC_MEAN] = mu;
        stats[LDK_RQMC_STD] = sigma;
        stats[LDK_RQMC_HALF] = t * sigma / sqrt((double)R);
    }
}

// Given points: one block per (tile of RQ_PTS_TILE points, replication),
// read straight from HBM: sixteen lanes share a point (dimensions j = q,
// q + 16, ...), their partial sums of c_j x_ij combine in a fixed order, and
// f is applied once per point.
constexpr int RQ_PTS_W = 16;                    // lanes per point
constexpr int RQ_PTS_GROUPS = KC_THREADS / RQ_PTS_W;  // point groups of a block
constexpr int RQ_PTS_TILE = RQ_PTS_GROUPS * RQ_PTS_W; // points per block: each group takes 16
constexpr int RQ_PTS_MAX_D = 128;               // coefficients per lane: d / 16 <= 8

// Group g of 16 lanes reads the rows of points first + g + 16 it (it < 16):
// lane q takes coordinates q, q + 16, ..., so a wave's four groups read four
// consecutive rows, whole cache lines per load.  The 16-lane sum of each
// dot product lands in every lane of the group; lane q keeps the one of
// it == q, and every lane then evaluates one integrand.
template <int F>
__global__ __launch_bounds__(KC_THREADS) void k_rqmc_pts(const double *__restrict__ x, int d,
                                                         int64_t n, const double *__restrict__ coef,
                                                         double phase, double *__restrict__ part)
{
    __shared__ double red[KC_THREADS / 64];
    const int r = blockIdx.y, t = threadIdx.x;
    const int q = t & (RQ_PTS_W - 1), g = t / RQ_PTS_W;
    double c[RQ_PTS_MAX_D / RQ_PTS_W];
#pragma unroll
    for (int k = 0; k < RQ_PTS_MAX_D / RQ_PTS_W; ++k) {
        const int j = q + RQ_PTS_W * k;
        c[k] = j < d ? coef[j] : 0.0;
    }
    const int64_t first = (int64_t)blockIdx.x * RQ_PTS_TILE + g;
    double mine = 0.0;
#pragma unroll 2
    for (int it = 0; it < RQ_PTS_W; ++it) {
        const int64_t p = first + (int64_t)RQ_PTS_W * it;
        double s = 0.0;
        if (p < n) {
            const double *row = x + ((size_t)r * n + p) * d;
#pragma unroll
            for (int k = 0; k < RQ_PTS_MAX_D / RQ_PTS_W; ++k) {
                const int j = q + RQ_PTS_W * k;
                if (j < d) s = fma(c[k], row[j], s);
            }
        }
        s += __shfl_xor(s, 1, 64);
        s += __shfl_xor(s, 2, 64);
        s += __shfl_xor(s, 4, 64);
        s += __shfl_xor(s, 8, 64);
        if (it == q) mine = s;
    }
    const int64_t pm = first + (int64_t)RQ_PTS_W * q;
    const double acc = pm < n ? integrand<F>(mine, d, phase) : 0.0;
    const double tot = block_sum<KC_THREADS>(acc, red);
    if (threadIdx.x == 0) part[(size_t)r * gridDim.x + blockIdx.x] = tot;
}

constexpr int RQ_IT_FULL = 8, RQ_IT_SMALL = 2;

int64_t tiles_of(int64_t n, int it) { return (n + KC_THREADS * it - 1) / (KC_THREADS * it); }

// Points per thread: 8, unless the grid would then hold fewer than two
// blocks per compute unit.
int rq_iters(int64_t n, int R)
{
    return tiles_of(n, RQ_IT_FULL) * R < 512 ? RQ_IT_SMALL : RQ_IT_FULL;
}

template <int F, int IT>
void launch_tiles(const KcolArgs &a, const double *coef, double phase, int64_t n, dim3 grid,
                  hipStream_t s, double *part)
{
    if (a.ps.kind == LDK_DNET_B2)
        hipLaunchKernelGGL((k_rqmc_tiles<LDK_DNET_B2, LDK_NATURAL, F, IT>), grid, dim3(KC_THREADS),
                           0, s, a, coef, phase, n, part);
    else if (a.ps.order == LDK_LINEAR)
        hipLaunchKernelGGL((k_rqmc_tiles<LDK_LATTICE, LDK_LINEAR, F, IT>), grid, dim3(KC_THREADS),
                           0, s, a, coef, phase, n, part);
    else
        hipLaunchKernelGGL((k_rqmc_tiles<LDK_LATTICE, LDK_NATURAL, F, IT>), grid,
                           dim3(KC_THREADS), 0, s, a, coef, phase, n, part);
}

}  // namespace

}  // namespace ldk

using namespace ldk;

namespace {

size_t align256_rq(size_t b) { return (b + 255) & ~(size_t)255; }

// Tile sums, then (LMS nets) each replication's scrambled columns S_j C_j,
// formed once instead of in every block of the grid.
size_t rqmc_ws(const PointsetArgs &a, int64_t n)
{
    size_t b = align256_rq((size_t)a.R * (size_t)tiles_of(n, RQ_IT_SMALL) * sizeof(double));
    if (a.kind == LDK_DNET_B2 && a.lms)
        b += (size_t)a.R * (size_t)a.d * (size_t)a.m_max * sizeof(uint64_t);
    return b;
}

}  // namespace

extern "C" size_t ldk_rqmc_workspace_bytes(const ldk_pointset *ps, int64_t n)
{
    PointsetArgs a;
    if (validate_pointset(ps, &a) || n < 0) return 0;
    return rqmc_ws(a, n);
}

extern "C" int ldk_rqmc(const ldk_pointset *ps, int64_t n, int integrand, const double *coef,
                        double u, double t, double *mu_r, double *stats, void *ws,
                        ldk_stream stream)
{
    KcolArgs a{};
    int st = validate_pointset(ps, &a.ps);
    if (st) return st;
    if (integrand != LDK_GENZ_CORNER_PEAK && integrand != LDK_GENZ_OSCILLATORY) return LDK_EINVAL;
    if (!(u >= -1.0e6 && u <= 1.0e6) || !(t >= 0.0 && t <= 1.0e300)) return LDK_EINVAL;
    const int64_t lim = (a.ps.kind == LDK_LATTICE && a.ps.order == LDK_NATURAL)
                            ? ((int64_t)1 << 62)
                            : ((int64_t)1 << a.ps.m_max);
    if (n < 1 || n > lim) return LDK_EINVAL;
    if (!coef || !mu_r || !stats || !ws) return LDK_EINVAL;
    const int it = rq_iters(n, a.ps.R);
    const int64_t tiles = tiles_of(n, it);
    // the grid is tiles x R blocks of KC_THREADS work items; a dispatch's
    // work-item count along x must fit 32 bits
    if (tiles > 0x7fffffff || (uint64_t)tiles * KC_THREADS > 0xffffffffull) return LDK_ENOTSUP;
    st = ensure_init();
    if (st) return st;
    a.n_min = 0;
    a.n_max = n;
    hipStream_t s = as_stream(stream);
    double *part = static_cast<double *>(ws);
    if (a.ps.kind == LDK_DNET_B2 && a.ps.lms && a.ps.m_max > 0 && ps->flags == 0) {
        // scramble the shared columns once per replication (interlacing of
        // order 1 is the scrambling alone); the tiles then read
        // per-replication columns and skip the scrambling.  A net with
        // per-replication columns and scrambles keeps lms: its tiles scramble
        // their own columns as they build their step tables.
        uint64_t *cols = reinterpret_cast<uint64_t *>(
            static_cast<unsigned char *>(ws) +
            align256_rq((size_t)a.ps.R * (size_t)tiles_of(n, RQ_IT_SMALL) * sizeof(double)));
        st = ldk_interlace(ps, 1, cols, stream);
        if (st) return st;
        a.ps.gen = cols;
        a.ps.gen_rstride = (int64_t)a.ps.d * a.ps.m_max;
        a.ps.lms = nullptr;
    }
    const dim3 grid((unsigned)tiles, (unsigned)a.ps.R);
    const double phase = 6.283185307179586476925286766559 * u;
    if (integrand == LDK_GENZ_CORNER_PEAK) {
        if (it == RQ_IT_SMALL) launch_tiles<LDK_GENZ_CORNER_PEAK, RQ_IT_SMALL>(a, coef, phase, n, grid, s, part);
        else launch_tiles<LDK_GENZ_CORNER_PEAK, RQ_IT_FULL>(a, coef, phase, n, grid, s, part);
    } else {
        if (it == RQ_IT_SMALL) launch_tiles<LDK_GENZ_OSCILLATORY, RQ_IT_SMALL>(a, coef, phase, n, grid, s, part);
        else launch_tiles<LDK_GENZ_OSCILLATORY, RQ_IT_FULL>(a, coef, phase, n, grid, s, part);
    }
    LDK_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_rqmc_final, dim3(1), dim3(RQ_FINAL_THREADS), 0, s, (const double *)part,
                       (int)tiles, a.ps.R, (double)n, t, mu_r, stats);
    LDK_LAUNCH_CHECK();
    return LDK_OK;
}

extern "C" size_t ldk_rqmc_points_workspace_bytes(int R, int64_t n)
{
    if (R < 1 || n < 1) return 0;
    return (size_t)R * (size_t)((n + RQ_PTS_TILE - 1) / RQ_PTS_TILE) * sizeof(double);
}

extern "C" int ldk_rqmc_points(int R, int64_t n, int d, const double *x, int integrand,
                               const double *coef, double u, double t, double *mu_r, double *stats,
                               void *ws, ldk_stream stream)
{
    if (R < 1 || R > 65535 || n < 1 || d < 1 || d > RQ_PTS_MAX_D || !x || !coef || !mu_r ||
        !stats || !ws)
        return LDK_EINVAL;
    if (integrand != LDK_GENZ_CORNER_PEAK && integrand != LDK_GENZ_OSCILLATORY) return LDK_EINVAL;
    if (!(u >= -1.0e6 && u <= 1.0e6) || !(t >= 0.0 && t <= 1.0e300)) return LDK_EINVAL;
    const int64_t tiles = (n + RQ_PTS_TILE - 1) / RQ_PTS_TILE;
    if (tiles > 0x7fffffff || (uint64_t)tiles * KC_THREADS > 0xffffffffull) return LDK_ENOTSUP;
    hipStream_t s = as_stream(stream);
    double *part = static_cast<double *>(ws);
    const dim3 grid((unsigned)tiles, (unsigned)R);
    const double phase = 6.283185307179586476925286766559 * u;
    if (integrand == LDK_GENZ_CORNER_PEAK)
        hipLaunchKernelGGL(k_rqmc_pts<LDK_GENZ_CORNER_PEAK>, grid, dim3(KC_THREADS), 0, s, x, d, n,
                           coef, phase, part);
    else
        hipLaunchKernelGGL(k_rqmc_pts<LDK_GENZ_OSCILLATORY>, grid, dim3(KC_THREADS), 0, s, x, d, n,
                           coef, phase, part);
    LDK_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_rqmc_final, dim3(1), dim3(RQ_FINAL_THREADS), 0, s, (const double *)part,
                       (int)tiles, R, (double)n, t, mu_r, stats);
    LDK_LAUNCH_CHECK();
    return LDK_OK;
}
