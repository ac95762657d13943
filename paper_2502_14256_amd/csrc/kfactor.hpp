// Factors of the product-weight kernels and the per-block point tables
// shared by the kernel column and its parameter gradient.
#pragma once

#include <type_traits>

#include "pointset.hpp"

namespace ldk {

namespace {
constexpr int KC_THREADS = 256;
constexpr int KC_LOG_THREADS = 8;
constexpr int KC_ITERS = 8;       // points per thread (spaced KC_THREADS apart)
constexpr int KC_DIM_CHUNK = 8;   // dimensions whose net tables sit in LDS at once (12 KiB)
constexpr int KC_TILE = KC_THREADS * KC_ITERS;
constexpr int KC_CODE_WORDS = LDK_MAX_D / 32;  // 2-bit order codes, 32 per word
}  // namespace

// ---- SI factor, Sec. 5.2:  K_a(x) = (2 pi)^{2a} / ((-1)^{a+1} (2a)!) B_{2a}(x) ----
// With w = x^2 - x the Bernoulli polynomials are cubics in w:
//   B_2 = w + 1/6,  B_4 = w^2 - 1/30,  B_6 = w^3 - w^2/2 + 1/42,
// so 1 + gamma K_a(x) = c0 + c1 w + c2 w^2 + c3 w^3 with per-dimension c.
struct SiPoly {
    double c0, c1, c2, c3;
};
__device__ __forceinline__ SiPoly si_poly(int alpha, double gamma)
{
    const double pi2 = 9.8696044010893586188344909998761511;
    if (alpha == 1) {  // 2 pi^2 B_2
        const double a = 2.0 * pi2 * gamma;
        return {1.0 + a * (1.0 / 6.0), a, 0.0, 0.0};
    }
    if (alpha == 2) {  // -2 pi^4 / 3 B_4
        const double a = (-2.0 / 3.0) * pi2 * pi2 * gamma;
        return {1.0 - a * (1.0 / 30.0), 0.0, a, 0.0};
    }
    const double a = (4.0 / 45.0) * pi2 * pi2 * pi2 * gamma;  // 4 pi^6 / 45 B_6
    return {1.0 + a * (1.0 / 42.0), 0.0, -0.5 * a, a};
}
// Fused multiply-add written out: every kernel that forms a factor forms it
// with the same roundings (the kernel column and its gradient divide one by
// the other, so they must agree bit for bit).
__device__ __forceinline__ float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ALPHA = 0: generic cubic (mixed orders); 1, 2: only the nonzero terms.
template <typename R, int ALPHA>
__device__ __forceinline__ R si_weighted(R x, R c0, R c1, R c2, R c3)
{
    const R w = fma_r(x, x, -x);
    if constexpr (ALPHA == 1) return fma_r(c1, w, c0);
    else if constexpr (ALPHA == 2) return fma_r(c2 * w, w, c0);
    else return fma_r(fma_r(fma_r(c3, w, c2), w, c1), w, c0);
}

// DSI product factor 1 + gamma K.
template <typename R>
__device__ __forceinline__ R dsi_weighted(R gam, R k) { return fma_r(gam, k, (R)1); }

// ---- DSI factor, Sec. 5.3 / Theorem 1 (base 2), alpha = 1 .. 4 ----
// beta = index of the first nonzero digit (clz + 1), t_nu = 2^{-nu beta},
// both 0 at x = 0; "-1+-" in the theorem read as "-1-".
// alpha = 1: K_1 = 1 - 3 t_1 (reading; the paper defers this form).
// The alpha = 4 series sum_{a>=0} (-1)^{xi_{a+1}} 8^{-a} is kept to 21 digits
// (the rest is below 2^-62) and read from three 128-entry tables of 7 digits:
// series = 8/7 - 2 (T0[d1..d7] + T1[d8..d14] + T2[d15..d21]).
// Each entry is a sum of at most 7 powers of 8 spanning 19 bits: exact in
// FP32, so the tables are stored as float (half the LDS traffic).
struct DsiTables {
    float t[3][128];
};
__device__ __forceinline__ void fill_dsi_tables(DsiTables &tab, int t, int nthreads)
{
    for (int w = t; w < 3 * 128; w += nthreads) {
        const int chunk = w >> 7, v = w & 127;
        double acc = 0.0;
        for (int b = 0; b < 7; ++b)  // bit 6 - b of v is digit 7 chunk + b + 1
            if ((v >> (6 - b)) & 1) acc += ldexp(1.0, -3 * (7 * chunk + b));
        tab.t[chunk][v] = (float)acc;
    }
}

// 2^-beta for 1 <= beta <= 64 from its exponent bits (exact).
__device__ __forceinline__ double pow2_neg(int beta)
{
    return __hiloint2double((1023 - beta) << 20, 0);
}
template <typename R>
__device__ __forceinline__ R pow2_neg_r(int beta);
template <>
__device__ __forceinline__ double pow2_neg_r<double>(int beta) { return pow2_neg(beta); }
template <>
__device__ __forceinline__ float pow2_neg_r<float>(int beta) { return __int_as_float((127 - beta) << 23); }

// A 32-bit value the optimiser cannot see through (no instruction): keeps
// a conversion of a 32-bit word from being widened into the much longer
// 64-bit integer-to-float sequence.
__device__ __forceinline__ uint32_t opaque32(uint32_t v)
{
    asm("" : "+v"(v));
    return v;
}

// A double constant held in scalar registers: a three-operand multiply-add
// cannot take a 64-bit literal, and with the literal the compiler falls back
// to the two-operand form plus a register copy.
__device__ __forceinline__ double scalar_const(double c)
{
    const uint64_t u = (uint64_t)__double_as_longlong(c);
    uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
    asm("" : "+s"(lo));
    asm("" : "+s"(hi));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Coordinate value x = u 2^-64.  FP64: rounded to nearest (two exact
// conversions, one fused multiply-add).  FP32: the top 32 digits rounded to
// 24 bits (absolute error below 2^-24 x + 2^-32, far inside the FP32
// tolerance; one conversion and one multiply).
template <typename R>
__device__ __forceinline__ R unit(uint64_t u);
template <>
__device__ __forceinline__ double unit<double>(uint64_t u)
{
    // hi 2^-32 + lo 2^-64: both terms exact, one rounding
    return __fma_rn((double)opaque32((uint32_t)(u >> 32)), scalar_const(0x1p-32),
                    (double)opaque32((uint32_t)u) * scalar_const(0x1p-64));
}
template <>
__device__ __forceinline__ float unit<float>(uint64_t u)
{
    return (float)opaque32((uint32_t)(u >> 32)) * 0x1p-32f;
}

// The same values from the two halves of u, with the low half's part
// lo_part(lo) computed once where several words share their low half:
// hi 2^-32 + lo 2^-64 rounded once is the value unit<double> returns.
template <typename R>
__device__ __forceinline__ R lo_part(uint32_t lo);
template <>
__device__ __forceinline__ double lo_part<double>(uint32_t lo)
{
    return (double)opaque32(lo) * scalar_const(0x1p-64);  // exact
}
template <>
__device__ __forceinline__ float lo_part<float>(uint32_t)
{
    return 0.0f;  // FP32 takes the top 32 digits only
}
template <typename R>
__device__ __forceinline__ R unit_hl(uint32_t hi, R lo_p);
template <>
__device__ __forceinline__ double unit_hl<double>(uint32_t hi, double lo_p)
{
    return __fma_rn((double)opaque32(hi), scalar_const(0x1p-32), lo_p);
}
template <>
__device__ __forceinline__ float unit_hl<float>(uint32_t hi, float)
{
    return (float)opaque32(hi) * 0x1p-32f;
}

template <typename R, int ALPHA>
__device__ __forceinline__ R dsi_factor(uint64_t delta, const DsiTables &tab)
{
    // beta = 1 + clz(delta) for delta != 0; beta = x = t_nu = 0 at delta = 0.
    // FP32 sees the top 32 digits only: where they are all zero, x = 0 and
    // t_nu <= 2^-33 lies below half an ulp of every term it enters (1 - 3 t1,
    // 1.5 - 2.5 t1, 1 - t_nu), so beta and t_nu are taken as 0 there, as at
    // delta = 0: one 32-bit count instead of a 64-bit one.  (For alpha = 4
    // the beta-weighted series term, exactly zero there, is then dropped
    // instead of carrying its FP32 rounding.)
    bool nz;
    int beta;
    if constexpr (std::is_same<R, float>::value) {
        const uint32_t hi = (uint32_t)(delta >> 32);
        nz = hi != 0;
        beta = nz ? __clz((int)hi) + 1 : 0;
    } else {
        nz = delta != 0;
        beta = nz ? clz64(delta) + 1 : 0;
    }
    const R x = unit<R>(delta);  // 0 at delta = 0
    const R b = (R)beta;
    const R t1 = nz ? pow2_neg_r<R>(beta) : (R)0;
    if constexpr (ALPHA == 1) {
        return (R)1 - (R)3 * t1;
    } else if constexpr (ALPHA == 2) {
        return (R)1.5 - (R)2.5 * t1 - b * x;
    } else if constexpr (ALPHA == 3) {
        const R t2 = t1 * t1;
        return ((b * x - (R)5 * ((R)1 - t1)) * x + (R)(43.0 / 18.0) * ((R)1 - t2)) - (R)1;
    } else {
        const R t2 = t1 * t1, t3 = t2 * t1;
        const uint32_t hi = (uint32_t)(delta >> 32);
        const R ones = ((R)tab.t[0][hi >> 25] + (R)tab.t[1][(hi >> 18) & 127]) +
                       (R)tab.t[2][(hi >> 11) & 127];
        const R series = (R)(8.0 / 7.0) - (R)2 * ones;
        const R poly = ((-(R)(2.0 / 3.0) * b * x + (R)5 * ((R)1 - t1)) * x -
                        (R)(43.0 / 9.0) * ((R)1 - t2)) * x;
        return poly + ((R)(701.0 / 294.0) * ((R)1 - t3) - (R)1) +
               b * (series * (R)(1.0 / 48.0) - (R)(1.0 / 42.0));
    }
}
template <typename R>
__device__ __forceinline__ R dsi_factor_any(int alpha, uint64_t delta, const DsiTables &tab)
{
    switch (alpha) {
    case 1: return dsi_factor<R, 1>(delta, tab);
    case 2: return dsi_factor<R, 2>(delta, tab);
    case 3: return dsi_factor<R, 3>(delta, tab);
    default: return dsi_factor<R, 4>(delta, tab);
    }
}

struct KcolArgs {
    PointsetArgs ps;
    const double *gamma;
    double zeta;
    int64_t n_min, n_max;
    const uint64_t *pts;  // [R][cnt][d] or nullptr (regenerate)
    const uint64_t *x0;   // [R][d] anchors (pts mode), or nullptr = row 0 of pts
    uint64_t acode[KC_CODE_WORDS];  // alpha_j - 1 in 2 bits, 32 dimensions per word
};

__device__ __forceinline__ int alpha_of(const KcolArgs &a, int j)
{
    return 1 + (int)((a.acode[j >> 5] >> (2 * (j & 31))) & 3u);
}

// Net tables of a chunk of dimensions.  The start point of thread t is
// z(code(tile0 + t)) = z(code(tile0)) ^ z(code(t)) (the index bits of tile0 and
// t are disjoint, also after Gray coding), read as one block-uniform word
// zb[jj] and two 16-entry nibble tables of z over the low 8 index bits.
struct NetLds {
    uint64_t ct[KC_DIM_CHUNK][64];  // scrambled columns S_j C_j
    union {
        uint64_t step[KC_DIM_CHUNK][64];  // XOR steps between a thread's points
        uint64_t srow[KC_DIM_CHUNK][65];  // rows of S_j (dead once ct is built)
    };
    uint64_t nib[KC_DIM_CHUNK][2][16];  // z of (nibble h of the low index byte)
    uint64_t zb[KC_DIM_CHUNK];          // z(code(tile0))
    DsiTables tab;
};

// SI weight without the leading 1: gamma K_a(x) = e0 + c1 w + c2 w^2 + c3 w^3
// (w = x^2 - x), so that small gamma K keeps its relative accuracy.
__device__ __forceinline__ SiPoly si_tpoly(int alpha, double gamma)
{
    SiPoly p = si_poly(alpha, gamma);
    const double pi2 = 9.8696044010893586188344909998761511;
    if (alpha == 1) p.c0 = 2.0 * pi2 * gamma * (1.0 / 6.0);
    else if (alpha == 2) p.c0 = -((-2.0 / 3.0) * pi2 * pi2 * gamma) * (1.0 / 30.0);
    else p.c0 = (4.0 / 45.0) * pi2 * pi2 * pi2 * gamma * (1.0 / 42.0);
    return p;
}

// Host: validate kernel + point-set arguments (as ldk_kernel_column states
// them) and fill KcolArgs; *uniform_alpha = the common order, or 0 if mixed.
int prepare_kernel_args(const ldk_kernel *k, const ldk_pointset *ps, const uint64_t *pts,
                        const uint64_t *x0, int64_t n_min, int64_t n_max, int dtype, KcolArgs *out,
                        int *uniform_alpha);

// Tables of dimensions jc .. jc+DB-1 for the block whose first point index
// has code code_tile: scrambled columns, XOR steps, nibble tables and the
// block's base point (see NetLds).  Every thread of the block must call it.
__device__ __forceinline__ void build_net_chunk(const KcolArgs &a, NetLds &L, int r, int jc, int DB,
                                                uint64_t code_tile)
{
    constexpr int s = KC_LOG_THREADS;
    const int d = a.ps.d, m = a.ps.m_max, t = threadIdx.x;
    const bool gray = a.ps.order == LDK_GRAY;
    __syncthreads();  // tables of the previous chunk are no longer read
    if (a.ps.lms) {
        for (int w = t; w < DB * 64; w += KC_THREADS)
            L.srow[w >> 6][w & 63] = a.ps.lms[((size_t)r * d + jc + (w >> 6)) * 64 + (w & 63)];
        __syncthreads();
    }
    // columns k >= m are zero; the DB m scrambled columns take one item
    // each, so no lane idles through a scrambling loop (the S rows are
    // padded: the lanes of a wave read rows of different dimensions)
    for (int w = t; w < DB * 64; w += KC_THREADS)
        if ((w & 63) >= m) L.ct[w >> 6][w & 63] = 0;
    for (int w = t; w < DB * m; w += KC_THREADS) {
        const int jj = w / m, k = w - jj * m;
        const uint64_t col = net_gen_column(a.ps, r, jc + jj, k);
        L.ct[jj][k] = a.ps.lms ? lms_column(L.srow[jj], col) : col;
    }
    __syncthreads();  // srow is dead from here on; step reuses its storage
    for (int w = t; w < DB * 64; w += KC_THREADS) {
        const int jj = w >> 6, c = w & 63;
        uint64_t v = 0;
        if (s + c < m) {
            if (gray) {
                v = L.ct[jj][s + c] ^ L.ct[jj][s - 1];
            } else {
                for (int k = s; k <= s + c; ++k) v ^= L.ct[jj][k];
            }
        }
        L.step[jj][c] = v;
    }
    for (int w = t; w < DB * 32; w += KC_THREADS) {
        const int jj = w >> 5, h = (w >> 4) & 1, v = w & 15;
        uint64_t z = 0;
        for (int k = 0; k < 4; ++k)
            if ((v >> k) & 1) z ^= L.ct[jj][4 * h + k];
        L.nib[jj][h][v] = z;
    }
    if (t < DB) L.zb[t] = net_point(L.ct[t], m, code_tile);
    __syncthreads();
}

}  // namespace ldk
