// First column of the product-weight Gram matrix,
//   k1_i = zeta prod_j (1 + gamma_j K_{alpha_j}(x_ij (-) x0_j)),
// with SI factors (Sec. 5.2, Bernoulli polynomials) for lattices and DSI
// factors (Sec. 5.3, Theorem 1) for base-2 digital nets.  This op is
// ALU-bound: the points are either read once or regenerated in registers.
#include "pointset.hpp"

namespace ldk {

namespace {
constexpr int KC_THREADS = 256;
constexpr int KC_ITERS = 8;       // points per thread (spaced KC_THREADS apart)
constexpr int KC_DIM_CHUNK = 32;  // dimensions whose net tables sit in LDS at once
}  // namespace

// ---- SI factor, Sec. 5.2:  K_a(x) = (2 pi)^{2a} / ((-1)^{a+1} (2a)!) B_{2a}(x) ----
// B_2 = x^2 - x + 1/6, B_4 = x^2 (1-x)^2 - 1/30, B_6 = x^6 - 3x^5 + 5/2 x^4 - 1/2 x^2 + 1/42.
template <typename R>
__device__ __forceinline__ R si_factor(int alpha, R x)
{
    const R pi2 = (R)9.8696044010893586188344909998761511;  // pi^2
    if (alpha < 1) return (R)__builtin_nan("");
    if (alpha == 1) return (R)2 * pi2 * ((x - (R)1) * x + (R)(1.0 / 6.0));
    const R x2 = x * x;
    if (alpha == 2) {
        const R w = (x - (R)1) * x;  // x^2 - x
        return (R)(-2.0 / 3.0) * pi2 * pi2 * (w * w - (R)(1.0 / 30.0));
    }
    if (alpha != 3) return (R)__builtin_nan("");  // unsupported order: poison the column
    // alpha == 3: (x^6 - 3x^5 + 5/2 x^4 - 1/2 x^2 + 1/42) * 4 pi^6 / 45
    const R b6 = (((((x - (R)3) * x + (R)2.5) * x) * x - (R)0.5) * x2 + (R)(1.0 / 42.0));
    return (R)(4.0 / 45.0) * pi2 * pi2 * pi2 * b6;
}

// sum_{a=0}^{20} (-1)^{xi_{a+1}} 8^{-a}: 21 leading digits of delta spread to
// every third bit (bit i of the digit field lands at bit 3 i), so that
// sum_{xi_{a+1} = 1} 8^{-a} = spread * 2^-60 exactly before rounding.
__device__ __forceinline__ uint64_t spread3_21(uint64_t b)
{
    b &= 0x1fffffull;
    b = (b | (b << 32)) & 0x1f00000000ffffull;
    b = (b | (b << 16)) & 0x1f0000ff0000ffull;
    b = (b | (b << 8)) & 0x100f00f00f00f00full;
    b = (b | (b << 4)) & 0x10c30c30c30c30c3ull;
    b = (b | (b << 2)) & 0x1249249249249249ull;
    return b;
}

// ---- DSI factor, Sec. 5.3 / Theorem 1 (base 2), alpha = 1 .. 4 ----
// beta = index of the first nonzero digit (clz + 1), t_nu = 2^{-nu beta},
// both 0 at x = 0; "-1+-" in the theorem read as "-1-".
// alpha = 1: K_1 = 1 - 3 t_1 (reading; the paper defers this form).
template <typename R>
__device__ __forceinline__ R dsi_factor(int alpha, uint64_t delta);

template <>
__device__ __forceinline__ double dsi_factor<double>(int alpha, uint64_t delta)
{
    int beta = 0;
    double x = 0.0;
    if (delta) {
        beta = clz64(delta) + 1;
        x = unit_f64(delta);
    }
    const double b = (double)beta;
    const double t1 = beta ? ldexp(1.0, -beta) : 0.0;
    if (alpha == 1) return 1.0 - 3.0 * t1;
    if (alpha == 2) return -1.0 - b * x + 2.5 * (1.0 - t1);
    if (alpha < 1) return __builtin_nan("");
    const double t2 = t1 * t1;
    if (alpha == 3) return -1.0 + b * x * x - 5.0 * (1.0 - t1) * x + (43.0 / 18.0) * (1.0 - t2);
    if (alpha != 4) return __builtin_nan("");  // unsupported order: poison the column
    const double t3 = t2 * t1;
    // series: sum_{a<21} 8^-a - 2 sum_{xi_{a+1}=1} 8^-a
    const uint64_t sp = spread3_21(delta >> 43);
    const double ones = unit_f64(sp) * 16.0;  // sp * 2^-60
    const double series = 1.1428571428571428571 - 2.0 * ones;
    return -1.0 - (2.0 / 3.0) * b * x * x * x + 5.0 * (1.0 - t1) * x * x -
           (43.0 / 9.0) * (1.0 - t2) * x + (701.0 / 294.0) * (1.0 - t3) +
           b * (series * (1.0 / 48.0) - 1.0 / 42.0);
}

template <>
__device__ __forceinline__ float dsi_factor<float>(int alpha, uint64_t delta)
{
    int beta = 0;
    float x = 0.0f;
    if (delta) {
        beta = clz64(delta) + 1;
        x = unit_f32(delta);
    }
    const float b = (float)beta;
    const float t1 = beta ? ldexpf(1.0f, -beta) : 0.0f;
    if (alpha == 1) return 1.0f - 3.0f * t1;
    if (alpha == 2) return -1.0f - b * x + 2.5f * (1.0f - t1);
    if (alpha < 1) return __builtin_nanf("");
    const float t2 = t1 * t1;
    if (alpha == 3)
        return -1.0f + b * x * x - 5.0f * (1.0f - t1) * x + (43.0f / 18.0f) * (1.0f - t2);
    if (alpha != 4) return __builtin_nanf("");  // unsupported order: poison the column
    const float t3 = t2 * t1;
    const uint64_t sp = spread3_21(delta >> 43);
    const float ones = unit_f32(sp) * 16.0f;
    const float series = 1.14285714285714285f - 2.0f * ones;
    return -1.0f - (2.0f / 3.0f) * b * x * x * x + 5.0f * (1.0f - t1) * x * x -
           (43.0f / 9.0f) * (1.0f - t2) * x + (701.0f / 294.0f) * (1.0f - t3) +
           b * (series * (1.0f / 48.0f) - 1.0f / 42.0f);
}

template <typename R>
__device__ __forceinline__ R unit(uint64_t u);
template <>
__device__ __forceinline__ double unit<double>(uint64_t u) { return unit_f64(u); }
template <>
__device__ __forceinline__ float unit<float>(uint64_t u) { return unit_f32(u); }

struct KcolArgs {
    PointsetArgs ps;
    const int32_t *alpha;
    const double *gamma;
    double zeta;
    int64_t n_min, n_max;
    const uint64_t *pts;  // [R][cnt][d] or nullptr (regenerate)
    const uint64_t *x0;   // [R][d] anchors (pts mode), or nullptr = row 0 of pts
};

// Block: replication r = blockIdx.y, points tile0 + t + KC_THREADS * l.
template <typename R>
__global__ __launch_bounds__(KC_THREADS) void k_kernel_column(KcolArgs a, R *__restrict__ out)
{
    __shared__ uint64_t ct[KC_DIM_CHUNK][64];
    __shared__ uint64_t step[KC_DIM_CHUNK][64];
    const int r = blockIdx.y;
    const int t = threadIdx.x;
    const int d = a.ps.d, m = a.ps.m_max;
    const bool net = a.ps.kind == LDK_DNET_B2;
    const bool regen = a.pts == nullptr;
    const int64_t cnt = a.n_max - a.n_min;
    const int64_t tile0 = a.n_min + (int64_t)blockIdx.x * KC_THREADS * KC_ITERS;
    const int64_t first = tile0 + t;
    constexpr int s = 8;  // log2(KC_THREADS): index stride between a thread's points
    static_assert((1 << s) == KC_THREADS, "stride");

    R prod[KC_ITERS];
#pragma unroll
    for (int l = 0; l < KC_ITERS; ++l) prod[l] = (R)a.zeta;

    for (int jc = 0; jc < d; jc += KC_DIM_CHUNK) {
        const int DB = min(KC_DIM_CHUNK, d - jc);
        if (regen && net) {
            __syncthreads();
            for (int w = t; w < DB * m; w += KC_THREADS) {
                const int jj = w / m, k = w % m;
                const uint64_t col = a.ps.gen[(size_t)(jc + jj) * m + k];
                ct[jj][k] = a.ps.lms ? lms_column(a.ps.lms + ((size_t)r * d + jc + jj) * 64, col)
                                     : col;
            }
            __syncthreads();
            for (int w = t; w < DB * 64; w += KC_THREADS) {
                const int jj = w / 64, c = w % 64;
                uint64_t v = 0;
                if (s + c < m) {
                    if (a.ps.order == LDK_GRAY) {
                        v = ct[jj][s + c] ^ ct[jj][s - 1];
                    } else {
                        for (int k = s; k <= s + c; ++k) v ^= ct[jj][k];
                    }
                }
                step[jj][c] = v;
            }
            __syncthreads();
        }
        for (int jj = 0; jj < DB; ++jj) {
            const int j = jc + jj;
            const int alpha = a.alpha[j];
            const R gam = (R)a.gamma[j];
            if (regen) {
                if (net) {
                    if (first >= a.n_max) continue;
                    const uint64_t code =
                        a.ps.order == LDK_GRAY ? gray_code((uint64_t)first) : (uint64_t)first;
                    uint64_t z = net_point(ct[jj], m, code);
                    int64_t i = first;
#pragma unroll
                    for (int l = 0; l < KC_ITERS; ++l) {
                        if (i < a.n_max) {
                            prod[l] *= (R)1 + gam * dsi_factor<R>(alpha, z);
                            if (i + KC_THREADS < a.n_max) z ^= step[jj][ctz64(((uint64_t)i >> s) + 1)];
                        }
                        i += KC_THREADS;
                    }
                } else {
                    const uint64_t g = a.ps.gen[j];
#pragma unroll
                    for (int l = 0; l < KC_ITERS; ++l) {
                        const int64_t i = first + (int64_t)l * KC_THREADS;
                        if (i < a.n_max) {
                            const uint64_t delta = lattice_point(g, (uint64_t)i, a.ps.order, m);
                            prod[l] *= (R)1 + gam * si_factor<R>(alpha, unit<R>(delta));
                        }
                    }
                }
            } else {
                const uint64_t u0 = a.x0 ? a.x0[(size_t)r * d + j] : a.pts[(size_t)r * cnt * d + j];
#pragma unroll
                for (int l = 0; l < KC_ITERS; ++l) {
                    const int64_t i = first + (int64_t)l * KC_THREADS;
                    if (i < a.n_max) {
                        const uint64_t u = a.pts[((size_t)r * cnt + (i - a.n_min)) * d + j];
                        const R f = net ? dsi_factor<R>(alpha, u ^ u0)
                                        : si_factor<R>(alpha, unit<R>(u - u0));
                        prod[l] *= (R)1 + gam * f;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int l = 0; l < KC_ITERS; ++l) {
        const int64_t i = first + (int64_t)l * KC_THREADS;
        if (i < a.n_max) out[(size_t)r * cnt + (i - a.n_min)] = prod[l];
    }
}

}  // namespace ldk

using namespace ldk;

extern "C" int ldk_kernel_column(const ldk_kernel *k, const ldk_pointset *ps, const uint64_t *pts,
                                 const uint64_t *x0, int64_t n_min, int64_t n_max, int dtype,
                                 void *out, ldk_stream stream)
{
    PointsetArgs p;
    int st = validate_pointset(ps, &p);
    if (st) return st;
    if (!k || k->kind != p.kind || k->d != p.d || !k->alpha || !k->gamma) return LDK_EINVAL;
    if (!(k->zeta > 0.0)) return LDK_EINVAL;
    if (dtype != LDK_F64 && dtype != LDK_F32) return LDK_EINVAL;
    if (n_min < 0 || n_max < n_min) return LDK_EINVAL;
    if (pts == nullptr) {
        const int64_t lim = (p.kind == LDK_LATTICE && p.order == LDK_NATURAL)
                                ? ((int64_t)1 << 62)
                                : ((int64_t)1 << p.m_max);
        if (n_max > lim) return LDK_EINVAL;
    } else if (x0 == nullptr && n_min != 0) {
        return LDK_EINVAL;  // the anchor must be given when row 0 is not point 0
    }
    if (n_max == n_min) return LDK_OK;  // empty window: out may be NULL
    if (!out) return LDK_EINVAL;
    const int64_t tiles = (n_max - n_min + KC_THREADS * KC_ITERS - 1) / (KC_THREADS * KC_ITERS);
    if (tiles > 0x7fffffff) return LDK_ENOTSUP;
    KcolArgs a{p, k->alpha, k->gamma, k->zeta, n_min, n_max, pts, x0};
    dim3 grid((unsigned)tiles, (unsigned)p.R);
    if (dtype == LDK_F64)
        hipLaunchKernelGGL(k_kernel_column<double>, grid, dim3(KC_THREADS), 0, as_stream(stream), a,
                           (double *)out);
    else
        hipLaunchKernelGGL(k_kernel_column<float>, grid, dim3(KC_THREADS), 0, as_stream(stream), a,
                           (float *)out);
    LDK_LAUNCH_CHECK();
    return LDK_OK;
}
