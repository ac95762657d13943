// Gradient of sum_i a_i k1_i in the kernel's parameters, the last step of the
// marginal-likelihood gradient (a = dL/dk1):
//   d k1_i / d log gamma_j = zeta t_ij prod_{l != j} f_il,   t = gamma K, f = 1 + t,
//   d k1_i / d log zeta    = k1_i = zeta prod_l f_il.
// ALU-bound like the kernel column.  Each block takes KC_TILE points of one
// replication and sweeps the dimensions twice: the first sweep forms every
// point's product of nonzero factors P and counts its exact zeros; the second
// re-evaluates t_ij and takes the product of the other factors as P / f_ij
// (no zero), P (the one zero is f_ij) or 0.  Per dimension, the point sum is
// reduced across the wavefront in FP64 and parked in lane j mod 64; every 64
// dimensions the block adds its waves in LDS and writes one partial per tile,
// and a second kernel adds the tiles in a fixed order.  Given the forward
// column k1 (formed by the kernel column from bit-identical factors), the
// first sweep is skipped: the product of the other factors is k1_i / f_ij.
#include "kfactor.hpp"

namespace ldk {

namespace {
constexpr int KG_WAVES = KC_THREADS / 64;

struct KgradArgs {
    KcolArgs k;
    const double *a;  // [R][cnt], dL/dk1
    const void *k1;   // [R][cnt] forward column (kernel-column dtype), or nullptr
    double *part;     // [R][tiles][d + 1]
    int64_t tile_base;
    int64_t tiles;
};

// One DPP lane move of a double (both halves), lanes the control leaves
// unwritten read 0.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_move(double v)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROW_MASK, 0xf,
                                               false);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Sum of v over the wavefront in a fixed order, returned in every lane.
// Lane moves go through DPP (no LDS round trips): swap neighbours, swap
// pairs, mirror within 8 and within 16 lanes (every lane of a row of 16 then
// holds the row's sum), then lane 15 of a row is added into the next row and
// lane 31 into the upper half; lane 63 ends with the total.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_move<0xb1>(v);        // quad_perm [1,0,3,2]
    v += dpp_move<0x4e>(v);        // quad_perm [2,3,0,1]
    v += dpp_move<0x141>(v);       // row_half_mirror
    v += dpp_move<0x140>(v);       // row_mirror
    v += dpp_move<0x142, 0xa>(v);  // row_bcast15 into rows 1 and 3
    v += dpp_move<0x143, 0xc>(v);  // row_bcast31 into rows 2 and 3
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Product of the other factors, P / f: FP32 multiplies by the hardware
// reciprocal (1 ulp; |f| is 0, which never reaches here, or far above the
// range where the reciprocal overflows), FP64 takes the correctly rounded
// quotient.
__device__ __forceinline__ float quot(float p, float f) { return p * __builtin_amdgcn_rcpf(f); }
__device__ __forceinline__ double quot(double p, double f) { return p / f; }

// ---- dimension sweeps: call visit(j, t[KC_ITERS], f[KC_ITERS]) for j = 0 .. d-1
// in order, t[l] = gamma_j K_j(delta) and f[l] = 1 + t[l] of point
// tile0 + threadIdx.x + KC_THREADS l, f formed exactly as the kernel column
// forms it ----

template <typename R, int ALPHA, int ORDER, typename Visit>
__device__ __forceinline__ void lattice_sweep(const KcolArgs &a, int64_t first, Visit &&visit)
{
    static_assert(KC_ITERS == 8 && KC_LOG_THREADS == 8, "offset table assumes 8 x 256");
    constexpr uint64_t br3[8] = {0, 4, 2, 6, 1, 5, 3, 7};
    const int d = a.ps.d, m = a.ps.m_max;
    const uint64_t bfirst = ORDER == LDK_NATURAL ? brev64((uint64_t)first) : (uint64_t)first;
    for (int j = 0; j < d; ++j) {
        const uint64_t g = a.ps.gen[j];
        const int alpha = ALPHA ? ALPHA : alpha_of(a, j);
        const SiPoly cf = si_tpoly(alpha, a.gamma[j]);
        const R e0 = (R)cf.c0, c1 = (R)cf.c1, c2 = (R)cf.c2, c3 = (R)cf.c3;
        const R c0 = (R)si_poly(alpha, a.gamma[j]).c0;
        uint64_t base, G;
        if constexpr (ORDER == LDK_NATURAL) {
            base = bfirst * g;
            G = g << 53;
        } else {
            base = m == 0 ? 0 : ((bfirst * g) << (64 - m));
            G = m <= 8 ? 0 : ((g << 8) << (64 - m));
        }
        R t[KC_ITERS], f[KC_ITERS];
        const R lo_p = lo_part<R>((uint32_t)base);  // shared low half (natural order)
#pragma unroll
        for (int l = 0; l < KC_ITERS; ++l) {
            R x;
            if constexpr (ORDER == LDK_NATURAL)
                x = unit_hl<R>((uint32_t)(base >> 32) + (uint32_t)br3[l] * (uint32_t)(G >> 32), lo_p);
            else
                x = unit<R>(base + (uint64_t)l * G);
            t[l] = si_weighted<R, ALPHA>(x, e0, c1, c2, c3);
            f[l] = si_weighted<R, ALPHA>(x, c0, c1, c2, c3);
        }
        visit(j, t, f);
    }
}

template <typename R, int ALPHA, typename Visit>
__device__ __forceinline__ void net_sweep(const KcolArgs &a, NetLds &L, int r, int64_t tile0,
                                          Visit &&visit)
{
    constexpr int s = KC_LOG_THREADS;
    const int d = a.ps.d, t = threadIdx.x;
    const bool gray = a.ps.order == LDK_GRAY;
    const uint64_t code_tile = gray ? gray_code((uint64_t)tile0) : (uint64_t)tile0;
    const uint32_t code_t = gray ? (uint32_t)gray_code((uint64_t)t) : (uint32_t)t;
    for (int jc = 0; jc < d; jc += KC_DIM_CHUNK) {
        const int DB = min(KC_DIM_CHUNK, d - jc);
        build_net_chunk(a, L, r, jc, DB, code_tile);
        for (int jj = 0; jj < DB; ++jj) {
            const int j = jc + jj;
            const R gam = (R)a.gamma[j];
            const int alpha = ALPHA ? ALPHA : alpha_of(a, j);
            uint64_t z = L.zb[jj] ^ L.nib[jj][0][code_t & 15] ^ L.nib[jj][1][(code_t >> 4) & 15];
            R tv[KC_ITERS], fv[KC_ITERS];
#pragma unroll
            for (int l = 0; l < KC_ITERS; ++l) {
                R k;
                if constexpr (ALPHA != 0)
                    k = dsi_factor<R, ALPHA>(z, L.tab);
                else
                    k = dsi_factor_any<R>(alpha, z, L.tab);
                tv[l] = gam * k;
                fv[l] = dsi_weighted(gam, k);
                // step to the next point; past the last index of the net the
                // step columns are zero and z just repeats (such points are
                // masked), so the step needs no bounds test
                const uint64_t nb = ((uint64_t)tile0 >> s) + (uint64_t)l + 1;
                if (l + 1 < KC_ITERS) z ^= L.step[jj][ctz64(nb)];
            }
            visit(j, tv, fv);
        }
    }
}

// Points read from memory (any order; anchors x0 or row 0).
template <typename R, bool NET, typename Visit>
__device__ __forceinline__ void points_sweep(const KcolArgs &a, const DsiTables &tab, int r,
                                             int64_t first, Visit &&visit)
{
    const int d = a.ps.d;
    const int64_t cnt = a.n_max - a.n_min;
    for (int j = 0; j < d; ++j) {
        const uint64_t u0 = a.x0 ? a.x0[(size_t)r * d + j] : a.pts[(size_t)r * cnt * d + j];
        const int alpha = alpha_of(a, j);
        const SiPoly cf = NET ? SiPoly{} : si_tpoly(alpha, a.gamma[j]);
        const R c0 = NET ? (R)1 : (R)si_poly(alpha, a.gamma[j]).c0;
        R t[KC_ITERS], f[KC_ITERS];
#pragma unroll
        for (int l = 0; l < KC_ITERS; ++l) {
            int64_t i = first + (int64_t)l * KC_THREADS;
            if (i >= a.n_max) i = a.n_max - 1;  // any valid row; masked out later
            const uint64_t u = a.pts[((size_t)r * cnt + (i - a.n_min)) * d + j];
            if constexpr (NET) {
                const R gam = (R)a.gamma[j];
                const R k = dsi_factor_any<R>(alpha, u ^ u0, tab);
                t[l] = gam * k;
                f[l] = dsi_weighted(gam, k);
            } else {
                const R x = unit<R>(u - u0);
                t[l] = si_weighted<R, 0>(x, (R)cf.c0, (R)cf.c1, (R)cf.c2, (R)cf.c3);
                f[l] = si_weighted<R, 0>(x, c0, (R)cf.c1, (R)cf.c2, (R)cf.c3);
            }
        }
        visit(j, t, f);
    }
}

// Source selector: SRC 0 lattice natural, 1 lattice linear, 2 net, 3 points
// (lattice), 4 points (net).
template <typename R, int ALPHA, int SRC, typename Visit>
__device__ __forceinline__ void sweep(const KcolArgs &a, NetLds &L, int r, int64_t tile0,
                                      int64_t first, Visit &&visit)
{
    if constexpr (SRC == 0) lattice_sweep<R, ALPHA, LDK_NATURAL>(a, first, visit);
    else if constexpr (SRC == 1) lattice_sweep<R, ALPHA, LDK_LINEAR>(a, first, visit);
    else if constexpr (SRC == 2) net_sweep<R, ALPHA>(a, L, r, tile0, visit);
    else points_sweep<R, SRC == 4>(a, L.tab, r, first, visit);
}

template <typename R, int ALPHA, int SRC, bool K1>
__global__ __launch_bounds__(KC_THREADS) void k_kernel_grad(KgradArgs g)
{
    __shared__ NetLds L;
    __shared__ double red[KG_WAVES][64];
    const KcolArgs &a = g.k;
    const int r = blockIdx.y, d = a.ps.d;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t cnt = a.n_max - a.n_min;
    const int64_t tile0 = g.tile_base + (int64_t)blockIdx.x * KC_TILE;
    const int64_t first = tile0 + threadIdx.x;
    if constexpr (SRC >= 2) {
        fill_dsi_tables(L.tab, threadIdx.x, KC_THREADS);
        __syncthreads();
    }
    R pnz[KC_ITERS], av[KC_ITERS];
    int nz[KC_ITERS];
    uint32_t valid = 0;
#pragma unroll
    for (int l = 0; l < KC_ITERS; ++l) {
        const int64_t i = first + (int64_t)l * KC_THREADS;
        const bool in = i >= a.n_min && i < a.n_max;
        valid |= (uint32_t)in << l;
        av[l] = in ? (R)g.a[(size_t)r * cnt + (i - a.n_min)] : (R)0;
        pnz[l] = (R)1;
        nz[l] = 0;
    }
    // With the forward column given, k1_i = zeta prod_l f_il already holds
    // the product, formed from the same factors bit for bit, so one sweep
    // suffices: zeta t_ij prod_{l != j} f_il = t_ij (k1_i / f_ij).  A block
    // with a zero k1_i (a zero factor, or underflow) takes the two sweeps.
    bool from_k1 = false;
    if constexpr (K1) {
        int zero = 0;
#pragma unroll
        for (int l = 0; l < KC_ITERS; ++l) {
            const int64_t i = first + (int64_t)l * KC_THREADS;
            if ((valid >> l) & 1u) {
                pnz[l] = static_cast<const R *>(g.k1)[(size_t)r * cnt + (i - a.n_min)];
                zero |= pnz[l] == (R)0;
            }
        }
        from_k1 = !__syncthreads_or(zero);
        if (!from_k1) {
#pragma unroll
            for (int l = 0; l < KC_ITERS; ++l) pnz[l] = (R)1;
        }
    }
    if (!from_k1) {
        // sweep 1: product of the nonzero factors and the number of zero factors
        sweep<R, ALPHA, SRC>(a, L, r, tile0, first,
                             [&](int, const R(&)[KC_ITERS], const R(&f)[KC_ITERS]) {
#pragma unroll
            for (int l = 0; l < KC_ITERS; ++l) {
                if (f[l] == (R)0) ++nz[l];
                else pnz[l] *= f[l];
            }
        });
    }
    // pnz already carries zeta when it came from k1
    const double zf = from_k1 ? 1.0 : a.zeta;
    double *part = g.part + ((size_t)r * g.tiles + blockIdx.x) * (d + 1);
    {
        // d/dlog zeta: sum_i a_i k1_i
        R zs = (R)0;
#pragma unroll
        for (int l = 0; l < KC_ITERS; ++l)
            if (((valid >> l) & 1u) && nz[l] == 0) zs += av[l] * pnz[l];
        const double w = wave_sum((double)zs * zf);
        if (lane == 0) red[wave][0] = w;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int q = 0; q < KG_WAVES; ++q) s += red[q][0];
            part[d] = s;
        }
        __syncthreads();
    }
    // sweep 2: t_ij times the product of the other factors
    double acc = 0.0;
    auto emit = [&](int j, R ps) {
        const double w = wave_sum((double)ps * zf);
        if ((j & 63) == lane) acc = w;
        if ((j & 63) == 63 || j == d - 1) {
            // block-uniform: every thread reaches these barriers
            const int j0 = j & ~63;
            red[wave][lane] = acc;
            __syncthreads();
            if (threadIdx.x < 64 && j0 + (int)threadIdx.x <= j) {
                double s = 0.0;
                for (int q = 0; q < KG_WAVES; ++q) s += red[q][threadIdx.x];
                part[j0 + threadIdx.x] = s;
            }
            __syncthreads();
        }
    };
    if (K1 && from_k1) {
        // no zero factor at any valid point of the tile
        sweep<R, ALPHA, SRC>(a, L, r, tile0, first,
                             [&](int j, const R(&t)[KC_ITERS], const R(&f)[KC_ITERS]) {
            R ps = (R)0;
#pragma unroll
            for (int l = 0; l < KC_ITERS; ++l) {
                const R c = av[l] * (t[l] * quot(pnz[l], f[l]));
                ps += ((valid >> l) & 1u) ? c : (R)0;
            }
            emit(j, ps);
        });
    } else {
        sweep<R, ALPHA, SRC>(a, L, r, tile0, first,
                             [&](int j, const R(&t)[KC_ITERS], const R(&f)[KC_ITERS]) {
            R ps = (R)0;
#pragma unroll
            for (int l = 0; l < KC_ITERS; ++l) {
                const R q = quot(pnz[l], f[l]);
                const R one_zero = (nz[l] == 1 && f[l] == (R)0) ? pnz[l] : (R)0;
                const R other = nz[l] == 0 ? q : one_zero;
                const R c = av[l] * (t[l] * other);
                ps += ((valid >> l) & 1u) ? c : (R)0;
            }
            emit(j, ps);
        });
    }
}

// grad[r][j] = sum over tiles of the partials, in a fixed order (four
// interleaved accumulators, combined in a fixed order).
__global__ __launch_bounds__(256) void k_grad_final(const double *__restrict__ part, int64_t tiles,
                                                    int d, double *__restrict__ grad)
{
    const int r = blockIdx.y;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j > d) return;
    const size_t stride = (size_t)(d + 1);
    const double *p = part + (size_t)r * tiles * stride + j;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t q = 0;
    for (; q + 4 <= tiles; q += 4) {
        s0 += p[(size_t)q * stride];
        s1 += p[(size_t)(q + 1) * stride];
        s2 += p[(size_t)(q + 2) * stride];
        s3 += p[(size_t)(q + 3) * stride];
    }
    for (; q < tiles; ++q) s0 += p[(size_t)q * stride];
    grad[(size_t)r * (d + 1) + j] = (s0 + s1) + (s2 + s3);
}

template <typename R, int ALPHA, int SRC>
void launch_grad_k1(const KgradArgs &g, dim3 grid, hipStream_t s)
{
    if (g.k1) hipLaunchKernelGGL((k_kernel_grad<R, ALPHA, SRC, true>), grid, dim3(KC_THREADS), 0, s, g);
    else hipLaunchKernelGGL((k_kernel_grad<R, ALPHA, SRC, false>), grid, dim3(KC_THREADS), 0, s, g);
}

template <typename R, int ALPHA>
void launch_grad_src(int src, const KgradArgs &g, dim3 grid, hipStream_t s)
{
    switch (src) {
    case 0: launch_grad_k1<R, ALPHA, 0>(g, grid, s); break;
    case 1: launch_grad_k1<R, ALPHA, 1>(g, grid, s); break;
    default: launch_grad_k1<R, ALPHA, 2>(g, grid, s); break;
    }
}

template <typename R>
void launch_grad(int src, int uniform, const KgradArgs &g, dim3 grid, hipStream_t s)
{
    if (src >= 3) {  // points given: generic orders
        if (src == 3) launch_grad_k1<R, 0, 3>(g, grid, s);
        else launch_grad_k1<R, 0, 4>(g, grid, s);
        return;
    }
    switch (uniform) {
    case 1: launch_grad_src<R, 1>(src, g, grid, s); break;
    case 2: launch_grad_src<R, 2>(src, g, grid, s); break;
    case 3: launch_grad_src<R, 3>(src, g, grid, s); break;
    case 4:
        if (src == 2) {
            launch_grad_k1<R, 4, 2>(g, grid, s);
            break;
        }
        [[fallthrough]];
    default: launch_grad_src<R, 0>(src, g, grid, s);
    }
}

// Tiles of KC_TILE points covering [n_min, n_max): aligned to absolute
// multiples of KC_TILE when regenerating, from n_min when points are given.
void grad_tiles(bool given, int64_t n_min, int64_t n_max, int64_t *base, int64_t *tiles)
{
    *base = given ? n_min : (n_min / KC_TILE) * KC_TILE;
    *tiles = (n_max - *base + KC_TILE - 1) / KC_TILE;
}

}  // namespace

}  // namespace ldk

using namespace ldk;

extern "C" size_t ldk_kernel_grad_workspace_bytes(int R, int d, int64_t n_min, int64_t n_max,
                                                  int points_given)
{
    if (R < 1 || d < 1 || d > LDK_MAX_D || n_min < 0 || n_max < n_min) return 0;
    int64_t base, tiles;
    grad_tiles(points_given != 0, n_min, n_max, &base, &tiles);
    return (size_t)R * (size_t)tiles * (size_t)(d + 1) * sizeof(double);
}

extern "C" int ldk_kernel_grad(const ldk_kernel *k, const ldk_pointset *ps, const uint64_t *pts,
                               const uint64_t *x0, int64_t n_min, int64_t n_max, int dtype,
                               const void *k1, const double *a, double *grad, void *ws,
                               ldk_stream stream)
{
    KgradArgs g{};
    int uniform = 0;
    const int st = prepare_kernel_args(k, ps, pts, x0, n_min, n_max, dtype, &g.k, &uniform);
    if (st) return st;
    const PointsetArgs &p = g.k.ps;
    if (!grad) return LDK_EINVAL;
    hipStream_t s = as_stream(stream);
    if (n_max == n_min) {
        // empty window: every sum is zero
        hipLaunchKernelGGL(k_grad_final, dim3((p.d + 1 + 255) / 256, p.R), dim3(256), 0, s,
                           (const double *)nullptr, (int64_t)0, p.d, grad);
        LDK_LAUNCH_CHECK();
        return LDK_OK;
    }
    if (!a || !ws) return LDK_EINVAL;
    const bool given = pts != nullptr;
    grad_tiles(given, n_min, n_max, &g.tile_base, &g.tiles);
    if (g.tiles > 0x7fffffff) return LDK_ENOTSUP;
    g.a = a;
    g.k1 = k1;
    g.part = static_cast<double *>(ws);
    const int src = given ? (p.kind == LDK_DNET_B2 ? 4 : 3)
                          : (p.kind == LDK_DNET_B2 ? 2 : (p.order == LDK_LINEAR ? 1 : 0));
    const dim3 grid((unsigned)g.tiles, (unsigned)p.R);
    if (dtype == LDK_F64) launch_grad<double>(src, uniform, g, grid, s);
    else launch_grad<float>(src, uniform, g, grid, s);
    LDK_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_grad_final, dim3((p.d + 1 + 255) / 256, p.R), dim3(256), 0, s,
                       (const double *)g.part, g.tiles, p.d, grad);
    LDK_LAUNCH_CHECK();
    return LDK_OK;
}
