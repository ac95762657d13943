// First column of the product-weight Gram matrix,
//   k1_i = zeta prod_j (1 + gamma_j K_{alpha_j}(x_ij (-) x0_j)),
// with SI factors (Sec. 5.2, Bernoulli polynomials) for lattices and DSI
// factors (Sec. 5.3, Theorem 1) for base-2 digital nets.  This op is
// ALU-bound: the points are either read once or regenerated in registers.
#include <type_traits>

#include "kfactor.hpp"

namespace ldk {

// ---------------------------------------------------------------------------
// Regenerating lattice variant.  Block: replication r = blockIdx.y; points
// i = tile0 + t + KC_THREADS l (l < KC_ITERS), tile0 a multiple of KC_TILE,
// so the bits of t, l and tile0 are disjoint and
//   natural: bitreverse(i) g = bitreverse(tile0 + t) g + bitreverse3(l) (g << 53),
//   linear:  (i g) << (64-m) = ((tile0 + t) g) << (64-m) + l ((g << 8) << (64-m)).
// The anchor is point 0, so delta = z(i) - z(0) = z(i): the shift cancels.
// ---------------------------------------------------------------------------
template <typename R, int ALPHA, int ORDER, bool FULL>
__device__ __forceinline__ void lattice_tile(const KcolArgs &a, int64_t first, R (&prod)[KC_ITERS])
{
    static_assert(KC_ITERS == 8 && KC_LOG_THREADS == 8, "offset table assumes 8 x 256");
    constexpr uint64_t br3[8] = {0, 4, 2, 6, 1, 5, 3, 7};
    const int d = a.ps.d, m = a.ps.m_max;
    const uint64_t bfirst = ORDER == LDK_NATURAL ? brev64((uint64_t)first) : (uint64_t)first;
    for (int j = 0; j < d; ++j) {
        const uint64_t g = a.ps.gen[j];
        const int alpha = ALPHA ? ALPHA : alpha_of(a, j);
        const SiPoly cf = si_poly(alpha, a.gamma[j]);
        const R c0 = (R)cf.c0, c1 = (R)cf.c1, c2 = (R)cf.c2, c3 = (R)cf.c3;
        uint64_t base, G;
        if constexpr (ORDER == LDK_NATURAL) {
            base = bfirst * g;
            G = g << 53;
        } else {
            base = m == 0 ? 0 : ((bfirst * g) << (64 - m));
            G = m <= 8 ? 0 : ((g << 8) << (64 - m));
        }
        // natural order: G has no low-half bits, so the points of a thread
        // share the low half of delta and differ in the high half only
        const R lo_p = lo_part<R>((uint32_t)base);
#pragma unroll
        for (int l = 0; l < KC_ITERS; ++l) {
            R x;
            if constexpr (ORDER == LDK_NATURAL)
                x = unit_hl<R>((uint32_t)(base >> 32) + (uint32_t)br3[l] * (uint32_t)(G >> 32), lo_p);
            else
                x = unit<R>(base + (uint64_t)l * G);
            const R f = si_weighted<R, ALPHA>(x, c0, c1, c2, c3);
            if (FULL) {
                prod[l] *= f;
            } else {
                const int64_t i = first + (int64_t)l * KC_THREADS;
                if (i >= a.n_min && i < a.n_max) prod[l] *= f;
            }
        }
    }
}

// Column tile bx of replication r (KC_TILE points from tile_base + bx KC_TILE).
template <typename R, int ALPHA, int ORDER>
__device__ __forceinline__ void kcol_lattice_block(const KcolArgs &a, int64_t tile_base,
                                                   R *__restrict__ out, int64_t bx, int r)
{
    const int64_t cnt = a.n_max - a.n_min;
    const int64_t tile0 = tile_base + bx * KC_TILE;
    const int64_t first = tile0 + threadIdx.x;
    R prod[KC_ITERS];
#pragma unroll
    for (int l = 0; l < KC_ITERS; ++l) prod[l] = (R)a.zeta;
    if (tile0 >= a.n_min && tile0 + KC_TILE <= a.n_max)
        lattice_tile<R, ALPHA, ORDER, true>(a, first, prod);
    else
        lattice_tile<R, ALPHA, ORDER, false>(a, first, prod);
#pragma unroll
    for (int l = 0; l < KC_ITERS; ++l) {
        const int64_t i = first + (int64_t)l * KC_THREADS;
        if (i >= a.n_min && i < a.n_max) out[(size_t)r * cnt + (i - a.n_min)] = prod[l];
    }
}

template <typename R, int ALPHA, int ORDER>
__global__ __launch_bounds__(KC_THREADS) void k_kcol_lattice(KcolArgs a, int64_t tile_base,
                                                            R *__restrict__ out)
{
    kcol_lattice_block<R, ALPHA, ORDER>(a, tile_base, out, blockIdx.x, blockIdx.y);
}

// Point words and first column of a lattice in one launch.  The column
// regenerates the points in registers and never reads the words, so the
// two halves are independent: column tiles (VALU bound) and point-word
// tiles (store bound).  The column tiles are spread evenly over the block
// indices (one per ~8 point tiles at n = 2^20, d = 32), so every stretch of
// the launch mixes the two and the column's arithmetic runs beside the
// stores, instead of after 256 MiB of stores (two launches), before them
// (column blocks first: 52 us against 48 here), or not at all beside them
// (two streams: the point launch takes every slot).
static_assert(GEN_THREADS == KC_THREADS, "one block shape for both halves");
template <typename R, int ALPHA, int ORDER>
__global__ __launch_bounds__(KC_THREADS) void k_points_kcol_lattice(KcolArgs a, int64_t tile_base,
                                                                   int64_t kc_tiles,
                                                                   R *__restrict__ k1, GenGrid g,
                                                                   uint64_t *__restrict__ pts)
{
    const int64_t b = blockIdx.x;
    const int64_t kc_blocks = kc_tiles * a.ps.R;
    const int64_t total = kc_blocks + g.tiles * g.chunks * g.R;
    // column blocks spread evenly over the grid: block b is one iff the
    // count floor((b+1) kc / total) of column blocks up to b steps at b
    const int64_t before = b * kc_blocks / total, upto = (b + 1) * kc_blocks / total;
    if (upto != before) {
        kcol_lattice_block<R, ALPHA, ORDER>(a, tile_base, k1, before % kc_tiles,
                                            (int)(before / kc_tiles));
        return;
    }
    const int64_t q = b - upto;
    gen_lattice_block<ORDER>(a.ps, a.n_min, a.n_max, g.P, g.pairs != 0, pts, q % g.tiles,
                             (int)((q / g.tiles) % g.chunks), (int)(q / (g.tiles * g.chunks)),
                             threadIdx.x);
}

// ---------------------------------------------------------------------------
// Regenerating net variant.  The scrambled columns of a chunk of dimensions
// sit in LDS (built from S rows staged in LDS); the step from point
// i = tile0 + t + KC_THREADS l to the next one flips index bits
// s .. s + ctz((tile0 >> s) + l + 1) (s = log2 KC_THREADS), a block-uniform
// table read.  The anchor is point 0 (z = 0), so delta = z(i).
// ---------------------------------------------------------------------------
template <typename R, int ALPHA, bool FULL>
__device__ __forceinline__ void net_tile(const KcolArgs &a, NetLds &L, int r, int64_t tile0,
                                         int64_t first, R (&prod)[KC_ITERS])
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
#pragma unroll
            for (int l = 0; l < KC_ITERS; ++l) {
                R k;
                if constexpr (ALPHA != 0)
                    k = dsi_factor<R, ALPHA>(z, L.tab);
                else
                    k = dsi_factor_any<R>(alpha, z, L.tab);
                const R f = dsi_weighted(gam, k);
                if (FULL) {
                    prod[l] *= f;
                } else {
                    const int64_t i = first + (int64_t)l * KC_THREADS;
                    if (i >= a.n_min && i < a.n_max) prod[l] *= f;
                }
                // step to the next point; past the last index of the net the
                // step columns are zero and z just repeats (such points are
                // masked), so the step needs no bounds test
                const uint64_t nb = ((uint64_t)tile0 >> s) + (uint64_t)l + 1;
                if (l + 1 < KC_ITERS) z ^= L.step[jj][ctz64(nb)];
            }
        }
    }
}

// Column tile bx of replication r of a net (every thread of the block calls it).
template <typename R, int ALPHA>
__device__ __forceinline__ void kcol_net_block(const KcolArgs &a, NetLds &L, int64_t tile_base,
                                               R *__restrict__ out, int64_t bx, int r)
{
    const int64_t cnt = a.n_max - a.n_min;
    const int64_t tile0 = tile_base + bx * KC_TILE;
    const int64_t first = tile0 + threadIdx.x;
    fill_dsi_tables(L.tab, threadIdx.x, KC_THREADS);
    R prod[KC_ITERS];
#pragma unroll
    for (int l = 0; l < KC_ITERS; ++l) prod[l] = (R)a.zeta;
    if (tile0 >= a.n_min && tile0 + KC_TILE <= a.n_max)
        net_tile<R, ALPHA, true>(a, L, r, tile0, first, prod);
    else
        net_tile<R, ALPHA, false>(a, L, r, tile0, first, prod);
#pragma unroll
    for (int l = 0; l < KC_ITERS; ++l) {
        const int64_t i = first + (int64_t)l * KC_THREADS;
        if (i >= a.n_min && i < a.n_max) out[(size_t)r * cnt + (i - a.n_min)] = prod[l];
    }
}

template <typename R, int ALPHA>
__global__ __launch_bounds__(KC_THREADS) void k_kcol_net(KcolArgs a, int64_t tile_base,
                                                        R *__restrict__ out)
{
    __shared__ NetLds L;
    kcol_net_block<R, ALPHA>(a, L, tile_base, out, blockIdx.x, blockIdx.y);
}

// Point words and first column of a net in one launch: column blocks and
// point-word blocks interleaved as for lattices (the column regenerates the
// points and never reads the words), one LDS region shared by the two
// block kinds.
template <typename R, int ALPHA>
__global__ __launch_bounds__(KC_THREADS) void k_points_kcol_net(KcolArgs a, int64_t tile_base,
                                                               int64_t kc_tiles, R *__restrict__ k1,
                                                               GenGrid g, uint64_t *__restrict__ pts)
{
    __shared__ union {
        NetLds k;
        GenNetLds g;
    } L;
    const int64_t b = blockIdx.x;
    const int64_t kc_blocks = kc_tiles * a.ps.R;
    const int64_t total = kc_blocks + g.tiles * g.chunks * g.R;
    const int64_t before = b * kc_blocks / total, upto = (b + 1) * kc_blocks / total;
    if (upto != before) {
        kcol_net_block<R, ALPHA>(a, L.k, tile_base, k1, before % kc_tiles, (int)(before / kc_tiles));
        return;
    }
    const int64_t q = b - upto;
    gen_net_block(a.ps, a.n_min, a.n_max, g.tile_base, g.P, g.logP, g.pairs, pts, q % g.tiles,
                  (int)((q / g.tiles) % g.chunks), (int)(q / (g.tiles * g.chunks)), threadIdx.x, L.g);
}

// ---------------------------------------------------------------------------
// Points given (any order; anchor rows x0).  Thread per point.
// ---------------------------------------------------------------------------
template <typename R, bool NET>
__global__ __launch_bounds__(KC_THREADS) void k_kcol_points(KcolArgs a, R *__restrict__ out)
{
    __shared__ DsiTables tab;
    if constexpr (NET) {
        fill_dsi_tables(tab, threadIdx.x, KC_THREADS);
        __syncthreads();
    }
    const int r = blockIdx.y;
    const int d = a.ps.d;
    const int64_t cnt = a.n_max - a.n_min;
    const int64_t i = a.n_min + (int64_t)blockIdx.x * KC_THREADS + threadIdx.x;
    if (i >= a.n_max) return;
    const uint64_t *row = a.pts + ((size_t)r * cnt + (i - a.n_min)) * d;
    R prod = (R)a.zeta;
    for (int j = 0; j < d; ++j) {
        const uint64_t u0 = a.x0 ? a.x0[(size_t)r * d + j] : a.pts[(size_t)r * cnt * d + j];
        const int alpha = alpha_of(a, j);
        if constexpr (NET) {
            prod *= dsi_weighted((R)a.gamma[j], dsi_factor_any<R>(alpha, row[j] ^ u0, tab));
        } else {
            const SiPoly cf = si_poly(alpha, a.gamma[j]);
            prod *= si_weighted<R, 0>(unit<R>(row[j] - u0), (R)cf.c0, (R)cf.c1, (R)cf.c2, (R)cf.c3);
        }
    }
    out[(size_t)r * cnt + (i - a.n_min)] = prod;
}

template <typename R, int ALPHA>
void launch_regen(const KcolArgs &a, int64_t tile_base, dim3 grid, hipStream_t s, void *out)
{
    if (a.ps.kind == LDK_DNET_B2)
        hipLaunchKernelGGL((k_kcol_net<R, ALPHA>), grid, dim3(KC_THREADS), 0, s, a, tile_base, (R *)out);
    else if (a.ps.order == LDK_LINEAR)
        hipLaunchKernelGGL((k_kcol_lattice<R, ALPHA, LDK_LINEAR>), grid, dim3(KC_THREADS), 0, s, a,
                           tile_base, (R *)out);
    else
        hipLaunchKernelGGL((k_kcol_lattice<R, ALPHA, LDK_NATURAL>), grid, dim3(KC_THREADS), 0, s, a,
                           tile_base, (R *)out);
}

template <typename R, int ALPHA>
void launch_points_kcol(const KcolArgs &a, int64_t tile_base, int64_t kc_tiles, const GenGrid &g,
                        unsigned blocks, hipStream_t s, void *k1, uint64_t *pts)
{
    if (a.ps.kind == LDK_DNET_B2)
        hipLaunchKernelGGL((k_points_kcol_net<R, ALPHA>), dim3(blocks), dim3(KC_THREADS), 0, s, a,
                           tile_base, kc_tiles, (R *)k1, g, pts);
    else if (a.ps.order == LDK_LINEAR)
        hipLaunchKernelGGL((k_points_kcol_lattice<R, ALPHA, LDK_LINEAR>), dim3(blocks),
                           dim3(KC_THREADS), 0, s, a, tile_base, kc_tiles, (R *)k1, g, pts);
    else
        hipLaunchKernelGGL((k_points_kcol_lattice<R, ALPHA, LDK_NATURAL>), dim3(blocks),
                           dim3(KC_THREADS), 0, s, a, tile_base, kc_tiles, (R *)k1, g, pts);
}

template <typename R>
void launch_points_kcol_alpha(int alpha, const KcolArgs &a, int64_t tile_base, int64_t kc_tiles,
                              const GenGrid &g, unsigned blocks, hipStream_t s, void *k1,
                              uint64_t *pts)
{
    switch (alpha) {  // lattice orders 1..3 and net orders 1..4; mixed orders 0
    case 1: launch_points_kcol<R, 1>(a, tile_base, kc_tiles, g, blocks, s, k1, pts); break;
    case 2: launch_points_kcol<R, 2>(a, tile_base, kc_tiles, g, blocks, s, k1, pts); break;
    case 3: launch_points_kcol<R, 3>(a, tile_base, kc_tiles, g, blocks, s, k1, pts); break;
    case 4:
        if (a.ps.kind == LDK_DNET_B2) {
            hipLaunchKernelGGL((k_points_kcol_net<R, 4>), dim3(blocks), dim3(KC_THREADS), 0, s, a,
                               tile_base, kc_tiles, (R *)k1, g, pts);
            break;
        }
        [[fallthrough]];
    default: launch_points_kcol<R, 0>(a, tile_base, kc_tiles, g, blocks, s, k1, pts);
    }
}

template <typename R>
void launch_regen_alpha(int kind, int alpha, const KcolArgs &a, int64_t tile_base, dim3 grid,
                        hipStream_t s, void *out)
{
    // lattice orders 1..3 and net orders 1..4 get specialised kernels; mixed
    // orders (alpha = 0) read the per-dimension code
    switch (alpha) {
    case 1: launch_regen<R, 1>(a, tile_base, grid, s, out); break;
    case 2: launch_regen<R, 2>(a, tile_base, grid, s, out); break;
    case 3: launch_regen<R, 3>(a, tile_base, grid, s, out); break;
    case 4:
        if (kind == LDK_DNET_B2) {
            hipLaunchKernelGGL((k_kcol_net<R, 4>), grid, dim3(KC_THREADS), 0, s, a, tile_base, (R *)out);
            break;
        }
        [[fallthrough]];
    default: launch_regen<R, 0>(a, tile_base, grid, s, out);
    }
}

}  // namespace ldk

using namespace ldk;

namespace ldk {

int prepare_kernel_args(const ldk_kernel *k, const ldk_pointset *ps, const uint64_t *pts,
                        const uint64_t *x0, int64_t n_min, int64_t n_max, int dtype, KcolArgs *out,
                        int *uniform_alpha)
{
    PointsetArgs p;
    int st = validate_pointset(ps, &p);
    if (st) return st;
    if (!k || k->kind != p.kind || k->d != p.d || !k->alpha || !k->gamma) return LDK_EINVAL;
    if (!(k->zeta > 0.0)) return LDK_EINVAL;
    if (dtype != LDK_F64 && dtype != LDK_F32) return LDK_EINVAL;
    if (n_min < 0 || n_max < n_min) return LDK_EINVAL;
    KcolArgs a{};
    a.ps = p;
    a.gamma = k->gamma;
    a.zeta = k->zeta;
    a.n_min = n_min;
    a.n_max = n_max;
    a.pts = pts;
    a.x0 = x0;
    // orders live on the host: validate, pack 2-bit codes, detect a uniform order
    const int amax = p.kind == LDK_LATTICE ? 3 : 4;
    int uniform = k->alpha[0];
    for (int j = 0; j < p.d; ++j) {
        const int al = k->alpha[j];
        if (al < 1 || al > amax) return LDK_EINVAL;
        if (al != uniform) uniform = 0;
        a.acode[j >> 5] |= (uint64_t)(al - 1) << (2 * (j & 31));
    }
    if (pts == nullptr) {
        const int64_t lim = (p.kind == LDK_LATTICE && p.order == LDK_NATURAL)
                                ? ((int64_t)1 << 62)
                                : ((int64_t)1 << p.m_max);
        if (n_max > lim) return LDK_EINVAL;
    } else if (x0 == nullptr && n_min != 0) {
        return LDK_EINVAL;  // the anchor must be given when row 0 is not point 0
    }
    *out = a;
    *uniform_alpha = uniform;
    return LDK_OK;
}

}  // namespace ldk

extern "C" int ldk_kernel_column(const ldk_kernel *k, const ldk_pointset *ps, const uint64_t *pts,
                                 const uint64_t *x0, int64_t n_min, int64_t n_max, int dtype,
                                 void *out, ldk_stream stream)
{
    KcolArgs a;
    int uniform = 0;
    const int st = prepare_kernel_args(k, ps, pts, x0, n_min, n_max, dtype, &a, &uniform);
    if (st) return st;
    const PointsetArgs &p = a.ps;
    if (n_max == n_min) return LDK_OK;  // empty window: out may be NULL
    if (!out) return LDK_EINVAL;
    hipStream_t s = as_stream(stream);
    if (pts != nullptr) {
        const int64_t blocks = (n_max - n_min + KC_THREADS - 1) / KC_THREADS;
        if (blocks > 0x7fffffff) return LDK_ENOTSUP;
        dim3 grid((unsigned)blocks, (unsigned)p.R);
        const bool net = p.kind == LDK_DNET_B2;
        if (dtype == LDK_F64) {
            if (net) hipLaunchKernelGGL((k_kcol_points<double, true>), grid, dim3(KC_THREADS), 0, s, a, (double *)out);
            else hipLaunchKernelGGL((k_kcol_points<double, false>), grid, dim3(KC_THREADS), 0, s, a, (double *)out);
        } else {
            if (net) hipLaunchKernelGGL((k_kcol_points<float, true>), grid, dim3(KC_THREADS), 0, s, a, (float *)out);
            else hipLaunchKernelGGL((k_kcol_points<float, false>), grid, dim3(KC_THREADS), 0, s, a, (float *)out);
        }
        LDK_LAUNCH_CHECK();
        return LDK_OK;
    }
    // tiles aligned to absolute multiples of KC_TILE
    const int64_t tile_base = (n_min / KC_TILE) * KC_TILE;
    const int64_t tiles = (n_max - tile_base + KC_TILE - 1) / KC_TILE;
    if (tiles > 0x7fffffff) return LDK_ENOTSUP;
    dim3 grid((unsigned)tiles, (unsigned)p.R);
    if (dtype == LDK_F64)
        launch_regen_alpha<double>(p.kind, uniform, a, tile_base, grid, s, out);
    else
        launch_regen_alpha<float>(p.kind, uniform, a, tile_base, grid, s, out);
    LDK_LAUNCH_CHECK();
    return LDK_OK;
}

extern "C" int ldk_points_column(const ldk_kernel *k, const ldk_pointset *ps, int64_t n_min,
                                 int64_t n_max, uint64_t *pts, int dtype, void *k1,
                                 ldk_stream stream)
{
    KcolArgs a;
    int uniform = 0;
    int st = prepare_kernel_args(k, ps, nullptr, nullptr, n_min, n_max, dtype, &a, &uniform);
    if (st) return st;
    const PointsetArgs &p = a.ps;
    const int64_t lim = (p.kind == LDK_LATTICE && p.order == LDK_NATURAL) ? ((int64_t)1 << 62)
                                                                          : ((int64_t)1 << p.m_max);
    if (n_min < 0 || n_max < n_min || n_max > lim) return LDK_EINVAL;
    if (n_max == n_min) return LDK_OK;  // empty window: the outputs may be NULL
    if (!pts || !k1) return LDK_EINVAL;
    const int64_t tile_base = (n_min / KC_TILE) * KC_TILE;
    const int64_t kc_tiles = (n_max - tile_base + KC_TILE - 1) / KC_TILE;
    const GenGrid g = gen_grid(p, n_min, n_max, pts);
    const int64_t blocks = kc_tiles * p.R + g.tiles * g.chunks * g.R;
    if (blocks > 0x7fffffff) return LDK_ENOTSUP;
    hipStream_t s = as_stream(stream);
    if (dtype == LDK_F64)
        launch_points_kcol_alpha<double>(uniform, a, tile_base, kc_tiles, g, (unsigned)blocks, s, k1,
                                         pts);
    else
        launch_points_kcol_alpha<float>(uniform, a, tile_base, kc_tiles, g, (unsigned)blocks, s, k1,
                                        pts);
    LDK_LAUNCH_CHECK();
    return LDK_OK;
}
