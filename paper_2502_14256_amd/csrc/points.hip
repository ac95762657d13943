// Randomized low-discrepancy point sets as exact 64-digit words:
// shifted rank-1 lattices (Sec. 4.2) and LMS + digitally shifted base-2
// digital nets in natural or Gray order (Sec. 4.3).
#include "pointset.hpp"

namespace ldk {

int validate_pointset(const ldk_pointset *ps, PointsetArgs *out)
{
    if (!ps || !out) return LDK_EINVAL;
    if (ps->R < 1 || ps->R > 65535 || ps->d < 1 || ps->d > LDK_MAX_D) return LDK_EINVAL;
    if (ps->m_max < 0 || ps->m_max > 62) return LDK_EINVAL;
    if (ps->flags != 0 && ps->flags != LDK_GEN_PER_REPLICATION) return LDK_EINVAL;
    if (ps->flags == LDK_GEN_PER_REPLICATION && ps->kind != LDK_DNET_B2) return LDK_EINVAL;
    // a net with m_max = 0 has no generating-matrix columns
    if (!ps->gen && !(ps->kind == LDK_DNET_B2 && ps->m_max == 0)) return LDK_EINVAL;
    if (ps->kind == LDK_LATTICE) {
        if (ps->order != LDK_NATURAL && ps->order != LDK_LINEAR) return LDK_EINVAL;
        if (ps->lms) return LDK_EINVAL;  // scrambling matrices belong to nets
    } else if (ps->kind == LDK_DNET_B2) {
        if (ps->order != LDK_NATURAL && ps->order != LDK_GRAY) return LDK_EINVAL;
    } else {
        return LDK_EINVAL;
    }
    const int64_t rstride =
        ps->flags == LDK_GEN_PER_REPLICATION ? (int64_t)ps->d * ps->m_max : 0;
    *out = PointsetArgs{ps->kind, ps->order, ps->R, ps->d,     ps->m_max,
                        ps->gen,  ps->lms,   ps->shift, rstride};
    return LDK_OK;
}

__global__ __launch_bounds__(GEN_THREADS) void k_gen_net(PointsetArgs a, int64_t n_min,
                                                         int64_t n_max, int64_t tile_base, int P,
                                                         int logP, int pairs,
                                                         uint64_t *__restrict__ out)
{
    __shared__ GenNetLds L;
    gen_net_block(a, n_min, n_max, tile_base, P, logP, pairs, out, blockIdx.x, blockIdx.y, blockIdx.z,
                  threadIdx.x, L);
}

template <int ORDER>
__global__ __launch_bounds__(GEN_THREADS) void k_gen_lattice(PointsetArgs a, int64_t n_min,
                                                             int64_t n_max, int P, int pairs,
                                                             uint64_t *__restrict__ out)
{
    gen_lattice_block<ORDER>(a, n_min, n_max, P, pairs != 0, out, blockIdx.x, blockIdx.y,
                             blockIdx.z, threadIdx.x);
}

// Interlaced, scrambled generating columns of a higher-order net (see
// ldk_interlace): one thread per output column (r, j, k); the ALPHA source
// columns are scrambled (64 parities each) and their digits interleaved.
template <int ALPHA>
__global__ __launch_bounds__(256) void k_interlace(PointsetArgs a, int d_out,
                                                  uint64_t *__restrict__ cols)
{
    const int m = a.m_max;
    const int64_t total = (int64_t)a.R * d_out * m;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= total) return;
    const int k = (int)(idx % m);
    const int j = (int)((idx / m) % d_out);
    const int r = (int)(idx / ((int64_t)m * d_out));
    uint64_t src[ALPHA];
#pragma unroll
    for (int q = 0; q < ALPHA; ++q) {
        const int sd = ALPHA * j + q;
        const uint64_t col = net_gen_column(a, r, sd, k);
        src[q] = a.lms ? lms_column(a.lms + ((size_t)r * a.d + sd) * 64, col) : col;
    }
    // digit t of the output is digit t / ALPHA of source t mod ALPHA
    uint64_t out = 0;
#pragma unroll
    for (int t = 0; t < 64; ++t) {
        const uint64_t bit = (src[t % ALPHA] >> (63 - t / ALPHA)) & 1u;
        out |= bit << (63 - t);
    }
    cols[idx] = out;
}

}  // namespace ldk

using namespace ldk;

extern "C" int ldk_interlace(const ldk_pointset *src, int alpha, uint64_t *cols, ldk_stream stream)
{
    PointsetArgs a;
    const int st = validate_pointset(src, &a);
    if (st) return st;
    if (a.kind != LDK_DNET_B2 || src->flags != 0) return LDK_EINVAL;
    if (alpha < 1 || alpha > 4 || a.d % alpha != 0) return LDK_EINVAL;
    const int d_out = a.d / alpha;
    const int64_t total = (int64_t)a.R * d_out * a.m_max;
    if (total == 0) return LDK_OK;  // m_max = 0: a net without columns
    if (!cols) return LDK_EINVAL;
    const int64_t blocks = (total + 255) / 256;
    if (blocks > 0x7fffffff) return LDK_ENOTSUP;
    const hipStream_t s = as_stream(stream);
    switch (alpha) {
    case 1: hipLaunchKernelGGL(k_interlace<1>, dim3((unsigned)blocks), dim3(256), 0, s, a, d_out, cols); break;
    case 2: hipLaunchKernelGGL(k_interlace<2>, dim3((unsigned)blocks), dim3(256), 0, s, a, d_out, cols); break;
    case 3: hipLaunchKernelGGL(k_interlace<3>, dim3((unsigned)blocks), dim3(256), 0, s, a, d_out, cols); break;
    default: hipLaunchKernelGGL(k_interlace<4>, dim3((unsigned)blocks), dim3(256), 0, s, a, d_out, cols); break;
    }
    LDK_LAUNCH_CHECK();
    return LDK_OK;
}

extern "C" int ldk_gen_points(const ldk_pointset *ps, int64_t n_min, int64_t n_max,
                              uint64_t *out, ldk_stream stream)
{
    PointsetArgs a;
    int st = validate_pointset(ps, &a);
    if (st) return st;
    if (n_min < 0 || n_max < n_min) return LDK_EINVAL;
    const int64_t lim = (a.kind == LDK_LATTICE && a.order == LDK_NATURAL)
                            ? ((int64_t)1 << 62)
                            : ((int64_t)1 << a.m_max);
    if (n_max > lim) return LDK_EINVAL;
    if (n_max == n_min) return LDK_OK;  // empty window: out may be NULL
    if (!out) return LDK_EINVAL;
    const GenGrid g = gen_grid(a, n_min, n_max, out);
    if (g.tiles > 0x7fffffff) return LDK_ENOTSUP;
    dim3 grid((unsigned)g.tiles, (unsigned)g.chunks, (unsigned)g.R);
    if (a.kind == LDK_LATTICE && a.order == LDK_LINEAR)
        hipLaunchKernelGGL(k_gen_lattice<LDK_LINEAR>, grid, dim3(GEN_THREADS), 0,
                           as_stream(stream), a, n_min, n_max, g.P, g.pairs, out);
    else if (a.kind == LDK_LATTICE)
        hipLaunchKernelGGL(k_gen_lattice<LDK_NATURAL>, grid, dim3(GEN_THREADS), 0,
                           as_stream(stream), a, n_min, n_max, g.P, g.pairs, out);
    else
        hipLaunchKernelGGL(k_gen_net, grid, dim3(GEN_THREADS), 0, as_stream(stream), a, n_min,
                           n_max, g.tile_base, g.P, g.logP, g.pairs, out);
    LDK_LAUNCH_CHECK();
    return LDK_OK;
}
