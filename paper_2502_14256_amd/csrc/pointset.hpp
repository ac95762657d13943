// Device-side point-set machinery shared by gen_points and the fused kernel
// column (points regenerated in registers instead of read from HBM).
#pragma once

#include "common.hpp"

namespace ldk {

// Host-validated, device-ready description of a point set.
struct PointsetArgs {
    int kind, order, R, d, m_max;
    const uint64_t *gen;    // lattice g[d] | net C[d][m_max] (or C[R][d][m_max])
    const uint64_t *lms;    // S[R][d][64] or nullptr
    const uint64_t *shift;  // [R][d] or nullptr
    int64_t gen_rstride;    // net columns: words between replications (0: shared)
};

// Column k of net dimension j in replication r (before scrambling).
__device__ __forceinline__ uint64_t net_gen_column(const PointsetArgs &a, int r, int j, int k)
{
    return a.gen[(size_t)r * a.gen_rstride + (size_t)j * a.m_max + k];
}

int validate_pointset(const ldk_pointset *ps, PointsetArgs *out);

// Natural-order digital-net step: the point index advances by P = 2^s, which
// flips index bits s .. s+c where c = ctz((i >> s) + 1); the point changes by
// the XOR of those scrambled columns.  Gray order: the Gray code changes in
// bits s-1 and s+c (only bit c when s = 0).
//   step[c] = XOR_{k=s}^{s+c} Ct_k            (natural)
//   step[c] = Ct_{s-1} ^ Ct_{s+c}  (s >= 1)   (Gray)
//
// Scrambled column (Sec. 4.3, linear matrix scrambling): bit 63-t of
// S_j C_j[:, k] is the parity of (row t of S_j) AND (column k of C_j).
__device__ __forceinline__ uint64_t lms_column(const uint64_t *__restrict__ S_rows,
                                               uint64_t col)
{
    uint64_t out = 0;
#pragma unroll 8
    for (int t = 0; t < 64; ++t) {
        const uint64_t bit = (uint64_t)(__popcll(S_rows[t] & col) & 1);
        out |= bit << (63 - t);
    }
    return out;
}

// Point of index `code` (already Gray-coded if needed) from scrambled
// columns ct[0..m): XOR of the columns whose index bit is set.
__device__ __forceinline__ uint64_t net_point(const uint64_t *ct, int m, uint64_t code)
{
    uint64_t z = 0;
    for (int k = 0; k < m; ++k)
        if ((code >> k) & 1u) z ^= ct[k];
    return z;
}

__device__ __forceinline__ uint64_t gray_code(uint64_t i) { return i ^ (i >> 1); }

// Lattice point z_i (without shift): natural order v(i) g = bitreverse64(i) g
// (mod 2^64); linear order ((i g) mod 2^m) 2^(64-m) = (i g) << (64 - m).
__device__ __forceinline__ uint64_t lattice_point(uint64_t g, uint64_t i, int order, int m)
{
    if (order == LDK_NATURAL) return brev64(i) * g;
    return m == 0 ? 0 : ((i * g) << (64 - m));
}

// Point-word tiling (gen_points, and the point half of the fused points +
// column launch): blocks of GEN_THREADS threads over (point tile, chunk of
// GEN_DIM_CHUNK dimensions, replication).  Thread (p, jj) of a block writes
// dimension j0 + jj of points tile + p + P k, P the largest power of two with
// P * dims <= GEN_THREADS: consecutive threads write consecutive words.
constexpr int GEN_THREADS = 256;
constexpr int GEN_DIM_CHUNK = 32;   // dimensions per block
constexpr int GEN_ITERS = 32;       // points per thread (lattices)
constexpr int GEN_ITERS_NET = 128;  // points per thread (nets: amortises the scrambling)

struct GenGrid {
    int64_t tiles;      // point tiles per (chunk, replication)
    int64_t tile_base;  // first index of tile 0 (nets: a multiple of P GEN_ITERS_NET)
    int chunks;         // dimension chunks
    int R;
    int P, logP;
    int pairs;          // words written two dimensions per 16-byte store
};

// out: the destination (16-byte stores need an even d and a 16-byte aligned
// destination).
inline GenGrid gen_grid(const PointsetArgs &a, int64_t n_min, int64_t n_max, const void *out)
{
    GenGrid g{};
    g.pairs = (a.d & 1) == 0 && ((uintptr_t)out & 15) == 0;
    int dims = a.d < GEN_DIM_CHUNK ? a.d : GEN_DIM_CHUNK;
    if (g.pairs) dims >>= 1;
    g.P = 1;
    while (2 * g.P * dims <= GEN_THREADS) g.P *= 2;
    while ((1 << g.logP) < g.P) ++g.logP;
    const int64_t span = (int64_t)g.P * (a.kind == LDK_LATTICE ? GEN_ITERS : GEN_ITERS_NET);
    g.tile_base = a.kind == LDK_LATTICE ? n_min : (n_min / span) * span;
    g.tiles = (n_max - g.tile_base + span - 1) / span;
    g.chunks = (a.d + GEN_DIM_CHUNK - 1) / GEN_DIM_CHUNK;
    g.R = a.R;
    return g;
}

// LDS of a net block: the scrambled columns S_j C_j of a chunk of
// dimensions, then the XOR steps between a thread's points (rows padded to
// 65 words: the lanes of a wave read different dimensions jj at one step
// index, and 64-word rows would put them all in one LDS bank).
struct GenNetLds {
    uint64_t ct[GEN_DIM_CHUNK][65];
    union {
        uint64_t step[GEN_DIM_CHUNK][65];
        uint64_t srow[GEN_DIM_CHUNK][65];  // rows of S_j, dead once ct is built
    } u;
};

// One lattice block of the tiling: point tile bx, dimension chunk by,
// replication r; thread t of GEN_THREADS.  With pairs (see GenGrid), a
// thread writes dimensions j, j + 1 of its points as one 16-byte store.
// ORDER >= 0 fixes the point order at compile time (it must equal a.order);
// a tile whose last point is below n_max stores with no per-point test.
template <int ORDER = -1>
__device__ __forceinline__ void gen_lattice_block(const PointsetArgs &a, int64_t n_min,
                                                  int64_t n_max, int P, bool pairs,
                                                  uint64_t *__restrict__ out, int64_t bx, int by,
                                                  int r, int t)
{
    const int order = ORDER >= 0 ? ORDER : a.order;
    if (pairs) {
        const int j0 = by * GEN_DIM_CHUNK;
        const int DB2 = min(GEN_DIM_CHUNK, a.d - j0) >> 1;  // dimension pairs
        const int p = t / DB2, jj = t % DB2;
        if (p >= P) return;
        const int j = j0 + 2 * jj;
        const int64_t cnt = n_max - n_min;
        const uint64_t g0 = a.gen[j], g1 = a.gen[j + 1];
        const uint64_t d0 = a.shift ? a.shift[(size_t)r * a.d + j] : 0;
        const uint64_t d1 = a.shift ? a.shift[(size_t)r * a.d + j + 1] : 0;
        const int64_t first = n_min + bx * P * GEN_ITERS + p;
        uint64_t *dst = out + ((size_t)r * cnt + (first - n_min)) * a.d + j;
        const size_t dstep = (size_t)P * a.d;
        auto put = [&](int64_t i, uint64_t *dp) {
            ulonglong2 w;
            w.x = lattice_point(g0, (uint64_t)i, order, a.m_max) + d0;
            w.y = lattice_point(g1, (uint64_t)i, order, a.m_max) + d1;
            *reinterpret_cast<ulonglong2 *>(dp) = w;
        };
        if (first + (int64_t)P * (GEN_ITERS - 1) < n_max) {
#pragma unroll
            for (int k = 0; k < GEN_ITERS; ++k) put(first + (int64_t)P * k, dst + dstep * k);
        } else {
            int64_t i = first;
            for (int k = 0; k < GEN_ITERS && i < n_max; ++k, i += P, dst += dstep) put(i, dst);
        }
        return;
    }
    const int j0 = by * GEN_DIM_CHUNK;
    const int DB = min(GEN_DIM_CHUNK, a.d - j0);
    const int p = t / DB, jj = t % DB;
    if (p >= P) return;
    const int j = j0 + jj;
    const int64_t cnt = n_max - n_min;
    const uint64_t g = a.gen[j];
    const uint64_t delta = a.shift ? a.shift[(size_t)r * a.d + j] : 0;
    const int64_t first = n_min + bx * P * GEN_ITERS + p;
    uint64_t *dst = out + ((size_t)r * cnt + (first - n_min)) * a.d + j;
    const size_t dstep = (size_t)P * a.d;
    int64_t i = first;
    for (int k = 0; k < GEN_ITERS && i < n_max; ++k) {
        *dst = lattice_point(g, (uint64_t)i, order, a.m_max) + delta;
        i += P;
        dst += dstep;
    }
}

// One net block of the tiling: point tile bx, dimension chunk by,
// replication r; thread t of GEN_THREADS walks the points
// i = tile + p + P * k, k < GEN_ITERS_NET, of dimension j0 + jj.  Every
// thread of the block calls it (it synchronises the block).
__device__ __forceinline__ void gen_net_block(const PointsetArgs &a, int64_t n_min, int64_t n_max,
                                              int64_t tile_base, int P, int logP, int pairs,
                                              uint64_t *__restrict__ out, int64_t bx, int by, int r,
                                              int t, GenNetLds &L)
{
    auto &ct = L.ct;
    auto &u = L.u;
    auto &step = u.step;
    const int j0 = by * GEN_DIM_CHUNK;
    const int DB = min(GEN_DIM_CHUNK, a.d - j0);
    const int m = a.m_max;

    if (a.lms) {
        for (int w = t; w < DB * 64; w += GEN_THREADS)
            u.srow[w >> 6][w & 63] = a.lms[((size_t)r * a.d + j0 + (w >> 6)) * 64 + (w & 63)];
        __syncthreads();
    }
    for (int w = t; w < DB * m; w += GEN_THREADS) {
        const int jj = w / m, k = w % m;
        const uint64_t col = net_gen_column(a, r, j0 + jj, k);
        ct[jj][k] = a.lms ? lms_column(u.srow[jj], col) : col;
    }
    __syncthreads();  // srow is dead from here on; step reuses its storage
    const int s = logP;
    for (int w = t; w < DB * 64; w += GEN_THREADS) {
        const int jj = w / 64, c = w % 64;
        uint64_t v = 0;
        if (s + c < m) {
            if (a.order == LDK_GRAY) {
                v = ct[jj][s + c] ^ (s >= 1 ? ct[jj][s - 1] : 0);
            } else {
                for (int k = s; k <= s + c; ++k) v ^= ct[jj][k];
            }
        }
        step[jj][c] = v;
    }
    __syncthreads();

    const int64_t cnt = n_max - n_min;
    if (pairs) {
        // two dimensions per thread, one 16-byte store per point (even d,
        // aligned destination): half the store instructions
        const int DB2 = DB >> 1;
        const int p = t / DB2, jj = 2 * (t % DB2);
        if (p >= P) return;
        const int j = j0 + jj;
        const int64_t first = tile_base + bx * P * GEN_ITERS_NET + p;
        if (first >= n_max) return;
        const uint64_t blk = ((uint64_t)tile_base >> s) + (uint64_t)bx * GEN_ITERS_NET;
        const uint64_t d0 = a.shift ? a.shift[(size_t)r * a.d + j] : 0;
        const uint64_t d1 = a.shift ? a.shift[(size_t)r * a.d + j + 1] : 0;
        const uint64_t code0 = a.order == LDK_GRAY ? gray_code((uint64_t)first) : (uint64_t)first;
        uint64_t z0 = net_point(ct[jj], m, code0), z1 = net_point(ct[jj + 1], m, code0);
        uint64_t *const row = out + (size_t)r * cnt * a.d + j;
        if (first >= n_min && first + (int64_t)P * (GEN_ITERS_NET - 1) < n_max) {
            // the whole tile is inside the window: every point is stored
            uint64_t *dst = row + (size_t)(first - n_min) * a.d;
            const size_t dstep = (size_t)P * a.d;
#pragma unroll 4
            for (int k = 0; k < GEN_ITERS_NET; ++k) {
                *reinterpret_cast<ulonglong2 *>(dst) = ulonglong2{z0 ^ d0, z1 ^ d1};
                if (k + 1 < GEN_ITERS_NET) {
                    const int c = ctz64(blk + (uint64_t)k + 1);
                    z0 ^= step[jj][c];
                    z1 ^= step[jj + 1][c];
                }
                dst += dstep;
            }
            return;
        }
        int64_t i = first;
        for (int k = 0; k < GEN_ITERS_NET; ++k) {
            if (i >= n_min) {
                ulonglong2 w2;
                w2.x = z0 ^ d0;
                w2.y = z1 ^ d1;
                *reinterpret_cast<ulonglong2 *>(row + (size_t)(i - n_min) * a.d) = w2;
            }
            const int64_t next = i + P;
            if (next >= n_max || k + 1 == GEN_ITERS_NET) break;
            const int c = ctz64(blk + (uint64_t)k + 1);
            z0 ^= step[jj][c];
            z1 ^= step[jj + 1][c];
            i = next;
        }
        return;
    }
    const int p = t / DB, jj = t % DB;
    if (p >= P) return;
    const int j = j0 + jj;
    // tiles start at multiples of P GEN_ITERS_NET (tile_base <= n_min), so
    // point k of every thread has i >> s = blk + k: the step index is the same
    // for the whole block (scalar work); points below n_min are not stored
    const int64_t first = tile_base + bx * P * GEN_ITERS_NET + p;
    if (first >= n_max) return;
    const uint64_t blk = ((uint64_t)tile_base >> s) + (uint64_t)bx * GEN_ITERS_NET;
    const uint64_t delta = a.shift ? a.shift[(size_t)r * a.d + j] : 0;
    const uint64_t code0 = a.order == LDK_GRAY ? gray_code((uint64_t)first) : (uint64_t)first;
    uint64_t z = net_point(ct[jj], m, code0);
    uint64_t *const row = out + (size_t)r * cnt * a.d + j;
    int64_t i = first;
    for (int k = 0; k < GEN_ITERS_NET; ++k) {
        if (i >= n_min) row[(size_t)(i - n_min) * a.d] = z ^ delta;
        const int64_t next = i + P;
        if (next >= n_max || k + 1 == GEN_ITERS_NET) break;
        z ^= step[jj][ctz64(blk + (uint64_t)k + 1)];
        i = next;
    }
}

}  // namespace ldk
