// Device-side point-set machinery shared by gen_points and the fused kernel
// column (points regenerated in registers instead of read from HBM).
#pragma once

#include "common.hpp"

namespace ldk {

// Host-validated, device-ready description of a point set.
struct PointsetArgs {
    int kind, order, R, d, m_max;
    const uint64_t *gen;    // lattice g[d] | net C[d][m_max]
    const uint64_t *lms;    // S[R][d][64] or nullptr
    const uint64_t *shift;  // [R][d] or nullptr
};

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

}  // namespace ldk
