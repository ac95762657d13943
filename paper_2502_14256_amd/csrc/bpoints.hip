// Point sets without the structure the fast transforms need; they feed QMC
// means (the RQMC estimate over given coordinates, ldk_rqmc_points).
//
// Digital sequences in a prime base b (Sec. 4.3 allows any prime base):
// point i has the base-b digits a_k of i (least significant first) and the
// digits z_t = sum_k C[t][k] a_k mod b, digit t weighing b^-(t+1).
//   Faure: one prime b >= d; dimension j (from 0) uses C = P^j mod b, P the
//   upper-triangular Pascal matrix, whose entries are binom(k, t) j^(k-t).
//   Halton (Sec. 4.4): dimension j uses the (j+1)-th prime and C = I, so z is
//   the digit expansion of the radical inverse of i.
// Randomizations, each optional, in this order: linear matrix scrambling
// z <- S z mod b (S lower triangular with a nonzero diagonal), a permutation
// of the digit values per digit position, a digital shift z_t + delta_t mod
// b.  T digits are kept, the largest T with b^T <= 2^53, so the coordinate is
// the integer v = sum_t z_t b^(T-1-t) < 2^53 divided by b^T, rounded once.
//
// A block takes 512 consecutive indices of one replication (two per thread)
// and walks the dimensions.  The digits of an index live in registers, four
// to a 32-bit word, so a row of S (or of Faure's C) times the digit vector is
// one v_dot4_u32_u8 per word; the sum stays below 2^21 and is reduced mod b
// with an exact 24-bit reciprocal product.  Per dimension the block stages
// S's rows, packed the same way, and the T x b table of the digit
// permutation and shift combined, in LDS; the Faure matrices come packed
// from a small kernel, formed once per call into the workspace.
//
// Nested uniform scrambling of a base-2 net (Sec. 4.3, NUS): the point word
// z = C i (64 digits), then digit t = 1..64 is flipped when the top bit of
// mix64(key XOR seed) is set, key = 2^(t-1) + the unscrambled digits before
// t as an integer; mix64 is the SplitMix64 finaliser (Steele, Lea and Flood,
// 2014, with Stafford's Mix13 constants).  For base 2 a permutation of the
// digit values is the identity or the flip, and this draws one independently
// for every prefix, as nested uniform scrambling asks.
#include "common.hpp"

// dynamic LDS of the tile kernels: the output tile
extern __shared__ __align__(16) unsigned char g_bp_lds[];

namespace ldk {

namespace {

constexpr int BP_T = LDK_BDIGITS_MAX;  // digit rows of the scramble layouts
constexpr int BP_MAX_D = 54;    // the first 54 primes are below 256
constexpr int BP_KMAX = 32;     // index digits (i < 2^32)
constexpr int BP_QW = BP_KMAX / 4;  // words of a packed digit row
constexpr int BP_TT = 512;      // threads of a tile block (Halton, Faure)
constexpr int BP_WAVES = BP_TT / 64;
constexpr int BP_P = 64;        // points per tile block, one per lane
constexpr int BP_DCH = 64;      // dimensions per output tile

struct BpArgs {
    int d, flags;
    int64_t n_min, cnt;
    uint32_t lms_off;  // byte offset of lms within its first word
    // per dimension (Halton; Faure uses entry 0 for every dimension), 32-bit
    // words so that a uniform index reads them with scalar loads
    uint32_t base[BP_MAX_D], T[BP_MAX_D], M[BP_MAX_D], L[BP_MAX_D];
    uint32_t mg[BP_MAX_D];  // ceil(2^L / b)
    double rb[BP_MAX_D];    // 1 / b, rounded
    double bT[BP_MAX_D];    // b^T, exact
    // Halton: wave w computes dimensions ord[q] for wbeg[w] <= q < wbeg[w + 1]
    uint32_t ord[BP_MAX_D], wbeg[BP_WAVES + 1];
};

// Faure matrix of dimension j = blockIdx.x, packed for the point kernel:
// C[t][k] = binom(k, t) j^(k-t) mod b for t <= k < T (zero elsewhere), rows
// t < 4 mj and columns k < 4 mj, four columns to a word: [d][4 mj][mj].
__global__ __launch_bounds__(64) void k_faure_cmat(int b, int T, int mj, uint32_t *__restrict__ cmat)
{
    __shared__ uint8_t binom[BP_T][BP_T];  // [k][t]
    __shared__ uint8_t pw[BP_T];
    const int j = blockIdx.x, t = threadIdx.x;
    if (t == 0) {
        int p = 1 % b;
        for (int e = 0; e < T; ++e) {
            pw[e] = (uint8_t)p;
            p = (p * (j % b)) % b;
        }
    }
    // Pascal's rule, one row k at a time: binom(k, t) = binom(k-1, t-1) + binom(k-1, t)
    for (int k = 0; k < T; ++k) {
        if (t < T) {
            int v;
            if (t > k) v = 0;
            else if (t == 0 || t == k) v = 1 % b;
            else v = (binom[k - 1][t - 1] + binom[k - 1][t]) % b;
            binom[k][t] = (uint8_t)v;
        }
        __syncthreads();
    }
    if (t < 4 * mj)
        for (int q = 0; q < mj; ++q) {
            uint32_t w = 0;
            for (int c = 0; c < 4; ++c) {
                const int k = 4 * q + c;
                if (t < T && k < T && k >= t) w |= (uint32_t)((binom[k][t] * pw[k - t]) % b) << (8 * c);
            }
            cmat[((size_t)j * 4 * mj + t) * mj + q] = w;
        }
}

// s mod b for s < 2^21 and b <= 251.  With L = 21 + ceil(log2 b) and
// mg = ceil(2^L / b) < 2^22, e = mg b - 2^L < b gives s e < 2^L, so
// floor(s mg / 2^L) = floor(s / b) exactly; both factors fit 24 bits.
__device__ __forceinline__ uint32_t mod_b(uint32_t s, uint32_t b, uint32_t mg, uint32_t L)
{
    const uint64_t p = (uint64_t)(s & 0xffffffu) * (uint64_t)(mg & 0xffffffu);
    const uint32_t q = __builtin_amdgcn_alignbit((uint32_t)(p >> 32), (uint32_t)p, L);
    return s - __umul24(q, b);
}

// floor(x / b) and the remainder for x < 2^32: x RN(1/b) in FP64 lies within
// 2^-20 of x / b, below the next integer (the fraction of x / b is at most
// 1 - 1/b), so truncation is exact except at multiples of b, where it can
// fall one short.
__device__ __forceinline__ uint32_t div_b(uint32_t x, uint32_t b, double rb, uint32_t &rem)
{
    uint32_t q = (uint32_t)((double)x * rb);
    uint32_t r = x - q * b;
    if (r >= b) {
        r -= b;
        ++q;
    }
    rem = r;
    return q;
}

// Base-b digits of an index, least significant first, four to a word
// (digit k in byte k % 4 of word k / 4); M digits, the rest zero.
template <int MJ>
__device__ __forceinline__ void index_digits_packed(uint32_t x, uint32_t b, double rb, int M,
                                                    uint32_t (&z)[MJ])
{
#pragma unroll
    for (int q = 0; q < MJ; ++q) z[q] = 0;
#pragma unroll
    for (int k = 0; k < 4 * MJ; ++k)
        if (k < M) {
            uint32_t dg;
            x = div_b(x, b, rb, dg);
            z[k >> 2] |= dg << (8 * (k & 3));
        }
}

// Lane t (t < T) fetches row t of S, packed four columns to a word over the
// columns below 4 MJ, keeping only k <= t (S is lower triangular): the row's
// bytes start o bytes past the word array W, and MJ + 1 words from the word
// boundary at or below cover them (within the row's 53 bytes).  Lanes t >= T
// hold zeros.
template <int MJ>
__device__ __forceinline__ void lane_row(const uint32_t *__restrict__ W, uint64_t o, int t, int T,
                                         uint32_t (&row)[MJ])
{
#pragma unroll
    for (int q = 0; q < MJ; ++q) row[q] = 0;
    if (t >= T) return;
    uint32_t wd[MJ + 1];
#pragma unroll
    for (int q = 0; q <= MJ; ++q) wd[q] = W[(o >> 2) + q];
    const uint32_t sh = (uint32_t)(o & 3) * 8;
#pragma unroll
    for (int q = 0; q < MJ; ++q) {
        const int lo = 4 * q;
        uint32_t x = (uint32_t)((((uint64_t)wd[q + 1] << 32) | wd[q]) >> sh);
        if (t < lo) x = 0;
        else if (t < lo + 3) x &= 0xffffffffu >> (8 * (3 - (t - lo)));
        row[q] = x;
    }
}

// K consecutive output digits t0 .. t0+K-1 (all below T) of one coordinate:
// w_t = (S z)_t mod b from row t of S (lane t's, by v_readlane), then
// pi_t(w_t) (K gathers in flight together), then + delta_t mod b, each
// joining the Horner sum.
template <int K, int MJ, int F>
__device__ __forceinline__ void digit_group(const uint32_t (&srows)[MJ], uint32_t dlane, const uint8_t *prow,
                                            const uint32_t (&z)[MJ], int t0, uint32_t b, uint32_t mg,
                                            uint32_t L, double bd, double &v)
{
    constexpr bool LMS = F & LDK_BR_LMS, DP = F & LDK_BR_DP, DS = F & LDK_BR_DS;
    uint32_t g[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int t = t0 + k;
        uint32_t s = 0;
#pragma unroll
        for (int q = 0; q < MJ; ++q) {
            uint32_t sr;
            if constexpr (LMS) sr = __builtin_amdgcn_readlane(srows[q], t);
            else sr = (t >> 2) == q ? 1u << (8 * (t & 3)) : 0u;
            s = __builtin_amdgcn_udot4(sr, z[q], s, false);
        }
        const uint32_t w = mod_b(s, b, mg, L);
        if constexpr (DP) g[k] = prow[t * 256 + w];
        else g[k] = w;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        uint32_t u = g[k];
        if constexpr (DS) {
            u += __builtin_amdgcn_readlane(dlane, t0 + k);
            if (u >= b) u -= b;
        }
        v = fma(v, bd, (double)u);
    }
}

// Coordinate of one point in dimension j of replication r (rj = r d + j):
// digit t of the output is w_t = (S z)_t mod b, then pi_t(w_t), then
// + delta_t mod b (each step as the flags F ask); Horner's rule in FP64 is
// exact (every partial sum is an integer below 2^53) and the one division
// rounds.  The wave's lanes first fetch one row of S and one delta each.
// With permutations the digits go four at a time (four gathers in flight),
// the last T mod 4 one at a time.
template <int MJ, int F>
__device__ __forceinline__ double coordinate(const BpArgs &a, const uint32_t *__restrict__ lmsw,
                                             const uint8_t *__restrict__ shift,
                                             const uint8_t *__restrict__ perm, const uint32_t (&z)[MJ],
                                             size_t rj, int T, uint32_t b, uint32_t mg, uint32_t L,
                                             double bT, int lane)
{
    constexpr bool LMS = F & LDK_BR_LMS, DP = F & LDK_BR_DP, DS = F & LDK_BR_DS;
    const uint8_t *prow = DP ? perm + rj * BP_T * 256 : nullptr;
    const double bd = (double)b;
    uint32_t srows[MJ] = {};
    if constexpr (LMS)
        lane_row<MJ>(lmsw, a.lms_off + ((uint64_t)rj * BP_T + lane) * BP_T, lane, T, srows);
    uint32_t dlane = 0;
    if constexpr (DS) dlane = lane < T ? shift[rj * BP_T + lane] : 0u;
    double v = 0.0;
    int t0 = 0;
    if constexpr (DP)
        for (; t0 + 4 <= T; t0 += 4) digit_group<4, MJ, F>(srows, dlane, prow, z, t0, b, mg, L, bd, v);
    for (; t0 < T; ++t0) digit_group<1, MJ, F>(srows, dlane, prow, z, t0, b, mg, L, bd, v);
    return v / bT;
}

// Write a finished tile: rows p < valid of dimensions j0 .. j0+dch-1 of the
// [R][cnt][d] output.  With every dimension in the tile the rows are one
// contiguous run.
__device__ __forceinline__ void flush_tile(double *__restrict__ out, const double *tile, int64_t cnt, int d,
                                           int r, int64_t i0, int j0, int dch, int tid)
{
    const int64_t rest = cnt - i0;
    const int valid = rest < BP_P ? (int)rest : BP_P;
    double *dst = out + ((size_t)r * cnt + i0) * d + j0;
    if (dch == d) {
        for (int e = tid; e < valid * dch; e += BP_TT) dst[e] = tile[e];
    } else {
        for (int e = tid; e < valid * dch; e += BP_TT) {
            const int p = e / dch;
            dst[(size_t)p * d + (e - p * dch)] = tile[e];
        }
    }
}

template <int MJ, int F>
__device__ __forceinline__ double halton_coordinate(const BpArgs &a, const uint32_t *__restrict__ lmsw,
                                                    const uint8_t *__restrict__ shift,
                                                    const uint8_t *__restrict__ perm, uint32_t i, int r,
                                                    int j, int lane)
{
    const uint32_t b = a.base[j];
    uint32_t z[MJ];
    index_digits_packed<MJ>(i, b, a.rb[j], a.M[j], z);
    return coordinate<MJ, F>(a, lmsw, shift, perm, z, (size_t)r * a.d + j, a.T[j], b, a.mg[j], a.L[j],
                             a.bT[j], lane);
}

// Halton: a block takes 64 consecutive indices of one replication, one per
// lane; its eight waves split the dimensions (a balanced order from the
// host) and write into an LDS tile of whole rows, which the block then
// stores as one contiguous run (d <= 54 fits one tile).
template <int F>
__global__ __launch_bounds__(BP_TT) void k_gen_halton(BpArgs a, const uint32_t *__restrict__ lmsw,
                                                      const uint8_t *__restrict__ shift,
                                                      const uint8_t *__restrict__ perm,
                                                      double *__restrict__ out)
{
    double *tile = reinterpret_cast<double *>(g_bp_lds);  // [64][d]
    const int tid = threadIdx.x, lane = tid & 63, r = blockIdx.y;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t i0 = (int64_t)blockIdx.x * BP_P;
    const int64_t ii = i0 + lane;
    const uint32_t i = (uint32_t)(a.n_min + (ii < a.cnt ? ii : 0));
    for (int q = a.wbeg[wave]; q < (int)a.wbeg[wave + 1]; ++q) {
        const int j = a.ord[q];
        const int mq = (a.M[j] + 3) >> 2;
        double x;
        switch (mq) {
        case 1: x = halton_coordinate<1, F>(a, lmsw, shift, perm, i, r, j, lane); break;
        case 2: x = halton_coordinate<2, F>(a, lmsw, shift, perm, i, r, j, lane); break;
        case 3: x = halton_coordinate<3, F>(a, lmsw, shift, perm, i, r, j, lane); break;
        case 4: x = halton_coordinate<4, F>(a, lmsw, shift, perm, i, r, j, lane); break;
        case 5: x = halton_coordinate<5, F>(a, lmsw, shift, perm, i, r, j, lane); break;
        case 6: x = halton_coordinate<6, F>(a, lmsw, shift, perm, i, r, j, lane); break;
        case 7: x = halton_coordinate<7, F>(a, lmsw, shift, perm, i, r, j, lane); break;
        default: x = halton_coordinate<8, F>(a, lmsw, shift, perm, i, r, j, lane); break;
        }
        tile[lane * a.d + j] = x;
    }
    __syncthreads();
    flush_tile(out, tile, a.cnt, a.d, r, i0, 0, a.d, tid);
}

// Faure: one base for every dimension, so a lane forms its index digits (MJ
// words) once; dimension j takes z = C_j a mod b from its packed matrix
// rows.  Tiles of up to 64 dimensions (d may reach 251).
template <int MJ, int F>
__global__ __launch_bounds__(BP_TT) void k_gen_faure(BpArgs a, const uint32_t *__restrict__ lmsw,
                                                     const uint8_t *__restrict__ shift,
                                                     const uint8_t *__restrict__ perm,
                                                          const uint32_t *__restrict__ cmat,
                                                          double *__restrict__ out)
{
    double *tile = reinterpret_cast<double *>(g_bp_lds);  // [64][min(d, 64)]
    const int tid = threadIdx.x, lane = tid & 63, r = blockIdx.y;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t i0 = (int64_t)blockIdx.x * BP_P;
    const int64_t ii = i0 + lane;
    const uint32_t i = (uint32_t)(a.n_min + (ii < a.cnt ? ii : 0));
    const uint32_t b = a.base[0], mg = a.mg[0], L = a.L[0];
    const int M = a.M[0], T = a.T[0];
    uint32_t ad[MJ];
    index_digits_packed<MJ>(i, b, a.rb[0], M, ad);
    for (int j0 = 0; j0 < a.d; j0 += BP_DCH) {
        const int dch = a.d - j0 < BP_DCH ? a.d - j0 : BP_DCH;
        for (int jj = wave; jj < dch; jj += BP_WAVES) {
            const int j = j0 + jj;
            // z_t = sum_{k >= t} C[t][k] a_k mod b (zero for t >= M: a_k = 0 there)
            const uint32_t *cj = cmat + (size_t)j * (4 * MJ * MJ);
            uint32_t z[MJ];
#pragma unroll
            for (int q = 0; q < MJ; ++q) z[q] = 0;
#pragma unroll
            for (int t = 0; t < 4 * MJ; ++t) {
                uint32_t s = 0;
#pragma unroll
                for (int q = 0; q < MJ; ++q) s = __builtin_amdgcn_udot4(cj[t * MJ + q], ad[q], s, false);
                z[t >> 2] |= mod_b(s, b, mg, L) << (8 * (t & 3));
            }
            tile[lane * dch + jj] = coordinate<MJ, F>(a, lmsw, shift, perm, z, (size_t)r * a.d + j, T, b, mg,
                                                      L, a.bT[0], lane);
        }
        __syncthreads();
        flush_tile(out, tile, a.cnt, a.d, r, i0, j0, dch, tid);
        __syncthreads();  // the tile is free for the next dimensions
    }
}

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// NUS: a block takes 64 consecutive indices of one replication, one per
// lane; its eight waves split the dimensions of each tile of up to 64 and
// the block stores the tile's rows (contiguous when d <= 64).
__global__ __launch_bounds__(BP_TT) void k_gen_nus(int d, int m, int64_t n_min, int64_t cnt,
                                                   const uint64_t *__restrict__ gen,
                                                   const uint64_t *__restrict__ seed, double *__restrict__ out)
{
    double *tile = reinterpret_cast<double *>(g_bp_lds);  // [64][min(d, 64)]
    const int tid = threadIdx.x, lane = tid & 63, r = blockIdx.y;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t i0 = (int64_t)blockIdx.x * BP_P;
    const int64_t ii = i0 + lane;
    const uint64_t i = (uint64_t)(n_min + (ii < cnt ? ii : 0));
    for (int j0 = 0; j0 < d; j0 += BP_DCH) {
        const int dch = d - j0 < BP_DCH ? d - j0 : BP_DCH;
        for (int jj = wave; jj < dch; jj += BP_WAVES) {
            const int j = j0 + jj;
            uint64_t z = 0;
            for (int k = 0; k < m; ++k)
                if ((i >> k) & 1u) z ^= gen[(size_t)j * m + k];
            const uint64_t s = seed[(size_t)r * d + j];
            // the flip of digit t keyed by the digits above it; the bit
            // position of digit t is 64 - t
            uint64_t flips = mix64(1ull ^ s) & 0x8000000000000000ull;
            for (int t = 2; t <= 64; ++t) {
                const uint64_t key = (1ull << (t - 1)) | (z >> (65 - t));
                flips |= (mix64(key ^ s) >> 63) << (64 - t);
            }
            tile[lane * dch + jj] = unit_f64(z ^ flips);
        }
        __syncthreads();
        flush_tile(out, tile, cnt, d, r, i0, j0, dch, tid);
        __syncthreads();  // the tile is free for the next dimensions
    }
}

bool is_prime(int v)
{
    if (v < 2) return false;
    for (int q = 2; q * q <= v; ++q)
        if (v % q == 0) return false;
    return true;
}

int digits_kept(int b)
{
    int T = 0;
    uint64_t p = 1;
    while (p <= ((uint64_t)1 << 53) / (uint64_t)b) {
        p *= (uint64_t)b;
        ++T;
    }
    return T;
}

// Digits needed for the indices below n_max (at least 1).
int index_digits(int b, int64_t n_max)
{
    int M = 1;
    uint64_t p = (uint64_t)b;
    while (p < (uint64_t)n_max) {
        p *= (uint64_t)b;
        ++M;
    }
    return M;
}

int validate_bpointset(const ldk_bpointset *ps, int64_t n_min, int64_t n_max)
{
    if (!ps) return LDK_EINVAL;
    if (ps->R < 1 || ps->R > 65535 || ps->d < 1 || n_min < 0 || n_max < n_min) return LDK_EINVAL;
    if (n_max > ((int64_t)1 << 32)) return LDK_ENOTSUP;
    switch (ps->kind) {
    case LDK_HALTON:
        if (ps->d > BP_MAX_D) return LDK_EINVAL;
        break;
    case LDK_FAURE:
        if (!is_prime(ps->base) || ps->base < ps->d || ps->base > 251) return LDK_EINVAL;
        break;
    case LDK_DNET_NUS:
        if (ps->m < 0 || ps->m > 32 || n_max > ((int64_t)1 << ps->m)) return LDK_EINVAL;
        if (!ps->gen || !ps->seed) return LDK_EINVAL;
        return LDK_OK;
    default:
        return LDK_EINVAL;
    }
    if (ps->flags & ~(LDK_BR_LMS | LDK_BR_DP | LDK_BR_DS)) return LDK_EINVAL;
    if (((ps->flags & LDK_BR_LMS) && !ps->lms) || ((ps->flags & LDK_BR_DP) && !ps->perm) ||
        ((ps->flags & LDK_BR_DS) && !ps->shift))
        return LDK_EINVAL;
    return LDK_OK;
}

}  // namespace

}  // namespace ldk

using namespace ldk;

extern "C" size_t ldk_bpoints_workspace_bytes(const ldk_bpointset *ps)
{
    if (!ps || ps->kind != LDK_FAURE || ps->d < 1) return 0;
    return (size_t)ps->d * BP_KMAX * BP_QW * sizeof(uint32_t);
}

extern "C" int ldk_gen_bpoints(const ldk_bpointset *ps, int64_t n_min, int64_t n_max, double *out,
                               void *ws, ldk_stream stream)
{
    int st = validate_bpointset(ps, n_min, n_max);
    if (st) return st;
    const int64_t cnt = n_max - n_min;
    if (cnt == 0) return LDK_OK;
    if (!out) return LDK_EINVAL;
    if (ps->kind == LDK_FAURE && !ws) return LDK_EINVAL;
    st = ensure_init();
    if (st) return st;
    hipStream_t s = as_stream(stream);
    if (ps->kind == LDK_DNET_NUS) {
        const int64_t blocks = (cnt + BP_P - 1) / BP_P;
        if (blocks > 0x7fffffff) return LDK_ENOTSUP;
        const size_t lds = (size_t)BP_P * (ps->d < BP_DCH ? ps->d : BP_DCH) * sizeof(double);
        hipLaunchKernelGGL(k_gen_nus, dim3((unsigned)blocks, (unsigned)ps->R), dim3(BP_TT), lds, s, ps->d,
                           ps->m, n_min, cnt, ps->gen, ps->seed, out);
        LDK_LAUNCH_CHECK();
        return LDK_OK;
    }
    const int64_t blocks = (cnt + BP_P - 1) / BP_P;
    if (blocks > 0x7fffffff) return LDK_ENOTSUP;
    const dim3 grid((unsigned)blocks, (unsigned)ps->R);
    BpArgs a{};
    a.d = ps->d;
    a.flags = ps->flags;
    a.n_min = n_min;
    a.cnt = cnt;
    // lms is read as 32-bit words from the word boundary at or below its
    // first byte (the same word, so within the allocation's page)
    const uintptr_t lp = reinterpret_cast<uintptr_t>(ps->lms);
    a.lms_off = (uint32_t)(lp & 3);
    const uint32_t *lmsw = reinterpret_cast<const uint32_t *>(lp & ~(uintptr_t)3);
    int prime = 1, m_max = 1;
    const int dims = ps->kind == LDK_FAURE ? 1 : ps->d;  // Faure: one base for all dimensions
    double cost[BP_MAX_D];
    for (int j = 0; j < dims; ++j) {
        int b = ps->base;
        if (ps->kind == LDK_HALTON) {
            do ++prime;
            while (!is_prime(prime));
            b = prime;
        }
        const int T = digits_kept(b), M = index_digits(b, n_max);
        int lg = 0;
        while ((1 << lg) < b) ++lg;
        if (M > BP_KMAX) return LDK_EINVAL;  // not reached for i < 2^32
        a.base[j] = (uint32_t)b;
        a.T[j] = (uint32_t)T;
        a.M[j] = (uint32_t)M;
        a.L[j] = (uint32_t)(21 + lg);
        a.mg[j] = (uint32_t)((((uint64_t)1 << (21 + lg)) + (uint64_t)b - 1) / (uint64_t)b);
        a.rb[j] = 1.0 / (double)b;
        double p = 1.0;
        for (int t = 0; t < T; ++t) p *= (double)b;
        a.bT[j] = p;
        m_max = M > m_max ? M : m_max;
        cost[j] = (double)T * (((M + 3) / 4) + 12) + 10.0 * M;  // VALU work per coordinate, roughly
    }
    if (ps->kind == LDK_HALTON) {
        // longest processing time first: dimensions by decreasing cost, each
        // to the wave with the least work so far; then each wave's list in turn
        int idx[BP_MAX_D], owner[BP_MAX_D];
        for (int j = 0; j < ps->d; ++j) idx[j] = j;
        for (int x = 1; x < ps->d; ++x)
            for (int y = x; y > 0 && cost[idx[y]] > cost[idx[y - 1]]; --y) {
                const int tmp = idx[y];
                idx[y] = idx[y - 1];
                idx[y - 1] = tmp;
            }
        double load[BP_WAVES] = {};
        for (int k = 0; k < ps->d; ++k) {
            int w = 0;
            for (int x = 1; x < BP_WAVES; ++x)
                if (load[x] < load[w]) w = x;
            owner[k] = w;
            load[w] += cost[idx[k]];
        }
        int q = 0;
        for (int w = 0; w < BP_WAVES; ++w) {
            a.wbeg[w] = (uint32_t)q;
            for (int k = 0; k < ps->d; ++k)
                if (owner[k] == w) a.ord[q++] = (uint32_t)idx[k];
        }
        a.wbeg[BP_WAVES] = (uint32_t)q;
    }
    const int mq = (m_max + 3) / 4;
    const int F = ps->flags & (LDK_BR_LMS | LDK_BR_DP | LDK_BR_DS);
    const int dmax = ps->kind == LDK_FAURE && ps->d > BP_DCH ? BP_DCH : ps->d;
    const size_t lds = (size_t)BP_P * dmax * sizeof(double);
    if (ps->kind == LDK_FAURE) {
        hipLaunchKernelGGL(k_faure_cmat, dim3((unsigned)ps->d), dim3(64), 0, s, ps->base,
                           digits_kept(ps->base), mq, static_cast<uint32_t *>(ws));
        LDK_LAUNCH_CHECK();
        const uint32_t *cm = static_cast<const uint32_t *>(ws);
#define BP_FAURE_F(MJ, FL)                                                                              \
    case FL:                                                                                            \
        hipLaunchKernelGGL((k_gen_faure<MJ, FL>), grid, dim3(BP_TT), lds, s, a, lmsw, ps->shift,        \
                           ps->perm, cm, out);                                                                    \
        break;
#define BP_FAURE(MJ)                                                                                    \
    case MJ:                                                                                            \
        switch (F) {                                                                                    \
            BP_FAURE_F(MJ, 0) BP_FAURE_F(MJ, 1) BP_FAURE_F(MJ, 2) BP_FAURE_F(MJ, 3)                     \
            BP_FAURE_F(MJ, 4) BP_FAURE_F(MJ, 5) BP_FAURE_F(MJ, 6) BP_FAURE_F(MJ, 7)                     \
        }                                                                                               \
        break;
        switch (mq) {
            BP_FAURE(1) BP_FAURE(2) BP_FAURE(3) BP_FAURE(4) BP_FAURE(5) BP_FAURE(6) BP_FAURE(7) BP_FAURE(8)
        default: return LDK_EINVAL;
        }
#undef BP_FAURE
#undef BP_FAURE_F
    } else {
#define BP_HALTON(FL)                                                                                   \
    case FL:                                                                                            \
        hipLaunchKernelGGL((k_gen_halton<FL>), grid, dim3(BP_TT), lds, s, a, lmsw, ps->shift, ps->perm,  \
                           out);                                                                        \
        break;
        switch (F) {
            BP_HALTON(0) BP_HALTON(1) BP_HALTON(2) BP_HALTON(3) BP_HALTON(4) BP_HALTON(5) BP_HALTON(6)
            BP_HALTON(7)
        }
#undef BP_HALTON
    }
    LDK_LAUNCH_CHECK();
    return LDK_OK;
}
