// Walsh-Hadamard transform of FP32 rows on the matrix cores, in split FP16.
//
// H_m is the Kronecker power of H_1 (Sec. 5.3: the recursion of H_m), so a
// length-2^m transform is a sequence of radix-16 stages y = H_16 x over the
// 4-bit digits of the index, in any order.  One stage on 16 vectors is the
// product Y = H_16 X of 16x16 matrices.  The FP32 data are split into two
// FP16 terms, X = X_hi + X_lo (X_lo = the rounding error of X_hi), and the
// stage is one matrix instruction with K = 32 over both terms,
//   Y = [H | H] [X_hi ; X_lo]     (v_mfma_f32_16x16x32_f16, FP32 sums),
// exact in the products (the entries of H are +-2^-k) and in the FP32
// accumulation up to rounding.  The K order of the instruction is free as
// long as both operands use the same one, so each lane keeps the high and low
// terms of its own four elements in one 8-wide operand and every element is
// read once.
//
// Register-resident stages (m >= 12): a workgroup of 4 waves takes a tile of
// 2^12 elements, 16 per lane.  Lane l holds, for each of its four 16x16
// blocks, four elements whose "K digit" (the digit the next stage transforms)
// is 4 (l / 16) + i, i < 4, and whose "N digit" is l mod 16.  A stage with the
// data as the right operand (D = H X) transforms the K digit in place; a stage
// with the data as the left operand (D = X H) transforms the K digit and
// leaves it at l mod 16 while the N digit moves to 4 (l / 16) + i.  So the low
// 8 bits of a row tile take two stages with no data movement, and each further
// digit costs one LDS exchange of the tile.  Partial digits (pass axes that
// are not a multiple of 4 bits) use a masked H_16 (H_2^k on the masked bits,
// the identity on the others).  The matrix is H / 2^k (k digit bits), so a
// stage never increases the largest magnitude: the tile is scaled once per
// pass by a power of two that puts its maximum just below 2^14 (the FP16
// range), and the store multiplies by 2^(pass bits) over that scale.
//
// Passes (m >= 12): a row pass over the low 12 bits (contiguous tiles), then
// column passes of a <= 8 axis bits over tiles of 2^a strided rows x
// 2^(12 - a) contiguous columns; the 4 lowest column bits of a tile are the
// N digit, so global loads and stores move 64-byte runs.  The solve and
// matvec (filter by scale / (lambda + sigma^2) or scale * lambda) run the top
// pass as forward stages, the filter in FP64 on the register values, and the
// same stages again (H_m is its own inverse up to 1/n).  Rows of fewer than
// 2^12 elements take a per-row LDS kernel with one exchange per stage.
#include <cmath>

#include "passkit.hpp"
#include "transform.hpp"

namespace ldk {

namespace {

typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));

constexpr int FM_THREADS = 256;
constexpr int FM_LOG_TILE = 12;
constexpr int FM_TILE = 1 << FM_LOG_TILE;
constexpr int FM_PER_THREAD = FM_TILE / FM_THREADS;

__device__ __forceinline__ int pad(int e) { return e + (e >> 4); }

struct FmArgs {
    const float *src;
    float *dst;
    int64_t rows;
    int m;
    PassGeom g;
    float scale;  // applied at the store (n^-1/2 on the last pass)
};

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// 2^e with e = 14 - ceil(log2(bound)): |x| * 2^e < 2^14 for |x| <= bound.
__device__ __forceinline__ float split_scale(float bound)
{
    if (!(bound > 0.0f)) return 1.0f;
    int e;
    const float f = frexpf(bound, &e);  // bound = f 2^e, 0.5 <= f < 1
    (void)f;
    const int k = 14 - e;
    return ldexpf(1.0f, k > 126 ? 126 : k);  // 2^126 keeps the scale finite
}

// Rows of fewer than 2^12 elements: one row per workgroup, the row in LDS,
// one LDS round trip per radix-16 stage (two K = 16 instructions, high and
// low terms), leftover bits as FP32 butterflies.
__global__ __launch_bounds__(FM_THREADS) void k_fwht_mfma_row(FmArgs a)
{
    __shared__ float tile[FM_TILE + FM_TILE / 16];
    __shared__ float red[FM_THREADS / 64];
    const int A = a.g.a, logW = a.g.logW, b0 = a.g.b0;
    const int W = 1 << logW;
    const int S = 1 << (A + logW);  // elements in this tile (<= FM_TILE)
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;

    const int64_t cb_count = (int64_t)1 << (b0 - logW);
    const int64_t outer_count = (int64_t)1 << (a.m - b0 - A);
    int64_t bid = kit::xcd_tile(blockIdx.x, gridDim.x);
    const int64_t cb = bid % cb_count;
    bid /= cb_count;
    const int64_t outer = bid % outer_count;
    const int64_t row = bid / outer_count;
    const int64_t base = row * ((int64_t)1 << a.m) + outer * ((int64_t)1 << (b0 + A)) + (cb << logW);
    const int64_t rstride = (int64_t)1 << b0;
    auto gidx = [&](int q) -> int64_t {
        return base + (int64_t)(q >> logW) * rstride + (q & (W - 1));
    };

    // ---- load (coalesced: q = t + 256 i) and the tile maximum
    float mx = 0.0f;
    for (int i = 0; i < FM_PER_THREAD; ++i) {
        const int q = t + FM_THREADS * i;
        if (q < S) {
            const float v = a.src[gidx(q)];
            tile[pad(q)] = v;
            mx = fmaxf(mx, fabsf(v));
        }
    }
    mx = wave_max(mx);
    if (lane == 0) red[wave] = mx;
    __syncthreads();
    float bound = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));

    // ---- leftover axis bits [0, rem) as FP32 butterflies
    const int rem = A & 3;
    for (int b = 0; b < rem; ++b) {
        const int h = 1 << b;
        for (int p = t; p < S / 2; p += FM_THREADS) {
            // pair p: axis bit b clear / set, other bits from p
            const int w = p & (W - 1), ro = p >> logW;
            const int r0 = ((ro >> b) << (b + 1)) | (ro & (h - 1));
            const int e0 = r0 * W + w, e1 = (r0 + h) * W + w;
            const float x = tile[pad(e0)], y = tile[pad(e1)];
            tile[pad(e0)] = x + y;
            tile[pad(e1)] = x - y;
        }
        __syncthreads();
        bound *= 2.0f;
    }

    // ---- radix-16 stages on the matrix cores
    // A = H_16: lane l holds A[l % 16][4 (l / 16) + i], i < 4 (the K = 16 operand layout)
    half4 hmat;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int k = 4 * (lane >> 4) + i;
        hmat[i] = (_Float16)((__popc((lane & 15) & k) & 1) ? -1.0f : 1.0f);
    }
    const int kb = 4 * (lane >> 4);  // digit values read by this lane: kb .. kb + 3
    const int col = lane & 15;       // vector within the instruction
    const int ob = 4 * (lane >> 4);        // digit values written: ob .. ob + 3
    const int nvec = S >> 4;
    for (int q = 0; q * 4 + rem < A; ++q) {
        const int p = rem + 4 * q;  // axis bit of this digit
        const float sc = split_scale(bound);
        const float inv = 1.0f / sc;  // exact: a power of two
        for (int mu = wave; mu * 16 < nvec; mu += FM_THREADS / 64) {
            // column `col` of this instruction is vector v; a tile of fewer
            // than 256 elements leaves columns without a vector (zeros in,
            // nothing out: a column of D depends on its own column of B only)
            const int v = 16 * mu + col;
            const bool live = v < nvec;
            const int w = v & (W - 1), ro = v >> logW;
            const int rlow = ro & ((1 << p) - 1), rhigh = (ro >> p) << (p + 4);
            half4 bhi, blo;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = rlow | ((kb + i) << p) | rhigh;
                const float x = live ? tile[pad(r * W + w)] * sc : 0.0f;
                const _Float16 hi = (_Float16)x;
                bhi[i] = hi;
                blo[i] = (_Float16)(x - (float)hi);
            }
            const float4v zero = {0.0f, 0.0f, 0.0f, 0.0f};
            float4v d = __builtin_amdgcn_mfma_f32_16x16x16f16(hmat, blo, zero, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_16x16x16f16(hmat, bhi, d, 0, 0, 0);
            if (live) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = rlow | ((ob + i) << p) | rhigh;
                    tile[pad(r * W + w)] = d[i] * inv;
                }
            }
        }
        __syncthreads();
        bound *= 16.0f;
    }

    // ---- store
    for (int i = 0; i < FM_PER_THREAD; ++i) {
        const int q = t + FM_THREADS * i;
        if (q < S) a.dst[gidx(q)] = tile[pad(q)] * a.scale;
    }
}

// ---------------------------------------------------------------------------
// Register-resident passes (m >= 12)
// ---------------------------------------------------------------------------
typedef _Float16 half8 __attribute__((ext_vector_type(8)));

// Tile index q (12 bits) of register slot 4 beta + i of lane l in wave w.
// ROW_A: K digit = bits 0-3, N digit = bits 4-7, beta = bits 8-9, w = bits 10-11.
__device__ __forceinline__ int q_row_a(int l, int w, int beta, int i)
{
    return i | ((l >> 4) << 2) | ((l & 15) << 4) | (beta << 8) | (w << 10);
}
// ROW_B: K digit = bits 4-7, N digit = bits 0-3 (ROW_A after a left-operand stage).
__device__ __forceinline__ int q_row_b(int l, int w, int beta, int i)
{
    return (l & 15) | ((i | ((l >> 4) << 2)) << 4) | (beta << 8) | (w << 10);
}
// COL(kb), 4 <= kb <= 8: N digit = bits 0-3, K digit = bits kb..kb+3, and
// beta | w << 2 in the other bits of [4, 12) in increasing order.
__device__ __forceinline__ int q_col(int kb, int l, int w, int beta, int i)
{
    const int K = i | ((l >> 4) << 2), o = beta | (w << 2), lo = kb - 4;
    return (l & 15) | (K << kb) | ((o & ((1 << lo) - 1)) << 4) | ((o >> lo) << (kb + 4));
}

enum { LAY_ROW_A = 0, LAY_ROW_B = 1, LAY_COL = 2 };

__device__ __forceinline__ int q_of(int lay, int kb, int l, int w, int beta, int i)
{
    return lay == LAY_ROW_A ? q_row_a(l, w, beta, i)
                            : lay == LAY_ROW_B ? q_row_b(l, w, beta, i) : q_col(kb, l, w, beta, i);
}

// LDS word of tile index q: bits 4-5 XOR a hash of bits 6-11, so that the four
// 16-lane groups of an exchange (2^6 .. 2^10 elements apart) use four
// different 16-bank groups.  A bijection of [0, 2^12).
__device__ __forceinline__ int swz(int q) { return q ^ ((((q >> 6) ^ (q >> 8) ^ (q >> 10)) & 3) << 4); }

// H_16 / 2^k restricted to the k digit bits in `mask` (H_2 / 2 on each
// masked bit, the identity on the others), laid out as the 8-wide operand of
// lane l: slot s holds row l mod 16, column 4 (l / 16) + (s mod 4), for both
// the high (s < 4) and the low (s >= 4) term.  The entries +-2^-k are exact
// in FP16, and a stage never increases the largest magnitude.  Symmetric, so
// the same register is the left operand (D = H X) and the right one (D = X H).
__device__ __forceinline__ half8 hmask_operand(int lane, int mask)
{
    half8 h;
    const int r = lane & 15;
    const float mag = 1.0f / (float)(1 << __popc(mask & 15));
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int c = 4 * (lane >> 4) + (s & 3);
        const bool zero = ((r ^ c) & ~mask & 15) != 0;
        h[s] = (_Float16)(zero ? 0.0f : ((__popc(r & c & mask) & 1) ? -mag : mag));
    }
    return h;
}

typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef float float2v __attribute__((ext_vector_type(2)));

// One radix-16 stage of the four blocks of this wave on values already
// scaled below 2^14.  LEFT: data as the left operand (the K digit ends at
// l mod 16).  Split: hi = FP16(x) and lo = FP16(x - hi), both rounded to
// nearest (two values per conversion); x - hi is exact and formed by one
// mixed-precision FMA with the FP16 operand (neg1 = -1, a run-time value so
// that the compiler keeps the fused form).  |x - hi - lo| <= 2^-23 |x| for
// values in the FP16 normal range.
template <bool LEFT>
__device__ __forceinline__ void f16_stage(float (&v)[16], half8 hm, float neg1)
{
#pragma unroll
    for (int beta = 0; beta < 4; ++beta) {
        half8 x;
#pragma unroll
        for (int i = 0; i < 4; i += 2) {
            const float a0 = v[4 * beta + i], a1 = v[4 * beta + i + 1];
            const float2v av = {a0, a1};
            const half2v h = __builtin_convertvector(av, half2v);
            const float2v r = {__builtin_fmaf((float)h[0], neg1, a0),
                               __builtin_fmaf((float)h[1], neg1, a1)};
            const half2v lo = __builtin_convertvector(r, half2v);
            x[i] = h[0];
            x[i + 1] = h[1];
            x[4 + i] = lo[0];
            x[4 + i + 1] = lo[1];
        }
        const float4v zero = {0.0f, 0.0f, 0.0f, 0.0f};
        const float4v d = LEFT ? __builtin_amdgcn_mfma_f32_16x16x32_f16(x, hm, zero, 0, 0, 0)
                               : __builtin_amdgcn_mfma_f32_16x16x32_f16(hm, x, zero, 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) v[4 * beta + i] = d[i];
    }
}

// Largest |v| over the workgroup's tile (red: 4 floats of LDS; one barrier).
__device__ __forceinline__ float tile_max(const float (&v)[16], float *red, int l, int w)
{
    float mx = 0.0f;
#pragma unroll
    for (int j = 0; j < 16; ++j) mx = fmaxf(mx, fabsf(v[j]));
    mx = wave_max(mx);
    if (l == 0) red[w] = mx;
    __syncthreads();
    return fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

// Element offset within a row of tile index q: columns (the low logW bits)
// stay, the row bits move to bit b0.  A map of bit fields, so the offset of
// the OR of disjoint fields is the sum of their offsets.
__device__ __forceinline__ uint32_t phi(int q, int logW, int b0)
{
    return ((uint32_t)(q >> logW) << b0) | (uint32_t)(q & ((1 << logW) - 1));
}

// Tile exchange through LDS from layout (la, ka) to layout (lb, kb).
__device__ __forceinline__ void f16_exchange(float (&v)[16], float *lds, int la, int ka, int lb,
                                             int kb, int l, int w, bool wait_readers)
{
    if (wait_readers) __syncthreads();  // earlier reads of the tile are done
#pragma unroll
    for (int beta = 0; beta < 4; ++beta)
#pragma unroll
        for (int i = 0; i < 4; ++i) lds[swz(q_of(la, ka, l, w, beta, i))] = v[4 * beta + i];
    __syncthreads();
#pragma unroll
    for (int beta = 0; beta < 4; ++beta)
#pragma unroll
        for (int i = 0; i < 4; ++i) v[4 * beta + i] = lds[swz(q_of(lb, kb, l, w, beta, i))];
}

struct F16Args {
    const float *src;
    float *dst;
    int m;
    int b0, a, logW;  // axis bits [b0, b0 + a) (12 for the row pass), tile columns 2^logW
    float scale;      // plain passes: multiplies the stored values
    float neg1;       // -1 (see f16_stage)
    // top pass of a solve (mode 0) or matvec (mode 1): filter between the
    // forward and the inverse stages
    const double *lam;
    int nrhs;
    int mode;
    double sigma2;
    double fscale;
    // plain passes, optional: store |x|^2 in FP64 here instead of x in dst
    double *pow;
};

// ROW: the row pass (a = 12, logW = 0); TOP: forward stages, filter, inverse
// stages; VEC: 16-byte aligned rows (vector loads and stores in ROW_A layout).
// Scaling: at the load the tile is multiplied by sc = 2^(14 - e), 2^e > the
// tile maximum, and the stages (H / 2^k) keep every value below 2^14; the
// true transform is the register value times 2^(digit bits) / sc.
template <bool ROW, bool TOP, bool VEC>
__global__ __launch_bounds__(256) void k_fwht16(F16Args a)
{
    __shared__ float lds[1 << 12];
    __shared__ float red[8];
    const int l = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const int logW = ROW ? 0 : a.logW, A = ROW ? 12 : a.a, b0 = ROW ? 0 : a.b0;
    // workgroup -> (row, outer block, column block)
    const int64_t cb_count = (int64_t)1 << (b0 - logW);
    const int64_t outer_count = (int64_t)1 << (a.m - b0 - A);
    int64_t bid = kit::xcd_tile(blockIdx.x, gridDim.x);
    const int64_t cb = bid % cb_count;
    bid /= cb_count;
    const int64_t outer = bid % outer_count;
    const int64_t row = bid / outer_count;
    const int64_t n = (int64_t)1 << a.m;
    const int64_t tbase = row * n + outer * ((int64_t)1 << (b0 + A)) + (cb << logW);
    const float *src = a.src + tbase;
    float *dst = a.dst + tbase;

    // layouts and digit masks of the stages
    //   row pass:    ROW_A -L-> ROW_B -R-> [exchange] COL(8) -R->
    //   column pass: COL(k1) -R-> [exchange, when a > 4] COL(8) -R->
    const int k1 = ROW ? 0 : (logW < 8 ? logW : 8);
    const int mask1 = ROW ? 15 : ((15 << (logW - k1)) & 15);
    const bool two = ROW || logW < 8;  // a second digit after an exchange
    const int mask2 = ROW ? 15 : ((15 << (logW - 4)) & 15);
    const int lay0 = ROW ? LAY_ROW_A : LAY_COL;
    float v[16];

    // ---- load: lane part of the offset in a register, slot part uniform
    {
        const uint32_t lo = phi(q_of(lay0, k1, l, 0, 0, 0), logW, b0);
#pragma unroll
        for (int beta = 0; beta < 4; ++beta) {
            if (ROW && VEC) {
                const float *p = src + phi(q_of(LAY_ROW_A, 0, 0, w, beta, 0), 0, 0);
                const float4v x = *reinterpret_cast<const float4v *>(p + lo);
#pragma unroll
                for (int i = 0; i < 4; ++i) v[4 * beta + i] = x[i];
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    v[4 * beta + i] = (src + phi(q_of(lay0, k1, 0, w, beta, i), logW, b0))[lo];
            }
        }
    }
    float sc = split_scale(tile_max(v, red, l, w));
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] *= sc;

    // ---- forward stages
    const half8 hm1 = hmask_operand(l, mask1);
    const half8 hm2 = two ? hmask_operand(l, mask2) : hm1;
    if (ROW) {
        f16_stage<true>(v, hm1, a.neg1);   // bits 0-3, ROW_A -> ROW_B
        f16_stage<false>(v, hm1, a.neg1);  // bits 4-7
        f16_exchange(v, lds, LAY_ROW_B, 0, LAY_COL, 8, l, w, false);
        f16_stage<false>(v, hm2, a.neg1);  // bits 8-11
    } else {
        f16_stage<false>(v, hm1, a.neg1);
        if (two) {
            f16_exchange(v, lds, LAY_COL, k1, LAY_COL, 8, l, w, false);
            f16_stage<false>(v, hm2, a.neg1);
        }
    }
    int lay = LAY_COL, kb = two ? 8 : k1;
    // true values = v * 2^A / sc
    float gain = ldexpf(1.0f, A) / sc;

    if (TOP) {
        // ---- filter: scale / (lambda + sigma^2) or scale * lambda, in FP64,
        // on the true values; then a new scale for the inverse stages
        const double *lam = a.lam + (row / a.nrhs) * n + (tbase - row * n);
        const uint32_t lo = phi(q_of(lay, kb, l, 0, 0, 0), logW, b0);
#pragma unroll
        for (int beta = 0; beta < 4; ++beta)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const double lv = (lam + phi(q_of(lay, kb, 0, w, beta, i), logW, b0))[lo];
                const double f = a.mode == 0 ? a.fscale / (lv + a.sigma2) : a.fscale * lv;
                v[4 * beta + i] *= (float)(f * (double)gain);
            }
        // (the barrier inside also ends the forward exchange's reads)
        sc = split_scale(tile_max(v, red + 4, l, w));
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] *= sc;
        gain = ldexpf(1.0f, A) / sc;
        // ---- the same stages in reverse order
        if (ROW) {
            f16_stage<false>(v, hm2, a.neg1);  // bits 8-11
            f16_exchange(v, lds, LAY_COL, 8, LAY_ROW_B, 0, l, w, false);
            f16_stage<true>(v, hm1, a.neg1);   // bits 4-7, ROW_B -> ROW_A
            f16_stage<false>(v, hm1, a.neg1);  // bits 0-3
            lay = LAY_ROW_A;
        } else {
            if (two) {
                f16_stage<false>(v, hm2, a.neg1);
                f16_exchange(v, lds, LAY_COL, 8, LAY_COL, k1, l, w, false);
                kb = k1;
            }
            f16_stage<false>(v, hm1, a.neg1);
        }
    } else {
        gain *= a.scale;
    }

    // ---- store
    const uint32_t lo = phi(q_of(lay, kb, l, 0, 0, 0), logW, b0);
#pragma unroll
    for (int beta = 0; beta < 4; ++beta) {
        if (ROW && TOP && VEC) {
            float *p = dst + phi(q_of(LAY_ROW_A, 0, 0, w, beta, 0), 0, 0);
            float4v x;
#pragma unroll
            for (int i = 0; i < 4; ++i) x[i] = v[4 * beta + i] * gain;
            *reinterpret_cast<float4v *>(p + lo) = x;
        } else if (!TOP && a.pow) {
            double *pw = a.pow + tbase;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const double x = (double)(v[4 * beta + i] * gain);
                (pw + phi(q_of(lay, kb, 0, w, beta, i), logW, b0))[lo] = x * x;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                (dst + phi(q_of(lay, kb, 0, w, beta, i), logW, b0))[lo] = v[4 * beta + i] * gain;
        }
    }
}

}  // namespace

// Passes of the register-resident transform (m >= 12): the row pass, then
// column passes of at most 8 bits.
struct F16Plan {
    int P;
    int b0[3], a[3];
};

static F16Plan f16_plan(int m)
{
    F16Plan p{};
    p.b0[0] = 0;
    p.a[0] = 12;
    p.P = 1;
    const int r = m - 12;
    const int C = (r + 7) / 8;
    int b0 = 12;
    for (int c = 0; c < C; ++c) {
        const int a = r / C + (c < r % C ? 1 : 0);
        p.b0[p.P] = b0;
        p.a[p.P++] = a;
        b0 += a;
    }
    return p;
}

template <bool TOP>
static int launch_f16(const F16Plan &pl, int p, F16Args a, int64_t rows, bool vec, hipStream_t s)
{
    a.b0 = pl.b0[p];
    a.a = pl.a[p];
    a.logW = 12 - a.a;
    const int64_t blocks = rows << (a.m - 12);
    if (blocks > 0x7fffffff) return LDK_ENOTSUP;
    const dim3 g((unsigned)blocks), b(256);
    if (p == 0) {
        if (vec) hipLaunchKernelGGL((k_fwht16<true, TOP, true>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_fwht16<true, TOP, false>), g, b, 0, s, a);
    } else {
        hipLaunchKernelGGL((k_fwht16<false, TOP, false>), g, b, 0, s, a);
    }
    LDK_LAUNCH_CHECK();
    return LDK_OK;
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// Plain transform of `rows` rows, m >= 12; the last pass scales by `scale`
// and, with pow, stores the squares there (FP64) instead of in out.
static int f16_transform(int m, int64_t rows, const float *in, float *out, float scale, hipStream_t s,
                         double *pow = nullptr)
{
    const F16Plan pl = f16_plan(m);
    const bool vec = aligned16(in) && aligned16(out);
    for (int p = 0; p < pl.P; ++p) {
        F16Args a{};
        a.src = p == 0 ? in : out;
        a.dst = out;
        a.m = m;
        a.scale = p == pl.P - 1 ? scale : 1.0f;
        a.neg1 = -1.0f;
        a.pow = p == pl.P - 1 ? pow : nullptr;
        const int st = launch_f16<false>(pl, p, a, rows, vec, s);
        if (st) return st;
    }
    return LDK_OK;
}

int fwht16_power(int m, int64_t rows, const float *y, float *tmp, double *pw, hipStream_t s)
{
    if (m < 12) return LDK_ENOTSUP;
    return f16_transform(m, rows, y, tmp, 1.0f, s, pw);
}

int fwht16_apply(int mode, int m, int64_t rows, int nrhs, const double *lam, double sigma2,
                 const float *y, float *c, hipStream_t s)
{
    if (m < 12) return LDK_ENOTSUP;
    const F16Plan pl = f16_plan(m);
    const bool vec = aligned16(y) && aligned16(c);
    const double fscale = 1.0 / (double)((int64_t)1 << m);
    // forward passes below the top one, the top pass, the inverse passes
    for (int p = 0; p < 2 * pl.P - 1; ++p) {
        const int q = p < pl.P ? p : 2 * pl.P - 2 - p;
        F16Args a{};
        a.src = p == 0 ? y : c;
        a.dst = c;
        a.m = m;
        a.scale = 1.0f;
        a.neg1 = -1.0f;
        a.lam = lam;
        a.nrhs = nrhs;
        a.mode = mode == PM_SOLVE ? 0 : 1;
        a.sigma2 = sigma2;
        a.fscale = fscale;
        const int st = p == pl.P - 1 ? launch_f16<true>(pl, q, a, rows, vec, s)
                                     : launch_f16<false>(pl, q, a, rows, vec, s);
        if (st) return st;
    }
    return LDK_OK;
}

}  // namespace ldk

using namespace ldk;

extern "C" int ldk_fwht_split16(int B, int m, const float *in, float *out, ldk_stream stream)
{
    if (B < 0 || m < 0 || m > LDK_MAX_M || B > 65535) return LDK_EINVAL;
    if (B == 0) return LDK_OK;
    if (!in || !out) return LDK_EINVAL;
    const hipStream_t s = as_stream(stream);
    if (m == 0) {
        if (in != out) LDK_HIP_CHECK(hipMemcpyAsync(out, in, sizeof(float) * (size_t)B,
                                                    hipMemcpyDeviceToDevice, s));
        return LDK_OK;
    }
    const float scale = (float)(1.0 / std::sqrt((double)((int64_t)1 << m)));
    if (m >= 12) return f16_transform(m, B, in, out, scale, s);
    const Plan pl = make_plan(m, FM_LOG_TILE);
    for (int p = 0; p < pl.P; ++p) {
        FmArgs a{};
        a.src = p == 0 ? in : out;
        a.dst = out;
        a.rows = B;
        a.m = m;
        a.g = pl.pass[p];
        a.scale = p == pl.P - 1 ? scale : 1.0f;
        const int64_t blocks = (int64_t)B << (m - a.g.a - a.g.logW);
        if (blocks > 0x7fffffff) return LDK_ENOTSUP;
        hipLaunchKernelGGL(k_fwht_mfma_row, dim3((unsigned)blocks), dim3(FM_THREADS), 0, s, a);
        LDK_LAUNCH_CHECK();
    }
    return LDK_OK;
}
