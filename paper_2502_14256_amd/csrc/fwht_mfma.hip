// Walsh-Hadamard transform of FP32 rows on the matrix cores, in split FP16.
//
// H_m is the Kronecker power of H_1 (Sec. 5.3: the recursion of H_m), so a
// length-2^m transform is a sequence of radix-16 stages y = H_16 x over the
// 4-bit digits of the index, in any order.  One stage on 16 vectors is the
// product Y = H_16 X of 16x16 matrices.  The FP32 data are split into two
// FP16 terms, X = X_hi + X_lo (X_lo = the rounding error of X_hi), and the
// stage is two accumulating matrix instructions with K = 16:
//   Y = H_16 X_lo + H_16 X_hi    (v_mfma_f32_16x16x16_f16, FP32 sums),
// exact in the products (H_16 is +-1) and in the FP32 accumulation up to
// rounding.  Each lane reads its four elements once and forms both terms
// (one [H_16 | H_16] instruction with K = 32 would put the high and low
// terms of an element in two lanes, so every element would be read twice).
// Before every stage the tile is scaled by a power of two so that
// |x| < 2^14 (the FP16 range), tracked from the tile maximum and the growth
// bound of 16 per stage, and the split is redone from the FP32 result: about
// 22 significant bits per stage.  A leftover of fewer than 4 index bits runs
// as FP32 butterflies.
//
// The passes follow the transform engine's plan (a row pass over the low
// bits, then column passes of 2^a strided rows x W contiguous columns, tiles
// of 4096 elements in LDS).  This is the same HBM traffic as the FP32
// butterfly passes (FP16 hi + lo is 4 bytes, like FP32): the matrix cores
// only replace the butterfly arithmetic and most of the LDS exchanges.
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

__global__ __launch_bounds__(FM_THREADS) void k_fwht_mfma(FmArgs a)
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

}  // namespace

}  // namespace ldk

using namespace ldk;

extern "C" int ldk_fwht_split16(int B, int m, const float *in, float *out, ldk_stream stream)
{
    if (B < 0 || m < 0 || m > LDK_MAX_M || B > 65535) return LDK_EINVAL;
    if (B == 0) return LDK_OK;
    if (!in || !out) return LDK_EINVAL;
    const Plan pl = make_plan(m, FM_LOG_TILE);
    const hipStream_t s = as_stream(stream);
    if (m == 0) {
        if (in != out) LDK_HIP_CHECK(hipMemcpyAsync(out, in, sizeof(float) * (size_t)B,
                                                    hipMemcpyDeviceToDevice, s));
        return LDK_OK;
    }
    const float scale = (float)(1.0 / std::sqrt((double)((int64_t)1 << m)));
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
        hipLaunchKernelGGL(k_fwht_mfma, dim3((unsigned)blocks), dim3(FM_THREADS), 0, s, a);
        LDK_LAUNCH_CHECK();
    }
    return LDK_OK;
}
