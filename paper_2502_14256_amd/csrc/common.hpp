// Shared device/host helpers of the ldk HIP library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/ldk.h"

namespace ldk {

// ---------------------------------------------------------------------------
// Host-side status handling
// ---------------------------------------------------------------------------
void set_hip_error(hipError_t e);
int ensure_init();  // builds the twiddle tables on the current device once
int noalloc_setup();  // device address of ldk_solve_noalloc's scratch (noalloc.hip)

#define LDK_HIP_CHECK(expr)                      \
    do {                                         \
        hipError_t _e = (expr);                  \
        if (_e != hipSuccess) {                  \
            ::ldk::set_hip_error(_e);            \
            return LDK_EDEVICE;                  \
        }                                        \
    } while (0)

// Check the launch that was just enqueued.
#define LDK_LAUNCH_CHECK() LDK_HIP_CHECK(hipGetLastError())

inline hipStream_t as_stream(ldk_stream s) { return reinterpret_cast<hipStream_t>(s); }

// ---------------------------------------------------------------------------
// Complex numbers (interleaved re, im)
// ---------------------------------------------------------------------------
template <typename R>
struct alignas(2 * sizeof(R)) cplx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename R>
__device__ __forceinline__ cplx<R> cmulc(cplx<R> a, cplx<R> b)
{
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}

// ---------------------------------------------------------------------------
// Twiddle tables.  W_N^p = exp(-2 pi i p / N).
//   tw_hi[q] = W_{2^13}^q,  tw_lo[q] = W_{2^26}^q   (q < 2^13)
// so W_{2^26}^P = tw_hi[P >> 13] * tw_lo[P & 8191].  Entries are correctly
// rounded (built on the host in extended precision by ldk_init).
// ---------------------------------------------------------------------------
constexpr int TW_BITS = 13;
constexpr int TW_MAX_LOG = 2 * TW_BITS;  // largest N = 2^26 handled by the tables
static_assert(TW_MAX_LOG == LDK_MAX_M, "twiddle tables must cover every transform length");
constexpr int TW_SIZE = 1 << TW_BITS;

extern __device__ cplx<double> g_tw_hi_f64[TW_SIZE];
extern __device__ cplx<double> g_tw_lo_f64[TW_SIZE];
extern __device__ cplx<float> g_tw_hi_f32[TW_SIZE];
extern __device__ cplx<float> g_tw_lo_f32[TW_SIZE];

template <typename R>
struct tw_tables;
template <>
struct tw_tables<double> {
    static __device__ __forceinline__ const cplx<double> *hi() { return g_tw_hi_f64; }
    static __device__ __forceinline__ const cplx<double> *lo() { return g_tw_lo_f64; }
};
template <>
struct tw_tables<float> {
    static __device__ __forceinline__ const cplx<float> *hi() { return g_tw_hi_f32; }
    static __device__ __forceinline__ const cplx<float> *lo() { return g_tw_lo_f32; }
};

// W_{2^k}^p for k <= 13 (one table read).
template <typename R>
__device__ __forceinline__ cplx<R> tw_small(uint32_t p, int k)
{
    return tw_tables<R>::hi()[(p << (TW_BITS - k)) & (TW_SIZE - 1)];
}
// W_{2^k}^p for k <= 26 (two reads, one product).
template <typename R>
__device__ __forceinline__ cplx<R> tw_any(uint64_t p, int k)
{
    const uint32_t P = (uint32_t)((p << (TW_MAX_LOG - k)) & ((1u << TW_MAX_LOG) - 1));
    return cmul(tw_tables<R>::hi()[P >> TW_BITS], tw_tables<R>::lo()[P & (TW_SIZE - 1)]);
}

// ---------------------------------------------------------------------------
// Bits
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t brev64(uint64_t v) { return __builtin_bitreverse64(v); }
__device__ __forceinline__ uint32_t brev_bits(uint32_t v, int bits)
{
    return bits == 0 ? 0u : (__builtin_bitreverse32(v) >> (32 - bits));
}
__device__ __forceinline__ int clz64(uint64_t v) { return __builtin_clzll(v); }
__device__ __forceinline__ int ctz64(uint64_t v) { return __builtin_ctzll(v); }

// x = u * 2^-64 rounded to nearest: hi * 2^32 + lo is formed exactly inside
// one fused multiply-add and rounded once.
__device__ __forceinline__ double unit_f64(uint64_t u)
{
    return __fma_rn((double)(uint32_t)(u >> 32), 4294967296.0, (double)(uint32_t)u) * 0x1p-64;
}
__device__ __forceinline__ float unit_f32(uint64_t u)
{
    return __fmaf_rn((float)(uint32_t)(u >> 32), 4294967296.0f, (float)(uint32_t)u) * 0x1p-64f;
}

}  // namespace ldk
