// Device building blocks of the pass kernels: element arithmetic, radix-2^g
// register stages, tile index maps, twiddles, LDS exchange, global IO.
#pragma once

#include <type_traits>

#include "transform.hpp"

namespace ldk {
namespace kit {

constexpr int LDS_PAD_SHIFT = 4;  // one padding element every 16

__device__ __forceinline__ int lds_idx(int q) { return q + (q >> LDS_PAD_SHIFT); }

// ---- element arithmetic -------------------------------------------------
template <typename R>
__device__ __forceinline__ R add(R a, R b) { return a + b; }
template <typename R>
__device__ __forceinline__ cplx<R> add(cplx<R> a, cplx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ R sub(R a, R b) { return a - b; }
template <typename R>
__device__ __forceinline__ cplx<R> sub(cplx<R> a, cplx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ R scl(R a, R s) { return a * s; }
template <typename R>
__device__ __forceinline__ cplx<R> scl(cplx<R> a, R s) { return {a.re * s, a.im * s}; }

// W_16^q = exp(-2 pi i q / 16), q = 0..7, as compile-time constants.
template <typename R, int q>
__device__ __forceinline__ cplx<R> mul_w16(cplx<R> v)
{
    constexpr double C1 = 0.92387953251128675613, S1 = 0.38268343236508977173;
    constexpr double H = 0.70710678118654752440;
    if constexpr (q == 0) return v;
    if constexpr (q == 4) return {v.im, -v.re};  // * (-i)
    if constexpr (q == 2) return {(R)H * (v.re + v.im), (R)H * (v.im - v.re)};
    if constexpr (q == 6) return {(R)H * (v.im - v.re), -(R)H * (v.re + v.im)};
    constexpr double c = q == 1 ? C1 : q == 3 ? S1 : q == 5 ? -S1 : -C1;
    constexpr double sn = q == 1 ? -S1 : q == 3 ? -C1 : q == 5 ? -C1 : -S1;
    return {(R)c * v.re - (R)sn * v.im, (R)c * v.im + (R)sn * v.re};
}
template <typename R, int q>
__device__ __forceinline__ cplx<R> mulc_w16(cplx<R> v)  // * conj(W_16^q)
{
    const cplx<R> t = mul_w16<R, q>(cplx<R>{v.re, -v.im});
    return {t.re, -t.im};
}

// Butterfly stage of span h = 2^b on the registers of one thread.
// FFT forward (DIT):  (u, w) -> (u + W_{2h}^j w, u - W_{2h}^j w), j = i mod h.
template <typename R, int E, int b, int i = 0>
__device__ __forceinline__ void fft_stage_fwd(cplx<R> (&v)[E])
{
    if constexpr (i < E) {
        constexpr int h = 1 << b;
        if constexpr ((i & h) == 0) {
            constexpr int j = i & (h - 1);
            const cplx<R> w = mul_w16<R, (j * (8 / h)) & 7>(v[i + h]);
            const cplx<R> u = v[i];
            v[i] = add(u, w);
            v[i + h] = sub(u, w);
        }
        fft_stage_fwd<R, E, b, i + 1>(v);
    }
}
// FFT inverse: (x, y) -> (x + y, conj(W_{2h}^j) (x - y)).
template <typename R, int E, int b, int i = 0>
__device__ __forceinline__ void fft_stage_inv(cplx<R> (&v)[E])
{
    if constexpr (i < E) {
        constexpr int h = 1 << b;
        if constexpr ((i & h) == 0) {
            constexpr int j = i & (h - 1);
            const cplx<R> x = v[i], y = v[i + h];
            v[i] = add(x, y);
            v[i + h] = mulc_w16<R, (j * (8 / h)) & 7>(sub(x, y));
        }
        fft_stage_inv<R, E, b, i + 1>(v);
    }
}
// FWHT butterfly (x, y) -> (x + y, x - y).
template <typename T, int E, int b, int i = 0>
__device__ __forceinline__ void wht_stage(T (&v)[E])
{
    if constexpr (i < E) {
        constexpr int h = 1 << b;
        if constexpr ((i & h) == 0) {
            const T x = v[i], y = v[i + h];
            v[i] = add(x, y);
            v[i + h] = sub(x, y);
        }
        wht_stage<T, E, b, i + 1>(v);
    }
}

// In-register transform over the low gs bits of the register index.
template <typename T, int E, int LOGE, bool INV, int b = 0>
__device__ __forceinline__ void reg_fwd(T (&v)[E], int gs)
{
    if constexpr (b < LOGE) {
        if (b < gs) {
            if constexpr (std::is_floating_point<T>::value)
                wht_stage<T, E, b>(v);
            else
                fft_stage_fwd<decltype(T::re), E, b>(v);
        }
        reg_fwd<T, E, LOGE, INV, b + 1>(v, gs);
    }
}
template <typename T, int E, int LOGE, int b = LOGE - 1>
__device__ __forceinline__ void reg_inv(T (&v)[E], int gs)
{
    if constexpr (b >= 0) {
        if (b < gs) {
            if constexpr (std::is_floating_point<T>::value)
                wht_stage<T, E, b>(v);
            else
                fft_stage_inv<decltype(T::re), E, b>(v);
        }
        reg_inv<T, E, LOGE, b - 1>(v, gs);
    }
}

// Workgroups are handed to the 8 XCDs (each with its own L2) round robin:
// workgroup b runs on XCD b mod 8.  Column passes read runs of one or a few
// cache lines per tile row, and neighbouring tiles share those lines; the
// swizzle gives each XCD a contiguous range of tiles so that the sharing
// stays inside one L2.  (Identity when the grid is not a multiple of 8.)
constexpr int XCD_COUNT = 8;
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb)
{
    if (nb % XCD_COUNT) return b;
    return (b % XCD_COUNT) * (nb / XCD_COUNT) + b / XCD_COUNT;
}

// Tile index of register i of thread t for a group of gs bits at tile bit
// `pos`: the digit c = i mod 2^gs is inserted at bit pos of o = sub*T + t.
__device__ __forceinline__ int group_q(int t, int i, int gs, int pos, int T)
{
    const int c = i & ((1 << gs) - 1);
    const int o = (i >> gs) * T + t;
    return (o & ((1 << pos) - 1)) | (c << pos) | ((o >> pos) << (pos + gs));
}

template <typename T>
struct real_of {
    using type = T;
};
template <typename R>
struct real_of<cplx<R>> {
    using type = R;
};

// Powers w^c, c = 0..E-1, by a binary product tree: w^{2^j} by squaring,
// w^c = w^{c - 2^j} w^{2^j} (at most 2 log2(E) roundings per entry).
template <typename R, int E>
__device__ __forceinline__ void powers(cplx<R> w, cplx<R> (&p)[E])
{
    p[0] = cplx<R>{(R)1, (R)0};
    if constexpr (E > 1) p[1] = w;
#pragma unroll
    for (int c = 2; c < E; ++c) {
        const int hi = 1 << (31 - __builtin_clz(c));  // largest power of two <= c
        p[c] = (c == hi) ? cmul(p[c >> 1], p[c >> 1]) : cmul(p[c - hi], p[hi]);
    }
}

// Group twiddle of the FFT schedule: the element with tile index q, axis
// index r = q >> logW and group digit c at axis bit s is multiplied by
// W_{2^{s+g}}^{(r mod 2^s) R_g(c)}.  For a full group every register of a
// thread shares r mod 2^s, so the twiddles are the powers of one base
// W_{2^{s+g}}^{r mod 2^s}.  Each full group g >= 1 of an A-bit axis has
// that base (group 0 sits at s = 0 and needs none), read once
// at kernel start so that the table latency overlaps the data loads instead
// of stalling each group; apply_group_twiddle multiplies by its powers.
constexpr int MAX_GROUPS = 4;
// The bases of groups 1 .. 3, as named fields.  Held in an array indexed by a
// group number known only at run time, they landed in scratch memory: each
// base load then waited for its data (and the scratch store) before the
// tile's own loads were issued, several memory latencies in a row at the
// start of every complex pass.
template <typename T>
struct GroupBases {
    T b1, b2, b3;
};
// The base of group g = 1 .. 3 (a run-time index), chosen among values:
// selecting among the fields through a reference let the compiler turn the
// choice back into an address, and the fields went back to scratch memory.
template <typename T>
__device__ __forceinline__ T pick_base(int g, T b1, T b2, T b3)
{
    return g == 1 ? b1 : (g == 2 ? b2 : b3);
}
template <typename R, int LOGE>
__device__ __forceinline__ void group_bases(GroupBases<cplx<R>> &B, int t, int A, int logW, int T_)
{
    const int G = (A + LOGE - 1) / LOGE;
    const int rem = A - LOGE * (G - 1);
    auto base = [&](int g) {
        const int s = rem + LOGE * (g - 1);
        const int q0 = group_q(t, 0, LOGE, logW + s, T_);
        const uint32_t rlow = (uint32_t)(q0 >> logW) & ((1u << s) - 1);
        return tw_small<R>(rlow, s + LOGE);
    };
    if (G > 1) B.b1 = base(1);
    if (G > 2) B.b2 = base(2);
    if (G > 3) B.b3 = base(3);
}
template <typename T, int E, int LOGE, bool CONJ>
__device__ __forceinline__ void apply_group_twiddle(T (&v)[E], const T &base)
{
    if constexpr (!std::is_floating_point<T>::value) {
        using R = typename real_of<T>::type;
        cplx<R> pw[E];
        powers<R, E>(base, pw);
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const cplx<R> w = pw[brev_bits((uint32_t)i, LOGE)];
            v[i] = CONJ ? cmulc(v[i], w) : cmul(v[i], w);
        }
    }
}

// Inter-pass twiddle W_{2^{b0+A}}^{k1 R_A(r)} for the coalesced pattern
// q = t + Tn i: the column k1 is fixed per thread and
// R_A(r) = R_{A-LOGE}(r0) 2^LOGE + R_LOGE(i), r0 = t >> logW, so the twiddles
// are base = W^{k1 R_{A-LOGE}(r0) 2^LOGE} times the powers of step = W^{k1}.
// pass_tw_fetch reads the two table products right behind the data loads,
// pass_tw_apply multiplies.
template <typename R>
struct PassTw {
    cplx<R> base, step;
};
template <typename R, int LOGE>
__device__ __forceinline__ PassTw<R> pass_tw_fetch(int t, uint64_t k1, int logW, int A, int b0)
{
    const uint64_t r0 = (uint64_t)(t >> logW);
    return PassTw<R>{tw_any<R>((k1 * brev_bits((uint32_t)r0, A - LOGE)) << LOGE, b0 + A),
                     tw_any<R>(k1, b0 + A)};
}
template <typename T, int E, int LOGE, bool CONJ>
__device__ __forceinline__ void pass_tw_apply(T (&v)[E], const PassTw<typename real_of<T>::type> &p)
{
    if constexpr (!std::is_floating_point<T>::value) {
        using R = typename real_of<T>::type;
        cplx<R> pw[E];
        powers<R, E>(p.step, pw);
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const cplx<R> w = cmul(p.base, pw[brev_bits((uint32_t)i, LOGE)]);
            v[i] = CONJ ? cmulc(v[i], w) : cmul(v[i], w);
        }
    }
}

template <typename T, int E>
__device__ __forceinline__ void lds_read(T (&v)[E], const T *lds, int t, int gs, int pos, int T_)
{
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = lds[lds_idx(group_q(t, i, gs, pos, T_))];
}
template <typename T, int E>
__device__ __forceinline__ void lds_write(const T (&v)[E], T *lds, int t, int gs, int pos, int T_)
{
#pragma unroll
    for (int i = 0; i < E; ++i) lds[lds_idx(group_q(t, i, gs, pos, T_))] = v[i];
}

// Global IO modes of a pass (complex working type; real types use IO_SAME):
//   IO_SAME    elements of the working type;
//   IO_REAL    real array: load as (x, 0), store the real part;
//   IO_PACKED  real array of 2 N per row holding a complex row of N as
//              (re at e, im at e + N): z_e = y_e + i y_{e+N};
//   IO_POWER   (store only) FP64 array receiving |x|^2, squared in FP64;
//   IO_COMBINE (store only, see the pass kernel) the n -> 2n update's butterfly.
// SRC_F32: the source holds floats widened to the FP64 working type.
enum IoMode { IO_SAME = 0, IO_REAL = 1, IO_PACKED = 2, IO_POWER = 3, IO_COMBINE = 4 };

template <typename T, int LD, bool SRC_F32>
__device__ __forceinline__ T load_elem(const void *p, int64_t idx, int64_t half)
{
    using R = typename real_of<T>::type;
    using S = typename std::conditional<SRC_F32, float, R>::type;
    if constexpr (std::is_floating_point<T>::value) {
        return (R) static_cast<const S *>(p)[idx];
    } else if constexpr (LD == IO_REAL) {
        return T{(R) static_cast<const S *>(p)[idx], (R)0};
    } else if constexpr (LD == IO_PACKED) {
        const S *q = static_cast<const S *>(p);
        return T{(R)q[idx], (R)q[idx + half]};
    } else {
        const cplx<S> v = static_cast<const cplx<S> *>(p)[idx];
        return T{(R)v.re, (R)v.im};
    }
}
template <typename T, int ST>
__device__ __forceinline__ void store_elem(void *p, int64_t idx, T v, int64_t half)
{
    if constexpr (ST == IO_POWER) {
        if constexpr (std::is_floating_point<T>::value)
            static_cast<double *>(p)[idx] = (double)v * (double)v;
        else
            static_cast<double *>(p)[idx] = (double)v.re * (double)v.re + (double)v.im * (double)v.im;
    } else if constexpr (std::is_floating_point<T>::value) {
        static_cast<T *>(p)[idx] = v;
    } else {
        using R = typename real_of<T>::type;
        if constexpr (ST == IO_REAL) {
            static_cast<R *>(p)[idx] = v.re;
        } else if constexpr (ST == IO_PACKED) {
            R *q = static_cast<R *>(p);
            q[idx] = v.re;
            q[idx + half] = v.im;
        } else {
            static_cast<T *>(p)[idx] = v;
        }
    }
}


}  // namespace kit
}  // namespace ldk
