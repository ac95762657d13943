// Pass kernels of the FWHT / FFTBR / IFFTBR engine (see transform.hpp).
#include <type_traits>

#include "transform.hpp"

namespace ldk {

// Dynamic LDS of the pass kernels (tile + padding).
extern __shared__ unsigned char g_pass_lds[];

namespace {

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

// Group twiddle of the FFT schedule: element with tile index q, axis index
// r = q >> logW, group digit c at axis bit s: W_{2^{s+gs}}^{(r mod 2^s) R_gs(c)}.
// For a full group every register of a thread shares r mod 2^s, so one table
// read gives w = W^{r mod 2^s} and the twiddles are its powers.
template <typename T, int E, int LOGE, bool CONJ>
__device__ __forceinline__ void group_twiddle(T (&v)[E], int t, int gs, int s, int logW, int T_)
{
    if constexpr (!std::is_floating_point<T>::value) {
        using R = typename real_of<T>::type;
        if (s == 0) return;
        if (gs == LOGE) {
            const int q0 = group_q(t, 0, gs, logW + s, T_);
            const uint32_t rlow = (uint32_t)(q0 >> logW) & ((1u << s) - 1);
            cplx<R> pw[E];
            powers<R, E>(tw_small<R>(rlow, s + gs), pw);
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const cplx<R> w = pw[brev_bits((uint32_t)i, LOGE)];
                v[i] = CONJ ? cmulc(v[i], w) : cmul(v[i], w);
            }
            return;
        }
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int q = group_q(t, i, gs, logW + s, T_);
            const uint32_t rlow = (uint32_t)(q >> logW) & ((1u << s) - 1);
            const uint32_t c = (uint32_t)i & ((1u << gs) - 1);
            const cplx<R> w = tw_small<R>(rlow * brev_bits(c, gs), s + gs);
            v[i] = CONJ ? cmulc(v[i], w) : cmul(v[i], w);
        }
    }
}

// Inter-pass twiddle W_{2^{b0+A}}^{k1 R_A(r)} for the coalesced pattern
// q = t + Tn i: the column k1 is fixed per thread and
// R_A(r) = R_{A-LOGE}(r0) 2^LOGE + R_LOGE(i), r0 = t >> logW, so the twiddles
// are W^{k1 R_{A-LOGE}(r0) 2^LOGE} times the powers of W^{k1}.
template <typename T, int E, int LOGE, bool CONJ>
__device__ __forceinline__ void pass_twiddle(T (&v)[E], int t, int64_t cb, int logW, int A, int b0)
{
    if constexpr (!std::is_floating_point<T>::value) {
        using R = typename real_of<T>::type;
        const uint64_t k1 = (uint64_t)((cb << logW) + (t & ((1 << logW) - 1)));
        const uint64_t r0 = (uint64_t)(t >> logW);
        const cplx<R> base = tw_any<R>((k1 * brev_bits((uint32_t)r0, A - LOGE)) << LOGE, b0 + A);
        cplx<R> pw[E];
        powers<R, E>(tw_any<R>(k1, b0 + A), pw);
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const cplx<R> w = cmul(base, pw[brev_bits((uint32_t)i, LOGE)]);
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

// SRC_F32: the source holds floats (real, or complex when !src_real) that are
// widened to the FP64 working type.
template <typename T, bool SRC_F32>
__device__ __forceinline__ T load_elem(const void *p, int64_t idx, bool src_real)
{
    using R = typename real_of<T>::type;
    using S = typename std::conditional<SRC_F32, float, R>::type;
    if constexpr (std::is_floating_point<T>::value) {
        return (R) static_cast<const S *>(p)[idx];
    } else {
        if (src_real) return T{(R) static_cast<const S *>(p)[idx], (R)0};
        const cplx<S> v = static_cast<const cplx<S> *>(p)[idx];
        return T{(R)v.re, (R)v.im};
    }
}
template <typename T>
__device__ __forceinline__ void store_elem(void *p, int64_t idx, T v, bool dst_real)
{
    if constexpr (std::is_floating_point<T>::value) {
        static_cast<T *>(p)[idx] = v;
    } else {
        using R = typename real_of<T>::type;
        if (dst_real)
            static_cast<R *>(p)[idx] = v.re;
        else
            static_cast<T *>(p)[idx] = v;
    }
}

// One pass over a tile: rows = 2^a along the axis, W = 2^logW columns.
template <typename T, int LOGE, int MODE, bool SRC_REAL, bool DST_REAL, bool SRC_F32>
__global__ __launch_bounds__(512) void k_pass(PassArgs a)
{
    using R = typename real_of<T>::type;
    constexpr int E = 1 << LOGE;
    constexpr bool FFT = !std::is_floating_point<T>::value;
    T *lds = reinterpret_cast<T *>(g_pass_lds);

    const int A = a.g.a, logW = a.g.logW, b0 = a.g.b0;
    const int S = 1 << (A + logW);
    const int Tn = S >> LOGE;  // threads
    const int t = threadIdx.x;

    // block -> (row, outer, column block)
    const int64_t cb_count = (int64_t)1 << (b0 - logW);
    const int64_t outer_count = (int64_t)1 << (a.m - b0 - A);
    int64_t bid = blockIdx.x;
    const int64_t cb = bid % cb_count;
    bid /= cb_count;
    const int64_t outer = bid % outer_count;
    const int64_t row = bid / outer_count;
    const int64_t base = outer * ((int64_t)1 << (b0 + A)) + (cb << logW);
    const int64_t rstride = (int64_t)1 << b0;

    // global index (within a row) of tile element q
    auto gidx = [&](int q) -> int64_t {
        return base + (int64_t)(q >> logW) * rstride + (q & ((1 << logW) - 1));
    };

    // groups over the axis bits: lowest group has rem bits, the rest LOGE bits
    const int G = (A + LOGE - 1) / LOGE;
    const int rem = A - LOGE * (G - 1);
    const int top_s = A - LOGE;  // axis bit where the top group starts

    T v[E];
    // ---- load (coalesced: q = t + Tn * i; the registers hold the top group)
#pragma unroll
    for (int i = 0; i < E; ++i)
        v[i] = load_elem<T, SRC_F32>(a.src, row * a.src_row + gidx(t + Tn * i), SRC_REAL);

    if constexpr (MODE != PM_INV) {
        if constexpr (FFT) {
            if (a.global_tw) pass_twiddle<T, E, LOGE, false>(v, t, cb, logW, A, b0);
        }
        if (G > 1) {
            lds_write(v, lds, t, LOGE, logW + top_s, Tn);
            __syncthreads();
            int s = 0;
            for (int gidx_ = 0; gidx_ < G - 1; ++gidx_) {
                const int gs = gidx_ == 0 ? rem : LOGE;
                lds_read(v, lds, t, gs, logW + s, Tn);
                group_twiddle<T, E, LOGE, false>(v, t, gs, s, logW, Tn);
                reg_fwd<T, E, LOGE, false>(v, gs);
                lds_write(v, lds, t, gs, logW + s, Tn);
                __syncthreads();
                s += gs;
            }
            lds_read(v, lds, t, LOGE, logW + top_s, Tn);
        }
        group_twiddle<T, E, LOGE, false>(v, t, LOGE, G > 1 ? top_s : 0, logW, Tn);
        reg_fwd<T, E, LOGE, false>(v, LOGE);
    }

    if constexpr (MODE == PM_SOLVE || MODE == PM_MATVEC) {
        const double *lam = a.lam + (row / a.nrhs) * ((int64_t)1 << a.m);
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const double l = lam[gidx(t + Tn * i)];
            const double f = MODE == PM_SOLVE ? a.scale / (l + a.sigma2) : a.scale * l;
            v[i] = scl(v[i], (R)f);
        }
    }

    if constexpr (MODE != PM_FWD) {
        reg_inv<T, E, LOGE>(v, LOGE);
        group_twiddle<T, E, LOGE, true>(v, t, LOGE, G > 1 ? top_s : 0, logW, Tn);
        if (G > 1) {
            if constexpr (MODE != PM_INV) __syncthreads();  // LDS reuse after the forward half
            lds_write(v, lds, t, LOGE, logW + top_s, Tn);
            __syncthreads();
            int s = top_s;
            for (int gi = G - 2; gi >= 0; --gi) {
                const int gs = gi == 0 ? rem : LOGE;
                s -= gs;
                lds_read(v, lds, t, gs, logW + s, Tn);
                reg_inv<T, E, LOGE>(v, gs);
                group_twiddle<T, E, LOGE, true>(v, t, gs, s, logW, Tn);
                lds_write(v, lds, t, gs, logW + s, Tn);
                __syncthreads();
            }
            lds_read(v, lds, t, LOGE, logW + top_s, Tn);
        }
        if constexpr (FFT) {
            if (a.global_tw) pass_twiddle<T, E, LOGE, true>(v, t, cb, logW, A, b0);
        }
    }

    // ---- store
    const R sc = (MODE == PM_FWD || MODE == PM_INV) ? (R)a.scale : (R)1;
#pragma unroll
    for (int i = 0; i < E; ++i) {
        T o = v[i];
        if (MODE == PM_FWD || MODE == PM_INV) o = scl(o, sc);
        store_elem<T>(a.dst, row * a.dst_row + gidx(t + Tn * i), o, DST_REAL);
    }
}

template <typename T, int LOGE, int MODE, bool SRC_F32>
int launch_t(bool src_real, bool dst_real, const PassArgs &a, hipStream_t s)
{
    const int S = 1 << (a.g.a + a.g.logW);
    const int threads = S >> LOGE;
    const int64_t blocks = a.rows * ((int64_t)1 << (a.m - a.g.a - a.g.logW));
    if (blocks > 0x7fffffff || threads > 512 || threads < 1) return LDK_ENOTSUP;
    const size_t lds = (size_t)(S + (S >> LDS_PAD_SHIFT)) * sizeof(T);
    if constexpr (std::is_floating_point<T>::value) {
        hipLaunchKernelGGL((k_pass<T, LOGE, MODE, false, false, SRC_F32>), dim3((unsigned)blocks),
                           dim3(threads), lds, s, a);
    } else {
        if (src_real && dst_real)
            hipLaunchKernelGGL((k_pass<T, LOGE, MODE, true, true, SRC_F32>), dim3((unsigned)blocks),
                               dim3(threads), lds, s, a);
        else if (src_real)
            hipLaunchKernelGGL((k_pass<T, LOGE, MODE, true, false, SRC_F32>), dim3((unsigned)blocks),
                               dim3(threads), lds, s, a);
        else if (dst_real)
            hipLaunchKernelGGL((k_pass<T, LOGE, MODE, false, true, SRC_F32>), dim3((unsigned)blocks),
                               dim3(threads), lds, s, a);
        else
            hipLaunchKernelGGL((k_pass<T, LOGE, MODE, false, false, SRC_F32>), dim3((unsigned)blocks),
                               dim3(threads), lds, s, a);
    }
    LDK_LAUNCH_CHECK();
    return LDK_OK;
}

template <typename T, int MODE, bool SRC_F32>
int launch_e(bool src_real, bool dst_real, const PassArgs &a, hipStream_t s)
{
    switch (a.g.logE) {
    case 1: return launch_t<T, 1, MODE, SRC_F32>(src_real, dst_real, a, s);
    case 2: return launch_t<T, 2, MODE, SRC_F32>(src_real, dst_real, a, s);
    case 3: return launch_t<T, 3, MODE, SRC_F32>(src_real, dst_real, a, s);
    case 4: return launch_t<T, 4, MODE, SRC_F32>(src_real, dst_real, a, s);
    default: return LDK_ENOTSUP;
    }
}

template <typename T>
int launch_m(int mode, bool src_real, bool dst_real, const PassArgs &a, hipStream_t s)
{
    switch (mode) {
    case PM_FWD: return launch_e<T, PM_FWD, false>(src_real, dst_real, a, s);
    case PM_INV: return launch_e<T, PM_INV, false>(src_real, dst_real, a, s);
    case PM_SOLVE: return launch_e<T, PM_SOLVE, false>(src_real, dst_real, a, s);
    case PM_MATVEC: return launch_e<T, PM_MATVEC, false>(src_real, dst_real, a, s);
    default: return LDK_EINVAL;
    }
}

}  // namespace

Plan make_plan(int m, int log_tile)
{
    Plan p{};
    p.m = m;
    if (m == 0) return p;
    constexpr int LOGE_MAX = 3;    // 8 elements per thread
    constexpr int LOG_THREADS = 9; // at most 512 threads per workgroup
    // row pass: the low a0 bits; column passes: the rest, split evenly into
    // chunks of at most 8 bits (at least 4 where possible)
    int a0 = m < log_tile ? m : log_tile;
    int r = m - a0;
    if (r > 0 && r < 4) {
        a0 = m - 4;
        r = 4;
    }
    p.pass[0] = PassGeom{0, a0, 0, a0 < LOGE_MAX ? a0 : LOGE_MAX};
    p.P = 1;
    const int C = (r + 7) / 8;
    int b0 = a0;
    for (int c = 0; c < C; ++c) {
        const int a = r / C + (c < r % C ? 1 : 0);
        const int logE = a < LOGE_MAX ? a : LOGE_MAX;
        // tile 2^a rows x 2^logW columns: at most 2^log_tile elements,
        // at most 2^LOG_THREADS threads (2^(a + logW - logE)), at most 2^b0 columns
        int logW = log_tile - a;
        if (logW > LOG_THREADS + logE - a) logW = LOG_THREADS + logE - a;
        if (logW > b0) logW = b0;
        p.pass[p.P++] = PassGeom{b0, a, logW, logE};
        b0 += a;
    }
    return p;
}

int log_tile_for(int kind, int dtype) { return (kind == LDK_LATTICE && dtype == LDK_F64) ? 11 : 12; }

int launch_pass(int kind, int dtype, int mode, bool src_real, bool dst_real, const PassArgs &a,
                hipStream_t s, bool src_f32)
{
    if (src_f32) {
        // FP64 forward transform of float data (eigenvalues from an FP32 column)
        if (dtype != LDK_F64 || mode != PM_FWD) return LDK_EINVAL;
        if (kind == LDK_DNET_B2) return launch_e<double, PM_FWD, true>(false, false, a, s);
        return launch_e<cplx<double>, PM_FWD, true>(src_real, dst_real, a, s);
    }
    if (kind == LDK_DNET_B2) {
        if (dtype == LDK_F64) return launch_m<double>(mode, false, false, a, s);
        return launch_m<float>(mode, false, false, a, s);
    }
    if (dtype == LDK_F64) return launch_m<cplx<double>>(mode, src_real, dst_real, a, s);
    return launch_m<cplx<float>>(mode, src_real, dst_real, a, s);
}

}  // namespace ldk
