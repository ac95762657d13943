// Real-input lattice transforms (Sec. 5.2, 5.4): the first Gram column and the
// responses are real, so a length-n FFTBR runs as a complex FFTBR of length
// N = n/2 on the packed row z_e = y_e + i y_{e+N}.
//
// In natural (radical inverse) order the first half of a row holds the even
// linear-order samples and the second half the odd ones, so FFTBR_N(z) is
// exactly Z = E + i O with E, O the DFTs of the even and odd samples, and
//   E_k = (Z_k + conj Z_{N-k}) / 2,   O_k = -i (Z_k - conj Z_{N-k}) / 2,
//   Y_k = E_k + W_n^k O_k,            Y_{k+N} = E_k - W_n^k O_k
// (Y the unnormalised length-n FFTBR of y).  The eigenvalues are
// lambda_k = Re Y_k and lambda_{k+N} = Re Y_{k+N}.  A solve filters with the
// symmetrised factor d_k = (f(lambda_k) + f(lambda_{n-k}))/2, which equals
// Re IFFTBR(Y (.) f(lambda)) exactly, then re-packs C_k = d_k Y_k as
//   E'_k = (C_k + C_{k+N}) / 2,   O'_k = conj(W_n^k) (C_k - C_{k+N}) / 2,
//   Z'_k = E'_k + i O'_k,
// and the inverse passes return c_e + i c_{e+N} = IFFTBR_N(Z')_e / N.
// Untangling, filtering and re-packing compose to one real-coefficient step
// per element: with s1 = d_k, s2 = d_{k+N} and W_n^k = c + i s,
//   Z'_k = p Z_k + i q conj(Z_{N-k}),  p = (s1+s2)/2 + s (s1-s2)/2,
//   q = c (s1-s2)/2
// (expand E' + i O' with conj(W) W = 1: the E + i O part is Z_k itself).
//
// The partner N - k of a frequency k = k1 + N1 k2 (k1 the column bits below
// b0, k2 the top pass's axis bits) is (N1 - k1) + N1 (N2 - 1 - k2) for k1 != 0
// and N1 ((N2 - k2) mod N2) for k1 = 0.  A top-pass tile therefore holds H
// columns and their H mirrors: tile cb takes columns cb H + 1 .. cb H + H and
// N1 - (cb+1) H .. N1 - cb H - 1; in the last tile the duplicate column N1/2
// of the second run is replaced by column 0.  Both self-mirrored columns
// (0 and N1/2) thus sit in the last tile; every element finds its partner in
// its own tile, through LDS.
//
// Two more modes serve the marginal likelihood: PM_POWER writes |Y_k|^2 (the
// power spectrum, FP64) instead of Re Y_k, and PM_ADJ is the inverse half
// alone: it reads a real spectrum g from a.lam, forms C = scale (g_k +
// g_{n-k}) / 2 (so the result is Re sum_k g_k W_n^{-k R(j)} for scale 2),
// re-packs it like the solve and runs the inverse top group.  PM_QFORM serves
// the cubature: it weights |Y_k|^2 by lambda_k or 1 / (lambda_k + sigma2)
// and sums the tile (into ld_part[row][cb]) instead of storing the spectrum,
// and the tile holding k = 0 stores Y_0 = sum_j y_j (into lam_out[row]).
#include "passkit.hpp"

namespace ldk {

extern __shared__ unsigned char g_real_lds[];

using namespace kit;

namespace {

// The real solve's (or matvec's) filter for frequency k < N of one
// eigenvalue row lam [2N]: s1 = (f(lambda_k) + f(lambda_{n-k}))/2 and s2 the
// same at k + N (f = scale / (lambda + sigma2) or scale lambda), combined
// with W_n^k into Z'_k = p Z_k + i q conj(Z_{N-k}), returned as (p, q).
template <typename T, int MODE>
__device__ __forceinline__ T filter_pq(const double *lam, int64_t k, int mp, double sigma2,
                                       double scale)
{
    using R = typename real_of<T>::type;
    const int64_t N = (int64_t)1 << mp, n = 2 * N;
    const T wk = tw_any<R>((uint64_t)k, mp + 1);
    const double la = lam[k], lb = lam[(n - k) & (n - 1)];
    const double lc = lam[k + N], ld = lam[(N - k) & (n - 1)];
    double s1, s2;
    if constexpr (MODE == PM_SOLVE) {
        // (1/(la+s2) + 1/(lb+s2)) / 2 with one division
        const double pa = la + sigma2, pb = lb + sigma2;
        const double pc = lc + sigma2, pd = ld + sigma2;
        s1 = 0.5 * scale * (pa + pb) / (pa * pb);
        s2 = 0.5 * scale * (pc + pd) / (pc * pd);
    } else {
        s1 = 0.5 * scale * (la + lb);
        s2 = 0.5 * scale * (lc + ld);
    }
    const R hs = (R)(0.5 * (s1 + s2)), hd = (R)(0.5 * (s1 - s2));
    // one explicit fused multiply-add: the same bits in every kernel
    return T{fma(hd, wk.im, hs), hd * wk.re};
}

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_filter_coef(const double *__restrict__ lam, int mp,
                                                     int64_t count, double sigma2, double scale,
                                                     T *__restrict__ coef)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= count) return;
    const int64_t N = (int64_t)1 << mp;
    const int64_t r = idx >> mp, k = idx & (N - 1);
    coef[idx] = filter_pq<T, MODE>(lam + r * 2 * N, k, mp, sigma2, scale);
}

// One tile (row, column block cb) of the top pass.  ld_part (PM_FWD only,
// may be NULL): receives this tile's sum of log(lambda + sigma2) over its 2 S
// eigenvalues at ld_part[row * cb_count + cb] (NaN if some lambda + s2 <= 0).
// CA, CLW >= 0: the axis bits and log2 tile width fixed at compile time (they
// must equal a.g.a and a.g.logW); the index maps, group loops and twiddle
// choices then fold to constants.
template <typename T, int LOGE, int MODE, int LD, int ST, bool SRC_F32, bool CF = false,
          int CA = -1, int CLW = -1>
__device__ __forceinline__ void real_top_body(const PassArgs &a, double *lam_out, int64_t row,
                                              int64_t cb, double *ld_part)
{
    using R = typename real_of<T>::type;
    constexpr int E = 1 << LOGE;
    T *lds = reinterpret_cast<T *>(g_real_lds);

    const int A = CA >= 0 ? CA : a.g.a, logW = CLW >= 0 ? CLW : a.g.logW, b0 = a.g.b0;
    const int mp = a.m;  // log2 N
    const int64_t N = (int64_t)1 << mp;
    const int64_t N1 = (int64_t)1 << b0;
    const int N2 = 1 << A;
    const int W = 1 << logW, H = W >> 1;
    const int S = 1 << (A + logW);
    const int Tn = S >> LOGE;
    const int t = threadIdx.x;
    const int64_t cb_count = N1 >> logW;
    const bool last = cb == cb_count - 1;

    auto col_of = [&](int w) -> int64_t {
        if (W == 1) return 0;
        if (w < H) return cb * H + w + 1;
        if (last && w == H) return 0;
        return N1 - (cb + 1) * H + (w - H);
    };
    auto gidx = [&](int q) -> int64_t { return col_of(q & (W - 1)) + (int64_t)(q >> logW) * N1; };

    const int G = (A + LOGE - 1) / LOGE;
    const int rem = A - LOGE * (G - 1);
    const int top_s = A - LOGE;

    const int64_t n = 2 * N;
    const double *lam = a.lam ? a.lam + (row / a.nrhs) * n : nullptr;

    T v[E];
    if constexpr (MODE != PM_ADJ) {
#pragma unroll
        for (int i = 0; i < E; ++i)
            v[i] = load_elem<T, LD, SRC_F32>(a.src, row * a.src_row + gidx(t + Tn * i), a.half);
    }
    // twiddle table reads issued right behind the data loads
    GroupBases<T> gb{};
    group_bases<R, LOGE>(gb, t, A, logW, Tn);
    PassTw<R> ptw{};
    if (b0 > 0) ptw = pass_tw_fetch<R, LOGE>(t, (uint64_t)col_of(t & (W - 1)), logW, A, b0);
    // Per-element twiddle W_n^k and spectral factors, fetched after the
    // data loads are issued and before the transform, so that their latency
    // overlaps the data loads and the groups.  The solve and matvec form
    // them after the forward transform instead, next to their one use: held
    // across the transform (with the eigenvalue loads in flight) they took
    // every register and spilled.
    constexpr bool LATE = MODE == PM_SOLVE || MODE == PM_MATVEC;
    T wkv[E];
    double f1[E], f2[E];
    // precomputed filter coefficients (p, q), when given: one pair per
    // element, read next to their use (held across the transform they would
    // cost 4 E registers)
    const T *crow = CF ? static_cast<const T *>(a.coef) + (row / a.nrhs) * N : nullptr;
#pragma unroll
    for (int i = 0; i < E && !LATE; ++i) {
        const int q = t + Tn * i;
        const int64_t k = col_of(q & (W - 1)) + N1 * (int64_t)(q >> logW);
        wkv[i] = tw_any<R>((uint64_t)k, mp + 1);
        if constexpr (MODE == PM_ADJ) {
            const double la = lam[k], lb = lam[(n - k) & (n - 1)];
            const double lc = lam[k + N], ld = lam[(N - k) & (n - 1)];
            f1[i] = 0.5 * a.scale * (la + lb);
            f2[i] = 0.5 * a.scale * (lc + ld);
        }
        if constexpr (MODE == PM_QFORM) {
            const double la = lam[k], lc = lam[k + N];
            if (a.qform_lam) {
                f1[i] = la;
                f2[i] = lc;
            } else {
                const double pa = la + a.sigma2, pc = lc + a.sigma2;
                f1[i] = pa > 0.0 ? 1.0 / pa : __builtin_nan("");
                f2[i] = pc > 0.0 ? 1.0 / pc : __builtin_nan("");
            }
        }
    }

    if constexpr (MODE != PM_ADJ) {
        if (b0 > 0) pass_tw_apply<T, E, LOGE, false>(v, ptw);

        // ---- forward transform over the axis bits (low groups first)
        if (G > 1) {
            lds_write(v, lds, t, LOGE, logW + top_s, Tn);
            __syncthreads();
            int s = 0;
            for (int gi = 0; gi < G - 1; ++gi) {
                const int gs = gi == 0 ? rem : LOGE;
                lds_read(v, lds, t, gs, logW + s, Tn);
                if (gi > 0) {
                    const auto gbase = pick_base(gi, gb.b1, gb.b2, gb.b3);
                    apply_group_twiddle<T, E, LOGE, false>(v, gbase);
                }
                reg_fwd<T, E, LOGE, false>(v, gs);
                lds_write(v, lds, t, gs, logW + s, Tn);
                __syncthreads();
                s += gs;
            }
            lds_read(v, lds, t, LOGE, logW + top_s, Tn);
            apply_group_twiddle<T, E, LOGE, false>(v, pick_base(G - 1, gb.b1, gb.b2, gb.b3));
        }
        reg_fwd<T, E, LOGE, false>(v, LOGE);

        // ---- real-spectrum step: every element reads its partner N - k
        __syncthreads();  // all threads are done reading the forward groups
        lds_write(v, lds, t, LOGE, logW + top_s, Tn);
        __syncthreads();
    }
    LogProd lsum;       // PM_FWD with ld_part: sum of log(lambda + s2)
    double qacc = 0.0;  // PM_QFORM: weighted sum of |Y|^2
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int q = t + Tn * i;
        const int w = q & (W - 1), k2 = q >> logW;
        const int64_t k1 = col_of(w);
        if constexpr (MODE == PM_ADJ) {
            // real spectrum g in a.lam: C = scale (g_k + g_{n-k}) / 2 at k and k + N
            const double s1 = f1[i], s2 = f2[i];
            const R ep = (R)(0.5 * (s1 + s2));
            const T op = cmulc(T{(R)(0.5 * (s1 - s2)), (R)0}, wkv[i]);
            v[i] = T{ep - op.im, op.re};
            continue;
        }
        int wp, k2p;
        if (k1 == 0) {
            wp = w;
            k2p = (N2 - k2) & (N2 - 1);
        } else if (k1 == N1 / 2) {
            wp = w;
            k2p = N2 - 1 - k2;
        } else {
            wp = 2 * H - 1 - w;
            k2p = N2 - 1 - k2;
        }
        const T zm = lds[lds_idx(k2p * W + wp)];
        const T zk = v[i];
        if constexpr (MODE == PM_SOLVE || MODE == PM_MATVEC) {
            // untangle, filter by s1 at k and s2 at k + N, re-pack, in one
            // step: Z'_k = p Z_k + i q conj(Z_{N-k}) with real
            // p = (s1 + s2)/2 + (s1 - s2)/2 Im W_n^k, q = (s1 - s2)/2 Re W_n^k
            R pc, qc;
            if constexpr (CF) {
                const T c2 = crow[k1 + N1 * (int64_t)k2];
                pc = c2.re;
                qc = c2.im;
            } else {
                const T c2 = filter_pq<T, MODE>(lam, k1 + N1 * (int64_t)k2, mp, a.sigma2, a.scale);
                pc = c2.re;
                qc = c2.im;
            }
            v[i] = T{pc * zk.re + qc * zm.im, pc * zk.im + qc * zm.re};
            continue;
        }
        const int64_t k = k1 + N1 * k2;
        const T ev{(zk.re + zm.re) * (R)0.5, (zk.im - zm.im) * (R)0.5};
        const T dv{(zk.re - zm.re) * (R)0.5, (zk.im + zm.im) * (R)0.5};
        const T od{dv.im, -dv.re};  // -i (Z_k - conj Z_{N-k}) / 2
        const T wk = wkv[i];
        const T wo = cmul(wk, od);
        const T yk{ev.re + wo.re, ev.im + wo.im};
        const T ykn{ev.re - wo.re, ev.im - wo.im};
        if constexpr (MODE == PM_FWD) {
            lam_out[row * n + k] = (double)yk.re;
            lam_out[row * n + k + N] = (double)ykn.re;
            if (ld_part) {
                lsum.add((double)yk.re + a.sigma2);
                lsum.add((double)ykn.re + a.sigma2);
            }
        } else if constexpr (MODE == PM_POWER) {
            lam_out[row * n + k] = (double)yk.re * (double)yk.re + (double)yk.im * (double)yk.im;
            lam_out[row * n + k + N] =
                (double)ykn.re * (double)ykn.re + (double)ykn.im * (double)ykn.im;
        } else if constexpr (MODE == PM_QFORM) {
            const double p1 = (double)yk.re * (double)yk.re + (double)yk.im * (double)yk.im;
            const double p2 = (double)ykn.re * (double)ykn.re + (double)ykn.im * (double)ykn.im;
            qacc = fma(f1[i], p1, qacc);
            qacc = fma(f2[i], p2, qacc);
            if (k == 0) lam_out[row] = (double)yk.re;  // Y_0: the row's sum
        }
    }
    if constexpr (MODE == PM_FWD) {
        if (ld_part) {
            // block sum in a fixed order: lanes, then waves
            __shared__ double red[8];
            double ls = lsum.value();
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) ls += __shfl_xor(ls, o, 64);
            if ((t & 63) == 0) red[t >> 6] = ls;
            __syncthreads();
            if (t == 0) {
                double s = 0.0;
                for (int w8 = 0; w8 < (Tn + 63) / 64; ++w8) s += red[w8];
                ld_part[row * cb_count + cb] = s;
            }
        }
        return;
    }
    if constexpr (MODE == PM_POWER) return;
    if constexpr (MODE == PM_QFORM) {
        // block sum in a fixed order: lanes, then waves (a block of fewer
        // than 64 threads sums its threads through LDS)
        __shared__ double qred[64];
        if (Tn >= 64) {
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) qacc += __shfl_xor(qacc, o, 64);
            if ((t & 63) == 0) qred[t >> 6] = qacc;
        } else {
            qred[t] = qacc;
        }
        __syncthreads();
        if (t == 0) {
            double sum = 0.0;
            const int terms = Tn >= 64 ? Tn / 64 : Tn;
            for (int w8 = 0; w8 < terms; ++w8) sum += qred[w8];
            ld_part[row * cb_count + cb] = sum;
        }
        return;
    }

    // ---- inverse transform over the axis bits (top group first)
    reg_inv<T, E, LOGE>(v, LOGE);
    if (G > 1) {
        apply_group_twiddle<T, E, LOGE, true>(v, pick_base(G - 1, gb.b1, gb.b2, gb.b3));
        if constexpr (MODE != PM_ADJ) __syncthreads();  // partner reads are done
        lds_write(v, lds, t, LOGE, logW + top_s, Tn);
        __syncthreads();
        int s = top_s;
        for (int gi = G - 2; gi >= 0; --gi) {
            const int gs = gi == 0 ? rem : LOGE;
            s -= gs;
            lds_read(v, lds, t, gs, logW + s, Tn);
            reg_inv<T, E, LOGE>(v, gs);
            if (gi > 0) {
                const auto gbase = pick_base(gi, gb.b1, gb.b2, gb.b3);
                apply_group_twiddle<T, E, LOGE, true>(v, gbase);
            }
            lds_write(v, lds, t, gs, logW + s, Tn);
            __syncthreads();
        }
        lds_read(v, lds, t, LOGE, logW + top_s, Tn);
    }
    if (b0 > 0) pass_tw_apply<T, E, LOGE, true>(v, ptw);
#pragma unroll
    for (int i = 0; i < E; ++i)
        store_elem<T, ST>(a.dst, row * a.dst_row + gidx(t + Tn * i), v[i], a.half);
}

// The fit's two top passes in one block (FP64, one right-hand side per
// column): threads [0, Tn) take tile cb of the column's transform and produce
// its eigenvalues (and log-det partial sum), threads [Tn, 2 Tn) take the
// same tile of the right-hand side's transform.  A tile holds every
// frequency's partner, so the eigenvalues the solve's filter needs at k,
// N - k, k + N and n - k are all produced in the same block; they pass
// through LDS (over the column half's tile, once its partner reads are
// done).  Both halves run the same forward schedule and reach every barrier;
// the column half idles through the inverse top group.
//   LDS: [column tile | rhs tile], each S + S/16 elements.
// CA, CLW >= 0: the axis bits and log2 tile width fixed at compile time (as
// for real_top_body).
template <int LOGE, int LD, int ST, int CA = -1, int CLW = -1>
__global__ __launch_bounds__(CA >= 0 ? (2 << (CA + CLW - LOGE)) : 512) void k_fit_top(
    PassArgs aK, PassArgs aY, double *lam_out, double *ld_part)
{
    using T = cplx<double>;
    using R = double;
    constexpr int E = 1 << LOGE;
    __shared__ double red[8];

    const int A = CA >= 0 ? CA : aK.g.a, logW = CLW >= 0 ? CLW : aK.g.logW, b0 = aK.g.b0;
    const int mp = aK.m;
    const int64_t N = (int64_t)1 << mp;
    const int64_t N1 = (int64_t)1 << b0;
    const int N2 = 1 << A;
    const int W = 1 << logW, H = W >> 1;
    const int S = 1 << (A + logW);
    const int Tn = S >> LOGE;
    const bool rhs = (int)threadIdx.x >= Tn;  // wave-uniform: Tn is a multiple of 64
    const int t = rhs ? (int)threadIdx.x - Tn : (int)threadIdx.x;
    const int64_t cb_count = N1 >> logW;
    const int64_t bid = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t row = bid / cb_count, cb = bid % cb_count;
    const bool last = cb == cb_count - 1;
    const int padS = S + (S >> LDS_PAD_SHIFT);
    T *lds = reinterpret_cast<T *>(g_real_lds) + (rhs ? padS : 0);
    double *lam_lds = reinterpret_cast<double *>(g_real_lds);  // [2][S] after the column's reads

    auto col_of = [&](int w) -> int64_t {
        if (W == 1) return 0;
        if (w < H) return cb * H + w + 1;
        if (last && w == H) return 0;
        return N1 - (cb + 1) * H + (w - H);
    };
    auto gidx = [&](int q) -> int64_t { return col_of(q & (W - 1)) + (int64_t)(q >> logW) * N1; };
    // position in the tile of the partner N - k of element q (q itself for k = 0)
    auto partner = [&](int q) -> int {
        const int w = q & (W - 1), k2 = q >> logW;
        const int64_t k1 = col_of(w);
        if (k1 == 0) return ((N2 - k2) & (N2 - 1)) * W + w;
        if (k1 == N1 / 2) return (N2 - 1 - k2) * W + w;
        return (N2 - 1 - k2) * W + (2 * H - 1 - w);
    };

    const int G = (A + LOGE - 1) / LOGE;
    const int rem = A - LOGE * (G - 1);
    const int top_s = A - LOGE;
    const int64_t n = 2 * N;

    const void *src = rhs ? aY.src : aK.src;
    const int64_t src_row = rhs ? aY.src_row : aK.src_row;
    T v[E];
#pragma unroll
    for (int i = 0; i < E; ++i)
        v[i] = load_elem<T, LD, false>(src, row * src_row + gidx(t + Tn * i), aK.half);
    GroupBases<T> gb{};
    group_bases<R, LOGE>(gb, t, A, logW, Tn);
    PassTw<R> ptw{};
    if (b0 > 0) ptw = pass_tw_fetch<R, LOGE>(t, (uint64_t)col_of(t & (W - 1)), logW, A, b0);
    T wkv[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int q = t + Tn * i;
        const int64_t k = col_of(q & (W - 1)) + N1 * (int64_t)(q >> logW);
        wkv[i] = tw_any<R>((uint64_t)k, mp + 1);
    }

    // ---- forward transform over the axis bits (both halves, own tiles)
    if (b0 > 0) pass_tw_apply<T, E, LOGE, false>(v, ptw);
    if (G > 1) {
        lds_write(v, lds, t, LOGE, logW + top_s, Tn);
        __syncthreads();
        int s = 0;
        // kept rolled: unrolled with the geometry fixed at compile time, the
        // 512-thread workgroup's 256 registers per wave no longer hold the
        // hoisted twiddle products and the kernel spills
#pragma nounroll
        for (int gi = 0; gi < G - 1; ++gi) {
            const int gs = gi == 0 ? rem : LOGE;
            lds_read(v, lds, t, gs, logW + s, Tn);
            if (gi > 0) {
                const auto gbase = pick_base(gi, gb.b1, gb.b2, gb.b3);
                apply_group_twiddle<T, E, LOGE, false>(v, gbase);
            }
            reg_fwd<T, E, LOGE, false>(v, gs);
            lds_write(v, lds, t, gs, logW + s, Tn);
            __syncthreads();
            s += gs;
        }
        lds_read(v, lds, t, LOGE, logW + top_s, Tn);
        apply_group_twiddle<T, E, LOGE, false>(v, pick_base(G - 1, gb.b1, gb.b2, gb.b3));
    }
    reg_fwd<T, E, LOGE, false>(v, LOGE);
    __syncthreads();  // all forward reads are done
    lds_write(v, lds, t, LOGE, logW + top_s, Tn);
    __syncthreads();

    // Untangled spectrum of element i: Y_k and Y_{k+N}.
    auto untangle = [&](int i, T &yk, T &ykn) {
        const T zm = lds[lds_idx(partner(t + Tn * i))];
        const T zk = v[i];
        const T ev{(zk.re + zm.re) * (R)0.5, (zk.im - zm.im) * (R)0.5};
        const T dv{(zk.re - zm.re) * (R)0.5, (zk.im + zm.im) * (R)0.5};
        const T od{dv.im, -dv.re};
        const T wo = cmul(wkv[i], od);
        yk = T{ev.re + wo.re, ev.im + wo.im};
        ykn = T{ev.re - wo.re, ev.im - wo.im};
    };

    // ---- column half: eigenvalues (global and LDS) and the log-det partial
    double la[E], lc[E];
    LogProd lsum;
    if (!rhs) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
            T yk, ykn;
            untangle(i, yk, ykn);
            const int q = t + Tn * i;
            const int64_t k = col_of(q & (W - 1)) + N1 * (int64_t)(q >> logW);
            la[i] = yk.re;
            lc[i] = ykn.re;
            lam_out[row * n + k] = la[i];
            lam_out[row * n + k + N] = lc[i];
            if (ld_part) {
                lsum.add(la[i] + aK.sigma2);
                lsum.add(lc[i] + aK.sigma2);
            }
        }
    }
    __syncthreads();  // the column's partner reads are done: its tile becomes lambda
    if (!rhs) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int q = t + Tn * i;
            lam_lds[q] = la[i];
            lam_lds[S + q] = lc[i];
        }
        if (ld_part) {
            double ls = lsum.value();
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) ls += __shfl_xor(ls, o, 64);
            if ((t & 63) == 0) red[t >> 6] = ls;
        }
    }
    __syncthreads();
    if (!rhs) {
        if (ld_part && t == 0) {
            double sacc = 0.0;
            for (int w8 = 0; w8 < (Tn + 63) / 64; ++w8) sacc += red[w8];
            ld_part[row * cb_count + cb] = sacc;
        }
    } else {
        // ---- rhs half: filter by the symmetrised 1/(lambda + s2) and re-pack,
        // as Z'_k = p Z_k + i q conj(Z_{N-k}) (see real_top_body)
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int q = t + Tn * i;
            const int qp = partner(q);
            const int64_t k = col_of(q & (W - 1)) + N1 * (int64_t)(q >> logW);
            // lambda at k, n - k, k + N and N - k; for k = 0, n - k is 0 and N - k is N
            const double l_k = lam_lds[q], l_kN = lam_lds[S + q];
            const double l_nk = k == 0 ? l_k : lam_lds[S + qp];
            const double l_Nk = k == 0 ? l_kN : lam_lds[qp];
            const double pa = l_k + aY.sigma2, pb = l_nk + aY.sigma2;
            const double pc = l_kN + aY.sigma2, pd = l_Nk + aY.sigma2;
            const double s1 = 0.5 * aY.scale * (pa + pb) / (pa * pb);
            const double s2 = 0.5 * aY.scale * (pc + pd) / (pc * pd);
            const double hs = 0.5 * (s1 + s2), hd = 0.5 * (s1 - s2);
            const double pk = hs + hd * wkv[i].im, qk = hd * wkv[i].re;
            const T zm = lds[lds_idx(qp)], zk = v[i];
            v[i] = T{pk * zk.re + qk * zm.im, pk * zk.im + qk * zm.re};
        }
        reg_inv<T, E, LOGE>(v, LOGE);
    }

    // ---- inverse transform over the axis bits (rhs half; both reach the barriers)
    if (G > 1) {
        if (rhs) apply_group_twiddle<T, E, LOGE, true>(v, pick_base(G - 1, gb.b1, gb.b2, gb.b3));
        __syncthreads();  // the rhs partner reads are done
        if (rhs) lds_write(v, lds, t, LOGE, logW + top_s, Tn);
        __syncthreads();
        int s = top_s;
#pragma nounroll  // (as the forward groups)
        for (int gi = G - 2; gi >= 0; --gi) {
            const int gs = gi == 0 ? rem : LOGE;
            s -= gs;
            if (rhs) {
                lds_read(v, lds, t, gs, logW + s, Tn);
                reg_inv<T, E, LOGE>(v, gs);
                if (gi > 0) {
                    const auto gbase = pick_base(gi, gb.b1, gb.b2, gb.b3);
                    apply_group_twiddle<T, E, LOGE, true>(v, gbase);
                }
                lds_write(v, lds, t, gs, logW + s, Tn);
            }
            __syncthreads();
        }
        if (rhs) lds_read(v, lds, t, LOGE, logW + top_s, Tn);
    }
    if (rhs) {
        if (b0 > 0) pass_tw_apply<T, E, LOGE, true>(v, ptw);
#pragma unroll
        for (int i = 0; i < E; ++i)
            store_elem<T, ST>(aY.dst, row * aY.dst_row + gidx(t + Tn * i), v[i], aY.half);
    }
}

template <int LOGE, int LD, int ST>
int launch_ft(const PassArgs &aK, const PassArgs &aY, double *lam_out, double *ld_part,
              hipStream_t s)
{
    const int S = 1 << (aK.g.a + aK.g.logW);
    const int Tn = S >> LOGE;
    const int64_t blocks = aK.rows * ((int64_t)1 << (aK.g.b0 - aK.g.logW));
    if (blocks > 0x7fffffff || Tn > 256 || Tn % 64 != 0) return LDK_ENOTSUP;
    if ((aK.g.a + LOGE - 1) / LOGE > MAX_GROUPS) return LDK_ENOTSUP;
    if (aK.g.b0 + aK.g.a != aK.m) return LDK_EINVAL;
    if (aK.g.b0 > 0 && aK.g.logW < 1) return LDK_ENOTSUP;
    const size_t lds = 2 * (size_t)(S + (S >> LDS_PAD_SHIFT)) * sizeof(cplx<double>);
    if constexpr (LOGE == 3 && LD == IO_SAME && ST == IO_SAME) {
        // the fit's top pass at n = 2^19 .. 2^20 (8 axis bits, 8-column tiles)
        if (aK.g.a == 8 && aK.g.logW == 3) {
            hipLaunchKernelGGL((k_fit_top<LOGE, LD, ST, 8, 3>), dim3((unsigned)blocks), dim3(2 * Tn),
                               lds, s, aK, aY, lam_out, ld_part);
            LDK_LAUNCH_CHECK();
            return LDK_OK;
        }
    }
    hipLaunchKernelGGL((k_fit_top<LOGE, LD, ST>), dim3((unsigned)blocks), dim3(2 * Tn), lds, s, aK,
                       aY, lam_out, ld_part);
    LDK_LAUNCH_CHECK();
    return LDK_OK;
}

// NR > 1 (with precomputed coefficients, nrhs a multiple of NR): a block
// runs the same tile of NR consecutive rows, which share an eigenvalue row,
// one after the other, so the later rows read the tile's coefficients from
// the L2 lines the first one brought in.
template <typename T, int LOGE, int MODE, int LD, int ST, bool SRC_F32, bool CF, int CA = -1,
          int CLW = -1, int NR = 1>
__global__ __launch_bounds__(CA >= 0 ? (1 << (CA + CLW - LOGE)) : 512) void k_real_top(
    PassArgs a, double *lam_out, double *ld_part)
{
    const int64_t cb_count = ((int64_t)1 << a.g.b0) >> a.g.logW;
    const int64_t bid = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t row0 = (bid / cb_count) * NR, cb = bid % cb_count;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        if (q > 0) __syncthreads();  // the tile's LDS is free again
        real_top_body<T, LOGE, MODE, LD, ST, SRC_F32, CF, CA, CLW>(a, lam_out, row0 + q, cb,
                                                                   ld_part);
    }
}

template <typename T, int LOGE, int MODE, int LD, int ST, bool SRC_F32, bool CF = false>
int launch_rt(const PassArgs &a, double *lam_out, hipStream_t s, double *ld_part = nullptr)
{
    const int S = 1 << (a.g.a + a.g.logW);
    const int threads = S >> LOGE;
    const int64_t blocks = a.rows * ((int64_t)1 << (a.g.b0 - a.g.logW));
    if (blocks > 0x7fffffff || threads > 512 || threads < 1) return LDK_ENOTSUP;
    if ((a.g.a + LOGE - 1) / LOGE > MAX_GROUPS) return LDK_ENOTSUP;  // group twiddle bases
    if (a.g.b0 + a.g.a != a.m) return LDK_EINVAL;  // must be the top pass
    if (a.g.b0 > 0 && a.g.logW < 1) return LDK_ENOTSUP;  // mirror runs need W >= 2
    const size_t lds = (size_t)(S + (S >> LDS_PAD_SHIFT)) * sizeof(T);
    if constexpr ((MODE == PM_SOLVE || (MODE == PM_FWD && !CF)) && LD == IO_SAME && ST == IO_SAME &&
                  !SRC_F32 && LOGE == 3) {
        // the solve's and the eigenvalues' top pass of the plans at n = 2^20
        // (FP64: 8 axis bits, 8-column tiles; FP32: 7 axis bits, 32-column
        // tiles): geometry fixed at compile time
        constexpr bool F64 = std::is_same<T, cplx<double>>::value;
        constexpr int TA = F64 ? 8 : 7, TLW = F64 ? 3 : 5;
        if (a.g.a == TA && a.g.logW == TLW) {
            bool pair = false;
            if constexpr (CF) pair = a.nrhs % 2 == 0;
            if constexpr (CF) {
                if (pair)
                    hipLaunchKernelGGL((k_real_top<T, LOGE, MODE, LD, ST, SRC_F32, CF, TA, TLW, 2>),
                                       dim3((unsigned)(blocks / 2)), dim3(threads), lds, s, a,
                                       lam_out, ld_part);
            }
            if (!pair)
                hipLaunchKernelGGL((k_real_top<T, LOGE, MODE, LD, ST, SRC_F32, CF, TA, TLW>),
                                   dim3((unsigned)blocks), dim3(threads), lds, s, a, lam_out,
                                   ld_part);
            LDK_LAUNCH_CHECK();
            return LDK_OK;
        }
    }
    hipLaunchKernelGGL((k_real_top<T, LOGE, MODE, LD, ST, SRC_F32, CF>), dim3((unsigned)blocks),
                       dim3(threads), lds, s, a, lam_out, ld_part);
    LDK_LAUNCH_CHECK();
    return LDK_OK;
}

template <typename T, int MODE, int LD, int ST, bool SRC_F32, bool CF = false>
int launch_rt_e(const PassArgs &a, double *lam_out, hipStream_t s, double *ld_part = nullptr)
{
    switch (a.g.logE) {
    case 1: return launch_rt<T, 1, MODE, LD, ST, SRC_F32, CF>(a, lam_out, s, ld_part);
    case 2: return launch_rt<T, 2, MODE, LD, ST, SRC_F32, CF>(a, lam_out, s, ld_part);
    case 3: return launch_rt<T, 3, MODE, LD, ST, SRC_F32, CF>(a, lam_out, s, ld_part);
    default: return LDK_ENOTSUP;
    }
}

template <typename T, int MODE>
int launch_rt_io(bool single, const PassArgs &a, double *lam_out, hipStream_t s)
{
    // one pass: packed real rows in and out; otherwise the complex work
    // rows, with the filter coefficients precomputed when given
    if (single) return launch_rt_e<T, MODE, IO_PACKED, IO_PACKED, false>(a, lam_out, s);
    if (a.coef) return launch_rt_e<T, MODE, IO_SAME, IO_SAME, false, true>(a, lam_out, s);
    return launch_rt_e<T, MODE, IO_SAME, IO_SAME, false>(a, lam_out, s);
}

}  // namespace

bool fit_top_supported(const PassGeom &g)
{
    const int S = 1 << (g.a + g.logW), Tn = S >> g.logE;
    const size_t lds = 2 * (size_t)(S + (S >> LDS_PAD_SHIFT)) * sizeof(cplx<double>);
    return (g.logE == 2 || g.logE == 3) && Tn % 64 == 0 && Tn <= 256 && lds <= LDS_PER_GROUP &&
           (g.a + g.logE - 1) / g.logE <= MAX_GROUPS && (g.b0 == 0 || g.logW >= 1);
}

int launch_fit_top(const PassArgs &aK, const PassArgs &aY, double *lam_out, double *ld_part,
                   hipStream_t s)
{
    if (!fit_top_supported(aK.g)) return LDK_ENOTSUP;
    if (aK.rows != aY.rows || aK.m != aY.m || aK.half != aY.half || aK.src_row != aY.src_row ||
        aY.nrhs != 1 || !lam_out)
        return LDK_EINVAL;
    const bool single = aK.g.b0 == 0;
    switch (aK.g.logE) {
    case 2:
        return single ? launch_ft<2, IO_PACKED, IO_PACKED>(aK, aY, lam_out, ld_part, s)
                      : launch_ft<2, IO_SAME, IO_SAME>(aK, aY, lam_out, ld_part, s);
    case 3:
        return single ? launch_ft<3, IO_PACKED, IO_PACKED>(aK, aY, lam_out, ld_part, s)
                      : launch_ft<3, IO_SAME, IO_SAME>(aK, aY, lam_out, ld_part, s);
    default: return LDK_ENOTSUP;
    }
}

int launch_filter_coef(int dtype, int mode, int mp, int64_t lam_rows, const double *lam,
                       double sigma2, double scale, void *coef, hipStream_t s)
{
    if (mp < 1 || lam_rows < 1 || !lam || !coef) return LDK_EINVAL;
    const int64_t count = lam_rows << mp;
    const int64_t blocks = (count + 255) / 256;
    if (blocks > 0x7fffffff) return LDK_ENOTSUP;
    const dim3 g((unsigned)blocks), b(256);
    if (dtype == LDK_F64) {
        if (mode == PM_SOLVE)
            hipLaunchKernelGGL((k_filter_coef<cplx<double>, PM_SOLVE>), g, b, 0, s, lam, mp, count,
                               sigma2, scale, static_cast<cplx<double> *>(coef));
        else
            hipLaunchKernelGGL((k_filter_coef<cplx<double>, PM_MATVEC>), g, b, 0, s, lam, mp, count,
                               sigma2, scale, static_cast<cplx<double> *>(coef));
    } else {
        if (mode == PM_SOLVE)
            hipLaunchKernelGGL((k_filter_coef<cplx<float>, PM_SOLVE>), g, b, 0, s, lam, mp, count,
                               sigma2, scale, static_cast<cplx<float> *>(coef));
        else
            hipLaunchKernelGGL((k_filter_coef<cplx<float>, PM_MATVEC>), g, b, 0, s, lam, mp, count,
                               sigma2, scale, static_cast<cplx<float> *>(coef));
    }
    LDK_LAUNCH_CHECK();
    return LDK_OK;
}

int launch_real_top(int dtype, int mode, const PassArgs &a, double *lam_out, hipStream_t s,
                    bool src_f32, double *ld_part)
{
    const bool single = a.g.b0 == 0;
    if (mode == PM_FWD) {
        // eigenvalues: FP64 working type
        if (dtype != LDK_F64 || !lam_out) return LDK_EINVAL;
        if (src_f32) {
            if (!single) return LDK_EINVAL;  // float sources only feed the first pass
            return launch_rt_e<cplx<double>, PM_FWD, IO_PACKED, IO_SAME, true>(a, lam_out, s,
                                                                                ld_part);
        }
        if (single)
            return launch_rt_e<cplx<double>, PM_FWD, IO_PACKED, IO_SAME, false>(a, lam_out, s,
                                                                                 ld_part);
        return launch_rt_e<cplx<double>, PM_FWD, IO_SAME, IO_SAME, false>(a, lam_out, s, ld_part);
    }
    if (mode == PM_QFORM) {
        // cubature quadratic forms: tile sums into ld_part, row sums into lam_out
        if (!lam_out || !ld_part || !a.lam || src_f32) return LDK_EINVAL;
        if (dtype == LDK_F64) {
            if (single) return launch_rt_e<cplx<double>, PM_QFORM, IO_PACKED, IO_SAME, false>(a, lam_out, s, ld_part);
            return launch_rt_e<cplx<double>, PM_QFORM, IO_SAME, IO_SAME, false>(a, lam_out, s, ld_part);
        }
        if (single) return launch_rt_e<cplx<float>, PM_QFORM, IO_PACKED, IO_SAME, false>(a, lam_out, s, ld_part);
        return launch_rt_e<cplx<float>, PM_QFORM, IO_SAME, IO_SAME, false>(a, lam_out, s, ld_part);
    }
    if (ld_part) return LDK_EINVAL;  // log-det partials come with the eigenvalues only
    if (src_f32) return LDK_EINVAL;
    if (mode == PM_POWER) {
        if (!lam_out) return LDK_EINVAL;
        if (dtype == LDK_F64) {
            if (single) return launch_rt_e<cplx<double>, PM_POWER, IO_PACKED, IO_SAME, false>(a, lam_out, s);
            return launch_rt_e<cplx<double>, PM_POWER, IO_SAME, IO_SAME, false>(a, lam_out, s);
        }
        if (single) return launch_rt_e<cplx<float>, PM_POWER, IO_PACKED, IO_SAME, false>(a, lam_out, s);
        return launch_rt_e<cplx<float>, PM_POWER, IO_SAME, IO_SAME, false>(a, lam_out, s);
    }
    if (!a.lam) return LDK_EINVAL;
    if (mode == PM_ADJ) {
        // adjoint of the eigenvalue map: FP64, real spectrum in a.lam
        if (dtype != LDK_F64) return LDK_EINVAL;
        if (single) return launch_rt_e<cplx<double>, PM_ADJ, IO_SAME, IO_PACKED, false>(a, nullptr, s);
        return launch_rt_e<cplx<double>, PM_ADJ, IO_SAME, IO_SAME, false>(a, nullptr, s);
    }
    if (mode != PM_SOLVE && mode != PM_MATVEC) return LDK_EINVAL;
    if (dtype == LDK_F64) {
        return mode == PM_SOLVE ? launch_rt_io<cplx<double>, PM_SOLVE>(single, a, nullptr, s)
                                : launch_rt_io<cplx<double>, PM_MATVEC>(single, a, nullptr, s);
    }
    return mode == PM_SOLVE ? launch_rt_io<cplx<float>, PM_SOLVE>(single, a, nullptr, s)
                            : launch_rt_io<cplx<float>, PM_MATVEC>(single, a, nullptr, s);
}

}  // namespace ldk
