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
// A block takes 256 consecutive indices of one replication and walks the
// dimensions; per dimension it stages that dimension's scrambles (and, for
// Faure, its matrix) in LDS, and every thread keeps its digit vector in an
// LDS column (runtime-indexed digits would otherwise go to scratch memory).
// The Faure matrices are formed once per call by a small kernel into the
// workspace.
//
// Nested uniform scrambling of a base-2 net (Sec. 4.3, NUS): the point word
// z = C i (64 digits), then digit t = 1..64 is flipped when the top bit of
// mix64(key XOR seed) is set, key = 2^(t-1) + the unscrambled digits before
// t as an integer; mix64 is the SplitMix64 finaliser (Steele, Lea and Flood,
// 2014, with Stafford's Mix13 constants).  For base 2 a permutation of the
// digit values is the identity or the flip, and this draws one independently
// for every prefix, as nested uniform scrambling asks.
#include "common.hpp"

namespace ldk {

namespace {

constexpr int BP_T = LDK_BDIGITS_MAX;  // digit rows of the scramble layouts
constexpr int BP_THREADS = 256;
constexpr int BP_MAX_D = 54;  // the first 54 primes are below 256

struct BpArgs {
    int kind, R, d, flags;
    int64_t n_min, cnt;
    const uint8_t *lms, *perm, *shift;
    const uint8_t *cmat;  // Faure: [d][53][53] (row t, column k)
    double *out;
    uint8_t base[BP_MAX_D], T[BP_MAX_D], M[BP_MAX_D];
    double bT[BP_MAX_D];  // b^T, exact
};

// Faure matrix of dimension j = blockIdx.x: C[t][k] = binom(k, t) j^(k-t) mod b.
__global__ __launch_bounds__(64) void k_faure_cmat(int b, int T, uint8_t *__restrict__ cmat)
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
    if (t < T)
        for (int k = 0; k < BP_T; ++k) {
            const int v = (k < T && k >= t) ? (binom[k][t] * pw[k - t]) % b : 0;
            cmat[((size_t)j * BP_T + t) * BP_T + k] = (uint8_t)v;
        }
}

template <int KIND>
__global__ __launch_bounds__(BP_THREADS) void k_gen_bpoints(BpArgs a)
{
    __shared__ uint8_t zs[BP_T][BP_THREADS];  // each thread's digit vector, one column
    __shared__ uint8_t sS[BP_T * BP_T];
    __shared__ uint8_t sP[BP_T * 256];
    __shared__ uint8_t sD[BP_T];
    __shared__ uint8_t sC[BP_T * BP_T];
    const int tid = threadIdx.x, r = blockIdx.y;
    const int64_t ii = (int64_t)blockIdx.x * BP_THREADS + tid;
    const bool live = ii < a.cnt;
    const uint32_t i = (uint32_t)(a.n_min + (live ? ii : 0));
    for (int j = 0; j < a.d; ++j) {
        const int b = a.base[j], T = a.T[j], M = a.M[j];
        const size_t rj = (size_t)r * a.d + j;
        __syncthreads();  // the previous dimension's reads of the staging are done
        if (a.flags & LDK_BR_LMS)
            for (int q = tid; q < BP_T * BP_T; q += BP_THREADS) sS[q] = a.lms[rj * BP_T * BP_T + q];
        if (a.flags & LDK_BR_DP)
            for (int q = tid; q < BP_T * 256; q += BP_THREADS) sP[q] = a.perm[rj * BP_T * 256 + q];
        if ((a.flags & LDK_BR_DS) && tid < BP_T) sD[tid] = a.shift[rj * BP_T + tid];
        if constexpr (KIND == LDK_FAURE)
            for (int q = tid; q < BP_T * BP_T; q += BP_THREADS) sC[q] = a.cmat[(size_t)j * BP_T * BP_T + q];
        __syncthreads();
        if (!live) continue;
        // base-b digits of i, least significant first (i < 2^32)
        uint32_t q = i;
        for (int k = 0; k < M; ++k) {
            const uint32_t nq = q / (uint32_t)b;
            zs[k][tid] = (uint8_t)(q - nq * (uint32_t)b);
            q = nq;
        }
        for (int k = M; k < T; ++k) zs[k][tid] = 0;
        if constexpr (KIND == LDK_FAURE) {
            // z_t = sum_{k >= t} C[t][k] a_k, in place in increasing t (z_t
            // needs a_t .. a_{M-1} only)
            for (int t = 0; t < M; ++t) {
                uint32_t s = 0;
                for (int k = t; k < M; ++k) s += (uint32_t)sC[t * BP_T + k] * zs[k][tid];
                zs[t][tid] = (uint8_t)(s % (uint32_t)b);
            }
        }
        if (a.flags & LDK_BR_LMS) {
            // w_t = sum_{k <= t} S[t][k] z_k, in place in decreasing t (w_t
            // needs z_0 .. z_t only); z_k = 0 for k >= M
            for (int t = T - 1; t >= 0; --t) {
                const int kmax = t < M - 1 ? t : M - 1;
                uint32_t s = 0;
                for (int k = 0; k <= kmax; ++k) s += (uint32_t)sS[t * BP_T + k] * zs[k][tid];
                zs[t][tid] = (uint8_t)(s % (uint32_t)b);
            }
        }
        uint64_t v = 0;
        for (int t = 0; t < T; ++t) {
            uint32_t z = zs[t][tid];
            if (a.flags & LDK_BR_DP) z = sP[t * 256 + z];
            if (a.flags & LDK_BR_DS) {
                z += sD[t];
                if (z >= (uint32_t)b) z -= (uint32_t)b;
            }
            v = v * (uint64_t)b + z;
        }
        a.out[((size_t)r * a.cnt + ii) * a.d + j] = (double)v / a.bT[j];
    }
}

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(BP_THREADS) void k_gen_nus(int d, int m, int64_t n_min, int64_t cnt,
                                                         const uint64_t *__restrict__ gen,
                                                         const uint64_t *__restrict__ seed,
                                                         double *__restrict__ out)
{
    const int r = blockIdx.y;
    const int64_t ii = (int64_t)blockIdx.x * BP_THREADS + threadIdx.x;
    if (ii >= cnt) return;
    const uint64_t i = (uint64_t)(n_min + ii);
    for (int j = 0; j < d; ++j) {
        uint64_t z = 0;
        for (int k = 0; k < m; ++k)
            if ((i >> k) & 1u) z ^= gen[(size_t)j * m + k];
        const uint64_t s = seed[(size_t)r * d + j];
        // the flip of digit t keyed by the digits above it; the bit position
        // of digit t is 64 - t
        uint64_t flips = mix64(1ull ^ s) & 0x8000000000000000ull;
        for (int t = 2; t <= 64; ++t) {
            const uint64_t key = (1ull << (t - 1)) | (z >> (65 - t));
            flips |= (mix64(key ^ s) >> 63) << (64 - t);
        }
        out[((size_t)r * cnt + ii) * d + j] = unit_f64(z ^ flips);
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
    return (size_t)ps->d * BP_T * BP_T;
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
    const int64_t blocks = (cnt + BP_THREADS - 1) / BP_THREADS;
    if (blocks > 0x7fffffff) return LDK_ENOTSUP;
    const dim3 grid((unsigned)blocks, (unsigned)ps->R);
    if (ps->kind == LDK_DNET_NUS) {
        hipLaunchKernelGGL(k_gen_nus, grid, dim3(BP_THREADS), 0, s, ps->d, ps->m, n_min, cnt, ps->gen,
                           ps->seed, out);
        LDK_LAUNCH_CHECK();
        return LDK_OK;
    }
    BpArgs a{};
    a.kind = ps->kind;
    a.R = ps->R;
    a.d = ps->d;
    a.flags = ps->flags;
    a.n_min = n_min;
    a.cnt = cnt;
    a.lms = ps->lms;
    a.perm = ps->perm;
    a.shift = ps->shift;
    a.cmat = static_cast<const uint8_t *>(ws);
    a.out = out;
    int prime = 1;
    for (int j = 0; j < ps->d; ++j) {
        int b = ps->base;
        if (ps->kind == LDK_HALTON) {
            do ++prime;
            while (!is_prime(prime));
            b = prime;
        }
        a.base[j] = (uint8_t)b;
        a.T[j] = (uint8_t)digits_kept(b);
        a.M[j] = (uint8_t)index_digits(b, n_max);
        double p = 1.0;
        for (int t = 0; t < a.T[j]; ++t) p *= (double)b;
        a.bT[j] = p;
    }
    if (ps->kind == LDK_FAURE) {
        hipLaunchKernelGGL(k_faure_cmat, dim3((unsigned)ps->d), dim3(64), 0, s, ps->base,
                           digits_kept(ps->base), static_cast<uint8_t *>(ws));
        LDK_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_gen_bpoints<LDK_FAURE>, grid, dim3(BP_THREADS), 0, s, a);
    } else {
        hipLaunchKernelGGL(k_gen_bpoints<LDK_HALTON>, grid, dim3(BP_THREADS), 0, s, a);
    }
    LDK_LAUNCH_CHECK();
    return LDK_OK;
}
