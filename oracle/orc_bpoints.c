/*
 * Oracle: point sets without the FWHT structure (they feed only QMC means).
 *
 * THIS IS TEST INFRASTRUCTURE (see orc.h).
 *
 *  - Digital sequences in a prime base b (Sec. 4.3, any prime base): the
 *    base-b digits a_k of the index i (least significant first) give the
 *    digits z_t = sum_k C[t][k] a_k mod b of the point, t = 0..T-1 (digit t
 *    has weight b^-(t+1)).
 *      Faure: one prime b >= d for every dimension, C_j = P^(j-1) mod b,
 *      P the upper-triangular Pascal matrix P[r][c] = binom(c, r).  Here the
 *      power is formed by repeated matrix products mod b.
 *      Halton (Sec. 4.4): dimension j has the j-th prime as its base and
 *      C_j = the identity, i.e. the radical inverse of i.
 *    Randomizations, in this order, each optional: linear matrix scrambling
 *    z <- S z mod b with S lower triangular (LMS), digit permutations
 *    z_t <- pi_t(z_t) (DP), digital shift z_t <- z_t + delta_t mod b (DS).
 *    T is the largest digit count with b^T <= 2^53, so the point is the
 *    integer v = sum_t z_t b^(T-1-t) < 2^53 divided by b^T: one rounding.
 *  - Nested uniform scrambling of a base-2 digital net (Sec. 4.3, NUS): the
 *    point word z = C i (64 digits), then digit t (t = 1..64, weight 2^-t)
 *    is flipped when a pseudo-random bit keyed by the unscrambled digits
 *    z_1 .. z_{t-1} says so: for base 2 a permutation of {0, 1} is either
 *    the identity or the flip, chosen independently for every prefix.  The
 *    bits come from a counter-based generator: the 64-bit finaliser of
 *    SplitMix64 (Steele, Lea and Flood, 2014; the mixing constants are
 *    Stafford's "Mix13"), applied to (prefix key XOR the replication's and
 *    dimension's seed); the prefix key of length t - 1 is 2^(t-1) + the
 *    prefix as an integer.  The top bit of the mixed word is the flip.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "orc.h"

#define BT_MAX 53

int orc_bdigits(int b)
{
    if (b < 2) return 0;
    /* largest T with b^T <= 2^53, by exact integer products */
    int T = 0;
    uint64_t p = 1;
    const uint64_t lim = (uint64_t)1 << 53;
    while (p <= lim / (uint64_t)b) {
        p *= (uint64_t)b;
        ++T;
    }
    return T;
}

int orc_nth_prime(int j)
{
    /* j = 1, 2, ... by trial division */
    int count = 0;
    for (int c = 2;; ++c) {
        int prime = 1;
        for (int q = 2; q * q <= c; ++q)
            if (c % q == 0) {
                prime = 0;
                break;
            }
        if (prime && ++count == j) return c;
    }
}

/* C = A B mod b, T x T */
static void matmul_mod(int T, int b, const int *A, const int *B, int *C)
{
    for (int r = 0; r < T; ++r)
        for (int c = 0; c < T; ++c) {
            long s = 0;
            for (int k = 0; k < T; ++k) s += (long)A[r * T + k] * B[k * T + c];
            C[r * T + c] = (int)(s % b);
        }
}

/* Faure generating matrix of dimension j (1-based): P^(j-1) mod b. */
static void faure_matrix(int T, int b, int j, int *C)
{
    int *P = calloc((size_t)T * T, sizeof(int));
    int *tmp = calloc((size_t)T * T, sizeof(int));
    /* binom(c, r) mod b by Pascal's rule, column by column */
    for (int c = 0; c < T; ++c)
        for (int r = 0; r <= c; ++r)
            P[r * T + c] = (r == 0 || r == c) ? 1 % b : (P[(r - 1) * T + (c - 1)] + P[r * T + (c - 1)]) % b;
    memset(C, 0, sizeof(int) * (size_t)T * T);
    for (int r = 0; r < T; ++r) C[r * T + r] = 1;
    for (int k = 1; k < j; ++k) {
        matmul_mod(T, b, C, P, tmp);
        memcpy(C, tmp, sizeof(int) * (size_t)T * T);
    }
    free(P);
    free(tmp);
}

int orc_bpoints(int kind, int R, int d, int base, int flags, int64_t n_min, int64_t n_max,
                const uint8_t *lms, const uint8_t *perm, const uint8_t *shift, double *out)
{
    if (R < 0 || d < 1 || n_min < 0 || n_max < n_min) return -1;
    if (kind != ORC_HALTON && kind != ORC_FAURE) return -1;
    if (kind == ORC_FAURE && (base < 2 || base > 255)) return -1;
    const int64_t cnt = n_max - n_min;
    int *C = malloc(sizeof(int) * BT_MAX * BT_MAX);
    int a[BT_MAX], z[BT_MAX], w[BT_MAX];
    for (int j = 0; j < d; ++j) {
        const int b = kind == ORC_HALTON ? orc_nth_prime(j + 1) : base;
        if (b > 255) {
            free(C);
            return -1;
        }
        const int T = orc_bdigits(b);
        if (kind == ORC_FAURE) {
            faure_matrix(T, b, j + 1, C);
        } else {
            memset(C, 0, sizeof(int) * (size_t)T * T);
            for (int t = 0; t < T; ++t) C[t * T + t] = 1;
        }
        double bT = 1.0;
        for (int t = 0; t < T; ++t) bT *= b; /* exact: b^T <= 2^53 */
        for (int r = 0; r < R; ++r) {
            const size_t rj = (size_t)r * d + j;
            for (int64_t ii = 0; ii < cnt; ++ii) {
                uint64_t i = (uint64_t)(n_min + ii);
                for (int k = 0; k < T; ++k) {
                    a[k] = (int)(i % (uint64_t)b);
                    i /= (uint64_t)b;
                }
                if (i != 0) { /* the index needs more than T digits */
                    free(C);
                    return -1;
                }
                for (int t = 0; t < T; ++t) {
                    long s = 0;
                    for (int k = 0; k < T; ++k) s += (long)C[t * T + k] * a[k];
                    z[t] = (int)(s % b);
                }
                if (flags & ORC_BR_LMS) {
                    const uint8_t *S = lms + rj * BT_MAX * BT_MAX;
                    for (int t = 0; t < T; ++t) {
                        long s = 0;
                        for (int k = 0; k <= t; ++k) s += (long)S[t * BT_MAX + k] * z[k];
                        w[t] = (int)(s % b);
                    }
                    memcpy(z, w, sizeof(int) * (size_t)T);
                }
                if (flags & ORC_BR_DP) {
                    const uint8_t *pi = perm + rj * BT_MAX * 256;
                    for (int t = 0; t < T; ++t) z[t] = pi[t * 256 + z[t]];
                }
                if (flags & ORC_BR_DS) {
                    const uint8_t *dl = shift + rj * BT_MAX;
                    for (int t = 0; t < T; ++t) z[t] = (z[t] + dl[t]) % b;
                }
                uint64_t v = 0;
                for (int t = 0; t < T; ++t) v = v * (uint64_t)b + (uint64_t)z[t];
                out[((size_t)r * cnt + ii) * d + j] = (double)v / bT;
            }
        }
    }
    free(C);
    return 0;
}

uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

int orc_nus_points(int R, int d, int m, int64_t n_min, int64_t n_max, const uint64_t *C,
                   const uint64_t *seed, uint64_t *out)
{
    if (R < 0 || d < 1 || m < 0 || m > 63 || n_min < 0 || n_max < n_min) return -1;
    if (n_max > ((int64_t)1 << m)) return -1;
    const int64_t cnt = n_max - n_min;
    for (int r = 0; r < R; ++r)
        for (int64_t ii = 0; ii < cnt; ++ii) {
            const uint64_t i = (uint64_t)(n_min + ii);
            for (int j = 0; j < d; ++j) {
                /* z = C_j i: XOR of the columns picked by the bits of i */
                uint64_t z = 0;
                for (int k = 0; k < m; ++k)
                    if ((i >> k) & 1u) z ^= C[(size_t)j * m + k];
                const uint64_t s = seed[(size_t)r * d + j];
                uint64_t x = 0;
                for (int t = 1; t <= 64; ++t) {
                    const uint64_t prefix = t == 1 ? 0 : z >> (65 - t);
                    const uint64_t key = ((uint64_t)1 << (t - 1)) | prefix;
                    const uint64_t flip = orc_mix64(key ^ s) >> 63;
                    const uint64_t digit = (z >> (64 - t)) & 1u;
                    x |= (digit ^ flip) << (64 - t);
                }
                out[((size_t)r * cnt + ii) * d + j] = x;
            }
        }
    return 0;
}
