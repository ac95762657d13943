/*
 * Oracle: low-discrepancy point sets (test infrastructure only).
 *
 * Written from the definitions of Sec. 4.1-4.3 of the paper, digit by digit.
 */
#include <stdlib.h>
#include <string.h>

#include "orc.h"

/* Sec. 4.2, lattice sequence: z_i = v(i) g mod 1 with v(i) the van der Corput
 * radical inverse of eq. (v), v(i) = sum_{t>=1} i_{t-1} 2^-t.
 * In 64-bit fixed point, digit i_{t-1} contributes g * 2^-t mod 1, i.e. the
 * word g << (64 - t) (bits shifted past 2^0 are the integer part, dropped).
 * Linear order (fixed n = 2^m): z_i = (i g / n) mod 1 = ((i g) mod n) 2^-m.
 * Shifted lattice: x_i = (z_i + Delta) mod 1 (unsigned wrap-around). */
int orc_lattice_points(int R, int d, int m, int order, int64_t n_min, int64_t n_max,
                       const uint64_t *g, const uint64_t *shift, uint64_t *out)
{
    if (R < 1 || d < 1 || m < 0 || m > 62 || n_min < 0 || n_max < n_min) return -1;
    if (order == ORC_LINEAR && n_max > ((int64_t)1 << m)) return -1;
    if (order != ORC_NATURAL && order != ORC_LINEAR) return -1;
    const int64_t cnt = n_max - n_min;
    /* points are independent (OpenMP in the CPU-baseline build only) */
#pragma omp parallel for collapse(2) schedule(static)
    for (int r = 0; r < R; ++r)
        for (int64_t ii = 0; ii < cnt; ++ii) {
            const uint64_t i = (uint64_t)(n_min + ii);
            for (int j = 0; j < d; ++j) {
                uint64_t z = 0;
                if (order == ORC_NATURAL) {
                    for (int t = 1; t <= 64; ++t) {
                        const uint64_t digit = (i >> (t - 1)) & 1u;
                        if (digit) z += (t == 64) ? g[j] : (g[j] << (64 - t));
                    }
                } else {
                    const unsigned __int128 n = (unsigned __int128)1 << m;
                    const unsigned __int128 prod = (unsigned __int128)i * g[j];
                    const uint64_t resid = (uint64_t)(prod % n);
                    z = (m == 0) ? 0 : (resid << (64 - m));
                }
                const uint64_t delta = shift ? shift[(size_t)r * d + j] : 0;
                out[((size_t)r * cnt + ii) * d + j] = z + delta;
            }
        }
    return 0;
}

/* Gray code of i (Sec. 4.3, Table 1): consecutive codes differ in one digit. */
uint64_t orc_gray(uint64_t i) { return i ^ (i >> 1); }

/* Bit (row t, column k) of a matrix stored as column words (row t at bit 63-t). */
static int col_bit(uint64_t col, int t) { return (int)((col >> (63 - t)) & 1u); }

/* Linear matrix scrambling, Sec. 4.3: Ct_j = S_j C_j mod 2, as a plain dense
 * 0/1 matrix product.  S_j rows are words (entry (t,s) at bit 63-s); C_j and
 * the result are column words. */
int orc_lms(int d, int m, const uint64_t *C, const uint64_t *S, uint64_t *Ct)
{
    for (int j = 0; j < d; ++j) {
        for (int k = 0; k < m; ++k) {
            uint64_t col = 0;
            for (int t = 0; t < 64; ++t) {
                int acc = 0;
                for (int s = 0; s < 64; ++s) {
                    const int s_ts = (int)((S[(size_t)j * 64 + t] >> (63 - s)) & 1u);
                    acc += s_ts * col_bit(C[(size_t)j * m + k], s);
                }
                if (acc & 1) col |= (uint64_t)1 << (63 - t);
            }
            Ct[(size_t)j * m + k] = col;
        }
    }
    return 0;
}

/* Digital net in base 2, Sec. 4.3: z_ij = F_64(C_j D_m(i) mod 2), i.e. the
 * GF(2) matrix-vector product of the (scrambled) generating matrix with the
 * digit vector of i, which is the XOR of the columns k whose digit i_k = 1.
 * Digital shift: x_ij = F_64((z_ij + Delta_j) mod 2), digitwise XOR.
 * Gray order: point i uses the digit vector of gray(i). */
int orc_dnet_points(int R, int d, int m_max, int order, int64_t n_min, int64_t n_max,
                    const uint64_t *C, const uint64_t *S, const uint64_t *shift,
                    uint64_t *out)
{
    if (R < 1 || d < 1 || m_max < 0 || m_max > 62 || n_min < 0 || n_max < n_min) return -1;
    if (n_max > ((int64_t)1 << m_max)) return -1;
    if (order != ORC_NATURAL && order != ORC_GRAY) return -1;
    const int64_t cnt = n_max - n_min;
    uint64_t *Ct = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)d * (m_max ? m_max : 1));
    if (!Ct) return -2;
    for (int r = 0; r < R; ++r) {
        if (S)
            orc_lms(d, m_max, C, S + (size_t)r * d * 64, Ct);
        else
            memcpy(Ct, C, sizeof(uint64_t) * (size_t)d * m_max);
#pragma omp parallel for schedule(static)
        for (int64_t ii = 0; ii < cnt; ++ii) {
            const uint64_t i = (uint64_t)(n_min + ii);
            const uint64_t code = (order == ORC_GRAY) ? orc_gray(i) : i;
            for (int j = 0; j < d; ++j) {
                uint64_t z = 0;
                for (int k = 0; k < m_max; ++k)
                    if ((code >> k) & 1u) z ^= Ct[(size_t)j * m_max + k];
                const uint64_t delta = shift ? shift[(size_t)r * d + j] : 0;
                out[((size_t)r * cnt + ii) * d + j] = z ^ delta;
            }
        }
    }
    free(Ct);
    return 0;
}
