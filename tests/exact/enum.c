/*
 * enum.c -- exact enumeration of every configuration of a small periodic
 * L x L lattice of the four-state model (section 2.1, eq. (3)), for the
 * statistical pins of the oracle.  Test infrastructure; written separately
 * from the oracle (its own site tables, bond sums and loops).
 *
 * The result is the density of states
 *   g[Q + N][Nc][BV + 2N][BJ + 2N]  (int64 counts)
 * with Q = sum S, Nc = sum S^2, BV = sum over bonds S S, BJ = sum over bonds
 * sigma sigma (each of the 2N bonds once).  Any Boltzmann average of a function
 * of (Q, Nc, BV, BJ) in any charge sector follows from it for every
 * (Delta, V, J, T).
 *
 * L = 3: direct loop over the 4^9 configurations.
 * L = 4: rows of 4 sites (256 row states); for fixed rows 0 and 2 the
 * contributions of row 1 (between rows 0 and 2) and of row 3 (between rows 2
 * and 0) take values from the same table, so their joint histogram is the
 * self-convolution of one compressed 256-entry table.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static const int CHG[4] = {0, 0, 1, -1};   /* S of code 0..3 */
static const int SPN[4] = {1, -1, 0, 0};   /* sigma of code 0..3 */

static int64_t dims_index(int L, int Q, int Nc, int BV, int BJ)
{
    int N = L * L;
    int64_t dNc = N + 1, dB = 4 * N + 1;
    return (((int64_t)(Q + N) * dNc + Nc) * dB + (BV + 2 * N)) * dB + (BJ + 2 * N);
}

int64_t exact_hist_size(int L)
{
    int N = L * L;
    return (int64_t)(2 * N + 1) * (N + 1) * (4 * N + 1) * (4 * N + 1);
}

static void enum_l3(int64_t *g)
{
    const int L = 3, N = 9;
    int c[9];
    for (int64_t cfg = 0; cfg < (1 << (2 * N)); ++cfg) {
        for (int i = 0; i < N; ++i) c[i] = (int)((cfg >> (2 * i)) & 3);
        int Q = 0, Nc = 0, BV = 0, BJ = 0;
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                int i = y * L + x, r = y * L + (x + 1) % L, d = ((y + 1) % L) * L + x;
                Q += CHG[c[i]];
                Nc += CHG[c[i]] * CHG[c[i]];
                BV += CHG[c[i]] * CHG[c[r]] + CHG[c[i]] * CHG[c[d]];
                BJ += SPN[c[i]] * SPN[c[r]] + SPN[c[i]] * SPN[c[d]];
            }
        g[dims_index(L, Q, Nc, BV, BJ)] += 1;
    }
}

static void enum_l4(int64_t *g)
{
    const int L = 4;
    int q[256], nc[256], bv[256], bj[256];
    static int vv[256][256], vj[256][256];
    for (int r = 0; r < 256; ++r) {
        q[r] = nc[r] = bv[r] = bj[r] = 0;
        for (int x = 0; x < 4; ++x) {
            int a = (r >> (2 * x)) & 3, b = (r >> (2 * ((x + 1) % 4))) & 3;
            q[r] += CHG[a];
            nc[r] += CHG[a] * CHG[a];
            bv[r] += CHG[a] * CHG[b];
            bj[r] += SPN[a] * SPN[b];
        }
    }
    for (int r = 0; r < 256; ++r)
        for (int s = 0; s < 256; ++s) {
            vv[r][s] = vj[r][s] = 0;
            for (int x = 0; x < 4; ++x) {
                int a = (r >> (2 * x)) & 3, b = (s >> (2 * x)) & 3;
                vv[r][s] += CHG[a] * CHG[b];
                vj[r][s] += SPN[a] * SPN[b];
            }
        }
    /* Linear index strides: index = base + sum of per-row offsets. */
    const int N = 16;
    const int64_t sBJ = 1, sBV = 4 * N + 1, sNc = sBV * (4 * N + 1), sQ = sNc * (N + 1);
    const int64_t base = dims_index(L, 0, 0, 0, 0);
    for (int r0 = 0; r0 < 256; ++r0) {
        for (int r2 = 0; r2 < 256; ++r2) {
            /* offsets of a middle row m between r0 and r2 */
            int64_t off[256];
            int64_t uniq[256];
            int64_t cnt[256];
            int nu = 0;
            for (int m = 0; m < 256; ++m) {
                int dBV = bv[m] + vv[r0][m] + vv[m][r2];
                int dBJ = bj[m] + vj[r0][m] + vj[m][r2];
                off[m] = q[m] * sQ + nc[m] * sNc + dBV * sBV + dBJ * sBJ;
            }
            for (int m = 0; m < 256; ++m) {
                int k = 0;
                while (k < nu && uniq[k] != off[m]) ++k;
                if (k == nu) { uniq[nu] = off[m]; cnt[nu] = 0; ++nu; }
                cnt[k] += 1;
            }
            int64_t own = base + (q[r0] + q[r2]) * sQ + (nc[r0] + nc[r2]) * sNc +
                          (bv[r0] + bv[r2]) * sBV + (bj[r0] + bj[r2]) * sBJ;
            for (int i = 0; i < nu; ++i)
                for (int k = 0; k < nu; ++k)
                    g[own + uniq[i] + uniq[k]] += cnt[i] * cnt[k];
        }
    }
}

/* Fill g (exact_hist_size(L) int64, zeroed by the caller). Returns 0 or -1. */
int exact_hist(int L, int64_t *g)
{
    if (L == 3) { enum_l3(g); return 0; }
    if (L == 4) { enum_l4(g); return 0; }
    return -1;
}
