/*
 * oracle.c -- sequential CPU oracle for the coupled-pair Metropolis algorithm
 * with an exact charge constraint (Budrin, Ulitko, Chikov, Panov, Moskvin,
 * "The Parallel Monte Carlo Algorithm Implementation on GPU for the Systems
 * with an Ising Hamiltonian under the Condition of a Constant Charge Density",
 * arXiv:2301.11735).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this code.  The product library never
 * links, imports or calls it, and it shares no code with the product.
 *
 * Everything here is plain, sequential and slow on purpose:
 *   - the state is one int8 code per site, row-major (site (x,y) at y*L+x);
 *   - pairs of a phase are visited one at a time, in pair-index order;
 *   - the energy change of a proposed pair move is recomputed from the
 *     definition of the energy, eq. (3), over the bonds that touch the pair;
 *   - the Metropolis threshold is recomputed with exp() for every proposal
 *     (no table).
 *
 * Site codes (section 2.1): 0 = magnetic s=+1/2 (sigma=+1), 1 = magnetic
 * s=-1/2 (sigma=-1), 2 = charge S=+1, 3 = charge S=-1.
 *
 * Readings of the paper that this file implements (the paper leaves them open):
 *   R1  every nearest-neighbour bond is counted once (2N bonds);
 *   R2  the J term is (J/4) sigma_i sigma_j as in eq. (3);
 *   R3  the proposal is uniform over the whole same-q set, the current
 *       configuration included;
 *   R4  the target charge Q is rounded to the parity of the charged count;
 *   R5  the concurrent pairs of a phase follow a fixed sublattice schedule
 *       with a random long-range displacement per phase, instead of the
 *       paper's random maps (section 3.2);
 *   R6  randomness is Philox4x32-10 keyed by the seed, with the counter
 *       naming the sweep, the phase and the pair.
 *   R15 penalty mode (section 2.2, the prior method): single-site
 *       checkerboard Metropolis on E - mu sum S, each site proposing one of
 *       its 4 codes, mu adjusted after every sweep by mu += kappa (Q - sum S)/N.
 *   R12 map mode (section 3.2 as printed): maps of max(1, floor(N/10))
 *       pairs built by the paper's sequential algorithm, the site draws
 *       taken from Philox words in counter order; a pair's two sites may be
 *       neighbours.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Philox4x32-10: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11.  Round: multiply counter words 0 and 2 by the two
 * round multipliers, xor the high halves with the other two counter words and
 * the round key; the key is bumped by the two Weyl constants between rounds. */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void philox_seeded(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                          uint32_t c3, uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox(ctr, key, out);
}

/* Counter domains (word 1 of the counter). */
#define DOM_SCHEDULE 0x100u
#define DOM_INIT     0x200u
#define DOM_GENERAL  0x300u
#define DOM_MAP      0x400u
#define DOM_MAPSTEP  0x500u
#define DOM_MU       0x600u

static uint32_t mulhi32(uint32_t a, uint32_t b)
{
    return (uint32_t)(((uint64_t)a * (uint64_t)b) >> 32);
}

/* ------------------------------------------------------------------ */
/* Site model, section 2.1 and eq. (3). */
static const int S_OF[4] = {0, 0, 1, -1};
static const int SIG_OF[4] = {1, -1, 0, 0};

/* Two-site configurations of each pair charge q = S_a + S_b, in the order the
 * paper lists them (section 3.1, "Algorithm"):
 *   q=+2: (+1,+1)
 *   q=+1: (+1,+1/2) (+1,-1/2) (+1/2,+1) (-1/2,+1)
 *   q= 0: (+1,-1) (-1,+1) (+1/2,+1/2) (-1/2,-1/2) (+1/2,-1/2) (-1/2,+1/2)
 *   q=-1: (-1,+1/2) (-1,-1/2) (+1/2,-1) (-1/2,-1)
 *   q=-2: (-1,-1)
 * Each entry is {code_a, code_b}. */
static const int SET_Q_PLUS1[4][2] = {{2, 0}, {2, 1}, {0, 2}, {1, 2}};
static const int SET_Q_ZERO[6][2] = {{2, 3}, {3, 2}, {0, 0}, {1, 1}, {0, 1}, {1, 0}};
static const int SET_Q_MINUS1[4][2] = {{3, 0}, {3, 1}, {0, 3}, {1, 3}};

/* The j-th configuration of the same-q set in the listing order above;
 * returns 0, or -1 for |q| = 2 (frozen) or j out of range. */
int orc_pair_config(int q, int j, int out[2])
{
    const int *pick;
    if (q == 1 && j >= 0 && j < 4) pick = SET_Q_PLUS1[j];
    else if (q == 0 && j >= 0 && j < 6) pick = SET_Q_ZERO[j];
    else if (q == -1 && j >= 0 && j < 4) pick = SET_Q_MINUS1[j];
    else return -1;
    out[0] = pick[0];
    out[1] = pick[1];
    return 0;
}

/* Metropolis acceptance threshold for an integer energy-change triple
 * (section 3.1: the classical Metropolis rule; eq. (3) for the energy):
 *   dE = Delta*nD + V*nV + (J/4)*nJ,
 *   dE <= 0 -> 0xFFFFFFFF ("always"),
 *   else    -> min(floor(exp(-dE/T) * 2^32), 0xFFFFFFFE).
 * A proposal is accepted iff thr == 0xFFFFFFFF or u < thr for a uniform
 * 32-bit draw u. */
static uint32_t threshold_of_dE(double dE, double T)
{
    if (dE <= 0.0) return 0xFFFFFFFFu;
    double x = exp(-dE / T) * 4294967296.0;
    double f = floor(x);
    if (f >= 4294967294.0) return 0xFFFFFFFEu;
    return (uint32_t)f;
}

uint32_t orc_threshold(double Delta, double V, double J, double T, int nD, int nV, int nJ)
{
    double dE = Delta * nD + V * nV + 0.25 * J * nJ;
    return threshold_of_dE(dE, T);
}

/* ------------------------------------------------------------------ */
/* Eq. (2): total charge Q = nN, made an integer (reading R4).  The charged
 * count Nc and Q must have equal parity because N+ - N- = Q and N+ + N- = Nc.
 *   Nc0 = n_charged_req if >= 0, else N/4;
 *   Q   = integer nearest to n*N with the parity of Nc0, ties to the smaller;
 *   if |Q| > Nc0 and no count was requested: Nc = |Q|; else Nc = Nc0.
 * Returns 0, or -1 if no valid (Q, Nc) exists. */
int orc_charge_target(int32_t L, double n, int64_t n_charged_req, int64_t *Q_out, int64_t *Nc_out)
{
    int64_t N = (int64_t)L * L;
    double target = n * (double)N;
    if (!(target == target) || fabs(target) > (double)N) return -1;
    int64_t Nc0 = n_charged_req >= 0 ? n_charged_req : N / 4;
    if (Nc0 > N) return -1;
    int64_t par = Nc0 & 1;
    /* the two integers of the right parity around target */
    int64_t lo = (int64_t)floor(target);
    if (((lo % 2) + 2) % 2 != par) lo -= 1;
    int64_t hi = lo + 2;
    double dlo = target - (double)lo, dhi = (double)hi - target;
    int64_t Q = (dhi < dlo) ? hi : lo;
    int64_t Nc = Nc0;
    if (llabs(Q) > Nc0) {
        if (n_charged_req >= 0) return -1;
        Nc = llabs(Q);
    }
    if (Nc > N || llabs(Q) > N) return -1;
    *Q_out = Q;
    *Nc_out = Nc;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Stage 1 of section 3.1: a configuration with the requested charge.  Reading:
 * every site i draws a 64-bit key K_i = (w0 << 32) | w1 from Philox with
 * counter (0, DOM_INIT, i, 0); sites are ranked by (K_i, i); ranks [0, N+)
 * become S=+1, ranks [N+, N+ + N-) become S=-1, and every other site is
 * magnetic with sigma from bit 0 of w2 (code = w2 & 1). */
typedef struct {
    uint64_t key;
    uint32_t idx;
} ranked_site;

static int cmp_ranked(const void *a, const void *b)
{
    const ranked_site *x = (const ranked_site *)a, *y = (const ranked_site *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
    return 0;
}

int orc_init(int32_t L, uint64_t seed, int64_t n_plus, int64_t n_minus, int8_t *codes)
{
    int64_t N = (int64_t)L * L;
    ranked_site *r = (ranked_site *)malloc(sizeof(ranked_site) * (size_t)N);
    if (!r) return -1;
    for (int64_t i = 0; i < N; ++i) {
        uint32_t w[4];
        philox_seeded(seed, 0u, DOM_INIT, (uint32_t)i, 0u, w);
        r[i].key = ((uint64_t)w[0] << 32) | w[1];
        r[i].idx = (uint32_t)i;
        codes[i] = (int8_t)(w[2] & 1u);
    }
    qsort(r, (size_t)N, sizeof(ranked_site), cmp_ranked);
    for (int64_t k = 0; k < n_plus + n_minus; ++k)
        codes[r[k].idx] = (int8_t)(k < n_plus ? 2 : 3);
    free(r);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Schedule of one sweep (reading R5; section 3.2 asks for concurrent pairs that
 * do not interact, and section 3.2's ergodicity remark asks for long-range
 * random partners).  Sweep s draws 12 words W[0..11] from Philox counters
 * (s_lo, DOM_SCHEDULE, t, s_hi), t = 0,1,2.  Then
 *   r     = 1 + (((W[0] >> 8) * 3) >> 24)          in {1,2,3}
 *   m_p   = mulhi(W[1+2p], L/4),  k_p = mulhi(W[2+2p], L/2)
 *   D_p   = ((r + 4 m_p) mod L, (1 + 2 k_p) mod L)  for phases p = 0..3.
 * Phase p pairs every a = (x, y) with x = p (mod 4), y even, to b = a + D_p. */
void orc_schedule(int32_t L, uint64_t seed, uint64_t sweep, int32_t *r_out, int32_t Dx[4], int32_t Dy[4])
{
    uint32_t W[12];
    for (uint32_t t = 0; t < 3; ++t)
        philox_seeded(seed, (uint32_t)sweep, DOM_SCHEDULE, t, (uint32_t)(sweep >> 32), &W[4 * t]);
    int32_t r = 1 + (int32_t)(((uint64_t)(W[0] >> 8) * 3u) >> 24);
    for (int p = 0; p < 4; ++p) {
        uint32_t m = mulhi32(W[1 + 2 * p], (uint32_t)(L / 4));
        uint32_t k = mulhi32(W[2 + 2 * p], (uint32_t)(L / 2));
        Dx[p] = (int32_t)(((int64_t)r + 4 * (int64_t)m) % L);
        Dy[p] = (int32_t)((1 + 2 * (int64_t)k) % L);
    }
    *r_out = r;
}

/* ------------------------------------------------------------------ */
/* Energy bookkeeping straight from eq. (3).  For a set of two sites {a, b}
 * the terms of E that involve them are
 *   Delta part: S_a^2 + S_b^2
 *   V part:     sum of S_i S_j over the bonds that touch a or b
 *   J part:     sum of sigma_i sigma_j over the same bonds
 * where a bond that joins a and b is counted once (reading R1).  The change
 * of these three integers is the change of the whole energy's integer parts. */
static void neighbours(int32_t L, int64_t i, int64_t nb[4])
{
    int64_t x = i % L, y = i / L;
    nb[0] = y * L + (x + 1) % L;
    nb[1] = y * L + (x + L - 1) % L;
    nb[2] = ((y + 1) % L) * L + x;
    nb[3] = ((y + L - 1) % L) * L + x;
}

static void local_terms(int32_t L, const int8_t *c, int64_t a, int64_t b, int64_t *tD, int64_t *tV, int64_t *tJ)
{
    int64_t nb[4];
    int64_t D = 0, Vs = 0, Js = 0;
    D += S_OF[c[a]] * S_OF[c[a]] + S_OF[c[b]] * S_OF[c[b]];
    neighbours(L, a, nb);
    for (int k = 0; k < 4; ++k) {
        Vs += S_OF[c[a]] * S_OF[c[nb[k]]];
        Js += SIG_OF[c[a]] * SIG_OF[c[nb[k]]];
    }
    neighbours(L, b, nb);
    for (int k = 0; k < 4; ++k) {
        if (nb[k] == a) continue; /* bond a-b already counted from a's side */
        Vs += S_OF[c[b]] * S_OF[c[nb[k]]];
        Js += SIG_OF[c[b]] * SIG_OF[c[nb[k]]];
    }
    *tD = D; *tV = Vs; *tJ = Js;
}

/* Integer energy-change triple (nD, nV, nJ) of setting sites a, b to codes
 * (ca1, cb1), from the definition of eq. (3); the codes are left unchanged. */
void orc_pair_delta(int32_t L, int8_t *c, int64_t a, int64_t b, int ca1, int cb1, int64_t out[3])
{
    int64_t D0, V0, J0, D1, V1, J1;
    int8_t ca0 = c[a], cb0 = c[b];
    local_terms(L, c, a, b, &D0, &V0, &J0);
    c[a] = (int8_t)ca1;
    c[b] = (int8_t)cb1;
    local_terms(L, c, a, b, &D1, &V1, &J1);
    c[a] = ca0;
    c[b] = cb0;
    out[0] = D1 - D0; out[1] = V1 - V0; out[2] = J1 - J0;
}

/* One coupled-pair Metropolis step on sites (a, b) (section 3.1, "Algorithm"):
 * q = S_a + S_b; |q| = 2 cannot change; otherwise draw one configuration of
 * the same-q set (index j from u_choice), compute the energy change and accept
 * with the Metropolis rule using u_acc.  Returns 1 if the move was accepted. */
static int pair_step(int32_t L, int8_t *c, int64_t a, int64_t b, uint32_t u_choice, uint32_t u_acc,
                     double Delta, double V, double J, double T, int64_t track[3])
{
    int q = S_OF[c[a]] + S_OF[c[b]];
    if (q == 2 || q == -2) return 0;
    uint32_t kq = (q == 0) ? 6u : 4u;
    uint32_t j = (uint32_t)(((uint64_t)(u_choice >> 8) * kq) >> 24);
    const int *pick;
    if (q == 1) pick = SET_Q_PLUS1[j];
    else if (q == 0) pick = SET_Q_ZERO[j];
    else pick = SET_Q_MINUS1[j];

    int64_t D0, V0, J0, D1, V1, J1;
    local_terms(L, c, a, b, &D0, &V0, &J0);
    int8_t ca0 = c[a], cb0 = c[b];
    c[a] = (int8_t)pick[0];
    c[b] = (int8_t)pick[1];
    local_terms(L, c, a, b, &D1, &V1, &J1);
    int nD = (int)(D1 - D0), nV = (int)(V1 - V0), nJ = (int)(J1 - J0);

    uint32_t thr = orc_threshold(Delta, V, J, T, nD, nV, nJ);
    int accept = (thr == 0xFFFFFFFFu) || (u_acc < thr);
    if (accept) {
        track[0] += nD; track[1] += nV; track[2] += nJ;
    } else {
        c[a] = ca0;
        c[b] = cb0;
    }
    return accept;
}

/* Sweeps of the structured chain (readings R5, R6).  In phase p of sweep s the
 * pair with a = (x, y), x = p (mod 4), y even, has index
 *   pairIdx = (y/2)*(L/4) + (x - p)/4
 * and b = a + D_p.  Philox counter (s_lo, p, pairIdx >> 1, s_hi) gives four
 * words; the pair uses words h and h+1 with h = 2*(pairIdx & 1): word h picks
 * the configuration, word h+1 is the acceptance draw.  Pairs are visited in
 * pairIdx order.  track[] accumulates the accepted (nD, nV, nJ). */
int orc_sweeps(int32_t L, double Delta, double V, double J, double T, uint64_t seed,
               uint64_t start_sweep, uint64_t n_sweeps, int8_t *codes, int64_t track[3])
{
    if (L < 4 || L % 4 != 0) return -1;
    for (uint64_t s = start_sweep; s < start_sweep + n_sweeps; ++s) {
        int32_t r, Dx[4], Dy[4];
        orc_schedule(L, seed, s, &r, Dx, Dy);
        for (int p = 0; p < 4; ++p) {
            for (int64_t y = 0; y < L; y += 2) {
                for (int64_t x = p; x < L; x += 4) {
                    int64_t pair_idx = (y / 2) * (L / 4) + (x - p) / 4;
                    int64_t a = y * L + x;
                    int64_t b = ((y + Dy[p]) % L) * L + (x + Dx[p]) % L;
                    uint32_t w[4];
                    philox_seeded(seed, (uint32_t)s, (uint32_t)p, (uint32_t)(pair_idx >> 1),
                                  (uint32_t)(s >> 32), w);
                    int h = 2 * (int)(pair_idx & 1);
                    pair_step(L, codes, a, b, w[h], w[h + 1], Delta, V, J, T, track);
                }
            }
        }
    }
    return 0;
}

/* General mode: the paper's sequential algorithm with one randomly chosen
 * coupled pair per step (section 3.1), any L >= 3, adjacent pairs allowed.
 * Step t uses Philox counter (t_lo, DOM_GENERAL, t_hi, 0):
 *   a = mulhi(w0, N), b' = mulhi(w1, N-1), b = b' + (b' >= a),
 *   w2 picks the configuration, w3 is the acceptance draw. */
int orc_general_steps(int32_t L, double Delta, double V, double J, double T, uint64_t seed,
                      uint64_t start_step, uint64_t n_steps, int8_t *codes, int64_t track[3])
{
    if (L < 3) return -1;
    uint32_t N = (uint32_t)((int64_t)L * L);
    for (uint64_t t = start_step; t < start_step + n_steps; ++t) {
        uint32_t w[4];
        philox_seeded(seed, (uint32_t)t, DOM_GENERAL, (uint32_t)(t >> 32), 0u, w);
        uint32_t a = mulhi32(w[0], N);
        uint32_t bp = mulhi32(w[1], N - 1u);
        uint32_t b = bp + (bp >= a ? 1u : 0u);
        pair_step(L, codes, a, b, w[2], w[3], Delta, V, J, T, track);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Observables of a configuration, all exact integers:
 *   out[0] sum_S   = sum_i S_i                       (eq. 2)
 *   out[1] n_ch    = sum_i S_i^2                     (Delta term of eq. 3)
 *   out[2] bond_SS = sum over bonds of S_i S_j       (V term of eq. 3)
 *   out[3] bond_ss = sum over bonds of sigma_i sigma_j (J term of eq. 3)
 *   out[4] M       = sum_i sigma_i                   (= 2 sum_i s_i)
 *   out[5] M_st    = sum_i (-1)^(x+y) sigma_i
 *   out[6] C_st    = sum_i (-1)^(x+y) S_i
 * Bonds are (x,y)-(x+1,y) and (x,y)-(x,y+1), periodic, each once. */
void orc_observables(int32_t L, const int8_t *codes, int64_t out[7])
{
    int64_t o[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t y = 0; y < L; ++y) {
        for (int64_t x = 0; x < L; ++x) {
            int c = codes[y * L + x];
            int cr = codes[y * L + (x + 1) % L];
            int cd = codes[((y + 1) % L) * L + x];
            int sgn = ((x + y) & 1) ? -1 : 1;
            o[0] += S_OF[c];
            o[1] += S_OF[c] * S_OF[c];
            o[2] += S_OF[c] * S_OF[cr] + S_OF[c] * S_OF[cd];
            o[3] += SIG_OF[c] * SIG_OF[cr] + SIG_OF[c] * SIG_OF[cd];
            o[4] += SIG_OF[c];
            o[5] += sgn * SIG_OF[c];
            o[6] += sgn * S_OF[c];
        }
    }
    memcpy(out, o, sizeof(o));
}

/* Energy of eq. (3) from the observables, in FP64. */
double orc_energy(double Delta, double V, double J, const int64_t obs[7])
{
    return Delta * (double)obs[1] + V * (double)obs[2] + 0.25 * J * (double)obs[3];
}

/* Run n_obs observation intervals of `every` sweeps each, writing the 7
 * observables after every interval to series[7*k .. 7*k+6].  A convenience
 * loop over orc_sweeps and orc_observables for the statistical tests. */
int orc_series(int32_t L, double Delta, double V, double J, double T, uint64_t seed,
               uint64_t start_sweep, uint64_t every, uint64_t n_obs, int8_t *codes,
               int64_t track[3], int64_t *series)
{
    for (uint64_t k = 0; k < n_obs; ++k) {
        int rc = orc_sweeps(L, Delta, V, J, T, seed, start_sweep + k * every, every, codes, track);
        if (rc) return rc;
        orc_observables(L, codes, &series[7 * k]);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Map mode (section 3.2, "Algorithm for building a map" and the processing
 * of maps).  A map is a list of coupled pairs no two of which interact: no
 * site of one pair is a site or a nearest neighbour of a site of another. */

/* Pairs per map: N/10 (section 3.2), at least one. */
int64_t orc_map_pairs(int32_t L)
{
    int64_t n = (int64_t)L * L / 10;
    return n < 1 ? 1 : n;
}

/* Build map m (section 3.2): pairs are accepted one at a time until the map
 * holds orc_map_pairs(L) of them.  Each site of a pair is the first draw that
 * lands on a site not yet marked; the first site is marked before its
 * partner is drawn, so a pair's two sites differ but may be neighbours; once
 * both are chosen, their neighbours are marked too, so no later pair can
 * touch or border an earlier one.
 * Draw k of map m is site mulhi(w, N) with w = word (k mod 4) of the Philox
 * counter (m_lo, DOM_MAP, floor(k/4), m_hi).  Writes pairs[2i] = a_i and
 * pairs[2i+1] = b_i; returns the number of draws consumed, or -1 if L < 3. */
int64_t orc_map_build(int32_t L, uint64_t seed, uint64_t m, int64_t *pairs)
{
    if (L < 3) return -1;
    const int64_t N = (int64_t)L * L, n_pairs = orc_map_pairs(L);
    uint8_t *marked = (uint8_t *)calloc((size_t)N, 1);
    if (!marked) return -1;
    uint64_t k = 0;
    uint32_t w[4] = {0, 0, 0, 0};
    for (int64_t i = 0; i < n_pairs; ++i) {
        int64_t site[2];
        for (int h = 0; h < 2; ++h) {
            for (;;) {
                if ((k & 3u) == 0)
                    philox_seeded(seed, (uint32_t)m, DOM_MAP, (uint32_t)(k >> 2), (uint32_t)(m >> 32), w);
                const int64_t cand = (int64_t)mulhi32(w[k & 3u], (uint32_t)N);
                ++k;
                if (!marked[cand]) {
                    marked[cand] = 1;
                    site[h] = cand;
                    break;
                }
            }
        }
        pairs[2 * i] = site[0];
        pairs[2 * i + 1] = site[1];
        for (int h = 0; h < 2; ++h) {
            int64_t nb[4];
            neighbours(L, site[h], nb);
            for (int d = 0; d < 4; ++d) marked[nb[d]] = 1;
        }
    }
    free(marked);
    return (int64_t)k;
}

/* Nearest-neighbour maps: the pairing of the paper's first version (section
 * 3.2), where the partner is a neighbour of the first site.  Pairs per map:
 * max(1, floor(N/20)).  Draws come from the same stream as orc_map_build:
 * a draw gives a = mulhi(w, N); if a is marked the next draw starts over;
 * otherwise the next draw gives the neighbour index d = w >> 30 (order: x+1,
 * x-1, y+1, y-1) and b = neighbour d of a; if b is marked the pair is
 * dropped and the next draw starts over; otherwise a, b and the neighbours
 * of both are marked and (a, b) is recorded.  Every pair marks at most 8
 * sites, so fewer than half the sites are ever marked, which leaves an
 * unmarked neighbour pair for every draw of the map to find. */
int64_t orc_nn_map_pairs(int32_t L)
{
    int64_t n = (int64_t)L * L / 20;
    return n < 1 ? 1 : n;
}

int64_t orc_nn_map_build(int32_t L, uint64_t seed, uint64_t m, int64_t *pairs)
{
    if (L < 3) return -1;
    const int64_t N = (int64_t)L * L, n_pairs = orc_nn_map_pairs(L);
    uint8_t *marked = (uint8_t *)calloc((size_t)N, 1);
    if (!marked) return -1;
    uint64_t k = 0;
    uint32_t w[4] = {0, 0, 0, 0};
    int64_t count = 0;
    while (count < n_pairs) {
        if ((k & 3u) == 0)
            philox_seeded(seed, (uint32_t)m, DOM_MAP, (uint32_t)(k >> 2), (uint32_t)(m >> 32), w);
        const int64_t a = (int64_t)mulhi32(w[k & 3u], (uint32_t)N);
        ++k;
        if (marked[a]) continue;
        if ((k & 3u) == 0)
            philox_seeded(seed, (uint32_t)m, DOM_MAP, (uint32_t)(k >> 2), (uint32_t)(m >> 32), w);
        const uint32_t d = w[k & 3u] >> 30;
        ++k;
        int64_t nb[4];
        neighbours(L, a, nb);
        const int64_t b = nb[d];
        if (marked[b]) continue;
        pairs[2 * count] = a;
        pairs[2 * count + 1] = b;
        ++count;
        marked[a] = 1;
        marked[b] = 1;
        for (int h = 0; h < 2; ++h) {
            int64_t q[4];
            neighbours(L, h ? b : a, q);
            for (int e = 0; e < 4; ++e) marked[q[e]] = 1;
        }
    }
    free(marked);
    return (int64_t)k;
}

/* Map steps start_map .. start_map + n_maps - 1: build each map, then apply
 * one coupled-pair Metropolis step to each of its pairs in map order.  Pair i
 * of map m uses Philox counter (m_lo, DOM_MAPSTEP, floor(i/2), m_hi): words
 * h and h+1 with h = 2*(i mod 2) are the configuration and acceptance draws.
 * The pairs of a map do not interact, so any order gives the same result. */
int orc_map_steps_mode(int32_t L, double Delta, double V, double J, double T, uint64_t seed, int nn,
                       uint64_t start_map, uint64_t n_maps, int8_t *codes, int64_t track[3])
{
    if (L < 3) return -1;
    const int64_t n_pairs = nn ? orc_nn_map_pairs(L) : orc_map_pairs(L);
    int64_t *pairs = (int64_t *)malloc((size_t)(2 * n_pairs) * sizeof(int64_t));
    if (!pairs) return -1;
    for (uint64_t m = start_map; m < start_map + n_maps; ++m) {
        if ((nn ? orc_nn_map_build(L, seed, m, pairs) : orc_map_build(L, seed, m, pairs)) < 0) {
            free(pairs);
            return -1;
        }
        for (int64_t i = 0; i < n_pairs; ++i) {
            uint32_t w[4];
            philox_seeded(seed, (uint32_t)m, DOM_MAPSTEP, (uint32_t)(i >> 1), (uint32_t)(m >> 32), w);
            const int h = 2 * (int)(i & 1);
            pair_step(L, codes, pairs[2 * i], pairs[2 * i + 1], w[h], w[h + 1], Delta, V, J, T, track);
        }
    }
    free(pairs);
    return 0;
}

int orc_map_steps(int32_t L, double Delta, double V, double J, double T, uint64_t seed,
                  uint64_t start_map, uint64_t n_maps, int8_t *codes, int64_t track[3])
{
    return orc_map_steps_mode(L, Delta, V, J, T, seed, 0, start_map, n_maps, codes, track);
}

/* Same for the map mode (nn = 1: nearest-neighbour maps); one observation
 * every `every` maps. */
int orc_map_series(int32_t L, double Delta, double V, double J, double T, uint64_t seed, int nn,
                   uint64_t start_map, uint64_t every, uint64_t n_obs, int8_t *codes,
                   int64_t track[3], int64_t *series)
{
    for (uint64_t k = 0; k < n_obs; ++k) {
        int rc = orc_map_steps_mode(L, Delta, V, J, T, seed, nn, start_map + k * every, every, codes, track);
        if (rc) return rc;
        orc_observables(L, codes, &series[7 * k]);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Penalty mode (section 2.2): the method the paper sets out to replace.  The
 * energy gets the term -mu sum_i S_i, sites are updated one at a time by the
 * classical Metropolis rule (no pairs, so the charge is free to change), and
 * mu is adjusted automatically to steer sum S towards Q.
 *   - a sweep is two half-sweeps over the checkerboard colours c = (x+y) mod 2,
 *     c = 0 first; site (x, y) of colour c has index k = y*(L/2) + floor(x/2);
 *   - site k of colour c in sweep s uses Philox counter (s_lo, 0x600 + c,
 *     floor(k/2), s_hi), words h, h+1 with h = 2*(k mod 2): the new code is
 *     word h >> 30 (one of the 4 codes, the current one included), word h+1
 *     is the acceptance draw;
 *   - dE = Delta nD + V nV + (J/4) nJ - mu dS with the site's changes of S^2,
 *     S * (sum of neighbour S), sigma * (sum of neighbour sigma) and S; the
 *     threshold follows orc_threshold's convention;
 *   - after the sweep, with sum S of the new configuration:
 *     mu = mu + kappa * (Q - sum S) / N (a proportional controller; the paper
 *     says only that mu is adjusted automatically).
 * mu_series[i] / sumS_series[i] (if not null) receive the mu used in sweep
 * start+i and the sum S after it.  track[] accumulates the accepted (nD, nV,
 * nJ) of the physical energy (the penalty term excluded). */
static uint32_t mu_threshold(double Delta, double V, double J, double T, double mu, int nD, int nV, int nJ, int dS)
{
    double dE = Delta * nD + V * nV + 0.25 * J * nJ - mu * dS;
    return threshold_of_dE(dE, T);
}

int orc_mu_sweeps(int32_t L, double Delta, double V, double J, double T, uint64_t seed, uint64_t start_sweep,
                  uint64_t n_sweeps, double kappa, int64_t Q, double *mu, int8_t *codes, int64_t track[3],
                  double *mu_series, int64_t *sumS_series)
{
    if (L < 4 || L % 2 != 0) return -1;
    const int64_t N = (int64_t)L * L, half = L / 2;
    for (uint64_t s = start_sweep; s < start_sweep + n_sweeps; ++s) {
        for (int c = 0; c < 2; ++c) {
            for (int64_t y = 0; y < L; ++y) {
                for (int64_t xh = 0; xh < half; ++xh) {
                    const int64_t x = 2 * xh + ((y + c) & 1);
                    const int64_t k = y * half + xh;
                    uint32_t w[4];
                    philox_seeded(seed, (uint32_t)s, DOM_MU + (uint32_t)c, (uint32_t)(k >> 1), (uint32_t)(s >> 32), w);
                    const int h = 2 * (int)(k & 1);
                    const int64_t i = y * L + x;
                    const int c0 = codes[i], c1 = (int)(w[h] >> 30);
                    int64_t nb[4];
                    neighbours(L, i, nb);
                    int sS = 0, sG = 0;
                    for (int d = 0; d < 4; ++d) {
                        sS += S_OF[codes[nb[d]]];
                        sG += SIG_OF[codes[nb[d]]];
                    }
                    const int dS = S_OF[c1] - S_OF[c0];
                    const int nD = S_OF[c1] * S_OF[c1] - S_OF[c0] * S_OF[c0];
                    const int nV = dS * sS;
                    const int nJ = (SIG_OF[c1] - SIG_OF[c0]) * sG;
                    const uint32_t thr = mu_threshold(Delta, V, J, T, *mu, nD, nV, nJ, dS);
                    if (thr == 0xFFFFFFFFu || w[h + 1] < thr) {
                        codes[i] = (int8_t)c1;
                        track[0] += nD;
                        track[1] += nV;
                        track[2] += nJ;
                    }
                }
            }
        }
        int64_t sumS = 0;
        for (int64_t i = 0; i < N; ++i) sumS += S_OF[codes[i]];
        if (mu_series) mu_series[s - start_sweep] = *mu;
        if (sumS_series) sumS_series[s - start_sweep] = sumS;
        *mu = *mu + kappa * (double)(Q - sumS) / (double)N;
    }
    return 0;
}

/* Same for the general mode; one observation every `every` single-pair steps. */
int orc_general_series(int32_t L, double Delta, double V, double J, double T, uint64_t seed,
                       uint64_t start_step, uint64_t every, uint64_t n_obs, int8_t *codes,
                       int64_t track[3], int64_t *series)
{
    for (uint64_t k = 0; k < n_obs; ++k) {
        int rc = orc_general_steps(L, Delta, V, J, T, seed, start_step + k * every, every, codes, track);
        if (rc) return rc;
        orc_observables(L, codes, &series[7 * k]);
    }
    return 0;
}
