"""Pins of the oracle's model pieces: pair sets, charge target, energy change,
schedule, init and the exact invariants (CPU only)."""
import itertools
import math

import numpy as np
import pytest

import oracle

S_OF = {0: 0, 1: 0, 2: 1, 3: -1}
SIG_OF = {0: 1, 1: -1, 2: 0, 3: 0}


# ---------------------------------------------------------------- pair sets
def _code(state):
    """Paper notation -> code: +1/-1 are charges, +0.5/-0.5 are spins."""
    return {1: 2, -1: 3, 0.5: 0, -0.5: 1}[state]


# The listing of section 3.1 ("Algorithm"), state by state.
PAPER_SETS = {
    1: [(1, 0.5), (1, -0.5), (0.5, 1), (-0.5, 1)],
    0: [(1, -1), (-1, 1), (0.5, 0.5), (-0.5, -0.5), (0.5, -0.5), (-0.5, 0.5)],
    -1: [(-1, 0.5), (-1, -0.5), (0.5, -1), (-0.5, -1)],
}


def test_pair_sets_follow_the_paper_listing():
    for q, listing in PAPER_SETS.items():
        got = [oracle.pair_config(q, j) for j in range(len(listing))]
        assert got == [(_code(a), _code(b)) for a, b in listing]
        assert oracle.pair_config(q, len(listing)) is None
    assert oracle.pair_config(2, 0) is None and oracle.pair_config(-2, 0) is None


def test_pair_sets_partition_all_sixteen_two_site_states():
    seen = []
    for q in (1, 0, -1):
        j = 0
        while (cfg := oracle.pair_config(q, j)) is not None:
            assert S_OF[cfg[0]] + S_OF[cfg[1]] == q
            seen.append(cfg)
            j += 1
    seen += [(2, 2), (3, 3)]  # q = +-2, frozen
    assert sorted(seen) == sorted(itertools.product(range(4), repeat=2))
    assert [sum(1 for c in seen if S_OF[c[0]] + S_OF[c[1]] == q) for q in (2, 1, 0, -1, -2)] == [1, 4, 6, 4, 1]


# ---------------------------------------------------------------- charge target (eq. 2)
@pytest.mark.parametrize("L,n,Q,Nc", [
    (32, 0.1, 102, 256),            # 256 charged, N+ - N- = 102
    (1024, 0.05, 52428, 262144),
    (8192, 0.1, 6710886, 16777216),
    (128, 0.0, 0, 4096),
    (128, 0.05, 820, 4096),
    (128, 0.30, 4916, 4916),        # |Q| above N/4: every charge positive
    (128, 0.35, 5734, 5734),
    (4, 0.125, 2, 4),
    (4, -0.125, -2, 4),
    (4, 0.0625, 0, 4),              # nN = 1 halfway between 0 and 2: ties go to the smaller
])
def test_charge_target(L, n, Q, Nc):
    assert oracle.charge_target(L, n) == (Q, Nc)


def test_charge_target_parity_and_nearest():
    rng = np.random.default_rng(3)
    for _ in range(500):
        L = int(rng.choice([4, 8, 12, 32, 64]))
        n = float(rng.uniform(-0.6, 0.6))
        Q, Nc = oracle.charge_target(L, n)
        N = L * L
        assert (Q - Nc) % 2 == 0 and abs(Q) <= Nc <= N
        # no integer of Nc's parity lies closer to nN
        assert abs(Q - n * N) <= 1.0 + 1e-9
    with pytest.raises(ValueError):
        oracle.charge_target(4, 2.0)
    with pytest.raises(ValueError):
        oracle.charge_target(8, 0.5, n_charged=4)  # |Q| = 32 > 4 requested charges


# ---------------------------------------------------------------- thresholds
def test_threshold_always_for_downhill_and_monotone_uphill():
    assert oracle.threshold(0.25, 0.5, 1.0, 0.8, 0, 0, 0) == 0xFFFFFFFF
    assert oracle.threshold(0.25, 0.5, 1.0, 0.8, -2, 0, 0) == 0xFFFFFFFF
    vals = [oracle.threshold(0.0, 1.0, 0.0, 1.0, 0, nV, 0) for nV in range(1, 17)]
    assert all(a > b for a, b in zip(vals, vals[1:]))
    # dE = 1 at T = 1: e^-1 * 2^32 = 1580030168.96...
    assert oracle.threshold(0.0, 1.0, 0.0, 1.0, 0, 1, 0) == 1580030168
    # the huge-Delta representation of a forbidden move never passes
    assert oracle.threshold(1e6, 0.5, 1.0, 2.5, 2, 0, 0) == 0


# ---------------------------------------------------------------- energy change vs eq. (3)
def _random_codes(rng, L, p_charge=0.4):
    c = rng.integers(0, 2, size=L * L).astype(np.int8)
    ch = rng.random(L * L) < p_charge
    c[ch] = rng.integers(2, 4, size=int(ch.sum()))
    return c


def _nbr_sums(L, c, i):
    x, y = i % L, i // L
    nb = [y * L + (x + 1) % L, y * L + (x - 1) % L, ((y + 1) % L) * L + x, ((y - 1) % L) * L + x]
    return sum(S_OF[int(c[j])] for j in nb), sum(SIG_OF[int(c[j])] for j in nb), nb


@pytest.mark.parametrize("L", [3, 4, 5, 8])
def test_pair_delta_equals_full_energy_difference(L):
    """Brute force: the local triple equals the change of the whole-lattice sums."""
    rng = np.random.default_rng(100 + L)
    for _ in range(300):
        c = _random_codes(rng, L)
        a, b = rng.choice(L * L, size=2, replace=False)
        ca1, cb1 = rng.integers(0, 4, size=2)
        d = oracle.pair_delta(L, c, int(a), int(b), int(ca1), int(cb1))
        o0 = oracle.observables(L, c)
        c2 = c.copy()
        c2[a], c2[b] = ca1, cb1
        o1 = oracle.observables(L, c2)
        assert list(d) == [o1[1] - o0[1], o1[2] - o0[2], o1[3] - o0[3]]


def test_pair_delta_matches_the_papers_pair_formulas():
    """Section 3.1: E_Delta, E_V for distant pairs; the adjacent-pair corrections
    -(S_a1-S_a0)^2 for V and +(sig_a1-sig_a0)(sig_b1-sig_b0) for J.  E_J is
    written in its general form dsig_a*sum<a> + dsig_b*sum<b>; the printed
    single-difference form is checked only where it coincides with that."""
    rng = np.random.default_rng(7)
    L = 6
    n_adjacent = n_distant = n_printed_form_differs = 0
    for _ in range(3000):
        c = _random_codes(rng, L)
        a = int(rng.integers(L * L))
        if rng.random() < 0.5:
            _, _, nb = _nbr_sums(L, c, a)
            b = int(nb[rng.integers(4)])
        else:
            b = int(rng.integers(L * L))
            if b == a:
                continue
        q = S_OF[int(c[a])] + S_OF[int(c[b])]
        if abs(q) == 2:
            continue
        k = 6 if q == 0 else 4
        ca1, cb1 = oracle.pair_config(q, int(rng.integers(k)))
        Sa0, Sb0, Sa1, Sb1 = S_OF[int(c[a])], S_OF[int(c[b])], S_OF[ca1], S_OF[cb1]
        sa0, sb0, sa1, sb1 = SIG_OF[int(c[a])], SIG_OF[int(c[b])], SIG_OF[ca1], SIG_OF[cb1]
        sumSa, sumsa, nba = _nbr_sums(L, c, a)
        sumSb, sumsb, _ = _nbr_sums(L, c, b)
        E_D = Sa1**2 + Sb1**2 - Sa0**2 - Sb0**2
        E_V = (Sa1 - Sa0) * (sumSa - sumSb)
        E_J = (sa1 - sa0) * sumsa + (sb1 - sb0) * sumsb
        if b in nba:
            n_adjacent += 1
            E_V -= (Sa1 - Sa0) ** 2
            E_J += (sa1 - sa0) * (sb1 - sb0)
        else:
            n_distant += 1
            printed = (sa1 - sa0) * (sumsa - sumsb)
            if printed != E_J:
                n_printed_form_differs += 1
                assert (sb1 - sb0) != -(sa1 - sa0)
        d = oracle.pair_delta(L, c, a, b, ca1, cb1)
        assert list(d) == [E_D, E_V, E_J]
    assert n_adjacent > 500 and n_distant > 500 and n_printed_form_differs > 0


# ---------------------------------------------------------------- schedule
def _phase_sites(L, Dx, Dy, p):
    a_sites, b_sites = [], []
    for y in range(0, L, 2):
        for x in range(p, L, 4):
            a_sites.append(y * L + x)
            b_sites.append(((y + Dy) % L) * L + (x + Dx) % L)
    return a_sites, b_sites


def _adjacent(L, i, j):
    xi, yi, xj, yj = i % L, i // L, j % L, j // L
    dx, dy = min((xi - xj) % L, (xj - xi) % L), min((yi - yj) % L, (yj - yi) % L)
    return dx + dy == 1


@pytest.mark.parametrize("L", [4, 8, 12, 16, 20])
def test_schedule_covers_each_site_once_and_pairs_never_interact(L):
    for s in range(40):
        r, Dx, Dy = oracle.schedule(L, 5, s)
        assert r in (1, 2, 3)
        assert all(d % 4 == r % 4 for d in Dx) and all(d % 2 == 1 for d in Dy)
        covered = []
        for p in range(4):
            A, B = _phase_sites(L, Dx[p], Dy[p], p)
            updated = A + B
            assert len(set(updated)) == len(updated) == L * L // 4
            us = set(updated)
            for i in updated:
                x, y = i % L, i // L
                for nb in (y * L + (x + 1) % L, y * L + (x - 1) % L, ((y + 1) % L) * L + x, ((y - 1) % L) * L + x):
                    assert nb not in us, "an updated site neighbours another updated site"
            covered += updated
        assert sorted(covered) == list(range(L * L))


@pytest.mark.parametrize("L", [4, 8, 16, 64])
def test_schedule_displacements_generate_the_whole_torus(L):
    gens = set()
    for s in range(60):
        _, Dx, Dy = oracle.schedule(L, 9, s)
        gens.update(zip(Dx.tolist(), Dy.tolist()))
    reach, frontier = {(0, 0)}, [(0, 0)]
    while frontier:
        x, y = frontier.pop()
        for gx, gy in gens:
            for sgn in (1, -1):
                n = ((x + sgn * gx) % L, (y + sgn * gy) % L)
                if n not in reach:
                    reach.add(n)
                    frontier.append(n)
    assert len(reach) == L * L


def test_schedule_draws_are_spread():
    L = 64
    rs, mx, ky = [], [], []
    for s in range(3000):
        r, Dx, Dy = oracle.schedule(L, 1, s)
        rs.append(r)
        mx += [(d - r) // 4 for d in Dx]
        ky += [(d - 1) // 2 for d in Dy]
    counts = np.bincount(rs, minlength=4)[1:]
    assert np.all(np.abs(counts - 1000) < 5 * math.sqrt(1000 * 2 / 3 * 1 / 3) * 1.0 + 1)
    assert set(mx) == set(range(L // 4)) and set(ky) == set(range(L // 2))


# ---------------------------------------------------------------- init (stage 1 of section 3.1)
@pytest.mark.parametrize("L,n", [(4, 0.125), (32, 0.1), (64, -0.2), (128, 0.35)])
def test_init_has_exact_counts(L, n):
    Q, Nc = oracle.charge_target(L, n)
    codes = oracle.init_codes(L, 17, (Nc + Q) // 2, (Nc - Q) // 2)
    assert np.sum(codes == 2) == (Nc + Q) // 2
    assert np.sum(codes == 3) == (Nc - Q) // 2
    o = oracle.observables(L, codes)
    assert o[0] == Q and o[1] == Nc


def test_init_positions_are_uniform():
    L, trials = 16, 400
    hits = np.zeros(L * L)
    for seed in range(trials):
        codes = oracle.init_codes(L, seed, 20, 12)
        hits += codes >= 2
    expected = trials * 32 / (L * L)
    chi2 = np.sum((hits - expected) ** 2 / expected)
    dof = L * L - 1
    assert abs(chi2 - dof) < 6 * math.sqrt(2 * dof)


# ---------------------------------------------------------------- exact invariants
@pytest.mark.parametrize("L,n,Delta,V,J,T", [
    (8, 0.1, 0.25, 0.5, 1.0, 0.8),
    (12, -0.2, -1.0, 0.7, 1.0, 0.3),
    (32, 0.1, 0.25, 0.5, 1.0, 0.8),
    (16, 0.0, 0.0, 0.0, 0.0, 1.0),
])
def test_charge_exact_and_tracker_equals_recomputed_energy(L, n, Delta, V, J, T):
    lat = oracle.OracleLattice(L, n, Delta, V, J, T, seed=4)
    o0 = lat.observables()
    for _ in range(50):
        lat.sweeps(1)
        o = lat.observables()
        assert o[0] == lat.Q
        assert list(lat.track) == [o[1] - o0[1], o[2] - o0[2], o[3] - o0[3]]


def test_resume_is_bit_exact():
    a = oracle.OracleLattice(16, 0.1, 0.25, 0.5, 1.0, 0.8, seed=21)
    a.sweeps(60)
    b = oracle.OracleLattice(16, 0.1, 0.25, 0.5, 1.0, 0.8, seed=21)
    b.sweeps(25)
    c = oracle.OracleLattice(16, 0.1, 0.25, 0.5, 1.0, 0.8, seed=21, start_sweep=25, codes=b.codes)
    c.sweeps(35)
    assert np.array_equal(a.codes, c.codes)


# ---------------------------------------------------------------- observables of known configurations
def test_observables_of_known_configurations():
    """Closed forms: the charge checkerboard, the spin Neel state, uniform
    states and stripes (every bond counted once, 2N bonds)."""
    L = 8
    N = L * L
    x, y = np.meshgrid(np.arange(L), np.arange(L))
    par = ((x + y) % 2).reshape(-1)
    checker = np.where(par == 0, 2, 3).astype(np.int8)      # +1 on even sites, -1 on odd
    assert oracle.observables(L, checker).tolist() == [0, N, -2 * N, 0, 0, 0, N]
    neel = par.astype(np.int8)                                # sigma = +1 on even, -1 on odd
    assert oracle.observables(L, neel).tolist() == [0, 0, 0, -2 * N, 0, N, 0]
    up = np.zeros(N, dtype=np.int8)
    assert oracle.observables(L, up).tolist() == [0, 0, 0, 2 * N, N, 0, 0]
    plus = np.full(N, 2, dtype=np.int8)
    assert oracle.observables(L, plus).tolist() == [N, N, 2 * N, 0, 0, 0, 0]
    stripes = np.where(y.reshape(-1) % 2 == 0, 0, 1).astype(np.int8)  # rows alternate spin up/down
    # horizontal bonds aligned (+N), vertical anti-aligned (-N); staggered sum over a row is 0
    assert oracle.observables(L, stripes).tolist() == [0, 0, 0, 0, 0, 0, 0]
    one = np.zeros(N, dtype=np.int8)
    one[3 * L + 5] = 3                                        # one -1 charge at (5,3) in spin-up sea
    o = oracle.observables(L, one)
    assert o[0] == -1 and o[1] == 1 and o[2] == 0 and o[3] == 2 * N - 4 and o[4] == N - 1
    # site (5,3) has x+y even: the staggered spin sum (0 before) loses +1; the staggered charge is -1
    assert o[5] == -1 and o[6] == -1


# ---------------------------------------------------------------- energy of eq. (3)
@pytest.mark.parametrize("Delta,V,J", [(0.25, 0.75, 1.5), (-1.25, 0.5, -3.0), (2.0, -0.375, 0.5)])
def test_energy_of_known_configurations(Delta, V, J):
    """E = Delta sum S^2 + V sum_bonds S S + (J/4) sum_bonds sigma sigma
    (eq. 3, 2N bonds) in closed form for configurations whose bond sums are
    known by counting: the charge checkerboard (every bond +-), all sites +1,
    the spin Neel state, all spins up, and the Neel state with one site made
    a charge (its four bonds drop out of the spin sum).  Dyadic couplings keep
    every value exact in FP64."""
    L = 8
    N = L * L
    x, y = np.meshgrid(np.arange(L), np.arange(L))
    par = ((x + y) % 2).reshape(-1)
    cases = {
        "checkerboard": (np.where(par == 0, 2, 3), Delta * N - 2 * V * N),
        "all +1": (np.full(N, 2), Delta * N + 2 * V * N),
        "neel": (par, -(J / 4) * 2 * N),
        "all up": (np.zeros(N), (J / 4) * 2 * N),
    }
    defect = par.copy()
    defect[2 * L + 3] = 2
    cases["neel + one charge"] = (defect, Delta + (J / 4) * (-2 * N + 4))
    for name, (codes, E) in cases.items():
        codes = np.ascontiguousarray(codes, dtype=np.int8)
        assert oracle.energy(Delta, V, J, oracle.observables(L, codes)) == E, name
