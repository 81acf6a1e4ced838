"""Pins of the oracle's map mode (section 3.2, random maps of non-interacting
coupled pairs), CPU only.

* Construction, by brute force over small lattices: max(1, N//10) pairs, all
  sites distinct, and no site of one pair equal or adjacent to a site of
  another pair (the property that lets a map's pairs run concurrently).
* The printed algorithm marks a pair's neighbours only after both sites are
  drawn, so a partner may neighbour the first site: on 4x4 (one pair per map)
  the first site is uniform and the partner is adjacent with probability 4/15.
* The chain a map sequence drives samples the Boltzmann distribution of the
  fixed-charge sector: exact enumeration on 3x3 and 4x4, Onsager's energy in
  the Delta -> infinity, n = 0 limit on 32x32 (102 pairs per map).
* Invariants: the charge never changes and the tracked energy triple equals
  the change of the recomputed one.
"""
import math

import numpy as np
import pytest

import oracle
from tests import exact
from tests.mcstats import block_heat_capacity, block_mean
from tests.test_oracle_stats import _check, _energies, onsager_energy_per_site


def _neighbours(L, i):
    x, y = i % L, i // L
    return {y * L + (x + 1) % L, y * L + (x - 1) % L, ((y + 1) % L) * L + x, ((y - 1) % L) * L + x}


@pytest.mark.parametrize("L", [3, 4, 5, 7, 8, 10, 16, 33])
def test_map_pairs_never_interact(L):
    N = L * L
    for m in (0, 1, 17):
        pairs, draws = oracle.map_build(L, 11, m)
        assert len(pairs) == max(1, N // 10)
        sites = pairs.reshape(-1).tolist()
        assert len(set(sites)) == len(sites), "a site appears twice in a map"
        assert all(0 <= s < N for s in sites)
        assert draws >= len(sites)
        cover = [{a, b} | _neighbours(L, a) | _neighbours(L, b) for a, b in pairs.tolist()]
        for j, (a, b) in enumerate(pairs.tolist()):
            for i in range(j):
                assert a not in cover[i] and b not in cover[i], f"pairs {i} and {j} of map {m} interact"


def test_map_first_site_uniform_and_partner_may_be_adjacent():
    L, N, n = 4, 16, 6000
    first = np.zeros(N, dtype=np.int64)
    adjacent = 0
    for m in range(n):
        (a, b), = oracle.map_build(L, 3, m)[0].tolist()
        assert a != b
        first[a] += 1
        adjacent += b in _neighbours(L, a)
    chi2 = float(((first - n / N) ** 2 / (n / N)).sum())
    assert chi2 < 50.0, f"first site not uniform (chi2 = {chi2:.1f}, 15 dof)"
    p = 4 / 15
    z = (adjacent / n - p) / math.sqrt(p * (1 - p) / n)
    assert abs(z) < 4, f"adjacent-partner rate {adjacent / n:.4f} vs 4/15 (z = {z:.2f})"


def test_map_steps_keep_charge_and_track_energy():
    L, n, Delta, V, J, T = 12, 0.1, 0.25, 0.5, 1.0, 0.9
    Q, Nc = oracle.charge_target(L, n)
    codes = oracle.init_codes(L, 5, (Nc + Q) // 2, (Nc - Q) // 2)
    o0 = oracle.observables(L, codes)
    track = np.zeros(3, dtype=np.int64)
    for k in range(20):
        oracle.map_steps(L, Delta, V, J, T, 5, codes, 3, start_map=3 * k, track=track)
        o = oracle.observables(L, codes)
        assert o[0] == Q
        assert track.tolist() == [o[1] - o0[1], o[2] - o0[2], o[3] - o0[3]]
    assert track.any(), "no move was ever accepted"


@pytest.mark.parametrize("L,Q,T", [(3, 1, 1.5), (3, 0, 0.8), (4, 2, 1.0), (4, 0, 0.5)])
def test_map_mode_matches_exact_enumeration(L, Q, T):
    N = L * L
    Delta, V, J = 0.25, 0.5, 1.0
    codes = np.zeros(N, dtype=np.int8)
    codes[:Q] = 2  # Q positive charges, the rest spin-up
    ser, _ = oracle.map_series(L, Delta, V, J, T, seed=41 + Q + L, codes=codes, every=5, n_obs=240000)
    assert np.all(ser[:, 0] == Q)
    ser = ser[20000:]
    ex = exact.sector_averages(L, Q, Delta, V, J, T)
    E = _energies(ser, Delta, V, J)
    _check("E", *block_mean(E), ex["E"])
    _check("Nc", *block_mean(ser[:, 1]), ex["Nc"])
    _check("BJ", *block_mean(ser[:, 3]), ex["BJ"])
    _check("C", *block_heat_capacity(E, N, T), ex["C"])


@pytest.mark.parametrize("T", [0.45, 1.0])
def test_map_mode_infinite_delta_reduces_to_onsager(T):
    L, J = 32, 1.0
    Tc = 2 * 0.25 * J / math.log(1 + math.sqrt(2))
    if T < Tc:
        x, y = np.meshgrid(np.arange(L), np.arange(L))
        codes = ((x + y) % 2).astype(np.int8).reshape(-1)  # Neel state: sigma = (-1)^(x+y)
    else:
        codes = (np.arange(L * L) % 2).astype(np.int8)
    ser, _ = oracle.map_series(L, 1e6, 0.5, J, T, seed=9, codes=codes, every=5, n_obs=7000)
    ser = ser[1000:]
    assert np.all(ser[:, 1] == 0)
    u = 0.25 * J * ser[:, 3] / (L * L)
    _check("u", *block_mean(u, n_blocks=25), onsager_energy_per_site(T, 0.25 * J))


# ---------------------------------------------------------------- nearest-neighbour maps
@pytest.mark.parametrize("L", [3, 4, 5, 8, 10, 16, 33])
def test_nn_map_pairs_are_adjacent_and_never_interact(L):
    N = L * L
    for m in (0, 3):
        pairs, draws = oracle.map_build(L, 13, m, nn=True)
        assert len(pairs) == max(1, N // 20)
        sites = pairs.reshape(-1).tolist()
        assert len(set(sites)) == len(sites)
        cover = [{a, b} | _neighbours(L, a) | _neighbours(L, b) for a, b in pairs.tolist()]
        for j, (a, b) in enumerate(pairs.tolist()):
            assert b in _neighbours(L, a), f"pair {j} of map {m} is not a neighbour pair"
            for i in range(j):
                assert a not in cover[i] and b not in cover[i]


def test_nn_map_first_site_and_direction_uniform():
    L, N, n = 4, 16, 6000
    first = np.zeros(N, dtype=np.int64)
    direction = np.zeros(4, dtype=np.int64)
    for m in range(n):
        (a, b), = oracle.map_build(L, 5, m, nn=True)[0].tolist()
        first[a] += 1
        x, y = a % L, a // L
        direction[[y * L + (x + 1) % L, y * L + (x - 1) % L, ((y + 1) % L) * L + x, ((y - 1) % L) * L + x].index(b)] += 1
    assert float(((first - n / N) ** 2 / (n / N)).sum()) < 50.0
    assert float(((direction - n / 4) ** 2 / (n / 4)).sum()) < 25.0


def _series_energy(L, Delta, V, J, T, Q, nn, seed, n_obs):
    N = L * L
    codes = np.zeros(N, dtype=np.int8)
    codes[:Q] = 2
    ser, _ = oracle.map_series(L, Delta, V, J, T, seed=seed, codes=codes, every=2, n_obs=n_obs, nn=nn)
    ser = ser[10000:]
    return _energies(ser, Delta, V, J)


def test_nn_maps_match_exact_where_they_mix():
    # weak charge repulsion: nearest-neighbour pairs still sample the sector
    L, N, Q, T = 4, 16, 2, 1.0
    Delta, V, J = 0.25, 0.5, 1.0
    E = _series_energy(L, Delta, V, J, T, Q, True, 5, 150000)
    ex = exact.sector_averages(L, Q, Delta, V, J, T)
    _check("E", *block_mean(E), ex["E"])
    _check("C", *block_heat_capacity(E, N, T), ex["C"])


def test_nn_maps_lose_the_low_temperature_states_random_pairs_reach():
    """Section 3.2: with partners restricted to nearest neighbours the 4x4
    low-temperature results miss the exact ones -- the chain freezes and the
    heat capacity loses its structure -- while long-range random pairs
    reproduce them.  Strong charge repulsion (V = 2) at T = 0.3, Q = 4."""
    L, N, Q, T = 4, 16, 4, 0.3
    Delta, V, J = 0.25, 2.0, 1.0
    ex = exact.sector_averages(L, Q, Delta, V, J, T)
    E_rand = _series_energy(L, Delta, V, J, T, Q, False, 5, 100000)
    _check("E random pairs", *block_mean(E_rand), ex["E"])
    _check("C random pairs", *block_heat_capacity(E_rand, N, T), ex["C"])
    E_nn = _series_energy(L, Delta, V, J, T, Q, True, 5, 100000)
    C_nn, _ = block_heat_capacity(E_nn, N, T)
    assert C_nn < 0.25 * ex["C"], f"nearest-neighbour pairs kept the fluctuations: C = {C_nn:.4f} vs {ex['C']:.4f}"
