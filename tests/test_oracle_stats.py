"""Statistical pins of the oracle's Markov chain against exact results (CPU).

* 3x3, general mode (one random pair per step, adjacent pairs included):
  Boltzmann averages from exact enumeration of all 4^9 states.
* 4x4, the structured sublattice schedule the GPU runs: exact enumeration of
  all 4^16 states (the lattice size the paper checks against, section 3.3).
* V = J = 0: closed-form sector partition function (free charges).
* Delta -> infinity, n = 0: the 2D Ising model with J_eff = J/4, Onsager's
  exact internal energy.
Seeds are fixed, so every pass/fail is reproducible; the bar is |z| < 4 with
block-averaged error bars.
"""
import math

import numpy as np
import pytest
from scipy.special import ellipk, gammaln

import oracle
from tests import exact
from tests.mcstats import block_heat_capacity, block_mean, zscore

Z_MAX = 4.0


def _check(name, est, err, ref):
    z = zscore(est, err, ref)
    assert abs(z) < Z_MAX, f"{name}: MC {est:.6f} +- {err:.6f} vs exact {ref:.6f} (z={z:.2f})"


def _energies(series, Delta, V, J):
    return Delta * series[:, 1] + V * series[:, 2] + 0.25 * J * series[:, 3]


# ---------------------------------------------------------------- 3x3 general mode
@pytest.mark.parametrize("Q,T", [(1, 0.5), (1, 1.5), (0, 0.8), (3, 1.0)])
def test_general_mode_3x3_matches_exact_enumeration(Q, T):
    L, N = 3, 9
    Delta, V, J = 0.25, 0.5, 1.0
    codes = np.zeros(N, dtype=np.int8)
    codes[:Q] = 2  # Q positive charges, the rest spin-up
    ser, _ = oracle.general_series(L, Delta, V, J, T, seed=31 + Q, codes=codes, every=5, n_obs=300000)
    assert np.all(ser[:, 0] == Q)
    ser = ser[20000:]
    ex = exact.sector_averages(L, Q, Delta, V, J, T)
    E = _energies(ser, Delta, V, J)
    _check("E", *block_mean(E), ex["E"])
    _check("Nc", *block_mean(ser[:, 1]), ex["Nc"])
    _check("BJ", *block_mean(ser[:, 3]), ex["BJ"])
    _check("C", *block_heat_capacity(E, N, T), ex["C"])


# ---------------------------------------------------------------- 4x4 structured schedule
# T >= 0.3 at n = 0: below that the chain sits in the charge-checkerboard ground
# state for the whole run and no finite sample resolves the exact average.
@pytest.mark.parametrize("n,T", [(0.0, 0.3), (0.0, 0.5), (0.125, 0.25), (0.125, 1.0), (0.25, 0.35), (0.25, 2.0)])
def test_structured_chain_4x4_matches_exact_enumeration(n, T):
    L, N = 4, 16
    Delta, V, J = 0.25, 0.5, 1.0
    lat = oracle.OracleLattice(L, n, Delta, V, J, T, seed=int(1000 * T) + int(100 * n))
    ser = lat.series(every=1, n_obs=300000)
    assert np.all(ser[:, 0] == lat.Q)
    ser = ser[10000:]
    ex = exact.sector_averages(L, lat.Q, Delta, V, J, T)
    E = _energies(ser, Delta, V, J)
    _check("E", *block_mean(E), ex["E"])
    _check("Nc", *block_mean(ser[:, 1]), ex["Nc"])
    _check("BV", *block_mean(ser[:, 2]), ex["BV"])
    _check("BJ", *block_mean(ser[:, 3]), ex["BJ"])
    _check("C", *block_heat_capacity(E, N, T), ex["C"])


def test_exact_enumeration_counts():
    """Sector sizes of the enumerations against the multinomial count
    sum_k N!/(N+! N-! N0!) 2^N0 over N+ - N- = Q."""
    for L in (3, 4):
        N = L * L
        g = exact.density_of_states(L)
        assert g.sum() == 4 ** N
        for Q in range(-N, N + 1):
            count = 0
            for n_minus in range(0, N + 1):
                n_plus = n_minus + Q
                n0 = N - n_plus - n_minus
                if n_plus < 0 or n0 < 0:
                    continue
                count += math.factorial(N) // (math.factorial(n_plus) * math.factorial(n_minus)
                                               * math.factorial(n0)) * 2 ** n0
            assert g[Q + N].sum() == count


# ---------------------------------------------------------------- V = J = 0 closed form
def _free_charge_exact(N, Q, Delta, T):
    """Z_Q = sum over N+ - N- = Q of N!/(N+! N-! N0!) 2^N0 exp(-Delta (N+ + N-)/T)."""
    logw, ncs = [], []
    for n_minus in range(0, N + 1):
        n_plus = n_minus + Q
        n0 = N - n_plus - n_minus
        if n_plus < 0 or n0 < 0:
            continue
        nc = n_plus + n_minus
        lw = (gammaln(N + 1) - gammaln(n_plus + 1) - gammaln(n_minus + 1) - gammaln(n0 + 1)
              + n0 * math.log(2.0) - Delta * nc / T)
        logw.append(lw)
        ncs.append(nc)
    logw, ncs = np.array(logw), np.array(ncs, dtype=np.float64)
    w = np.exp(logw - logw.max())
    w /= w.sum()
    mean = float((w * ncs).sum())
    var = float((w * ncs * ncs).sum() - mean * mean)
    return mean, var


@pytest.mark.parametrize("Delta,n", [(0.5, 0.1), (-0.3, 0.0), (0.0, 0.2)])
def test_free_charges_match_closed_form(Delta, n):
    L, T = 16, 1.0
    lat = oracle.OracleLattice(L, n, Delta, 0.0, 0.0, T, seed=77)
    ser = lat.series(every=1, n_obs=40000)[2000:]
    mean, var = _free_charge_exact(L * L, lat.Q, Delta, T)
    _check("Nc", *block_mean(ser[:, 1]), mean)
    _check("var Nc", *block_heat_capacity(ser[:, 1], 1, 1.0), var)


# ---------------------------------------------------------------- Onsager limit
def onsager_energy_per_site(T, Jeff):
    """Internal energy per site of the square-lattice Ising model (Onsager 1944)."""
    b = 2.0 * Jeff / T
    kappa = 2.0 * math.sinh(b) / math.cosh(b) ** 2
    K = ellipk(kappa * kappa)
    return -Jeff / math.tanh(b) * (1.0 + (2.0 / math.pi) * (2.0 * math.tanh(b) ** 2 - 1.0) * K)


def test_onsager_closed_form_values():
    # T_c = 2 J_eff / ln(1 + sqrt 2) with J_eff = 1/4; energy at T_c is -sqrt(2) J_eff
    Tc = 2 * 0.25 / math.log(1 + math.sqrt(2))
    assert abs(Tc - 0.567296) < 1e-6
    assert abs(onsager_energy_per_site(Tc * (1 + 1e-5), 0.25) + math.sqrt(2) * 0.25) < 1e-3
    assert abs(onsager_energy_per_site(0.05, 0.25) + 0.5) < 1e-9  # ground state: 2 bonds per site


@pytest.mark.parametrize("T", [0.3, 0.45, 0.8, 1.0])
def test_infinite_delta_reduces_to_onsager(T):
    L, J = 64, 1.0
    Tc = 2 * 0.25 * J / math.log(1 + math.sqrt(2))
    codes = None
    if T < Tc:
        # Start ordered: a quench from random spins leaves metastable stripe
        # domains on the torus that a finite run at T << Tc does not anneal.
        x, y = np.meshgrid(np.arange(L), np.arange(L))
        codes = ((x + y) % 2).astype(np.int8).reshape(-1)  # Neel state: sigma = (-1)^(x+y)
    lat = oracle.OracleLattice(L, 0.0, 1e6, 0.5, J, T, seed=5, n_charged=0, codes=codes)
    ser = lat.series(every=1, n_obs=6000)[1000:]
    assert np.all(ser[:, 1] == 0)
    u = 0.25 * J * ser[:, 3] / (L * L)
    _check("u", *block_mean(u, n_blocks=25), onsager_energy_per_site(T, 0.25 * J))
