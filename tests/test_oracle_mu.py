"""Pins of the oracle's penalty mode (section 2.2: the prior method, with
-mu sum S in the energy, single-site checkerboard Metropolis and mu adjusted
between sweeps), CPU only.

* With the controller off (kappa = 0) the chain samples the grand-canonical
  ensemble at fixed mu: exact averages over all charge sectors of the 4x4
  density of states, weighted by exp(-(E - mu Q)/T).
* With the controller on, the charge averages to its target.
* The paper's objection reproduces: under the controller the energy keeps
  fluctuating as T -> 0, so the heat capacity grows as T falls, while the
  exact heat capacity of the fixed-charge sector vanishes.
* The tracked energy triple equals the change of the recomputed one.
"""
import numpy as np
import pytest

import oracle
from tests import exact
from tests.mcstats import block_heat_capacity, block_mean
from tests.test_oracle_stats import _check

L, N = 4, 16


def _grand_canonical(Delta, V, J, T, mu):
    g = exact.density_of_states(L).astype(np.float64)  # [Q+N, Nc, BV+2N, BJ+2N]
    q = (np.arange(2 * N + 1) - N)[:, None, None, None]
    nc = np.arange(N + 1)[None, :, None, None]
    bv = (np.arange(4 * N + 1) - 2 * N)[None, None, :, None]
    bj = (np.arange(4 * N + 1) - 2 * N)[None, None, None, :]
    E = Delta * nc + V * bv + 0.25 * J * bj
    mask = g > 0
    logw = np.where(mask, np.log(np.where(mask, g, 1.0)) - (E - mu * q) / T, -np.inf)
    w = np.exp(logw - logw[mask].max())
    Z = w.sum()
    avg = lambda X: float((w * X).sum() / Z)  # noqa: E731
    return {"E": avg(E), "C": (avg(E * E) - avg(E) ** 2) / (N * T * T), "Q": avg(q * np.ones_like(E)),
            "Nc": avg(nc * np.ones_like(E))}


def _run(Delta, V, J, T, kappa, Q, mu0, sweeps, seed=3, burn=2000):
    codes = oracle.init_codes(L, seed, 2, 2)
    mu = mu0
    track = np.zeros(3, dtype=np.int64)
    E, S, Nc = [], [], []
    for s in range(burn + sweeps):
        mu, _, _, _ = oracle.mu_sweeps(L, Delta, V, J, T, seed, codes, 1, kappa, Q, mu, start_sweep=s, track=track)
        if s >= burn:
            o = oracle.observables(L, codes)
            E.append(Delta * o[1] + V * o[2] + 0.25 * J * o[3])
            S.append(o[0])
            Nc.append(o[1])
    return np.asarray(E), np.asarray(S), np.asarray(Nc), mu


@pytest.mark.parametrize("mu,T", [(0.3, 1.0), (-0.6, 0.7)])
def test_fixed_mu_samples_the_grand_canonical_ensemble(mu, T):
    Delta, V, J = 0.25, 0.5, 1.0
    E, S, Nc, _ = _run(Delta, V, J, T, 0.0, 0, mu, 60000)
    ex = _grand_canonical(Delta, V, J, T, mu)
    _check("E", *block_mean(E), ex["E"])
    _check("sum S", *block_mean(S), ex["Q"])
    _check("Nc", *block_mean(Nc), ex["Nc"])
    _check("C", *block_heat_capacity(E, N, T), ex["C"])


def test_controller_holds_the_charge_on_average():
    E, S, _, _ = _run(0.25, 0.5, 1.0, 1.0, 0.5, 2, 0.0, 30000)
    est, err = block_mean(S)
    assert abs(est - 2) < 4 * err + 0.02, (est, err)
    assert S.std() > 0.5, "the charge should fluctuate under the penalty method"


def test_penalty_heat_capacity_grows_as_temperature_falls():
    Delta, V, J, Q = 0.25, 0.5, 1.0, 2
    C = {}
    for T in (0.4, 0.2, 0.1):
        E, _, _, _ = _run(Delta, V, J, T, 0.5, Q, 0.0, 20000)
        C[T] = block_heat_capacity(E, N, T)[0]
    ex = exact.sector_averages(L, Q, Delta, V, J, 0.1)
    assert C[0.1] > C[0.2] > C[0.4], C
    assert C[0.1] > 10 * ex["C"], (C[0.1], ex["C"])


def test_penalty_mode_tracks_energy():
    Delta, V, J, T = 0.25, 0.5, 1.0, 0.8
    codes = oracle.init_codes(8, 5, 10, 6)
    o0 = oracle.observables(8, codes)
    track = np.zeros(3, dtype=np.int64)
    mu, mus, sums, track = oracle.mu_sweeps(8, Delta, V, J, T, 5, codes, 50, 0.5, 4, 0.1, track=track)
    o = oracle.observables(8, codes)
    assert track.tolist() == [o[1] - o0[1], o[2] - o0[2], o[3] - o0[3]]
    assert sums[-1] == o[0]
    assert mus[0] == 0.1 and abs(mu - (mus[-1] + 0.5 * (4 - sums[-1]) / 64)) < 1e-15
