"""GPU parity of the penalty mode (section 2.2, the prior method) against the
oracle through the C-ABI: states, observables, tracker, and the whole mu and
sum-S trajectory bit for bit; plus the paper's objection on the GPU path.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2301_11735_amd as lat
import workloads

pytestmark = pytest.mark.gpu

SMALL = workloads.SMALL


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("spec,kappa,mu0", [
    (SMALL.with_(L=4, n=0.125), 0.5, 0.0),
    (SMALL.with_(L=8, n=-0.1, seed=9, T=0.4), 1.0, -0.2),
    (SMALL.with_(L=32), 0.5, 0.1),
    (SMALL.with_(L=100, Delta=-0.7, V=-0.3, T=1.7, seed=12), 0.25, 0.3),
    (SMALL.with_(L=256, seed=13, T=0.9), 0.5, 0.0),
], ids=lambda v: f"L{v.L}" if hasattr(v, "L") else str(v))
def test_penalty_sweeps_match_oracle(spec, kappa, mu0):
    _say(f"case penalty L={spec.L} kappa={kappa} mu0={mu0}")
    g = lat.Lattice(spec.L, spec.n, spec.Delta, spec.V, spec.J, spec.T, spec.seed, encoding=lat.ENC_INT8)
    o = oracle.OracleLattice(spec.L, spec.n, spec.Delta, spec.V, spec.J, spec.T, spec.seed)
    mu_g, mu_o, done = mu0, mu0, 0
    for k in (1, 2, 5, 10):
        mu_g, mus_g, sums_g = g.mu_sweeps(done, k, kappa, mu_g)
        mu_o, mus_o, sums_o, _ = oracle.mu_sweeps(spec.L, spec.Delta, spec.V, spec.J, spec.T, spec.seed, o.codes, k,
                                                  kappa, o.Q, mu_o, start_sweep=done, track=o.track)
        done += k
        assert np.array_equal(sums_g, sums_o), f"after {done}"
        assert np.array_equal(mus_g, mus_o) and mu_g == mu_o, f"after {done}"
        assert np.array_equal(g.read_state(), o.codes), f"after {done}"
        go = g.observables()
        assert go.ints() == o.observables().tolist()
        assert [go.track_nD, go.track_nV, go.track_nJ] == o.track.tolist()
    g.destroy()


def test_penalty_mode_rejects_2bit_lattices():
    g = lat.Lattice(64, 0.1, 0.25, 0.5, 1.0, 1.0, 1, encoding=lat.ENC_2BIT)
    with pytest.raises(lat.LatticeError):
        g.mu_sweeps(0, 1, 0.5, 0.0)
    g.destroy()


def test_penalty_heat_capacity_grows_as_temperature_falls():
    """4x4, n = 1/8: as T falls, the penalty method's heat capacity grows (mu
    keeps the charge, and with it the energy, fluctuating) while the exact
    heat capacity of the fixed-charge sector vanishes."""
    from paper_2301_11735_amd import thermo
    from tests import exact

    _say("case penalty C(T) on 4x4")
    rows = thermo.penalty_scan(4, 0.125, 0.25, 0.5, 1.0, [0.4, 0.2, 0.1], replicas=4, sweeps=4000, burn=500,
                               kappa=0.5)
    C = {r["T"]: r["C"] for r in rows}
    assert C[0.1] > C[0.2] > C[0.4], C
    ex = exact.sector_averages(4, 2, 0.25, 0.5, 1.0, 0.1)
    assert C[0.1] > 10 * ex["C"], (C[0.1], ex["C"])
