"""GPU parity of the map mode (section 3.2 random maps, built on the device)
against the oracle's sequential construction and pair updates, through the
C-ABI.  The bar is bit-exact: codes, the seven observables and the tracker.
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


def _make(spec):
    return lat.Lattice(spec.L, spec.n, spec.Delta, spec.V, spec.J, spec.T, spec.seed, encoding=spec.encoding,
                       n_charged=spec.n_charged)


def _oracle(spec):
    return oracle.OracleLattice(spec.L, spec.n, spec.Delta, spec.V, spec.J, spec.T, spec.seed,
                                n_charged=spec.n_charged)


def _oracle_maps(spec, o, first, n, nn=False):
    oracle.map_steps(spec.L, spec.Delta, spec.V, spec.J, spec.T, spec.seed, o.codes, n, start_map=first,
                     track=o.track, nn=nn)


def _assert_same(g, o, where):
    gs = g.read_state()
    if not np.array_equal(gs, o.codes):
        bad = np.flatnonzero(gs != o.codes)
        raise AssertionError(f"{where}: {bad.size} sites differ, first at {bad[:8].tolist()}")
    go = g.observables()
    assert go.ints() == o.observables().tolist(), where
    assert [go.track_nD, go.track_nV, go.track_nJ] == o.track.tolist(), where


@pytest.mark.parametrize("spec", [
    SMALL.with_(L=4, n=0.125),                                   # one pair per map
    SMALL.with_(L=8, n=-0.1, seed=9),
    SMALL.with_(L=12, n=0.2, T=0.4, seed=10),
    SMALL.with_(L=32),                                           # 102 pairs per map
    SMALL.with_(L=100, Delta=-0.7, V=-0.3, T=1.7, seed=12),
    SMALL.with_(L=256, seed=13, T=0.9),                          # 6553 pairs, 65536 sites
    SMALL.with_(L=64, encoding=1, n=0.3, T=0.5, seed=21),
    SMALL.with_(L=192, encoding=1, Delta=0.9, V=-0.8, T=2.2, seed=22),
], ids=lambda s: f"{'2bit' if s.encoding else 'int8'}-L{s.L}")
@pytest.mark.parametrize("partner", [lat.MAP_ANY, lat.MAP_NEIGHBOUR], ids=["any", "neighbour"])
def test_map_steps_match_oracle(spec, partner):
    _say(f"case maps L={spec.L} enc={spec.encoding} seed={spec.seed} partner={partner}")
    g, o = _make(spec), _oracle(spec)
    done = 0
    for k in (1, 2, 5, 12):
        g.map_steps(done, k, partner)
        _oracle_maps(spec, o, done, k, nn=partner == lat.MAP_NEIGHBOUR)
        done += k
        _assert_same(g, o, f"after {done} maps")
    g.destroy()


def test_maps_and_sweeps_interleave():
    """Map steps and structured sweeps on one lattice in any order, map
    indices given explicitly (a resume continues at the next index)."""
    _say("case maps and sweeps interleaved")
    spec = SMALL.with_(L=64, encoding=0, seed=31, T=0.7)
    g, o = _make(spec), _oracle(spec)
    g.sweep(3)
    o.sweeps(3)
    g.map_steps(0, 4)
    _oracle_maps(spec, o, 0, 4)
    g.sweep(2)
    o.sweeps(2)
    g.map_steps(4, 3)
    _oracle_maps(spec, o, 4, 3)
    _assert_same(g, o, "interleaved")
    assert g.observables().sweep == 5


def test_map_batch_equals_oracle_and_alone():
    """One launch over lattices of different L, encodings and parameters."""
    _say("case map batch")
    rng = np.random.default_rng(8)
    specs = []
    for i, (L, enc) in enumerate([(4, 0), (12, 0), (64, 1), (100, 0), (128, 1), (256, 0), (32, 0)]):
        specs.append(SMALL.with_(L=L, encoding=enc, seed=1500 + i, n=float(rng.uniform(-0.3, 0.3)),
                                 Delta=float(rng.uniform(-1, 1)), V=float(rng.uniform(-1, 1)),
                                 T=float(rng.uniform(0.2, 2.5))))
    gs = [_make(s) for s in specs]
    os_ = [_oracle(s) for s in specs]
    lat.map_steps_batch(gs, 7, 6)
    lat.map_steps_batch(gs, 13, 4, lat.MAP_NEIGHBOUR)
    for s, g, o in zip(specs, gs, os_):
        _oracle_maps(s, o, 7, 6)
        _oracle_maps(s, o, 13, 4, nn=True)
        _assert_same(g, o, f"batch L={s.L}")
    alone = _make(specs[4])
    alone.map_steps(7, 6)
    alone.map_steps(13, 4, lat.MAP_NEIGHBOUR)
    assert np.array_equal(alone.read_state(), gs[4].read_state())


def test_map_mode_rejects_large_lattices():
    g = _make(SMALL.with_(L=512, encoding=1))
    with pytest.raises(lat.LatticeError):
        g.map_steps(0, 1)
    g.destroy()


def test_neighbour_pairs_lose_the_low_temperature_fluctuations():
    """The paper's first pairing (partners restricted to nearest neighbours)
    freezes on 4x4 at low temperature: every replica stays in one
    configuration and the heat capacity collapses, while random partners give
    the exact energy and heat capacity.  64 replicas each, V = 2, Q = 4,
    T = 0.3; C per replica from its own series, then averaged."""
    from tests import exact

    _say("case neighbour pairs vs random pairs on 4x4")
    L, N, Q, T = 4, 16, 4, 0.3
    Delta, V, J = 0.25, 2.0, 1.0
    ex = exact.sector_averages(L, Q, Delta, V, J, T)
    res = {}
    for partner in (lat.MAP_ANY, lat.MAP_NEIGHBOUR):
        gs = [lat.Lattice(L, 0.25, Delta, V, J, T, 2000 + r, n_charged=4) for r in range(64)]
        obs = lat.BatchObservables(len(gs))
        lat.map_steps_batch(gs, 0, 2000, partner)
        E = []
        for k in range(2000):
            lat.map_steps_batch(gs, 2000 + 10 * k, 10, partner)
            E.append([o.E for o in obs(gs)])
        E = np.asarray(E)
        e_rep, c_rep = E.mean(axis=0), E.var(axis=0) / (N * T * T)
        n = e_rep.size
        res[partner] = (e_rep.mean(), e_rep.std(ddof=1) / np.sqrt(n), c_rep.mean(), c_rep.std(ddof=1) / np.sqrt(n))
    e, e_err, c, c_err = res[lat.MAP_ANY]
    assert abs(e - ex["E"]) < 4 * e_err + 0.01 * abs(ex["E"]), (e, e_err, ex["E"])
    assert abs(c - ex["C"]) < 4 * c_err + 0.05 * ex["C"], (c, c_err, ex["C"])
    c_nn = res[lat.MAP_NEIGHBOUR][2]
    assert c_nn < 0.25 * ex["C"], (c_nn, ex["C"])
