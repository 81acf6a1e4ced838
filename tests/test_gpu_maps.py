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


def _oracle_maps(spec, o, first, n):
    oracle.map_steps(spec.L, spec.Delta, spec.V, spec.J, spec.T, spec.seed, o.codes, n, start_map=first,
                     track=o.track)


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
def test_map_steps_match_oracle(spec):
    _say(f"case maps L={spec.L} enc={spec.encoding} seed={spec.seed}")
    g, o = _make(spec), _oracle(spec)
    done = 0
    for k in (1, 2, 5, 12):
        g.map_steps(done, k)
        _oracle_maps(spec, o, done, k)
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
    for s, g, o in zip(specs, gs, os_):
        _oracle_maps(s, o, 7, 6)
        _assert_same(g, o, f"batch L={s.L}")
    alone = _make(specs[4])
    alone.map_steps(7, 6)
    assert np.array_equal(alone.read_state(), gs[4].read_state())


def test_map_mode_rejects_large_lattices():
    g = _make(SMALL.with_(L=512, encoding=1))
    with pytest.raises(lat.LatticeError):
        g.map_steps(0, 1)
    g.destroy()
