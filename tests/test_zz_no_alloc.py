"""The allocation-free batched observables call against the one that takes a
caller device buffer, through the C-ABI, on lattices of every sweep path.

lattice_observables_batch_noalloc stages its records in a static device array
of the library; its output must equal lattice_observables_batch's on the same
lattices, record for record, on two calls in a row (the second with fewer
lattices, so stale records of the first call must not leak into it), and both
must equal the oracle.
"""
import sys

import pytest

import oracle
import paper_2301_11735_amd as lat
import workloads

pytestmark = pytest.mark.gpu

SMALL = workloads.SMALL


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rec(o):
    return (o.sweep, *o.ints(), o.track_nD, o.track_nV, o.track_nJ, o.E)


def test_noalloc_observables_equal_buffered_and_oracle():
    specs = [
        SMALL.with_(L=64, encoding=1, seed=2001),                    # on-chip path, 2-bit
        SMALL.with_(L=100, encoding=0, n=-0.2, seed=2002),           # on-chip path, int8, L % 64 != 0
        SMALL.with_(L=512, encoding=0, T=1.4, seed=2003),            # multi-block words, int8 on its 2-bit copy
        SMALL.with_(L=576, encoding=1, Delta=-0.5, seed=2004),       # multi-block words, 2-bit
        SMALL.with_(L=256, encoding=1, V=-0.7, T=0.6, seed=2005),
        SMALL.with_(L=32, encoding=0, seed=2006),
    ]
    _say("case noalloc observables: " + ", ".join(f"L={s.L}/enc{s.encoding}" for s in specs))
    gs = [lat.Lattice(s.L, s.n, s.Delta, s.V, s.J, s.T, s.seed, encoding=s.encoding) for s in specs]
    os_ = [oracle.OracleLattice(s.L, s.n, s.Delta, s.V, s.J, s.T, s.seed) for s in specs]
    buffered = lat.BatchObservables(len(gs))
    # first call: every lattice; second call: the last three only, after more sweeps
    for subset, sweeps in ((list(range(len(gs))), 3), ([3, 4, 5], 2)):
        sub_g = [gs[i] for i in subset]
        lat.sweep_batch(sub_g, sweeps)
        for i in subset:
            os_[i].sweeps(sweeps)
        want = buffered(sub_g)
        got = lat.observables_batch_noalloc(sub_g)
        assert len(got) == len(subset)
        for i, w, g in zip(subset, want, got):
            assert _rec(g) == _rec(w), f"L={specs[i].L} enc={specs[i].encoding}"
            o = os_[i]
            assert g.ints() == o.observables().tolist()
            assert [g.track_nD, g.track_nV, g.track_nJ] == o.track.tolist()
            assert g.E == o.energy()
    for g in gs:
        g.destroy()


def test_noalloc_observables_reject_more_than_the_static_array_holds():
    g = lat.Lattice(64, 0.1, 0.25, 0.5, 1.0, 0.8, 7, encoding=1)
    with pytest.raises(lat.LatticeError) as exc:
        lat.observables_batch_noalloc([g] * 1025)
    assert "1024" in str(exc.value)
    assert lat.observables_batch_noalloc([]) == []
    g.destroy()
