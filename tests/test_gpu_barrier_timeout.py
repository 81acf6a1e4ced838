"""The time-out path of the persistent multi-block word kernel's device-wide
barriers, forced from the host: LATTICE_BARRIER_TICKS=0 bounds every wait by
zero ticks of the device wall clock, so a block that would have to wait
raises the lattice's error flag and goes on (every kernel still ends).  The
state is then invalid, and every read of it must say so with LAT_EHIP:
lattice_observables, lattice_observables_batch, lattice_observables_batch_noalloc
and lattice_series_read.  A
lattice made afterwards, with the normal bound, is unaffected."""
import sys

import numpy as np
import pytest

import oracle
import paper_2301_11735_amd as lat
import workloads

pytestmark = pytest.mark.gpu

SPEC = workloads.SMALL.with_(L=512, encoding=1, seed=41)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _make():
    s = SPEC
    return lat.Lattice(s.L, s.n, s.Delta, s.V, s.J, s.T, s.seed, encoding=s.encoding)


def test_barrier_time_out_is_reported_by_every_read(monkeypatch):
    monkeypatch.setenv("LATTICE_WORDS_PERSISTENT", "1")
    monkeypatch.setenv("LATTICE_BARRIER_TICKS", "0")
    _say("case barrier time-out forced: sweep, then observables")
    g = _make()
    g.sweep(20)
    with pytest.raises(lat.LatticeError) as e:
        g.observables()
    assert e.value.code == lat.LAT_EHIP
    with pytest.raises(lat.LatticeError) as e:
        lat.BatchObservables(1)([g])
    assert e.value.code == lat.LAT_EHIP
    with pytest.raises(lat.LatticeError) as e:
        lat.observables_batch_noalloc([g])
    assert e.value.code == lat.LAT_EHIP
    g.destroy()

    _say("case barrier time-out forced: observation series")
    g = _make()
    buf = g.sweep_series(4, 2, read=False)
    with pytest.raises(lat.LatticeError) as e:
        g.read_series(buf, 4)
    assert e.value.code == lat.LAT_EHIP
    g.destroy()

    _say("case normal bound afterwards")
    monkeypatch.delenv("LATTICE_BARRIER_TICKS")
    g = _make()
    s = SPEC
    o = oracle.OracleLattice(s.L, s.n, s.Delta, s.V, s.J, s.T, s.seed)
    g.sweep(5)
    o.sweeps(5)
    assert np.array_equal(g.read_state(), o.codes)
    assert g.observables().ints() == o.observables().tolist()
    g.destroy()
