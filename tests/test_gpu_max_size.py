"""The largest lattice the library accepts (L = 32768, 2^30 sites) on the
GPU, in both encodings.  The oracle cannot follow the chain at this size, so
the checks are properties that hold at any size: the charge sum stays at its
target (the coupled-pair moves conserve it), the tracker's three components
equal the changes of the recomputed charged-site count and bond sums (eq. 3
terms), and the codes read back agree with the recomputed sums.  Smaller
lattices up to L = 8192 are compared with the oracle bit for bit in
test_gpu_parity.py."""
import sys
import time

import numpy as np
import pytest

import paper_2301_11735_amd as lat

pytestmark = pytest.mark.gpu

L_MAX = 32768


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(encoding):
    n, Delta, V, J, T, seed = 0.1, 0.25, 0.5, 1.0, 1.2, 11
    Q, Nc = lat.charge_target(L_MAX, n)
    _say(f"case max size L={L_MAX} enc={encoding}: create")
    t0 = time.perf_counter()
    g = lat.Lattice(L_MAX, n, Delta, V, J, T, seed, encoding=encoding)
    _say(f"  created in {time.perf_counter() - t0:.1f} s")
    try:
        o0 = g.observables()
        assert o0.sum_S == Q and o0.n_charged == Nc
        assert [o0.track_nD, o0.track_nV, o0.track_nJ] == [0, 0, 0]
        g.sweep(2)
        o = g.observables()
        _say(f"  after 2 sweeps: n_charged {o.n_charged}, bonds {o.bond_SS} {o.bond_ss}")
        assert o.sweep == 2
        assert o.sum_S == Q
        assert o.track_nD == o.n_charged - o0.n_charged
        assert o.track_nV == o.bond_SS - o0.bond_SS
        assert o.track_nJ == o.bond_ss - o0.bond_ss
        assert o.track_nJ != 0  # the chain moved
        codes = g.read_state()
        assert codes.size == L_MAX * L_MAX
        counts = np.bincount(codes.ravel().astype(np.uint8), minlength=4)
        assert counts.size == 4  # codes are 0..3 only
        assert counts[2] - counts[3] == o.sum_S and counts[2] + counts[3] == o.n_charged
        assert counts[0] - counts[1] == o.M
        return o.as_dict()
    finally:
        g.destroy()


def test_largest_lattice_keeps_its_invariants():
    """Both encodings at L = 32768: the invariants above, and the same chain
    (int8 lattices run on a packed 2-bit copy: identical observables)."""
    a = _run(lat.ENC_2BIT)
    b = _run(lat.ENC_INT8)
    assert a == b
