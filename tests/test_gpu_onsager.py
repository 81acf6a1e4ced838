"""The GPU path at scale against a closed form: with Delta -> infinity and
n = 0 no site is charged, the model is the square-lattice Ising model of the
spins with coupling J/4 (eq. 3), and the energy per site must match
Onsager's exact result (the same limit the oracle is pinned to at L = 64).
L = 1024 runs on the one-launch-per-phase kernels (2-bit), where finite-size
corrections away from T_c are far below the statistical error.
"""
import math
import sys

import numpy as np
import pytest

import paper_2301_11735_amd as lat
from tests.mcstats import block_mean
from tests.test_oracle_stats import onsager_energy_per_site

pytestmark = pytest.mark.gpu

J = 1.0
TC = 2 * 0.25 * J / math.log(1 + math.sqrt(2))  # 0.5673 in units of the code's J


@pytest.mark.parametrize("T", [0.45, 0.8, 1.0])
def test_large_lattice_energy_matches_onsager(T):
    L = 1024
    print(f"case Onsager L={L} T={T}", flush=True)
    sys.stdout.flush()
    init = None
    if T < TC:
        # ordered start (sigma = (-1)^(x+y)): a quench from random spins leaves
        # stripe domains on the torus that a finite run below T_c keeps
        x, y = np.meshgrid(np.arange(L), np.arange(L))
        init = ((x + y) % 2).astype(np.int8).reshape(-1)
    g = lat.Lattice(L, 0.0, 1e6, 0.5, J, T, 17, encoding=lat.ENC_2BIT, n_charged=0, init_codes=init)
    g.sweep(2000)
    e = []
    for _ in range(400):
        g.sweep(5)
        o = g.observables()
        assert o.n_charged == 0 and o.sum_S == 0
        e.append(0.25 * J * o.bond_ss / (L * L))
    g.destroy()
    est, err = block_mean(np.asarray(e), n_blocks=20)
    exact = onsager_energy_per_site(T, 0.25 * J)
    print(f"T={T}: e = {est:.6f} +- {err:.6f}, Onsager {exact:.6f}", flush=True)
    # 4 standard errors of 20 block means, plus 1e-4 for what 20 blocks
    # leave of the series' autocorrelation
    assert abs(est - exact) < 4 * err + 1e-4, (T, est, err, exact)
