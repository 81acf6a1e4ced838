"""Seeded synthetic workloads: parameter sets and request streams.

This module holds none of the method's arithmetic.  It only names the
lattices to simulate (size, couplings, temperature, density, seed, sweep
counts), so that the tests, the benchmark and the oracle runs all draw the
same inputs.  The lattice contents themselves are produced by the method's
own seeded init (stage 1 of section 3.1), on each side separately.
"""
from __future__ import annotations

from dataclasses import asdict, dataclass, replace

import numpy as np

INT8 = 0
TWOBIT = 1


@dataclass(frozen=True)
class LatticeSpec:
    L: int
    n: float
    Delta: float
    V: float
    J: float
    T: float
    seed: int
    encoding: int = INT8
    n_charged: int = -1
    sweeps: int = 1
    every: int = 1

    def with_(self, **kw) -> "LatticeSpec":
        return replace(self, **kw)

    def asdict(self) -> dict:
        return asdict(self)


# Small plain run: L=32, 256 charged sites with sum S = 102, observables every 10 sweeps.
SMALL = LatticeSpec(L=32, n=0.1, Delta=0.25, V=0.5, J=1.0, T=0.8, seed=1, encoding=INT8, sweeps=10000, every=10)
# Single mid lattice: L=1024, int8, observables every sweep.
MID = LatticeSpec(L=1024, n=0.05, Delta=0.0, V=0.5, J=1.0, T=1.0, seed=2, encoding=INT8, sweeps=2000, every=1)
# Large single lattice: L=8192 (67M sites), 2-bit states, observables every 50 sweeps.
LARGE = LatticeSpec(L=8192, n=0.1, Delta=0.25, V=0.5, J=1.0, T=1.2, seed=3, encoding=TWOBIT, sweeps=1000, every=50)


def batched_specs(count: int = 256, L: int = 128, sweeps: int = 5000) -> list[LatticeSpec]:
    """256 independent L=128 lattices: id = 32*j + i with T_i = 0.2 + 1.8*i/31
    (32 temperatures) and n_j = 0.05*j (8 densities); seeds 1000 + id."""
    out = []
    for lid in range(count):
        i, j = lid % 32, lid // 32
        T = 0.2 + 1.8 * i / 31.0
        n = 0.05 * (j % 8)
        out.append(LatticeSpec(L=L, n=n, Delta=0.25, V=0.5, J=1.0, T=T, seed=1000 + lid,
                               encoding=TWOBIT, sweeps=sweeps, every=50))
    return out


@dataclass(frozen=True)
class Request:
    index: int
    arrival_s: float
    spec: LatticeSpec


def request_stream(rate_per_s: float = 200.0, duration_s: float = 60.0, seed: int = 7,
                   sizes=(64, 128, 256, 512), sweep_range=(500, 5000)) -> list[Request]:
    """Poisson arrivals of uneven simulation requests (served workload):
    L uniform in `sizes`, T ~ U[0.1, 2.5], n ~ U[0, 0.4], Delta, V ~ U[-1, 1],
    J = 1, sweeps uniform in `sweep_range`, request seed 10^6 + index, 2-bit."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t >= duration_s:
            break
        idx = len(out)
        spec = LatticeSpec(
            L=int(rng.choice(sizes)),
            n=float(rng.uniform(0.0, 0.4)),
            Delta=float(rng.uniform(-1.0, 1.0)),
            V=float(rng.uniform(-1.0, 1.0)),
            J=1.0,
            T=float(rng.uniform(0.1, 2.5)),
            seed=10**6 + idx,
            encoding=TWOBIT,
            sweeps=int(rng.integers(sweep_range[0], sweep_range[1] + 1)),
            every=0,
        )
        out.append(Request(index=idx, arrival_s=t, spec=spec))
    return out
