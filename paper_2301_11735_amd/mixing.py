"""Mixing of the two pair schedules on the GPU: the structured sublattice
schedule (one sweep = N site updates) against the paper's random maps
(section 3.2; five maps = 10 * floor(N/10) ~ N site updates).

For each schedule a batch of replicas (same parameters, different seeds) is
run from its own seeded start.  After a burn-in, the energy is read once per
unit of N site updates, and its integrated autocorrelation time is estimated
per replica with Sokal's automatic window.  The cost of an effectively
independent energy sample is then tau_int * 2 units of work, and dividing by
the measured update rate gives it in seconds.  Update rates are timed
separately, without observable reads.

Usage:
    python -m paper_2301_11735_amd.mixing [--L 64] [--T 0.7 1.2 2.0] [--n 0.1] [--replicas 64]
                                          [--units 3000] [--burn 500]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_2301_11735_amd as lat  # noqa: E402

MAPS_PER_UNIT = 5


def tau_int(x: np.ndarray, c: float = 6.0) -> float:
    """Integrated autocorrelation time of a series (in samples), with Sokal's
    automatic window: the smallest W with W >= c * tau(W)."""
    x = np.asarray(x, dtype=np.float64) - np.mean(x)
    n = x.size
    if n < 4 or not np.any(x):
        return 0.5
    f = np.fft.rfft(x, 2 * n)
    acf = np.fft.irfft(f * np.conj(f))[:n]
    acf /= acf[0]
    tau = 0.5
    for w in range(1, n):
        tau += acf[w]
        if w >= c * tau:
            return float(tau)
    return float(tau)


def _make(L, n, Delta, V, J, T, seeds, encoding):
    return [lat.Lattice(L, n, Delta, V, J, T, s, encoding=encoding) for s in seeds]


def _advance(schedule, lats, unit_index, units):
    if schedule == "sweeps":
        lat.sweep_batch(lats, units)
    else:
        lat.map_steps_batch(lats, unit_index * MAPS_PER_UNIT, units * MAPS_PER_UNIT)


def run(schedule: str, L: int, n: float, Delta: float, V: float, J: float, T: float, replicas: int, units: int,
        burn: int, seed0: int, encoding: int = 0) -> dict:
    import torch

    N = L * L
    per_unit = N if schedule == "sweeps" else MAPS_PER_UNIT * 2 * max(1, N // 10)
    seeds = [seed0 + i for i in range(replicas)]

    # update rate, no observable reads
    lats = _make(L, n, Delta, V, J, T, seeds, encoding)
    _advance(schedule, lats, 0, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _advance(schedule, lats, 2, 50)
    torch.cuda.synchronize()
    rate = replicas * 50 * per_unit / (time.perf_counter() - t0)
    for g in lats:
        g.destroy()

    # energy series
    lats = _make(L, n, Delta, V, J, T, seeds, encoding)
    obs = lat.BatchObservables(replicas)
    _advance(schedule, lats, 0, burn)
    E = np.zeros((units, replicas))
    for u in range(units):
        _advance(schedule, lats, burn + u, 1)
        E[u] = [o.E for o in obs(lats)]
    for g in lats:
        g.destroy()
    taus = np.array([tau_int(E[:, r]) for r in range(replicas)])
    tau, tau_err = float(taus.mean()), float(taus.std(ddof=1) / np.sqrt(replicas)) if replicas > 1 else 0.0
    return {
        "schedule": schedule,
        "site_updates_per_unit": per_unit,
        "tau_int_units": tau,
        "tau_int_err": tau_err,
        "E_per_site": float(E.mean() / N),
        "E_per_site_err": float(E.mean(axis=0).std(ddof=1) / np.sqrt(replicas) / N) if replicas > 1 else 0.0,
        "site_updates_per_s": rate,
        # the batch yields `replicas` independent samples per 2 tau units of work
        "batch_seconds_per_independent_sample": 2.0 * tau * per_unit / rate,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--L", type=int, default=64)
    ap.add_argument("--T", type=float, nargs="+", default=[0.7, 1.2, 2.0])
    ap.add_argument("--n", type=float, default=0.1)
    ap.add_argument("--Delta", type=float, default=0.25)
    ap.add_argument("--V", type=float, default=0.5)
    ap.add_argument("--J", type=float, default=1.0)
    ap.add_argument("--replicas", type=int, default=64)
    ap.add_argument("--units", type=int, default=3000)
    ap.add_argument("--burn", type=int, default=500)
    args = ap.parse_args()
    for T in args.T:
        for schedule in ("sweeps", "maps"):
            r = run(schedule, args.L, args.n, args.Delta, args.V, args.J, T, args.replicas, args.units, args.burn,
                    seed0=9000)
            r.update(L=args.L, T=T, n=args.n, Delta=args.Delta, V=args.V, J=args.J, replicas=args.replicas,
                     units=args.units, burn=args.burn)
            print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
