"""Thermodynamics from replica batches (arXiv:2301.11735 section 2.2 and the
averaging over lattice copies of section 3.2): temperature scans of the
energy, heat capacity, susceptibilities and charge order, with errors from
the spread over independent replicas.

Every (temperature, replica) pair is one lattice of a single batch; after a
burn-in the batch runs as replays of one HIP graph whose intervals each
advance every lattice by `every` sweeps and reduce its observables on the
device, so a whole series comes back with one copy per replay.  Per replica
the time averages give

    e    = <E>/N
    C    = (<E^2> - <E>^2) / (N T^2)
    chi  = (<M^2> - <M>^2) / (N T)          M = sum sigma
    chis = (<Ms^2> - <Ms>^2) / (N T)        Ms = sum (-1)^(x+y) sigma
    nc   = <N_c>/N,  cs2 = <C_st^2>/N^2     C_st = sum (-1)^(x+y) S

and the estimate at each temperature is the mean over replicas with its
standard error (replicas are independent chains from different seeds).

The penalty mode (section 2.2's prior method) has its own scan,
penalty_scan(), for comparison.

Usage:
    python -m paper_2301_11735_amd.thermo --L 16 --n 0.1 --T 0.2 0.4 0.8 1.6 [--replicas 32]
                                          [--sweeps 4000] [--burn 1000] [--every 1] [--penalty --kappa 0.5]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_2301_11735_amd as lat  # noqa: E402


def _mean_err(x: np.ndarray):
    x = np.asarray(x, dtype=np.float64)
    err = float(x.std(ddof=1) / np.sqrt(x.size)) if x.size > 1 else 0.0
    return float(x.mean()), err


def scan(L: int, n: float, Delta: float, V: float, J: float, temps, replicas: int = 32, sweeps: int = 4000,
         burn: int = 1000, every: int = 1, seed0: int = 1, encoding: int | None = None, n_charged: int = -1,
         chunk: int = 200) -> list:
    """Run the scan; returns one dict per temperature."""
    if encoding is None:
        encoding = lat.ENC_2BIT if L % 64 == 0 else lat.ENC_INT8
    temps = [float(t) for t in temps]
    N = L * L
    lats, keys = [], []
    for it, T in enumerate(temps):
        for r in range(replicas):
            seed = seed0 + it * replicas + r
            lats.append(lat.Lattice(L, n, Delta, V, J, T, seed, encoding=encoding, n_charged=n_charged))
            keys.append(it)
    keys = np.asarray(keys)
    if burn > 0:
        lat.sweep_batch(lats, burn)
    chunk = max(1, min(chunk, sweeps // every))
    n_chunks = max(1, sweeps // (every * chunk))
    graph = lat.BatchGraph(lats, every, chunk)
    parts = []
    for _ in range(n_chunks):
        graph.launch(1)
        parts.append(graph.read_array())
    graph.destroy()
    rec = np.concatenate(parts, axis=0)  # (samples, lattices)
    for g in lats:
        g.destroy()

    E = rec["E"].astype(np.float64)
    M = rec["M"].astype(np.float64)
    Ms = rec["M_stag"].astype(np.float64)
    Nc = rec["n_charged"].astype(np.float64)
    Cs = rec["C_stag"].astype(np.float64)
    out = []
    for it, T in enumerate(temps):
        cols = np.flatnonzero(keys == it)
        e = E[:, cols].mean(axis=0) / N
        C = E[:, cols].var(axis=0) / (N * T * T)
        chi = M[:, cols].var(axis=0) / (N * T)
        chis = Ms[:, cols].var(axis=0) / (N * T)
        nc = Nc[:, cols].mean(axis=0) / N
        cs2 = (Cs[:, cols] ** 2).mean(axis=0) / (N * N)
        row = {"T": T, "L": L, "n": n, "Delta": Delta, "V": V, "J": J, "replicas": replicas,
               "samples_per_replica": int(rec.shape[0]), "every": every, "burn": burn}
        for name, v in (("e", e), ("C", C), ("chi", chi), ("chi_st", chis), ("nc", nc), ("cst2", cs2)):
            row[name], row[name + "_err"] = _mean_err(v)
        out.append(row)
    return out


def penalty_scan(L: int, n: float, Delta: float, V: float, J: float, temps, replicas: int = 4, sweeps: int = 2000,
                 burn: int = 500, kappa: float = 0.5, mu0: float = 0.0, seed0: int = 1) -> list:
    """The same estimates for the penalty mode (section 2.2, the prior method:
    single-site updates of E - mu sum S with mu steered towards the target
    charge after every sweep).  Replicas run one after another (the controller
    reads the charge back every sweep); each is sampled once per sweep."""
    N = L * L
    out = []
    for it, T in enumerate(temps):
        per = {k: [] for k in ("e", "C", "nc", "q", "mu")}
        for r in range(replicas):
            g = lat.Lattice(L, n, Delta, V, J, float(T), seed0 + it * replicas + r, encoding=lat.ENC_INT8)
            mu, _, _ = g.mu_sweeps(0, burn, kappa, mu0)
            E, Nc, S, M = [], [], [], []
            for s in range(sweeps):
                mu, mus, sums = g.mu_sweeps(burn + s, 1, kappa, mu)
                o = g.observables()
                E.append(o.E)
                Nc.append(o.n_charged)
                S.append(sums[0])
                M.append(mus[0])
            g.destroy()
            E = np.asarray(E)
            per["e"].append(E.mean() / N)
            per["C"].append(E.var() / (N * T * T))
            per["nc"].append(np.mean(Nc) / N)
            per["q"].append(np.mean(S) / N)
            per["mu"].append(np.mean(M))
        row = {"T": float(T), "L": L, "n": n, "Delta": Delta, "V": V, "J": J, "kappa": kappa, "replicas": replicas,
               "samples_per_replica": sweeps, "burn": burn, "method": "penalty"}
        for name, v in per.items():
            row[name], row[name + "_err"] = _mean_err(v)
        out.append(row)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--L", type=int, default=16)
    ap.add_argument("--n", type=float, default=0.1)
    ap.add_argument("--Delta", type=float, default=0.25)
    ap.add_argument("--V", type=float, default=0.5)
    ap.add_argument("--J", type=float, default=1.0)
    ap.add_argument("--T", type=float, nargs="+", default=[0.2, 0.4, 0.6, 0.8, 1.2, 1.6, 2.4])
    ap.add_argument("--replicas", type=int, default=32)
    ap.add_argument("--sweeps", type=int, default=4000)
    ap.add_argument("--burn", type=int, default=1000)
    ap.add_argument("--every", type=int, default=1)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--penalty", action="store_true",
                    help="also scan the penalty mode (section 2.2) with --kappa, 4 replicas")
    ap.add_argument("--kappa", type=float, default=0.5)
    args = ap.parse_args()
    for row in scan(args.L, args.n, args.Delta, args.V, args.J, args.T, args.replicas, args.sweeps, args.burn,
                    args.every, args.seed):
        print(json.dumps(row), flush=True)
    if args.penalty:
        for row in penalty_scan(args.L, args.n, args.Delta, args.V, args.J, args.T, 4, args.sweeps, args.burn,
                                args.kappa, seed0=args.seed):
            print(json.dumps(row), flush=True)


if __name__ == "__main__":
    main()
