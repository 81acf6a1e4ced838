"""Charge-drop formation (arXiv:2301.11735, section 4): when the magnetic
exchange is much stronger than the charge interaction (J >> V), the doped
charge collects in one compact region while the rest of the lattice orders
antiferromagnetically; when V >> J the like charges repel and spread out.

anneal() takes replicas of one parameter set down a ladder of temperatures
in one batch: on each rung the lattices are re-created at the new
temperature from the previous rung's codes, continuing their sweep count, and
advanced together.  The start is either the seeded random configuration of
the method's stage 1, or an antiferromagnet doped at random: Neel-ordered
spins with the charges placed on randomly chosen sites (start="neel"), so
that no antiphase domain walls form on cooling through the Neel temperature
(charges gather on such walls as stripes, a long-lived state that competes
with the drop).  drop_stats() measures a configuration on the host:

    drop   largest 4-connected cluster of charged sites / number of charged
           sites (periodic lattice): about 1 for one drop, about 1/N_c for
           isolated charges
    perim  charge-spin bonds per charged site: 4 for isolated charges,
           about 4/sqrt(N_c) for one compact square drop
    af     |sum (-1)^(x+y) sigma| / number of spin sites: 1 for perfect
           antiferromagnetic order of the spins around the charge

Usage:
    python -m paper_2301_11735_amd.drop [--L 64] [--n 0.1] [--replicas 16] [--sweeps 20000] [--start neel|random]
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

# Temperatures of the default ladder, from above the Neel temperature of the
# spins (about 0.57 J for J_eff = J/4) down to well below it.
LADDER = (1.2, 1.0, 0.8, 0.6, 0.5, 0.4, 0.3, 0.2, 0.15, 0.1)


# Temperatures of the ladder for a start from the doped antiferromagnet: all
# below the Neel temperature.
NEEL_LADDER = (0.4, 0.3, 0.2, 0.15, 0.12, 0.1, 0.08)


def doped_neel(L: int, n_plus: int, n_minus: int, seed: int) -> np.ndarray:
    """Neel-ordered spins (code 0 where x + y is even, 1 where odd) with
    n_plus sites of charge +1 and n_minus of charge -1 at distinct random
    sites (numpy generator seeded with `seed`); row-major codes."""
    y, x = np.indices((L, L))
    codes = ((x + y) % 2).astype(np.int8).ravel()
    sites = np.random.default_rng(seed).permutation(L * L)[: n_plus + n_minus]
    codes[sites[:n_plus]] = 2
    codes[sites[n_plus:]] = 3
    return codes


def anneal(L: int, n: float, Delta: float, V: float, J: float, temps=LADDER, sweeps_per_T: int = 3000,
           replicas: int = 16, seed0: int = 1, n_charged: int = -1, encoding: int | None = None,
           start: str = "random"):
    """Returns (codes, observables, rungs) of every replica after the ladder;
    rungs[i] is summary() of the configurations after rung i."""
    if encoding is None:
        encoding = lat.ENC_2BIT if L % 64 == 0 else lat.ENC_INT8
    if start == "neel":
        Q, Nc = lat.charge_target(L, n, n_charged)
        init = [doped_neel(L, (Nc + Q) // 2, (Nc - Q) // 2, seed0 + r) for r in range(replicas)]
    else:
        init = [None] * replicas
    lats = [lat.Lattice(L, n, Delta, V, J, float(temps[0]), seed0 + r, encoding=encoding, n_charged=n_charged,
                        init_codes=init[r]) for r in range(replicas)]
    done, rungs = 0, []
    for i, T in enumerate(temps):
        if i > 0:
            codes = [g.read_state() for g in lats]
            for g in lats:
                g.destroy()
            lats = [lat.Lattice(L, n, Delta, V, J, float(T), seed0 + r, encoding=encoding, start_sweep=done,
                                init_codes=codes[r]) for r in range(replicas)]
        lat.sweep_batch(lats, sweeps_per_T)
        done += sweeps_per_T
        rungs.append({"T": float(T), "sweeps": done, **summary([g.read_state() for g in lats], L)})
    codes = [g.read_state() for g in lats]
    obs = [g.observables() for g in lats]
    for g in lats:
        g.destroy()
    return codes, obs, rungs


def charge_clusters(codes, L: int) -> np.ndarray:
    """Sizes of the 4-connected clusters of charged sites (codes 2, 3) on the
    periodic L x L lattice, largest first."""
    c = np.asarray(codes).reshape(L, L) >= 2
    parent = np.arange(L * L)

    def find(i):
        while parent[i] != i:
            parent[i] = parent[parent[i]]
            i = parent[i]
        return i

    ys, xs = np.nonzero(c)
    for y, x in zip(ys.tolist(), xs.tolist()):
        i = y * L + x
        for yy, xx in ((y, (x + 1) % L), ((y + 1) % L, x)):
            if c[yy, xx]:
                a, b = find(i), find(yy * L + xx)
                if a != b:
                    parent[a] = b
    roots = np.array([find(y * L + x) for y, x in zip(ys.tolist(), xs.tolist())], dtype=np.int64)
    if roots.size == 0:
        return np.zeros(0, dtype=np.int64)
    return np.sort(np.bincount(roots)[np.unique(roots)])[::-1]


def drop_stats(codes, L: int) -> dict:
    c = np.asarray(codes).reshape(L, L)
    charged = c >= 2
    n_c = int(charged.sum())
    sizes = charge_clusters(c, L)
    mixed = 0
    for sh in ((0, 1), (1, 0)):
        other = np.roll(charged, (-sh[0], -sh[1]), axis=(0, 1))
        mixed += int((charged != other).sum())
    sigma = np.where(c == 0, 1, np.where(c == 1, -1, 0))
    yy, xx = np.indices((L, L))
    stag = 1 - 2 * ((xx + yy) % 2)
    n_spin = L * L - n_c
    return {
        "n_charged": n_c,
        "drop": float(sizes[0] / n_c) if n_c else 0.0,
        "clusters": int(sizes.size),
        "perim": float(mixed / n_c) if n_c else 0.0,
        "af": float(abs((sigma * stag).sum()) / n_spin) if n_spin else 0.0,
    }


def summary(codes, L: int) -> dict:
    """Means and standard errors of drop_stats over replicas."""
    rows = [drop_stats(c, L) for c in codes]
    out = {}
    for k in ("drop", "perim", "af", "clusters"):
        v = np.array([r[k] for r in rows], dtype=np.float64)
        out[k] = float(v.mean())
        out[k + "_err"] = float(v.std(ddof=1) / np.sqrt(v.size)) if v.size > 1 else 0.0
        out[k + "_min"] = float(v.min())
        out[k + "_max"] = float(v.max())
    out["replicas"] = len(rows)
    return out


# The two regimes compared: exchange much stronger than the charge
# repulsion, and the reverse.  Delta = 3 > 2V keeps +- pairs from forming
# (with V = 1 and a small Delta the lattice would fill with a charge-ordered
# checkerboard instead), so both runs hold the same |Q| charges of one sign.
CASES = (("J>>V", 1.0, 0.05), ("V>>J", 0.1, 1.0))
DROP_DELTA = 3.0


def run_cases(L: int = 64, n: float = 0.1, sweeps_per_T: int = 20000, replicas: int = 16, seed0: int = 1,
              temps=NEEL_LADDER, start: str = "neel") -> list:
    Q, _ = lat.charge_target(L, n)
    out = []
    for name, J, V in CASES:
        codes, _, rungs = anneal(L, n, DROP_DELTA, V, J, temps, sweeps_per_T, replicas, seed0, n_charged=abs(Q),
                                 start=start)
        out.append({"case": name, "L": L, "n": n, "Q": Q, "J": J, "V": V, "Delta": DROP_DELTA, "start": start,
                    "ladder": list(temps), "sweeps_per_T": sweeps_per_T, **summary(codes, L), "rungs": rungs})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--L", type=int, default=64)
    ap.add_argument("--n", type=float, default=0.1)
    ap.add_argument("--replicas", type=int, default=16)
    ap.add_argument("--sweeps", type=int, default=20000, help="sweeps per rung of the temperature ladder")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--start", choices=("neel", "random"), default="neel")
    args = ap.parse_args()
    temps = NEEL_LADDER if args.start == "neel" else LADDER
    for row in run_cases(args.L, args.n, args.sweeps, args.replicas, args.seed, temps, args.start):
        print(json.dumps(row), flush=True)


if __name__ == "__main__":
    main()
