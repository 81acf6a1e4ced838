"""GPU temperature scans (paper_2301_11735_amd.thermo) on 4x4 lattices against
exact results: the fixed-charge sector by exact enumeration (tests/exact),
and the Delta -> infinity, n = 0 limit (an antiferromagnetic Ising model with
J_eff = J/4) by enumerating all 2^16 spin states here.  Estimates are means
over 64 independent replicas; the bar is |z| < 4 with a 1% allowance for the
finite-series bias of the per-replica variance estimators.
"""
import sys

import numpy as np
import pytest

from paper_2301_11735_amd import thermo
from tests import exact

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _close(name, est, err, ref, T):
    z = (est - ref) / max(err, 1e-12)
    assert abs(est - ref) < 4 * err + 0.01 * abs(ref), f"T={T} {name}: {est:.6f} +- {err:.6f} vs exact {ref:.6f} (z={z:.2f})"


def test_scan_4x4_matches_exact_enumeration():
    L, N, Q = 4, 16, 2
    Delta, V, J, n = 0.25, 0.5, 1.0, 0.125
    temps = [0.5, 1.0, 2.0]
    _say("case thermo 4x4 sector scan")
    rows = thermo.scan(L, n, Delta, V, J, temps, replicas=64, sweeps=8000, burn=500, every=1, seed0=700)
    for row in rows:
        ex = exact.sector_averages(L, Q, Delta, V, J, row["T"])
        _close("e", row["e"], row["e_err"], ex["E"] / N, row["T"])
        _close("C", row["C"], row["C_err"], ex["C"], row["T"])
        _close("nc", row["nc"], row["nc_err"], ex["Nc"] / N, row["T"])


def _ising_4x4(J_eff, T):
    L, N = 4, 16
    states = np.arange(1 << N, dtype=np.int64)
    sig = 1 - 2 * ((states[:, None] >> np.arange(N)) & 1)
    idx = np.arange(N).reshape(L, L)
    right = np.roll(idx, -1, axis=1).reshape(-1)
    down = np.roll(idx, -1, axis=0).reshape(-1)
    bonds = (sig * sig[:, right]).sum(axis=1) + (sig * sig[:, down]).sum(axis=1)
    E = J_eff * bonds
    stag = 1 - 2 * ((np.arange(N) // L + np.arange(N) % L) % 2)
    M = sig.sum(axis=1)
    Ms = (sig * stag).sum(axis=1)
    w = np.exp(-(E - E.min()) / T)
    Z = w.sum()
    avg = lambda X: float((w * X).sum() / Z)  # noqa: E731
    return {"e": avg(E) / N, "C": (avg(E * E) - avg(E) ** 2) / (N * T * T),
            "chi": avg(M * M) / (N * T), "chi_st": avg(Ms * Ms) / (N * T)}


@pytest.mark.parametrize("T", [1.0, 2.0])
def test_scan_ising_limit_4x4_matches_enumeration(T):
    L, J = 4, 1.0
    _say(f"case thermo 4x4 Ising limit T={T}")
    row, = thermo.scan(L, 0.0, 1e6, 0.5, J, [T], replicas=64, sweeps=8000, burn=500, every=1, seed0=900,
                       n_charged=0)
    assert row["nc"] == 0.0
    ex = _ising_4x4(0.25 * J, T)
    for name in ("e", "C", "chi", "chi_st"):
        _close(name, row[name], row[name + "_err"], ex[name], T)


def test_heat_capacity_curve_4x4_matches_exact():
    """C(T) of the 4x4 sector n = 1/8 across the range where the exact curve has
    its structure; prints the table (T, C from 64 replicas, exact C).  Below
    T = 0.5 the chain leaves its low-energy states rarely, so those points get a
    long burn-in and a long series; every point's error bar must stay under 30%
    of C, so that agreement within it means something."""
    L, N, Q = 4, 16, 2
    Delta, V, J, n = 0.25, 0.5, 1.0, 0.125
    _say("case thermo 4x4 C(T) curve")
    rows = thermo.scan(L, n, Delta, V, J, [0.25, 0.35], replicas=64, sweeps=160000, burn=20000, every=2, seed0=1000)
    rows += thermo.scan(L, n, Delta, V, J, [0.5, 0.7, 1.0, 1.4, 2.0, 3.0], replicas=64, sweeps=8000, burn=500,
                        every=1, seed0=1100)
    _say("T  C_gpu  C_err  C_exact  z_C  e_gpu  e_err  e_exact  z_e")
    for row in rows:
        ex = exact.sector_averages(L, Q, Delta, V, J, row["T"])
        e_ex = ex["E"] / N
        _say(f"{row['T']:.2f} {row['C']:.5f} {row['C_err']:.5f} {ex['C']:.5f} "
             f"{(row['C'] - ex['C']) / row['C_err']:+.2f} {row['e']:.5f} {row['e_err']:.5f} {e_ex:.5f} "
             f"{(row['e'] - e_ex) / row['e_err']:+.2f}")
        assert row["C_err"] < 0.3 * ex["C"], f"T={row['T']}: error bar {row['C_err']:.4f} too wide for C={ex['C']:.4f}"
        _close("C", row["C"], row["C_err"], ex["C"], row["T"])
        _close("e", row["e"], row["e_err"], e_ex, row["T"])


def test_charge_collects_into_a_drop_when_exchange_dominates():
    """Section 4's charge drop on a 64 x 64 lattice at n = 0.1 (410 charges of
    one sign; Delta = 3 keeps +- pairs from forming), 16 replicas started from
    a Neel antiferromagnet doped at random and cooled to T = 0.08: with
    J >> V (J = 1, V = 0.05) the charge gathers into one compact cluster inside
    an antiferromagnetic background; with V >> J (J = 0.1, V = 1) the like
    charges stay apart.  The measures (largest charged cluster / charges,
    charge-spin bonds per charge, staggered spin order) are pinned on the CPU
    by tests/test_drop_stats.py."""
    from paper_2301_11735_amd import drop

    _say("case charge drop 64x64")
    rows = {r["case"]: r for r in drop.run_cases(64, 0.1, 20000, 16, 1)}
    jv, vj = rows["J>>V"], rows["V>>J"]
    for r in (jv, vj):
        _say(f"{r['case']}: drop {r['drop']:.3f} +- {r['drop_err']:.3f} (min {r['drop_min']:.3f}), "
             f"perim {r['perim']:.3f}, af {r['af']:.4f}, clusters {r['clusters']:.1f}")
    assert jv["drop"] > 0.75 and jv["drop_min"] > 0.5   # most of the charge in one cluster
    assert jv["perim"] < 1.0                              # compact: few charge-spin bonds per charge
    assert jv["af"] > 0.99                                # the rest stays antiferromagnetic
    assert vj["drop_max"] < 0.01 and vj["perim"] > 3.9   # isolated charges
