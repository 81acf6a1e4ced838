"""Block-averaged Monte Carlo error bars for the statistical pins (test helper)."""
from __future__ import annotations

import numpy as np


def block_mean(x: np.ndarray, n_blocks: int = 50):
    """Mean and standard error from n_blocks consecutive block means."""
    x = np.asarray(x, dtype=np.float64)
    B = len(x) // n_blocks
    blocks = x[: B * n_blocks].reshape(n_blocks, B).mean(axis=1)
    return float(blocks.mean()), float(blocks.std(ddof=1) / np.sqrt(n_blocks))


def block_heat_capacity(E: np.ndarray, N: int, T: float, n_blocks: int = 50):
    """C = (<E^2> - <E>^2) / (N T^2) with a jackknife error over blocks."""
    E = np.asarray(E, dtype=np.float64)
    B = len(E) // n_blocks
    E = E[: B * n_blocks].reshape(n_blocks, B)
    s1 = E.sum(axis=1)
    s2 = (E * E).sum(axis=1)
    tot1, tot2, n = s1.sum(), s2.sum(), E.size

    def c_of(a1, a2, m):
        mu = a1 / m
        return (a2 / m - mu * mu) / (N * T * T)

    full = c_of(tot1, tot2, n)
    jk = np.array([c_of(tot1 - s1[i], tot2 - s2[i], n - B) for i in range(n_blocks)])
    err = np.sqrt((n_blocks - 1) / n_blocks * np.sum((jk - jk.mean()) ** 2))
    return float(full), float(err)


def zscore(est: float, err: float, exact: float) -> float:
    return (est - exact) / max(err, 1e-12)
