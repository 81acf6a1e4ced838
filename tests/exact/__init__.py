"""Exact enumeration of small lattices and exact Boltzmann averages (test infrastructure).

``enum.c`` counts every configuration of a 3x3 or 4x4 periodic lattice by
(Q, Nc, BV, BJ); the helpers below turn that density of states into exact
canonical averages in a fixed charge sector for any (Delta, V, J, T).
"""
from __future__ import annotations

import ctypes
import functools
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "enum.c")
_LIB = os.path.join(_HERE, "libexact.so")


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = f"{_LIB}.tmp{os.getpid():x}"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


@functools.lru_cache(maxsize=None)
def density_of_states(L: int) -> np.ndarray:
    """g[Q+N, Nc, BV+2N, BJ+2N] as int64 (N = L*L)."""
    build(force=False)
    lib = ctypes.CDLL(_LIB)
    lib.exact_hist_size.argtypes = [ctypes.c_int]
    lib.exact_hist_size.restype = ctypes.c_int64
    lib.exact_hist.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]
    lib.exact_hist.restype = ctypes.c_int
    N = L * L
    g = np.zeros(int(lib.exact_hist_size(L)), dtype=np.int64)
    rc = lib.exact_hist(L, g.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    assert rc == 0
    return g.reshape(2 * N + 1, N + 1, 4 * N + 1, 4 * N + 1)


def sector_averages(L: int, Q: int, Delta: float, V: float, J: float, T: float) -> dict:
    """Exact <E>, <E^2>, C = (<E^2>-<E>^2)/(N T^2), <Nc>, <BV>, <BJ> in charge sector Q."""
    N = L * L
    g = density_of_states(L)[Q + N].astype(np.float64)  # [Nc, BV, BJ]
    nc = np.arange(N + 1)[:, None, None]
    bv = (np.arange(4 * N + 1) - 2 * N)[None, :, None]
    bj = (np.arange(4 * N + 1) - 2 * N)[None, None, :]
    E = Delta * nc + V * bv + 0.25 * J * bj
    mask = g > 0
    logw = np.where(mask, np.log(np.where(mask, g, 1.0)) - E / T, -np.inf)
    w = np.exp(logw - logw[mask].max())
    Z = w.sum()
    avg = lambda X: float((w * X).sum() / Z)  # noqa: E731
    e1 = avg(E)
    e2 = avg(E * E)
    return {
        "E": e1,
        "E2": e2,
        "C": (e2 - e1 * e1) / (N * T * T),
        "Nc": avg(nc * np.ones_like(E)),
        "BV": avg(bv * np.ones_like(E)),
        "BJ": avg(bj * np.ones_like(E)),
    }


_PIN_SRC = os.path.join(_HERE, "philox_pin.cpp")
_PIN_LIB = os.path.join(_HERE, "libphilox_pin.so")
ROCM_INCLUDE = os.environ.get("ROCM_PATH", "/opt/rocm") + "/include"


def build_philox_pin(force: bool = True) -> str | None:
    """Build the rocRAND-backed Philox reference; None if the headers are absent."""
    if not os.path.exists(os.path.join(ROCM_INCLUDE, "rocrand", "rocrand_philox4x32_10.h")):
        return None
    if force or not os.path.exists(_PIN_LIB) or os.path.getmtime(_PIN_LIB) < os.path.getmtime(_PIN_SRC):
        tmp = f"{_PIN_LIB}.tmp{os.getpid():x}"
        subprocess.check_call(["g++", "-O1", "-fPIC", "-shared", "-D__HIP_PLATFORM_AMD__",
                               "-I" + ROCM_INCLUDE, "-o", tmp, _PIN_SRC])
        os.replace(tmp, _PIN_LIB)
    return _PIN_LIB


def rocrand_philox(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    """rocRAND Philox4x32-10 of n counters (n,4) under n keys (n,2) -> (n,4) uint32."""
    path = build_philox_pin(force=False)
    lib = ctypes.CDLL(path)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib.pin_philox.argtypes = [u32p, u32p, u32p, ctypes.c_int]
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros_like(c)
    lib.pin_philox(c.ctypes.data_as(u32p), k.ctypes.data_as(u32p), out.ctypes.data_as(u32p), c.shape[0])
    return out
