"""Sequential CPU oracle for the coupled-pair Metropolis algorithm (arXiv:2301.11735).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library (``paper_2301_11735_amd``) never imports it and shares no code with it.

The arithmetic lives in ``oracle.c`` (plain C, one int8 code per site, pairs
visited one at a time); this module only marshals arguments through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

# FP contraction stays off so that Delta*nD + V*nV + 0.25*J*nJ is rounded
# term by term, exactly as written.
GCC_FLAGS = ["-O2", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off", "-fno-fast-math"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it (gcc, host only)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = f"{_LIB_PATH}.tmp{os.getpid():x}"  # per process: parallel test workers may build at once
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _configure(L: ctypes.CDLL) -> ctypes.CDLL:
    u32p = ctypes.POINTER(ctypes.c_uint32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    i8p = ctypes.POINTER(ctypes.c_int8)
    d, u64, i32, i64 = ctypes.c_double, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64
    L.orc_philox.argtypes = [u32p, u32p, u32p]
    L.orc_philox.restype = None
    L.orc_threshold.argtypes = [d, d, d, d, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.orc_threshold.restype = ctypes.c_uint32
    L.orc_charge_target.argtypes = [i32, d, i64, i64p, i64p]
    L.orc_charge_target.restype = ctypes.c_int
    L.orc_init.argtypes = [i32, u64, i64, i64, i8p]
    L.orc_init.restype = ctypes.c_int
    L.orc_schedule.argtypes = [i32, u64, u64, i32p, i32p, i32p]
    L.orc_schedule.restype = None
    L.orc_sweeps.argtypes = [i32, d, d, d, d, u64, u64, u64, i8p, i64p]
    L.orc_sweeps.restype = ctypes.c_int
    L.orc_general_steps.argtypes = [i32, d, d, d, d, u64, u64, u64, i8p, i64p]
    L.orc_general_steps.restype = ctypes.c_int
    L.orc_observables.argtypes = [i32, i8p, i64p]
    L.orc_observables.restype = None
    L.orc_pair_delta.argtypes = [i32, i8p, i64, i64, ctypes.c_int, ctypes.c_int, i64p]
    L.orc_pair_delta.restype = None
    L.orc_pair_config.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    L.orc_pair_config.restype = ctypes.c_int
    L.orc_energy.argtypes = [d, d, d, i64p]
    L.orc_energy.restype = d
    L.orc_series.argtypes = [i32, d, d, d, d, u64, u64, u64, u64, i8p, i64p, i64p]
    L.orc_series.restype = ctypes.c_int
    L.orc_general_series.argtypes = [i32, d, d, d, d, u64, u64, u64, u64, i8p, i64p, i64p]
    L.orc_general_series.restype = ctypes.c_int
    L.orc_map_pairs.argtypes = [i32]
    L.orc_map_pairs.restype = i64
    L.orc_map_build.argtypes = [i32, u64, u64, i64p]
    L.orc_map_build.restype = i64
    L.orc_map_steps.argtypes = [i32, d, d, d, d, u64, u64, u64, i8p, i64p]
    L.orc_map_steps.restype = ctypes.c_int
    L.orc_map_steps_mode.argtypes = [i32, d, d, d, d, u64, ctypes.c_int, u64, u64, i8p, i64p]
    L.orc_map_steps_mode.restype = ctypes.c_int
    L.orc_nn_map_pairs.argtypes = [i32]
    L.orc_nn_map_pairs.restype = i64
    L.orc_nn_map_build.argtypes = [i32, u64, u64, i64p]
    L.orc_nn_map_build.restype = i64
    dp = ctypes.POINTER(ctypes.c_double)
    L.orc_mu_sweeps.argtypes = [i32, d, d, d, d, u64, u64, u64, d, i64, dp, i8p, i64p, dp, i64p]
    L.orc_mu_sweeps.restype = ctypes.c_int
    L.orc_map_series.argtypes = [i32, d, d, d, d, u64, ctypes.c_int, u64, u64, u64, i8p, i64p, i64p]
    L.orc_map_series.restype = ctypes.c_int
    return L


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        build(force=False)
        _lib = _configure(ctypes.CDLL(_LIB_PATH))
    return _lib


def use_library(path: str | None):
    """Test hook for mutation tests: make every call go to the C library at
    `path` (a deliberately broken copy of oracle.c), or back to the real one
    with None.  Returns nothing; not thread-safe."""
    global _lib
    _lib = None if path is None else _configure(ctypes.CDLL(path))


def _p(arr: np.ndarray, ctype):
    return arr.ctypes.data_as(ctypes.POINTER(ctype))


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(_p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32), _p(out, ctypes.c_uint32))
    return out


def threshold(Delta, V, J, T, nD, nV, nJ) -> int:
    return int(lib().orc_threshold(Delta, V, J, T, nD, nV, nJ))


def charge_target(L: int, n: float, n_charged: int = -1):
    Q = ctypes.c_int64()
    Nc = ctypes.c_int64()
    rc = lib().orc_charge_target(L, n, n_charged, ctypes.byref(Q), ctypes.byref(Nc))
    if rc != 0:
        raise ValueError(f"no valid charge target for L={L} n={n} n_charged={n_charged}")
    return Q.value, Nc.value


def init_codes(L: int, seed: int, n_plus: int, n_minus: int) -> np.ndarray:
    codes = np.zeros(L * L, dtype=np.int8)
    if lib().orc_init(L, seed, n_plus, n_minus, _p(codes, ctypes.c_int8)) != 0:
        raise MemoryError("orc_init failed")
    return codes


def schedule(L: int, seed: int, sweep: int):
    r = ctypes.c_int32()
    dx = np.zeros(4, dtype=np.int32)
    dy = np.zeros(4, dtype=np.int32)
    lib().orc_schedule(L, seed, sweep, ctypes.byref(r), _p(dx, ctypes.c_int32), _p(dy, ctypes.c_int32))
    return r.value, dx, dy


def observables(L: int, codes: np.ndarray) -> np.ndarray:
    assert codes.dtype == np.int8 and codes.size == L * L and codes.flags.c_contiguous
    out = np.zeros(7, dtype=np.int64)
    lib().orc_observables(L, _p(codes, ctypes.c_int8), _p(out, ctypes.c_int64))
    return out


def pair_delta(L: int, codes: np.ndarray, a: int, b: int, ca1: int, cb1: int) -> np.ndarray:
    """(nD, nV, nJ) of moving sites a, b to codes ca1, cb1 (codes unchanged)."""
    out = np.zeros(3, dtype=np.int64)
    lib().orc_pair_delta(L, _p(codes, ctypes.c_int8), a, b, ca1, cb1, _p(out, ctypes.c_int64))
    return out


def pair_config(q: int, j: int):
    """The j-th two-site configuration (code_a, code_b) of the pair-charge-q set, or None."""
    out = (ctypes.c_int * 2)()
    if lib().orc_pair_config(q, j, out) != 0:
        return None
    return int(out[0]), int(out[1])


def energy(Delta, V, J, obs) -> float:
    o = np.ascontiguousarray(obs, dtype=np.int64)
    return float(lib().orc_energy(Delta, V, J, _p(o, ctypes.c_int64)))


@dataclass
class OracleLattice:
    """One lattice advanced by the sequential oracle; mirrors the library's create/sweep/observe."""

    L: int
    n: float
    Delta: float
    V: float
    J: float
    T: float
    seed: int
    n_charged: int = -1
    start_sweep: int = 0
    codes: np.ndarray | None = None

    def __post_init__(self):
        if self.codes is None:
            self.Q, self.Nc = charge_target(self.L, self.n, self.n_charged)
            n_plus = (self.Nc + self.Q) // 2
            n_minus = (self.Nc - self.Q) // 2
            self.codes = init_codes(self.L, self.seed, n_plus, n_minus)
        else:
            self.codes = np.ascontiguousarray(self.codes, dtype=np.int8).reshape(-1).copy()
            o = observables(self.L, self.codes)
            self.Q, self.Nc = int(o[0]), int(o[1])
        self.sweep = self.start_sweep
        self.track = np.zeros(3, dtype=np.int64)

    def sweeps(self, k: int):
        rc = lib().orc_sweeps(self.L, self.Delta, self.V, self.J, self.T, self.seed, self.sweep, k,
                              _p(self.codes, ctypes.c_int8), _p(self.track, ctypes.c_int64))
        if rc != 0:
            raise ValueError("orc_sweeps: L must be a multiple of 4 and >= 4")
        self.sweep += k

    def observables(self) -> np.ndarray:
        return observables(self.L, self.codes)

    def energy(self) -> float:
        return energy(self.Delta, self.V, self.J, self.observables())

    def series(self, every: int, n_obs: int) -> np.ndarray:
        out = np.zeros((n_obs, 7), dtype=np.int64)
        rc = lib().orc_series(self.L, self.Delta, self.V, self.J, self.T, self.seed, self.sweep, every, n_obs,
                              _p(self.codes, ctypes.c_int8), _p(self.track, ctypes.c_int64),
                              _p(out, ctypes.c_int64))
        if rc != 0:
            raise ValueError("orc_series failed")
        self.sweep += every * n_obs
        return out


def general_series(L, Delta, V, J, T, seed, codes, every, n_obs, start_step=0):
    """General-mode (one random pair per step) observation series; codes updated in place."""
    track = np.zeros(3, dtype=np.int64)
    out = np.zeros((n_obs, 7), dtype=np.int64)
    rc = lib().orc_general_series(L, Delta, V, J, T, seed, start_step, every, n_obs,
                                  _p(codes, ctypes.c_int8), _p(track, ctypes.c_int64), _p(out, ctypes.c_int64))
    if rc != 0:
        raise ValueError("orc_general_series failed")
    return out, track


def map_pairs(L: int, nn: bool = False) -> int:
    """Pairs per map: max(1, N // 10) (section 3.2), or max(1, N // 20) for nearest-neighbour maps."""
    return int(lib().orc_nn_map_pairs(L) if nn else lib().orc_map_pairs(L))


def map_build(L: int, seed: int, m: int, nn: bool = False):
    """Map m of the map mode (nn: nearest-neighbour partners): an (n_pairs, 2)
    array of site indices and the number of draws the construction consumed."""
    pairs = np.zeros((map_pairs(L, nn), 2), dtype=np.int64)
    build = lib().orc_nn_map_build if nn else lib().orc_map_build
    k = build(L, seed, m, _p(pairs, ctypes.c_int64))
    if k < 0:
        raise ValueError("map build failed")
    return pairs, int(k)


def map_steps(L, Delta, V, J, T, seed, codes, n_maps, start_map=0, track=None, nn=False):
    """Apply maps start_map .. start_map+n_maps-1 (section 3.2) to codes in place."""
    track = np.zeros(3, dtype=np.int64) if track is None else track
    rc = lib().orc_map_steps_mode(L, Delta, V, J, T, seed, int(nn), start_map, n_maps, _p(codes, ctypes.c_int8),
                                  _p(track, ctypes.c_int64))
    if rc != 0:
        raise ValueError("orc_map_steps failed")
    return track


def map_series(L, Delta, V, J, T, seed, codes, every, n_obs, start_map=0, nn=False):
    """Map-mode observation series (one row every `every` maps); codes updated in place."""
    track = np.zeros(3, dtype=np.int64)
    out = np.zeros((n_obs, 7), dtype=np.int64)
    rc = lib().orc_map_series(L, Delta, V, J, T, seed, int(nn), start_map, every, n_obs,
                              _p(codes, ctypes.c_int8), _p(track, ctypes.c_int64), _p(out, ctypes.c_int64))
    if rc != 0:
        raise ValueError("orc_map_series failed")
    return out, track


def mu_sweeps(L, Delta, V, J, T, seed, codes, n_sweeps, kappa, Q, mu, start_sweep=0, track=None):
    """Penalty-mode sweeps (section 2.2, reading R15) on codes in place.  Returns
    (final mu, mu used in each sweep, sum S after each sweep, track)."""
    track = np.zeros(3, dtype=np.int64) if track is None else track
    mu_c = ctypes.c_double(mu)
    mus = np.zeros(n_sweeps, dtype=np.float64)
    sums = np.zeros(n_sweeps, dtype=np.int64)
    rc = lib().orc_mu_sweeps(L, Delta, V, J, T, seed, start_sweep, n_sweeps, kappa, Q, ctypes.byref(mu_c),
                             _p(codes, ctypes.c_int8), _p(track, ctypes.c_int64), _p(mus, ctypes.c_double),
                             _p(sums, ctypes.c_int64))
    if rc != 0:
        raise ValueError("orc_mu_sweeps failed")
    return mu_c.value, mus, sums, track
