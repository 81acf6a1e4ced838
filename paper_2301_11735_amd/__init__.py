"""Python binding of liblattice.so (include/lattice.h): the coupled-pair
Metropolis sweep with an exact charge constraint (arXiv:2301.11735) on MI355X.

Argument marshalling only.  Every step of a sweep runs in the library's HIP
kernels; PyTorch supplies the device buffers and the stream.  There is no CPU
fallback: without the built library, or without a GPU, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblattice.so")

LAT_OK, LAT_EINVAL, LAT_ENOMEM, LAT_EHIP, LAT_ESTATE = 0, -1, -2, -3, -4
ENC_INT8, ENC_2BIT = 0, 1

EXPORTS = (
    "lattice_state_bytes",
    "lattice_scratch_bytes",
    "lattice_charge_target",
    "lattice_create",
    "lattice_sweep",
    "lattice_observables",
    "lattice_read_state",
    "lattice_sweep_series",
    "lattice_series_read",
    "lattice_sweep_batch",
    "lattice_observables_batch",
    "lattice_observables_batch_noalloc",
    "lattice_batch_graph_create",
    "lattice_batch_graph_launch",
    "lattice_batch_graph_read",
    "lattice_batch_graph_destroy",
    "lattice_map_steps",
    "lattice_map_steps_batch",
    "lattice_mu_sweeps",
    "lattice_destroy",
    "lattice_last_error",
    "lat_server_create",
    "lat_server_submit",
    "lat_server_step",
    "lat_server_poll",
    "lat_server_release",
    "lat_server_stats",
    "lat_server_destroy",
)
REQ_QUEUED, REQ_RESIDENT, REQ_FINISHED, REQ_FAILED = 0, 1, 2, 3
MAP_ANY, MAP_NEIGHBOUR = 0, 1


class LatParams(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32),
        ("encoding", ctypes.c_int32),
        ("n", ctypes.c_double),
        ("Delta", ctypes.c_double),
        ("V", ctypes.c_double),
        ("J", ctypes.c_double),
        ("T", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("n_charged", ctypes.c_int64),
        ("start_sweep", ctypes.c_uint64),
        ("init_codes", ctypes.POINTER(ctypes.c_int8)),
    ]


class LatObs(ctypes.Structure):
    _fields_ = [
        ("sweep", ctypes.c_uint64),
        ("sum_S", ctypes.c_int64),
        ("n_charged", ctypes.c_int64),
        ("bond_SS", ctypes.c_int64),
        ("bond_ss", ctypes.c_int64),
        ("M", ctypes.c_int64),
        ("M_stag", ctypes.c_int64),
        ("C_stag", ctypes.c_int64),
        ("track_nD", ctypes.c_int64),
        ("track_nV", ctypes.c_int64),
        ("track_nJ", ctypes.c_int64),
        ("E", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}

    def ints(self) -> list:
        """(sum_S, n_charged, bond_SS, bond_ss, M, M_stag, C_stag) in the oracle's order."""
        return [self.sum_S, self.n_charged, self.bond_SS, self.bond_ss, self.M, self.M_stag, self.C_stag]


class LatRequestInfo(ctypes.Structure):
    _fields_ = [
        ("id", ctypes.c_uint64),
        ("status", ctypes.c_int32),
        ("error", ctypes.c_int32),
        ("sweeps_total", ctypes.c_uint32),
        ("sweeps_done", ctypes.c_uint32),
        ("t_submit", ctypes.c_double),
        ("t_admit", ctypes.c_double),
        ("t_finish", ctypes.c_double),
        ("obs", LatObs),
    ]


class LatServerStats(ctypes.Structure):
    _fields_ = [
        ("queued", ctypes.c_int32),
        ("resident", ctypes.c_int32),
        ("pool_used", ctypes.c_uint64),
        ("steps", ctypes.c_uint64),
        ("site_updates", ctypes.c_uint64),
    ]


class LatticeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"liblattice error {code}: {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Load liblattice.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2301_11735_amd/build.py")
        # torch first: the library then binds to the HIP runtime torch has
        # loaded, so that one runtime serves both in this process
        import torch  # noqa: F401

        L = ctypes.CDLL(LIB_PATH)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        L.lattice_state_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
        L.lattice_state_bytes.restype = sz
        L.lattice_scratch_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
        L.lattice_scratch_bytes.restype = sz
        L.lattice_charge_target.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_int64,
                                            ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.lattice_charge_target.restype = ctypes.c_int
        L.lattice_create.argtypes = [ctypes.POINTER(LatParams), vp, sz, vp, sz, vp, ctypes.POINTER(vp)]
        L.lattice_create.restype = ctypes.c_int
        L.lattice_sweep.argtypes = [vp, ctypes.c_uint32]
        L.lattice_sweep.restype = ctypes.c_int
        L.lattice_observables.argtypes = [vp, ctypes.POINTER(LatObs)]
        L.lattice_observables.restype = ctypes.c_int
        L.lattice_read_state.argtypes = [vp, ctypes.POINTER(ctypes.c_int8)]
        L.lattice_read_state.restype = ctypes.c_int
        L.lattice_sweep_series.argtypes = [vp, ctypes.c_uint32, ctypes.c_uint32, vp, sz]
        L.lattice_sweep_series.restype = ctypes.c_int
        L.lattice_series_read.argtypes = [vp, vp, ctypes.c_uint32, ctypes.POINTER(LatObs)]
        L.lattice_series_read.restype = ctypes.c_int
        L.lattice_sweep_batch.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.c_uint32, vp]
        L.lattice_sweep_batch.restype = ctypes.c_int
        L.lattice_observables_batch.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, vp, sz, ctypes.POINTER(LatObs), vp]
        L.lattice_observables_batch.restype = ctypes.c_int
        L.lattice_observables_batch_noalloc.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(LatObs), vp]
        L.lattice_observables_batch_noalloc.restype = ctypes.c_int
        L.lattice_batch_graph_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint32,
                                                 vp, sz, vp, ctypes.POINTER(vp)]
        L.lattice_batch_graph_create.restype = ctypes.c_int
        L.lattice_batch_graph_launch.argtypes = [vp, ctypes.c_uint32]
        L.lattice_batch_graph_launch.restype = ctypes.c_int
        L.lattice_batch_graph_read.argtypes = [vp, ctypes.POINTER(LatObs)]
        L.lattice_batch_graph_read.restype = ctypes.c_int
        L.lattice_batch_graph_destroy.argtypes = [vp]
        L.lattice_batch_graph_destroy.restype = ctypes.c_int
        L.lattice_map_steps.argtypes = [vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32]
        L.lattice_map_steps.restype = ctypes.c_int
        L.lattice_map_steps_batch.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint32,
                                              ctypes.c_int32, vp]
        L.lattice_map_steps_batch.restype = ctypes.c_int
        dp = ctypes.POINTER(ctypes.c_double)
        L.lattice_mu_sweeps.argtypes = [vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double, dp, dp,
                                        ctypes.POINTER(ctypes.c_int64)]
        L.lattice_mu_sweeps.restype = ctypes.c_int
        L.lattice_destroy.argtypes = [vp]
        L.lattice_destroy.restype = ctypes.c_int
        L.lat_server_create.argtypes = [vp, sz, ctypes.c_int32, ctypes.c_uint64, vp, ctypes.POINTER(vp)]
        L.lat_server_create.restype = ctypes.c_int
        L.lat_server_submit.argtypes = [vp, ctypes.POINTER(LatParams), ctypes.c_uint32, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_uint64)]
        L.lat_server_submit.restype = ctypes.c_int
        L.lat_server_step.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
        L.lat_server_step.restype = ctypes.c_int
        L.lat_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(LatRequestInfo), ctypes.POINTER(ctypes.c_int8)]
        L.lat_server_poll.restype = ctypes.c_int
        L.lat_server_release.argtypes = [vp, ctypes.c_uint64]
        L.lat_server_release.restype = ctypes.c_int
        L.lat_server_stats.argtypes = [vp, ctypes.POINTER(LatServerStats)]
        L.lat_server_stats.restype = ctypes.c_int
        L.lat_server_destroy.argtypes = [vp]
        L.lat_server_destroy.restype = ctypes.c_int
        L.lattice_last_error.argtypes = []
        L.lattice_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != LAT_OK:
        raise LatticeError(rc, lib().lattice_last_error().decode())


def state_bytes(L: int, encoding: int) -> int:
    return int(lib().lattice_state_bytes(L, encoding))


def scratch_bytes(L: int, encoding: int) -> int:
    return int(lib().lattice_scratch_bytes(L, encoding))


def charge_target(L: int, n: float, n_charged: int = -1):
    Q, Nc = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().lattice_charge_target(L, n, n_charged, ctypes.byref(Q), ctypes.byref(Nc)))
    return Q.value, Nc.value


def _stream_handle(stream) -> int:
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class Lattice:
    """One lattice on the GPU.  Buffers are torch uint8 tensors owned here;
    the library borrows them until destroy()."""

    def __init__(self, L: int, n: float, Delta: float, V: float, J: float, T: float, seed: int,
                 encoding: int = ENC_INT8, n_charged: int = -1, start_sweep: int = 0, init_codes=None,
                 device: str = "cuda", stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("a ROCm GPU is required (torch.cuda.is_available() is False)")
        self.L, self.encoding = L, encoding
        self.params = dict(L=L, n=n, Delta=Delta, V=V, J=J, T=T, seed=seed, encoding=encoding,
                           n_charged=n_charged, start_sweep=start_sweep)
        sb = state_bytes(L, encoding)
        if sb == 0:
            raise ValueError(f"L={L} is not valid for encoding {encoding}")
        self.state = torch.empty(sb, dtype=torch.uint8, device=device)
        self.scratch = torch.empty(scratch_bytes(L, encoding), dtype=torch.uint8, device=device)
        self.stream = stream
        p = LatParams(L=L, encoding=encoding, n=n, Delta=Delta, V=V, J=J, T=T, seed=seed, n_charged=n_charged,
                      start_sweep=start_sweep, init_codes=None)
        self._init = None
        if init_codes is not None:
            self._init = np.ascontiguousarray(init_codes, dtype=np.int8).reshape(-1)
            if self._init.size != L * L:
                raise ValueError("init_codes must hold L*L codes")
            p.init_codes = self._init.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
        h = ctypes.c_void_p()
        _check(lib().lattice_create(ctypes.byref(p), self.state.data_ptr(), self.state.numel(),
                                    self.scratch.data_ptr(), self.scratch.numel(), _stream_handle(stream),
                                    ctypes.byref(h)))
        self._h = h

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise LatticeError(LAT_ESTATE, "lattice destroyed")
        return self._h

    def sweep(self, sweeps: int = 1):
        _check(lib().lattice_sweep(self.handle, sweeps))

    def mu_sweeps(self, first_sweep: int, n_sweeps: int, kappa: float, mu: float):
        """Penalty-mode sweeps (the prior method of section 2.2).  Returns (next mu,
        mu of each sweep, sum S after each sweep)."""
        m = ctypes.c_double(mu)
        mus = np.zeros(n_sweeps, dtype=np.float64)
        sums = np.zeros(n_sweeps, dtype=np.int64)
        _check(lib().lattice_mu_sweeps(self.handle, first_sweep, n_sweeps, kappa, ctypes.byref(m),
                                       mus.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       sums.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return m.value, mus, sums

    def map_steps(self, first_map: int, n_maps: int = 1, partner: int = 0):
        """Apply maps first_map .. first_map+n_maps-1 of the map mode (partner MAP_ANY or MAP_NEIGHBOUR)."""
        _check(lib().lattice_map_steps(self.handle, first_map, n_maps, partner))

    def sweep_series(self, intervals: int, every: int = 1, read: bool = True):
        """`intervals` times: `every` sweeps, then the observables into a device
        record (no host synchronisation between intervals).  Returns the
        records as a list of LatObs (read=True), else the device buffer for
        read_series()."""
        import torch

        buf = torch.empty(88 * max(1, intervals), dtype=torch.uint8, device=self.state.device)
        _check(lib().lattice_sweep_series(self.handle, intervals, every, buf.data_ptr(), buf.numel()))
        return self.read_series(buf, intervals) if read else buf

    def read_series(self, buf, intervals: int, as_array: bool = False):
        """The records of a device series as a list of LatObs, or (as_array)
        as a numpy structured array over the same memory (no per-record
        Python objects)."""
        out = (LatObs * max(1, intervals))()
        _check(lib().lattice_series_read(self.handle, buf.data_ptr(), intervals, out))
        if as_array:
            return np.frombuffer(out, dtype=_obs_dtype(), count=intervals)
        return list(out)[:intervals]

    def observables(self) -> LatObs:
        o = LatObs()
        _check(lib().lattice_observables(self.handle, ctypes.byref(o)))
        return o

    def read_state(self) -> np.ndarray:
        out = np.empty(self.L * self.L, dtype=np.int8)
        _check(lib().lattice_read_state(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))))
        return out

    def destroy(self):
        if self._h is not None:
            _check(lib().lattice_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _handles(lattices):
    return (ctypes.c_void_p * len(lattices))(*[lat.handle.value for lat in lattices])


def map_steps_batch(lattices, first_map: int, n_maps: int, partner: int = 0, stream=None):
    """Apply maps first_map .. first_map+n_maps-1 (map mode; partner MAP_ANY or
    MAP_NEIGHBOUR) to several lattices in one call."""
    _check(lib().lattice_map_steps_batch(_handles(lattices), len(lattices), first_map, n_maps, partner,
                                         _stream_handle(stream)))


def sweep_batch(lattices, sweeps: int, stream=None):
    """Advance several lattices by `sweeps` sweeps each in one call."""
    _check(lib().lattice_sweep_batch(_handles(lattices), len(lattices), sweeps, _stream_handle(stream)))


_OBS_DTYPE = None


def _obs_dtype():
    """numpy dtype of LatObs, built once (record arrays are views of the
    library's output with it)."""
    global _OBS_DTYPE
    if _OBS_DTYPE is None:
        _OBS_DTYPE = np.dtype(LatObs)
    return _OBS_DTYPE


class BatchObservables:
    """Reusable device output buffer for observables_batch()."""

    def __init__(self, capacity: int, device: str = "cuda"):
        import torch

        self.capacity = capacity
        self.buf = torch.empty(80 * max(1, capacity), dtype=torch.uint8, device=device)

    def _read(self, lattices, stream):
        n = len(lattices)
        if n > self.capacity:
            raise ValueError("more lattices than the buffer holds")
        out = (LatObs * max(1, n))()
        _check(lib().lattice_observables_batch(_handles(lattices), n, self.buf.data_ptr(), self.buf.numel(), out,
                                               _stream_handle(stream)))
        return out, n

    def __call__(self, lattices, stream=None) -> list:
        out, n = self._read(lattices, stream)
        return list(out)[:n]

    def array(self, lattices, stream=None):
        """The same records as a numpy structured array (no per-record
        Python objects)."""
        out, n = self._read(lattices, stream)
        return np.frombuffer(out, dtype=_obs_dtype(), count=n)


def observables_batch_noalloc(lattices, stream=None) -> list:
    """Observables of up to 1024 lattices (as BatchObservables) with the
    library's static device staging: no device buffer is allocated."""
    n = len(lattices)
    out = (LatObs * max(1, n))()
    _check(lib().lattice_observables_batch_noalloc(_handles(lattices), n, out, _stream_handle(stream)))
    return list(out)[:n]


class BatchGraph:
    """`intervals` observation intervals of a batch (each: `sweeps` sweeps of
    every lattice, then their observables) captured into one HIP graph;
    launch() replays it, read() returns the observables of the last replay as
    a list of `intervals` lists (one record per lattice)."""

    def __init__(self, lattices, sweeps: int, intervals: int = 1, stream=None, device: str = "cuda"):
        import torch

        self._lats = list(lattices)  # keep the lattices (and their buffers) alive
        self.intervals = intervals
        self.buf = torch.empty(80 * max(1, len(self._lats)) * intervals, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        _check(lib().lattice_batch_graph_create(_handles(self._lats), len(self._lats), sweeps, intervals,
                                                self.buf.data_ptr(), self.buf.numel(), _stream_handle(stream),
                                                ctypes.byref(h)))
        self._h = h

    def launch(self, times: int = 1):
        _check(lib().lattice_batch_graph_launch(self._h, times))

    def read(self) -> list:
        n = len(self._lats)
        out = (LatObs * (n * self.intervals))()
        _check(lib().lattice_batch_graph_read(self._h, out))
        flat = list(out)
        return [flat[k * n:(k + 1) * n] for k in range(self.intervals)]

    def read_array(self):
        """The same records as a numpy structured array of shape (intervals, lattices)."""
        n = len(self._lats)
        out = (LatObs * (n * self.intervals))()
        _check(lib().lattice_batch_graph_read(self._h, out))
        return np.frombuffer(out, dtype=_obs_dtype(), count=n * self.intervals).reshape(self.intervals, n)

    def destroy(self):
        if self._h:
            _check(lib().lattice_batch_graph_destroy(self._h))
            self._h = None


class Server:
    """Continuous-batching request server (lat_server_*) over a torch-owned
    device pool of `pool_bytes`."""

    def __init__(self, pool_bytes: int, max_slots: int = 256, quantum_updates: int = 1 << 22, device: str = "cuda",
                 stream=None):
        import torch

        self.pool = torch.empty(pool_bytes, dtype=torch.uint8, device=device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib().lat_server_create(self.pool.data_ptr(), pool_bytes, max_slots, quantum_updates,
                                       _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self._sizes = {}

    def submit(self, L, n, Delta, V, J, T, seed, sweeps, encoding=ENC_2BIT, n_charged=-1, keep_state=False) -> int:
        p = LatParams(L=L, encoding=encoding, n=n, Delta=Delta, V=V, J=J, T=T, seed=seed, n_charged=n_charged,
                      start_sweep=0, init_codes=None)
        rid = ctypes.c_uint64()
        _check(lib().lat_server_submit(self._h, ctypes.byref(p), sweeps, int(keep_state), ctypes.byref(rid)))
        self._sizes[rid.value] = L * L
        return rid.value

    def step(self) -> int:
        n = ctypes.c_int32()
        _check(lib().lat_server_step(self._h, ctypes.byref(n)))
        return n.value

    def poll(self, rid: int, with_state: bool = False):
        info = LatRequestInfo()
        codes = None
        ptr = None
        if with_state:
            codes = np.empty(self._sizes[rid], dtype=np.int8)
            ptr = codes.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
        _check(lib().lat_server_poll(self._h, rid, ctypes.byref(info), ptr))
        return (info, codes) if with_state else info

    def release(self, rid: int):
        _check(lib().lat_server_release(self._h, rid))
        self._sizes.pop(rid, None)

    def stats(self) -> LatServerStats:
        st = LatServerStats()
        _check(lib().lat_server_stats(self._h, ctypes.byref(st)))
        return st

    def destroy(self):
        if self._h is not None:
            _check(lib().lat_server_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
