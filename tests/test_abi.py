"""The C-ABI library loads on the CPU, exports every symbol include/lattice.h
declares, and its host-side logic (charge target, argument checks) agrees
with the oracle and the header.  No GPU call is made here."""
import ctypes
import os
import re

import pytest

import oracle
import paper_2301_11735_amd as lat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lattice.h")

pytestmark = pytest.mark.skipif(not os.path.exists(lat.LIB_PATH), reason="liblattice.so not built")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:lattice|lat_server)_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    assert _declared_functions() == sorted(lat.EXPORTS)


def test_library_exports_every_declared_symbol():
    dll = ctypes.CDLL(lat.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(dll, name), name


def test_state_and_scratch_sizes():
    assert lat.state_bytes(32, lat.ENC_INT8) == 1024
    assert lat.state_bytes(8192, lat.ENC_2BIT) == 8192 * 8192 // 4
    assert lat.state_bytes(30, lat.ENC_INT8) == 0
    assert lat.state_bytes(96, lat.ENC_2BIT) == 0      # 2-bit needs L % 64 == 0
    assert lat.state_bytes(2, lat.ENC_INT8) == 0
    assert lat.scratch_bytes(32, lat.ENC_INT8) >= 933 * 8 + 96 * 8 + 80  # device tables + tracker + sums


@pytest.mark.parametrize("L,n,nc", [(32, 0.1, -1), (1024, 0.05, -1), (8192, 0.1, -1), (128, 0.3, -1),
                                    (4, -0.125, -1), (64, 0.0, 0), (12, 0.37, -1), (16, 0.01, 7)])
def test_charge_target_matches_oracle(L, n, nc):
    try:
        want = oracle.charge_target(L, n, nc)
    except ValueError:
        with pytest.raises(lat.LatticeError):
            lat.charge_target(L, n, nc)
        return
    assert lat.charge_target(L, n, nc) == want


def _create_rc(**kw):
    p = lat.LatParams(L=32, encoding=0, n=0.1, Delta=0.25, V=0.5, J=1.0, T=0.8, seed=1, n_charged=-1,
                      start_sweep=0, init_codes=None)
    for k, v in kw.items():
        setattr(p, k, v)
    h = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(1)  # never dereferenced: validation fails first
    rc = lat.lib().lattice_create(ctypes.byref(p), ctypes.addressof(buf), 1 << 40, ctypes.addressof(buf),
                                  1 << 40, None, ctypes.byref(h))
    return rc, lat.lib().lattice_last_error().decode(), h.value


@pytest.mark.parametrize("kw", [dict(L=30), dict(L=0), dict(L=96, encoding=1), dict(encoding=7),
                                dict(T=0.0), dict(T=-1.0), dict(Delta=float("inf")), dict(J=float("nan")),
                                dict(n=1.5), dict(n=0.5, n_charged=4), dict(n_charged=2000)])
def test_create_rejects_invalid_arguments_before_touching_memory(kw):
    rc, msg, h = _create_rc(**kw)
    assert rc == lat.LAT_EINVAL and msg and h is None


def test_create_rejects_small_buffers():
    p = lat.LatParams(L=32, encoding=0, n=0.1, Delta=0.25, V=0.5, J=1.0, T=0.8, seed=1, n_charged=-1,
                      start_sweep=0, init_codes=None)
    h = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(1)
    rc = lat.lib().lattice_create(ctypes.byref(p), ctypes.addressof(buf), 1023, ctypes.addressof(buf), 1 << 20,
                                  None, ctypes.byref(h))
    assert rc == lat.LAT_ENOMEM
    rc = lat.lib().lattice_create(ctypes.byref(p), ctypes.addressof(buf), 1024, ctypes.addressof(buf), 100,
                                  None, ctypes.byref(h))
    assert rc == lat.LAT_ENOMEM


def test_calls_on_null_handles_fail_cleanly():
    L = lat.lib()
    assert L.lattice_sweep(None, 1) == lat.LAT_ESTATE
    assert L.lattice_destroy(None) == lat.LAT_ESTATE
    assert L.lattice_observables(None, ctypes.byref(lat.LatObs())) == lat.LAT_ESTATE
    assert L.lattice_sweep_batch(None, 1, 1, None) == lat.LAT_EINVAL
    assert L.lattice_sweep_batch(None, 0, 1, None) == lat.LAT_OK


def test_batch_graph_rejects_bad_arguments_without_a_device():
    L = lat.lib()
    vp = ctypes.c_void_p
    h = vp()
    d = ctypes.c_void_p(16)  # never dereferenced: every call below fails before any device work
    assert L.lattice_batch_graph_create(None, 1, 1, 1, None, 80, None, None) == lat.LAT_EINVAL
    assert L.lattice_batch_graph_create(None, 0, 1, 1, None, 80, None, ctypes.byref(h)) == lat.LAT_EINVAL
    assert h.value is None
    fake = (vp * 1)(None)
    assert L.lattice_batch_graph_create(fake, 1, 0, 1, d, 80, None, ctypes.byref(h)) == lat.LAT_EINVAL
    assert L.lattice_batch_graph_create(fake, 1, 5, 0, d, 80, None, ctypes.byref(h)) == lat.LAT_EINVAL
    assert L.lattice_batch_graph_create(fake, 1, 5, 1, d, 79, None, ctypes.byref(h)) == lat.LAT_ENOMEM
    assert L.lattice_batch_graph_create(fake, 1, 5, 3, d, 239, None, ctypes.byref(h)) == lat.LAT_ENOMEM
    assert L.lattice_batch_graph_create(fake, 1, 5, 3, d, 240, None, ctypes.byref(h)) == lat.LAT_ESTATE
    assert L.lattice_batch_graph_launch(None, 1) == lat.LAT_ESTATE
    assert L.lattice_batch_graph_read(None, ctypes.byref(lat.LatObs())) == lat.LAT_ESTATE
    assert L.lattice_batch_graph_destroy(None) == lat.LAT_ESTATE


def test_map_calls_on_null_handles_fail_cleanly():
    L = lat.lib()
    assert L.lattice_map_steps(None, 0, 1, 0) == lat.LAT_ESTATE
    assert L.lattice_map_steps_batch(None, 1, 0, 1, 0, None) == lat.LAT_EINVAL
    assert L.lattice_map_steps_batch(None, 0, 0, 1, 0, None) == lat.LAT_OK
    assert L.lattice_map_steps_batch(None, 0, 0, 1, 7, None) == lat.LAT_EINVAL
    fake = (ctypes.c_void_p * 1)(None)
    assert L.lattice_map_steps_batch(fake, 1, 0, 1, 1, None) == lat.LAT_ESTATE


def test_penalty_calls_on_null_handles_fail_cleanly():
    L = lat.lib()
    mu = ctypes.c_double(0.0)
    assert L.lattice_mu_sweeps(None, 0, 1, 0.5, ctypes.byref(mu), None, None) == lat.LAT_ESTATE


def _server_without_device():
    """A server whose pool pointer is never dereferenced: submit only queues."""
    h = ctypes.c_void_p()
    rc = lat.lib().lat_server_create(ctypes.c_void_p(1 << 20), 1 << 20, 4, 1 << 16, None, ctypes.byref(h))
    assert rc == lat.LAT_OK
    return h


@pytest.mark.parametrize("kw", [dict(n=1.5), dict(Delta=float("nan")), dict(V=float("inf")), dict(T=0.0),
                                dict(n=0.5, n_charged=4), dict(n_charged=64 * 64 + 2), dict(L=96),
                                dict(L=1024)])
def test_server_refuses_a_request_that_could_never_be_admitted(kw):
    """Bad parameters are refused at submit (LAT_EINVAL), so that they never
    reach admission, where they would block the queue; good requests before
    and after them still queue."""
    srv = _server_without_device()
    good = lat.LatParams(L=64, encoding=1, n=0.1, Delta=0.25, V=0.5, J=1.0, T=0.8, seed=1, n_charged=-1,
                         start_sweep=0, init_codes=None)
    rid = ctypes.c_uint64()
    assert lat.lib().lat_server_submit(srv, ctypes.byref(good), 10, 0, ctypes.byref(rid)) == lat.LAT_OK
    bad = lat.LatParams(L=64, encoding=1, n=0.1, Delta=0.25, V=0.5, J=1.0, T=0.8, seed=2, n_charged=-1,
                        start_sweep=0, init_codes=None)
    for k, v in kw.items():
        setattr(bad, k, v)
    assert lat.lib().lat_server_submit(srv, ctypes.byref(bad), 10, 0, ctypes.byref(rid)) == lat.LAT_EINVAL
    assert lat.lib().lattice_last_error().decode()
    assert lat.lib().lat_server_submit(srv, ctypes.byref(good), 10, 0, ctypes.byref(rid)) == lat.LAT_OK
    st = lat.LatServerStats()
    assert lat.lib().lat_server_stats(srv, ctypes.byref(st)) == lat.LAT_OK
    assert st.queued == 2


def test_server_refuses_init_codes_outside_the_code_range():
    srv = _server_without_device()
    codes = (ctypes.c_int8 * (64 * 64))(*([0] * (64 * 64 - 1) + [5]))
    p = lat.LatParams(L=64, encoding=1, n=0.0, Delta=0.25, V=0.5, J=1.0, T=0.8, seed=1, n_charged=-1,
                      start_sweep=0, init_codes=ctypes.cast(codes, ctypes.POINTER(ctypes.c_int8)))
    rid = ctypes.c_uint64()
    assert lat.lib().lat_server_submit(srv, ctypes.byref(p), 10, 0, ctypes.byref(rid)) == lat.LAT_EINVAL


_ENOMEM_CHILD = r"""
import ctypes, resource, sys
sys.path.insert(0, {root!r})
import paper_2301_11735_amd as lat
L = lat.lib()
limit = 3 << 30
resource.setrlimit(resource.RLIMIT_AS, (limit, limit))
p = lat.LatParams(L=16384, encoding=1, n=0.1, Delta=0.25, V=0.5, J=1.0, T=0.8, seed=1, n_charged=-1,
                  start_sweep=0, init_codes=None)
h = ctypes.c_void_p()
rc = L.lattice_create(ctypes.byref(p), ctypes.c_void_p(1 << 20), 1 << 40, ctypes.c_void_p(1 << 20), 1 << 40, None,
                      ctypes.byref(h))
print(rc, L.lattice_last_error().decode(), h.value, flush=True)
"""


def test_host_memory_exhaustion_is_an_error_code_not_an_abort():
    """The seeded init of an L=16384 lattice needs about 4.6 GB of host
    memory; under a 3 GiB address-space limit the allocation fails before any
    device call, and the C-ABI returns LAT_ENOMEM instead of letting the C++
    exception terminate the caller."""
    import subprocess
    import sys

    out = subprocess.run([sys.executable, "-c", _ENOMEM_CHILD.format(root=ROOT)], capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    rc, rest = out.stdout.split(" ", 1)
    assert int(rc) == lat.LAT_ENOMEM, out.stdout
    assert "out of host memory" in rest and rest.strip().endswith("None")
