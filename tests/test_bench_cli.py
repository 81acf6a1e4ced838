"""Host-side behaviour of bench.py, CPU only: it refuses more than one GPU,
and the traffic summary scales the phase kernel's FETCH_SIZE / WRITE_SIZE
by what the same counters read for a device copy of known size, and is only
reported while it was taken on the current kernel sources."""
import csv
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert out.returncode == 2
    assert "one GPU" in out.stderr


def _csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, c, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_traffic_summary_scales_by_the_copy(tmp_path, monkeypatch):
    phase = "void lat::(anonymous namespace)::k_phase_2bit<1>(lat::PhaseArgs, int)"
    copy = "__amd_rocclr_copyBuffer"
    # the 256 MiB copy reads 131072 fetch units and 262144 write units: 2048 and 1024 bytes per unit
    _csv(tmp_path / "f.csv", [(phase, "FETCH_SIZE", 100.0), (phase, "FETCH_SIZE", 300.0), ("k_other", "FETCH_SIZE", 9e9)])
    _csv(tmp_path / "w.csv", [(phase, "WRITE_SIZE", 50.0), (phase, "WRITE_SIZE", 50.0)])
    _csv(tmp_path / "cf.csv", [(copy, "FETCH_SIZE", 131072.0)] * 3 + [(copy, "FETCH_SIZE", 3.0)])
    _csv(tmp_path / "cw.csv", [(copy, "WRITE_SIZE", 262144.0)] * 3 + [(copy, "WRITE_SIZE", 2.0)])
    out = tmp_path / "traffic.txt"
    bench.write_traffic_summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "cf.csv"),
                                str(tmp_path / "cw.csv"), out=str(out))
    vals = dict(line.split("=", 1) for line in out.read_text().splitlines() if "=" in line and not line.startswith("#"))
    assert int(vals["fetch_bytes_per_launch"]) == 200 * 2048
    assert int(vals["write_bytes_per_launch"]) == 50 * 1024
    assert vals["phase_sources_sha256"] == bench.kernel_source_digest()

    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(out))
    assert bench.measured_traffic() == 200 * 2048 + 50 * 1024
    out.write_text(out.read_text().replace(bench.kernel_source_digest(), "0" * 64))
    assert bench.measured_traffic() is None


def test_valu_summary_is_keyed_to_the_kernel_sources(tmp_path, monkeypatch):
    phase = "void lat::(anonymous namespace)::k_phase_2bit<1>(lat::PhaseArgs, int)"
    _csv(tmp_path / "v.csv", [(phase, "SQ_INSTS_VALU", 7.0e6), (phase, "SQ_INSTS_VALU", 7.2e6),
                              ("k_obs_2bit", "SQ_INSTS_VALU", 1.0)])
    out = tmp_path / "valu.txt"
    bench.write_valu_summary(str(tmp_path / "v.csv"), out=str(out))
    monkeypatch.setattr(bench, "VALU_SUMMARY", str(out))
    assert bench.measured_valu_insts() == 7.1e6
    out.write_text(out.read_text().replace(bench.kernel_source_digest(), "0" * 64))
    assert bench.measured_valu_insts() is None
