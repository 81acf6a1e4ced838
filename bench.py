"""Benchmark: site updates/s of the coupled-pair Metropolis sweep on the large
single lattice (L = 8192, 67M sites, 2-bit states) on one MI355X.

One step = one observation interval of the workload: 50 sweeps (4 phase
launches each) followed by the grid-wide observable reduction.  The lattice is
created (init, threshold table) before the timed region, so its inputs are
resident in HBM when timing starts.

The same line also carries the single mid lattice (L = 1024 int8, observables
after every sweep), the batched workload (256 lattices of L = 128,
lattices/s) and the served stream (Poisson arrivals, p50/p99
time-to-result), the other parts of the metric.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-batched] [--no-mid] [--serve-seconds S]
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads  # noqa: E402

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 full-rate 32-bit
# integer VALU lane-operations per second; 1024 SIMDs issue one wave64 VALU
# instruction per 4 cycles each.
VALU_PEAK_OPS = 256 * 64 * 2.4e9
N_SIMD, CLOCK_HZ = 1024, 2.4e9
HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes per site update at 2 bits per site: the state read and
# written once, 0.5 B (the roofline's per-unit figure).
BYTES_PER_SITE_UPDATE_2BIT = 0.5
# The RNG floor of the method's integer work: half a Philox4x32-10 call per
# pair, i.e. a quarter call per site update; a call is 10 rounds of two
# 32x32->64 multiplies and two three-input xors, all full-rate on gfx950, so
# 40 lane-ops per call.  Reported only as a lower bound on ALU use.
PHILOX_OPS_PER_SITE_UPDATE = 10.0
# LDS bytes per site update in the phase kernel: per pair one 16-byte
# transition entry and one 8-byte threshold entry (12 B per update), and the
# b-word exchange, a 4-byte write and a 4-byte read per thread for its 32
# updates (0.25 B).  The tables' staging (9 KB per block, about 2% more at
# L = 8192) is left out.  Peak: 128 B per clock per CU x 256 CUs x 2.4 GHz.
LDS_BYTES_PER_SITE_UPDATE = 12.25
LDS_PEAK_GBS = 128 * 256 * 2.4


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_phase_2bit_L8192_traffic.txt")
VALU_SUMMARY = os.path.join(ROOT, "profiles", "k_phase_2bit_L8192_valu.txt")


PHASE_KERNEL_SOURCES = ("phase.hip", "device_common.h", "kernels.h", "philox.h")


def kernel_source_digest() -> str:
    """SHA-256 over the sources the phase kernel is compiled from."""
    import hashlib

    h = hashlib.sha256()
    for name in PHASE_KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2301_11735_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def _summary_values(path):
    """key = value lines of a committed counter summary, or None if it is
    missing or was taken on another phase-kernel source."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("phase_sources_sha256") != kernel_source_digest():
        return None
    return vals


def measured_traffic():
    """HBM bytes per phase launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, or None if it was taken on another kernel source."""
    vals = _summary_values(TRAFFIC_SUMMARY)
    try:
        return float(vals["fetch_bytes_per_launch"]) + float(vals["write_bytes_per_launch"])
    except (TypeError, KeyError, ValueError):
        return None


def measured_valu_insts():
    """VALU wave-instructions per phase launch (rocprofv3 SQ_INSTS_VALU) from
    the committed summary, or None if it was taken on another kernel source."""
    vals = _summary_values(VALU_SUMMARY)
    try:
        return float(vals["valu_insts_per_launch"])
    except (TypeError, KeyError, ValueError):
        return None


def write_valu_summary(csv_path, out=VALU_SUMMARY):
    """Mean SQ_INSTS_VALU of the L=8192 phase kernel per dispatch, keyed to
    the digest of its sources."""
    import statistics

    v = [x for k, x in _counter_rows(csv_path) if "k_phase_2bit" in k]
    n_updates = workloads.LARGE.L ** 2 / 4
    lines = [
        "# VALU wave-instructions of k_phase_2bit at L=8192 (one phase launch updates N/4 = 16.8M sites)",
        "# counter: rocprofv3 --pmc SQ_INSTS_VALU on",
        "#   python3 bench.py --steps 4 --warmup 1 --no-cpu-baseline --no-batched --no-mid --no-maps --no-penalty"
        " --serve-seconds 0",
        "# written by: python3 bench.py --valu-summary <counter csv>",
        f"# phase dispatches: {len(v)}; mean {statistics.mean(v):.1f} min {min(v):.1f} max {max(v):.1f}",
        f"# lane-ops per site update (x64 lanes / N/4): {statistics.mean(v) * 64 / n_updates:.2f}",
        f"# phase_sources_sha256 covers csrc/{', csrc/'.join(PHASE_KERNEL_SOURCES)}",
        f"phase_sources_sha256={kernel_source_digest()}",
        f"valu_insts_per_launch={statistics.mean(v):.0f}",
    ]
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _counter_rows(path):
    import csv

    return [(r["Kernel_Name"], float(r["Counter_Value"])) for r in csv.DictReader(open(path))]


def write_traffic_summary(fetch_csv, write_csv, cfetch_csv, cwrite_csv, out=TRAFFIC_SUMMARY):
    """Scale the phase kernel's FETCH_SIZE / WRITE_SIZE (KiB-like units per
    dispatch) by what the same counters read for a device copy of a known
    size, and write bytes per launch with the digest of the kernel source."""
    import statistics

    copy_bytes = 256 << 20

    def per_dispatch(path, name):
        return [v for k, v in _counter_rows(path) if name in k]

    def copy_factor(path):
        # the three largest copyBuffer dispatches are the 256 MiB copies
        vals = sorted(per_dispatch(path, "copyBuffer"))[-3:]
        return copy_bytes / statistics.median(vals)

    f = per_dispatch(fetch_csv, "k_phase_2bit")
    w = per_dispatch(write_csv, "k_phase_2bit")
    ff, fw = copy_factor(cfetch_csv), copy_factor(cwrite_csv)
    fetch_b, write_b = statistics.mean(f) * ff, statistics.mean(w) * fw
    lines = [
        "# HBM-side traffic of k_phase_2bit at L=8192 (one phase launch updates N/4 = 16.8M sites)",
        "# counters: rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE, one pass each, on",
        "#   python3 bench.py --steps 4 --warmup 1 --no-cpu-baseline --no-batched --serve-seconds 0",
        "# calibration: the same counters on python3 bench.py --calibrate-copy-mib 256 (a 268435456-byte",
        "#   device copy reads and writes that many bytes); factor = bytes / counter value",
        "# written by: python3 bench.py --traffic-summary <fetch csv> <write csv> <copy fetch csv> <copy write csv>",
        f"# phase dispatches: fetch {len(f)}, write {len(w)}",
        f"# FETCH_SIZE mean {statistics.mean(f):.1f} min {min(f):.1f} max {max(f):.1f}; copy factor {ff:.4f}",
        f"# WRITE_SIZE mean {statistics.mean(w):.1f} min {min(w):.1f} max {max(w):.1f}; copy factor {fw:.4f}",
        f"# phase_sources_sha256 covers csrc/{', csrc/'.join(PHASE_KERNEL_SOURCES)}",
        f"phase_sources_sha256={kernel_source_digest()}",
        f"fetch_bytes_per_launch={fetch_b:.0f}",
        f"write_bytes_per_launch={write_b:.0f}",
    ]
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def write_counter_summary(out_md, csvs, trace_stats=None):
    """Per-dispatch means of every counter in the given rocprofv3 --pmc CSVs,
    per kernel, as a markdown table, with the derived per-site figures of the
    L=8192 phase kernel."""
    import csv
    import re
    import statistics
    from collections import defaultdict

    vals = defaultdict(lambda: defaultdict(list))
    for path in csvs:
        for r in csv.DictReader(open(path)):
            name = re.sub(r"\(.*", "", r["Kernel_Name"].replace("lat::(anonymous namespace)::", "").replace("void ", ""))
            vals[name][r["Counter_Name"]].append(float(r["Counter_Value"]))
    lines = ["| kernel | counter | dispatches | mean per dispatch |", "|---|---|---|---|"]
    keep = ("k_phase_2bit", "k_sweep_lds_w", "k_obs_2bit", "k_obs_batch", "k_fold_sums")
    for k in sorted(v for v in vals if v.startswith(keep)):
        for c in sorted(vals[k]):
            v = vals[k][c]
            lines.append(f"| {k} | {c} | {len(v)} | {statistics.mean(v):.6g} |")
    ph = vals.get("k_phase_2bit<1>", {})
    if "SQ_INSTS_VALU" in ph:
        n_updates = workloads.LARGE.L ** 2 / 4
        insts = statistics.mean(ph["SQ_INSTS_VALU"])
        lines += ["", f"k_phase_2bit at L={workloads.LARGE.L}: one dispatch updates N/4 = {n_updates:.0f} sites.",
                  f"* VALU wave-instructions per dispatch: {insts:.4g}; lane-ops per site update "
                  f"(x64 lanes): {insts * 64 / n_updates:.1f}"]
        if "SQ_INSTS_LDS" in ph:
            lines.append(f"* LDS instructions per site update (wave-instr x64 / updates): "
                         f"{statistics.mean(ph['SQ_INSTS_LDS']) * 64 / n_updates:.2f}")
        if "SQ_LDS_BANK_CONFLICT" in ph and "SQ_LDS_IDX_ACTIVE" in ph:
            lines.append(f"* SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE: "
                         f"{statistics.mean(ph['SQ_LDS_BANK_CONFLICT']) / max(1.0, statistics.mean(ph['SQ_LDS_IDX_ACTIVE'])):.3f}")
        if "SQ_WAIT_INST_LDS" in ph and "SQ_WAVE_CYCLES" in ph:
            lines.append(f"* SQ_WAIT_INST_LDS / SQ_WAVE_CYCLES: "
                         f"{statistics.mean(ph['SQ_WAIT_INST_LDS']) / statistics.mean(ph['SQ_WAVE_CYCLES']):.4f}")
        if "TCC_HIT_sum" in ph and "TCC_MISS_sum" in ph:
            hit, miss = statistics.mean(ph["TCC_HIT_sum"]), statistics.mean(ph["TCC_MISS_sum"])
            lines.append(f"* L2 hit rate: {hit / (hit + miss):.3f}")
        if trace_stats:
            us = float(trace_stats)
            lines.append(f"* VALU issue utilisation at 2.4 GHz over the traced {us:.2f} us average: "
                         f"{insts * 4 / (1024 * us * 1e-6 * 2.4e9):.3f} (a wave64 VALU instruction occupies a "
                         f"16-lane SIMD for 4 cycles; 1024 SIMDs)")
    open(out_md, "a").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _progress(msg: str):
    """One line on stderr per finished leg (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sweeps", type=int, default=20)
    ap.add_argument("--cpu-all-cores-sweeps", type=int, default=600,
                    help="sweeps per lattice of the batched workload in the all-cores oracle run (0 skips it)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-mid", action="store_true")
    ap.add_argument("--no-maps", action="store_true")
    ap.add_argument("--no-penalty", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="0 skips the served run")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only copy a device buffer of this many MiB 3 times (HBM counter calibration) and exit")
    ap.add_argument("--counter-summary", nargs="+", metavar=("OUT_MD", "CSV"),
                    help="write per-kernel means of rocprofv3 --pmc counter_collection.csv files to OUT_MD and exit")
    ap.add_argument("--valu-summary", metavar="CSV",
                    help="write the VALU summary from a rocprofv3 --pmc SQ_INSTS_VALU counter_collection.csv and exit")
    ap.add_argument("--traffic-summary", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="write the traffic summary from four rocprofv3 --pmc counter_collection.csv files and exit")
    return ap.parse_args()


def host_cores() -> int:
    """Cores this process may run on (the affinity mask, else the count)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(spec: workloads.LatticeSpec, sweeps: int) -> dict:
    """The oracle (single thread) on the same lattice: init untimed, then
    `sweeps` sweeps timed."""
    import oracle

    o = oracle.OracleLattice(spec.L, spec.n, spec.Delta, spec.V, spec.J, spec.T, spec.seed)
    t0 = time.perf_counter()
    o.sweeps(sweeps)
    dt = time.perf_counter() - t0
    return {
        "value": spec.L * spec.L * sweeps / dt,
        "unit": "site updates/s",
        "cores": 1,
        "host_cores": host_cores(),
        "kind": "oracle",
        "sample": f"{sweeps} sweeps of the L={spec.L} lattice (same parameters and seed), init not timed",
    }


def cpu_all_cores(sweeps: int, workers: int) -> dict:
    """The unmodified sequential oracle on every host core at once: the
    batched workload's 256 lattices, one lattice per worker thread at a time
    (the oracle's C sweeps run outside the Python lock), `sweeps` sweeps each;
    init not timed."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    specs = workloads.batched_specs()
    lats = [oracle.OracleLattice(s.L, s.n, s.Delta, s.V, s.J, s.T, s.seed) for s in specs]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(lambda o: o.sweeps(sweeps), lats))
    dt = time.perf_counter() - t0
    updates = sum(s.L * s.L for s in specs) * sweeps
    return {
        "value": updates / dt,
        "unit": "site updates/s",
        "cores": workers,
        "kind": "oracle",
        "sample": f"the batched workload's 256 L=128 lattices, {sweeps} of their 5000 sweeps each, "
                  f"one sequential oracle run per core",
        "lattices_per_s_equivalent": updates / dt / (specs[0].L ** 2 * specs[0].sweeps),
    }


def batched_run(torch, lat, b2b_sample: int = 8, b2b_sweeps: int = 1000) -> dict:
    """The batched workload: 256 L=128 lattices (32 temperatures x 8
    densities), 5000 sweeps each, observables every 50 sweeps.  Timed two
    ways on fresh lattices: the whole job as one replay of a HIP graph holding
    its 100 intervals (batched sweep launch + batched observable reduction
    into that interval's slot, the series read back once at the end), and
    eagerly, one batched sweep call and one observables read per interval.
    Lattice creation, graph capture and the launch-shape autotuning (the first
    calls for a new batch shape) are not timed.  Beside them, a sample of the
    same lattices run back to back through the single-lattice call."""
    specs = workloads.batched_specs()
    every, total = specs[0].every, specs[0].sweeps
    intervals = total // every
    updates = sum(s.L * s.L for s in specs) * total

    def fresh():
        return [lat.Lattice(s.L, s.n, s.Delta, s.V, s.J, s.T, s.seed, encoding=s.encoding) for s in specs]

    # autotune the batch shape on throw-away lattices
    warm = fresh()
    wobs = lat.BatchObservables(len(warm))
    for _ in range(6):
        lat.sweep_batch(warm, every)
        wobs(warm)
    for g in warm:
        g.destroy()

    # The timed regions read the records into structured arrays (the
    # library's device-to-host copy and record conversion); turning 25,600
    # records into Python objects would add 10-20 ms of interpreter work.
    lats = fresh()
    graph = lat.BatchGraph(lats, every, intervals)
    torch.cuda.synchronize()
    gc.collect()
    t0 = time.perf_counter()
    graph.launch(1)
    series = graph.read_array()  # synchronises
    dt_graph = time.perf_counter() - t0
    graph.destroy()
    last_graph = series[-1].copy()
    for g in lats:
        g.destroy()

    lats = fresh()
    obs = lat.BatchObservables(len(lats))
    torch.cuda.synchronize()
    gc.collect()
    t0 = time.perf_counter()
    for _ in range(intervals):
        lat.sweep_batch(lats, every)
        last = obs.array(lats)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for i, s in enumerate(specs):
        Q, _ = lat.charge_target(s.L, s.n)
        assert last["sum_S"][i] == Q
    assert last.tobytes() == last_graph.tobytes(), "graph and eager runs differ"
    for g in lats:
        g.destroy()
    out = {
        "workload": "256 lattices L=128 2-bit, T in [0.2,2.0] x n in {0..0.35}, 5000 sweeps, observables every 50",
        "lattices_per_s": len(specs) / dt_graph,
        "site_updates_per_s": updates / dt_graph,
        "seconds": dt_graph,
        "form": "one HIP graph replay holding all 100 intervals (sweeps + observables), series read once",
        "eager": {"lattices_per_s": len(specs) / dt, "site_updates_per_s": updates / dt, "seconds": dt},
    }
    if b2b_sample > 0:
        sample = specs[:: len(specs) // b2b_sample][:b2b_sample]
        busy = 0.0
        for s in sample:
            g = lat.Lattice(s.L, s.n, s.Delta, s.V, s.J, s.T, s.seed, encoding=s.encoding)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(b2b_sweeps // every):
                g.sweep(every)
                g.observables()
            torch.cuda.synchronize()
            busy += time.perf_counter() - t1
            g.destroy()
        b2b = sum(s.L * s.L for s in sample) * (b2b_sweeps // every * every) / busy
        out["back_to_back"] = {
            "sample": f"{len(sample)} of the lattices, {b2b_sweeps} sweeps each, one lattice_sweep at a time",
            "site_updates_per_s": b2b,
        }
        out["batched_over_back_to_back"] = out["site_updates_per_s"] / b2b
    return out


def mid_run(torch, lat, reps: int = 3) -> dict:
    """The single mid lattice: L=1024 int8 (seed 2), 2000 sweeps with the
    observables after every sweep, run as one device-side observation series
    (per interval the sweep's phase launches, then the observable reduction
    into that interval's record; the 2000 records are read back once at the
    end).  Creation and a warm-up on a throw-away lattice are not timed; the
    same chain runs `reps` times on fresh lattices and the median counts
    (host-side stalls of tens of ms were seen in single runs)."""
    s = workloads.MID
    warm = lat.Lattice(s.L, s.n, s.Delta, s.V, s.J, s.T, s.seed, encoding=s.encoding)
    warm.sweep_series(20, s.every)
    warm.destroy()
    times = []
    Q, _ = lat.charge_target(s.L, s.n)
    for _ in range(reps):
        g = lat.Lattice(s.L, s.n, s.Delta, s.V, s.J, s.T, s.seed, encoding=s.encoding)
        o0 = g.observables()
        torch.cuda.synchronize()
        gc.collect()
        t0 = time.perf_counter()
        buf = g.sweep_series(s.sweeps // s.every, s.every, read=False)
        recs = g.read_series(buf, s.sweeps // s.every, as_array=True)  # synchronises
        times.append(time.perf_counter() - t0)
        assert (recs["sum_S"] == Q).all(), "charge constraint violated"
        assert recs[-1]["sweep"] == s.sweeps
        assert recs[-1]["track_nD"] == recs[-1]["n_charged"] - o0.n_charged, "tracker drifted from the recomputed energy"
        g.destroy()
    dt = sorted(times)[len(times) // 2]
    return {
        "workload": f"single mid lattice L={s.L} int8, J=1 V=0.5 Delta=0 T=1 n=0.05 seed {s.seed}, "
                    f"{s.sweeps} sweeps, observables after every sweep (device-side series, read once); "
                    f"median of {reps} runs of the same chain",
        "site_updates_per_s": s.L * s.L * s.sweeps / dt,
        "ms_per_sweep": 1e3 * dt / s.sweeps,
        "seconds": dt,
        "seconds_all": times,
    }


def map_run(torch, lat, n_maps: int = 100) -> dict:
    """Map mode (the paper's random maps, built on the device) on the batched
    workload's 256 lattices of L=128: n_maps maps each in one launch."""
    specs = workloads.batched_specs()
    lats = [lat.Lattice(s.L, s.n, s.Delta, s.V, s.J, s.T, s.seed, encoding=s.encoding) for s in specs]
    lat.map_steps_batch(lats, 0, 2)  # warm-up (not counted)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.map_steps_batch(lats, 2, n_maps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for g in lats:
        g.destroy()
    pairs = max(1, specs[0].L ** 2 // 10)
    updates = len(specs) * n_maps * 2 * pairs
    return {
        "workload": f"256 lattices L=128 2-bit (the batched workload), {n_maps} maps of {pairs} pairs each, one launch",
        "maps_per_s": len(specs) * n_maps / dt,
        "site_updates_per_s": updates / dt,
        "seconds": dt,
    }


def penalty_run(torch, lat, L: int = 4096, sweeps: int = 20) -> dict:
    """Penalty mode (section 2.2's prior method: single-site checkerboard
    Metropolis, mu adjusted after every sweep) on one int8 lattice with the
    large lattice's parameters.  Wall-clock rate, including the per-sweep
    host rebuild of the mu table and the charge read-back."""
    s = workloads.LARGE
    g = lat.Lattice(L, s.n, s.Delta, s.V, s.J, s.T, s.seed, encoding=lat.ENC_INT8)
    mu, _, _ = g.mu_sweeps(0, 2, 0.5, 0.0)  # warm-up (not counted)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.mu_sweeps(2, sweeps, 0.5, mu)
    dt = time.perf_counter() - t0
    g.destroy()
    return {
        "workload": f"one int8 lattice L={L}, J=1 V=0.5 Delta=0.25 T=1.2 n=0.1 seed 3, kappa 0.5, {sweeps} sweeps",
        "site_updates_per_s": L * L * sweeps / dt,
        "ms_per_sweep": 1e3 * dt / sweeps,
    }


def served_run(seconds: float) -> dict:
    from paper_2301_11735_amd import serve as serve_mod

    reqs = workloads.request_stream(200.0, seconds, 7)
    done, wall, st = serve_mod.serve(reqs, 8 << 20, 256, 1 << 22, progress=False)
    lats = [d["latency"] for d in done.values()]
    updates = sum(d["L"] ** 2 * d["sweeps"] for d in done.values())

    def pct(v, q):
        v = sorted(v)
        return float(v[min(len(v) - 1, int(q * len(v)))]) if v else None

    by_L = {}
    for L in sorted({d["L"] for d in done.values()}):
        v = [d["latency"] for d in done.values() if d["L"] == L]
        by_L[str(L)] = {"requests": len(v), "p50_s": pct(v, 0.5), "p99_s": pct(v, 0.99)}
    out = {
        "workload": f"Poisson 200 req/s for {seconds:g} s, L in {{64,128,256,512}}, 500-5000 sweeps, 8 MiB pool, 256 slots",
        "requests": len(reqs),
        "completed": len(done),
        "p50_s": pct(lats, 0.5),
        "p99_s": pct(lats, 0.99),
        "by_L": by_L,
        "site_updates_per_s": updates / wall,
    }
    # the same requests one at a time with plain lattices (a sample spread
    # over the stream), and whether each result equals the served one
    sample = [r for r in reqs[:: max(1, len(reqs) // 100)] if r.index in done][:100]
    if sample:
        b2b, busy = serve_mod.back_to_back(sample)
        work = sum(r.spec.L ** 2 * r.spec.sweeps for r in sample)
        out["back_to_back"] = {
            "sample": f"{len(sample)} requests spread over the stream, one plain lattice at a time",
            "site_updates_per_s": work / busy,
            "same_results": all(b2b[r.index]["obs"] == done[r.index]["obs"] for r in sample),
        }
        out["served_over_back_to_back"] = out["site_updates_per_s"] / (work / busy)
    return out


def main():
    args = parse()
    if args.traffic_summary:
        write_traffic_summary(*args.traffic_summary)
        return
    if args.valu_summary:
        write_valu_summary(args.valu_summary)
        return
    if args.counter_summary:
        out_md, *rest = args.counter_summary
        us = os.environ.get("PHASE_KERNEL_TRACE_US")
        write_counter_summary(out_md, rest, us)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    if args.calibrate_copy_mib > 0:
        # A plain device-to-device copy of known size: what FETCH_SIZE and
        # WRITE_SIZE read for it scales the counters of the phase kernel.
        n = args.calibrate_copy_mib << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": n, "copies": 3}), flush=True)
        return

    import paper_2301_11735_amd as lat

    spec = workloads.LARGE
    every = spec.every
    N = spec.L * spec.L
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    g = lat.Lattice(spec.L, spec.n, spec.Delta, spec.V, spec.J, spec.T, spec.seed, encoding=spec.encoding,
                    stream=stream)
    o0 = g.observables()

    for _ in range(args.warmup):
        g.sweep(every)
        g.observables()
    torch.cuda.synchronize()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    obs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1, e2 in ev:
        e0.record(stream)
        g.sweep(every)
        e1.record(stream)
        obs.append(g.observables())  # synchronises the stream
        e2.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    sweep_ms = sum(e0.elapsed_time(e1) for e0, e1, _ in ev)
    phase_us = sweep_ms * 1e3 / (args.steps * every * 4)
    value = N * every * args.steps / wall
    per_launch_updates = N / 4  # one phase updates N/8 pairs
    algo_bytes = per_launch_updates * BYTES_PER_SITE_UPDATE_2BIT
    hbm_achieved = algo_bytes / (phase_us * 1e-6) / 1e9
    valu_insts = measured_valu_insts()

    last = obs[-1]
    Q, _ = lat.charge_target(spec.L, spec.n)
    assert last.sum_S == Q, "charge constraint violated"
    assert last.track_nD == last.n_charged - o0.n_charged, "tracker drifted from the recomputed energy"

    line = {
        "metric": "site updates/sec at L=8192",
        "value": value,
        "unit": "site updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "large single lattice L=8192 (67M sites), 2-bit states, J=1 V=0.5 Delta=0.25 T=1.2 "
                        "n=0.1 seed 3, step = 50 sweeps + observable reduction",
            "L": spec.L,
            "sweeps_per_step": every,
            "encoding": "2bit",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": hbm_achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": hbm_achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(),
            "kernel": "k_phase_2bit",
            "avg_launch_us": phase_us,
            "algorithmic_bytes_per_launch": algo_bytes,
            # what binds the kernel: VALU issue (SQ_INSTS_VALU of the committed
            # counter summary over the live launch time)
            # LDS traffic of the table gathers and the b-word exchange
            "lds": {
                "bytes_per_site_update": LDS_BYTES_PER_SITE_UPDATE,
                "achieved": per_launch_updates * LDS_BYTES_PER_SITE_UPDATE / (phase_us * 1e-6) / 1e9,
                "peak": LDS_PEAK_GBS,
                "unit": "GB/s",
                "frac": per_launch_updates * LDS_BYTES_PER_SITE_UPDATE / (phase_us * 1e-6) / 1e9 / LDS_PEAK_GBS,
            },
            "valu": {
                "issue_frac": valu_insts * 4 / (N_SIMD * phase_us * 1e-6 * CLOCK_HZ) if valu_insts else None,
                "lane_ops_per_site_update": valu_insts * 64 / per_launch_updates if valu_insts else None,
                "philox_floor_frac_lower_bound":
                    per_launch_updates * PHILOX_OPS_PER_SITE_UPDATE / (phase_us * 1e-6) / VALU_PEAK_OPS,
            },
        },
    }
    g.destroy()
    _progress(f"large lattice: {value:.4g} site updates/s, phase {phase_us:.2f} us")
    if not args.no_mid:
        line["mid"] = mid_run(torch, lat)
        _progress(f"mid lattice: {line['mid']['site_updates_per_s']:.4g} site updates/s")
    if not args.no_batched:
        line["batched"] = batched_run(torch, lat)
        _progress(f"batched: {line['batched']['lattices_per_s']:.5g} lattices/s")
    if not args.no_maps:
        line["map_mode"] = map_run(torch, lat)
        _progress("map mode done")
    if not args.no_penalty:
        line["penalty_mode"] = penalty_run(torch, lat)
        _progress("penalty mode done")
    if args.serve_seconds > 0:
        line["served"] = served_run(args.serve_seconds)
        _progress(f"served: p50 {line['served']['p50_s']:.3f} s, p99 {line['served']['p99_s']:.3f} s")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(spec, args.cpu_sweeps)
        _progress(f"cpu baseline: {line['cpu_baseline']['value']:.4g} site updates/s on 1 core")
        if args.cpu_all_cores_sweeps > 0:
            # the machine's CPU share per GPU is 16 cores, whatever the host reports
            line["cpu_baseline"]["all_cores"] = cpu_all_cores(args.cpu_all_cores_sweeps, min(16, host_cores()))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
