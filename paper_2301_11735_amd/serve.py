"""Serve a Poisson stream of uneven simulation requests with the library's
continuous-batching server (lat_server_*) and report time-to-result.

The request loop runs in real time: requests are submitted when their arrival
time comes, every server step advances all resident lattices in one batched
launch, and finished requests are harvested between steps.  With --baseline
the same requests (or a sample of them) are also served back to back, one
plain lattice at a time, for comparison.

Usage:
    python -m paper_2301_11735_amd.serve [--rate 200] [--duration 60] [--pool-mib 8] [--slots 256]
                                         [--quantum 4194304] [--baseline-sample 200]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_2301_11735_amd as lat  # noqa: E402
import workloads  # noqa: E402


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else float("nan")


def serve(requests, pool_bytes, slots, quantum, keep_state=False, progress=True):
    """Run the stream through a Server in real time.  Returns per-request
    records (arrival, admit, finish, latency, observables) and totals."""
    import torch

    srv = lat.Server(pool_bytes, max_slots=slots, quantum_updates=quantum)
    t0 = time.monotonic()
    i, pending, done, failed = 0, {}, {}, {}
    last_report = t0
    while i < len(requests) or pending:
        now = time.monotonic() - t0
        while i < len(requests) and requests[i].arrival_s <= now:
            r = requests[i]
            s = r.spec
            rid = srv.submit(s.L, s.n, s.Delta, s.V, s.J, s.T, s.seed, s.sweeps, encoding=s.encoding,
                             keep_state=keep_state)
            pending[rid] = r
            i += 1
        if pending:
            finished = srv.step()
            st = srv.stats() if finished == 0 else None
            # poll when requests finished, or when some left the server without
            # finishing (a request whose set-up failed at admission)
            if finished > 0 or st.queued + st.resident < len(pending):
                for rid in list(pending):
                    res = srv.poll(rid, with_state=keep_state)
                    info, codes = res if keep_state else (res, None)
                    if info.status == lat.REQ_FINISHED:
                        r = pending.pop(rid)
                        done[r.index] = dict(arrival=r.arrival_s, admit=info.t_admit - t0, finish=info.t_finish - t0,
                                             latency=info.t_finish - t0 - r.arrival_s, obs=info.obs.as_dict(),
                                             codes=codes, L=r.spec.L, sweeps=r.spec.sweeps)
                        srv.release(rid)
                    elif info.status == lat.REQ_FAILED:
                        r = pending.pop(rid)
                        failed[r.index] = info.error
                        srv.release(rid)
        elif i < len(requests):
            time.sleep(max(0.0, min(0.01, requests[i].arrival_s - (time.monotonic() - t0))))
        if progress and time.monotonic() - last_report > 5.0:
            st = srv.stats()
            print(f"[serve] t={time.monotonic() - t0:6.1f}s submitted={i} done={len(done)} resident={st.resident} "
                  f"queued={st.queued}", file=sys.stderr, flush=True)
            last_report = time.monotonic()
    torch.cuda.synchronize()
    wall = time.monotonic() - t0
    st = srv.stats()
    srv.destroy()
    if failed:
        print(f"[serve] {len(failed)} requests failed at admission: {sorted(failed.items())[:8]}", file=sys.stderr,
              flush=True)
    return done, wall, st


def back_to_back(requests):
    """Serve requests one at a time with plain lattices, in arrival order,
    each starting when it has arrived and the previous one has finished."""
    import torch

    t_free, out = 0.0, {}
    busy = 0.0
    for r in requests:
        s = r.spec
        t_start_wall = time.monotonic()
        g = lat.Lattice(s.L, s.n, s.Delta, s.V, s.J, s.T, s.seed, encoding=s.encoding)
        g.sweep(s.sweeps)
        o = g.observables()
        g.destroy()
        torch.cuda.synchronize()
        service = time.monotonic() - t_start_wall
        busy += service
        start = max(r.arrival_s, t_free)
        t_free = start + service
        out[r.index] = dict(latency=t_free - r.arrival_s, service=service, obs=o.as_dict())
    return out, busy


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--duration", type=float, default=60.0)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--pool-mib", type=float, default=8.0)
    ap.add_argument("--slots", type=int, default=256)
    ap.add_argument("--quantum", type=int, default=1 << 22)
    ap.add_argument("--baseline-sample", type=int, default=200)
    args = ap.parse_args()

    reqs = workloads.request_stream(args.rate, args.duration, args.seed)
    done, wall, st = serve(reqs, int(args.pool_mib * 2**20), args.slots, args.quantum)
    lats = [d["latency"] for d in done.values()]
    updates = sum(d["L"] ** 2 * d["sweeps"] for d in done.values())
    line = {
        "workload": f"served Poisson stream {args.rate}/s for {args.duration}s (seed {args.seed})",
        "requests": len(reqs),
        "completed": len(done),
        "wall_s": wall,
        "site_updates_per_s": updates / wall,
        "p50_s": percentile(lats, 50),
        "p99_s": percentile(lats, 99),
        "by_L": {str(L): {"requests": len(v), "p50_s": percentile(v, 50), "p99_s": percentile(v, 99),
                          "max_s": max(v)}
                 for L in sorted({d["L"] for d in done.values()})
                 for v in [[d["latency"] for d in done.values() if d["L"] == L]]},
        "steps": st.steps,
        "pool_mib": args.pool_mib,
        "slots": args.slots,
        "quantum_updates": args.quantum,
    }
    if args.baseline_sample > 0:
        rng = np.random.default_rng(1)
        sample = sorted(rng.choice(len(reqs), size=min(args.baseline_sample, len(reqs)), replace=False))
        sub = [reqs[k] for k in sample]
        b2b, busy = back_to_back(sub)
        updates_b = sum(r.spec.L ** 2 * r.spec.sweeps for r in sub)
        line["back_to_back"] = {
            "sample": len(sub),
            "site_updates_per_s": updates_b / busy,
            "mean_service_s": busy / len(sub),
            "same_results": all(b2b[r.index]["obs"] == done[r.index]["obs"] for r in sub if r.index in done),
        }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
