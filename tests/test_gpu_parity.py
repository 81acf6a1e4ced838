"""GPU parity: the HIP path (through the C-ABI) against the sequential oracle.

The bar is bit-exact: the state codes, all seven integer observables and the
incremental energy tracker must be identical after every observed sweep.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2301_11735_amd as lat
import workloads

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(spec: workloads.LatticeSpec, init_codes=None, start_sweep=0):
    g = lat.Lattice(spec.L, spec.n, spec.Delta, spec.V, spec.J, spec.T, spec.seed, encoding=spec.encoding,
                    n_charged=spec.n_charged, start_sweep=start_sweep, init_codes=init_codes)
    o = oracle.OracleLattice(spec.L, spec.n, spec.Delta, spec.V, spec.J, spec.T, spec.seed,
                             n_charged=spec.n_charged, start_sweep=start_sweep, codes=init_codes)
    return g, o


def _assert_same(g, o, where=""):
    gs = g.read_state()
    if not np.array_equal(gs, o.codes):
        bad = np.flatnonzero(gs != o.codes)
        raise AssertionError(f"{where}: {bad.size} sites differ, first at {bad[:8].tolist()}")
    go = g.observables()
    assert go.ints() == o.observables().tolist(), where
    assert [go.track_nD, go.track_nV, go.track_nJ] == o.track.tolist(), where
    assert go.E == o.energy(), where


def _run_parity(spec, checkpoints):
    _say(f"case L={spec.L} enc={spec.encoding} n={spec.n} T={spec.T} seed={spec.seed} checkpoints={checkpoints}")
    g, o = _pair(spec)
    _assert_same(g, o, "init")
    done = 0
    for c in checkpoints:
        g.sweep(c - done)
        o.sweeps(c - done)
        done = c
        _assert_same(g, o, f"after {c} sweeps")
    g.destroy()


SMALL = workloads.SMALL


@pytest.mark.parametrize("spec", [
    SMALL.with_(L=4, n=0.125),
    SMALL.with_(L=8, n=-0.1, seed=9),
    SMALL.with_(L=12, n=0.2, seed=10),          # L/4 odd: a Philox call spans two rows
    SMALL.with_(L=20, T=0.3, seed=11),
    SMALL,                                      # L=32, n=0.1 (sum S = 102)
    SMALL.with_(L=100, Delta=-0.7, V=-0.3, T=1.7, seed=12),
    SMALL.with_(L=256, seed=13),
], ids=lambda s: f"int8-L{s.L}")
def test_int8_matches_oracle(spec):
    _run_parity(spec, [1, 2, 5, 10, 25])


@pytest.mark.parametrize("spec", [
    SMALL.with_(L=64, encoding=1),
    SMALL.with_(L=128, encoding=1, n=0.3, T=0.4, seed=21),
    SMALL.with_(L=192, encoding=1, Delta=0.9, V=-0.8, T=2.2, seed=22),   # 3 words per class row
    SMALL.with_(L=256, encoding=1, n=-0.2, seed=23),
    SMALL.with_(L=512, encoding=1, T=1.2, seed=24),
], ids=lambda s: f"2bit-L{s.L}")
def test_2bit_matches_oracle(spec):
    _run_parity(spec, [1, 2, 5, 10, 25])


def test_small_config_observable_series():
    """SMALL: observables every 10 sweeps for the first 500 sweeps."""
    _say("case SMALL series")
    g, o = _pair(SMALL)
    for k in range(50):
        g.sweep(10)
        o.sweeps(10)
        go = g.observables()
        assert go.ints() == o.observables().tolist(), k
        assert [go.track_nD, go.track_nV, go.track_nJ] == o.track.tolist(), k
    _assert_same(g, o, "end")


def test_int8_and_2bit_run_the_same_chain():
    spec = SMALL.with_(L=128, seed=31)
    _say("case int8 vs 2bit L=128")
    a = lat.Lattice(spec.L, spec.n, spec.Delta, spec.V, spec.J, spec.T, spec.seed, encoding=0)
    b = lat.Lattice(spec.L, spec.n, spec.Delta, spec.V, spec.J, spec.T, spec.seed, encoding=1)
    for _ in range(4):
        a.sweep(7)
        b.sweep(7)
        assert np.array_equal(a.read_state(), b.read_state())
        assert a.observables().as_dict() == b.observables().as_dict()


@pytest.mark.parametrize("encoding,L", [(0, 32), (1, 128)])
def test_resume_from_read_state_is_bit_exact(encoding, L):
    _say(f"case resume enc={encoding} L={L}")
    spec = SMALL.with_(L=L, encoding=encoding, seed=41)
    full = lat.Lattice(spec.L, spec.n, spec.Delta, spec.V, spec.J, spec.T, spec.seed, encoding=encoding)
    full.sweep(30)
    part = lat.Lattice(spec.L, spec.n, spec.Delta, spec.V, spec.J, spec.T, spec.seed, encoding=encoding)
    part.sweep(12)
    mid = part.read_state()
    resumed = lat.Lattice(spec.L, spec.n, spec.Delta, spec.V, spec.J, spec.T, spec.seed, encoding=encoding,
                          start_sweep=12, init_codes=mid)
    resumed.sweep(18)
    assert np.array_equal(full.read_state(), resumed.read_state())


def test_sweep_batch_equals_separate_sweeps():
    _say("case batch")
    specs = [SMALL.with_(L=L, encoding=e, seed=50 + i, T=0.5 + 0.3 * i)
             for i, (L, e) in enumerate([(32, 0), (64, 1), (128, 1), (20, 0)])]
    batch = [lat.Lattice(s.L, s.n, s.Delta, s.V, s.J, s.T, s.seed, encoding=s.encoding) for s in specs]
    alone = [lat.Lattice(s.L, s.n, s.Delta, s.V, s.J, s.T, s.seed, encoding=s.encoding) for s in specs]
    lat.sweep_batch(batch, 9)
    for a in alone:
        a.sweep(9)
    for a, b in zip(alone, batch):
        assert np.array_equal(a.read_state(), b.read_state())


@pytest.mark.parametrize("kw", [
    dict(n=0.0, n_charged=0, Delta=1e6),       # no charges: pure Ising spins
    dict(n=0.0, n_charged=32 * 32),            # every site charged
    dict(n=1.0),                               # every site +1: all pairs frozen
    dict(T=1e-3),                              # quench
    dict(T=1e6, Delta=0.0, V=0.0, J=0.0),      # everything accepted
], ids=["no-charge", "all-charged", "all-plus", "cold", "hot"])
def test_degenerate_cases(kw):
    spec = SMALL.with_(**kw)
    _run_parity(spec, [1, 3, 10])
    spec2 = spec.with_(L=64, encoding=1, n_charged=(64 * 64 if spec.n_charged == 32 * 32 else spec.n_charged))
    _run_parity(spec2, [1, 3, 10])


def test_empty_and_zero_work_calls_change_nothing():
    """Calls with nothing to do, on lattices of the three paths (on-chip
    L = 64, multi-block word L = 320, phase kernel L = 4096): zero sweeps,
    an empty batch and a batch given zero sweeps, observables of no lattices
    (buffered and allocation-free), an observation series of zero intervals.
    Afterwards each lattice carries on exactly as the oracle does."""
    specs = [SMALL.with_(L=64, encoding=1, seed=1800), SMALL.with_(L=320, encoding=0, seed=1801),
             SMALL.with_(L=4096, encoding=1, T=1.1, seed=1802)]
    gs = [_make(s) for s in specs]
    os_ = [_oracle(s) for s in specs]
    _say("case empty and zero-work calls")
    for g in gs:
        g.sweep(0)
        assert g.sweep_series(0, 1) == []
    lat.sweep_batch([], 5)
    lat.sweep_batch(gs, 0)
    assert lat.BatchObservables(4)([]) == []
    assert lat.observables_batch_noalloc([]) == []
    for s, g, o in zip(specs, gs, os_):
        _assert_same(g, o, f"untouched L={s.L}")
        assert g.observables().sweep == 0
    lat.sweep_batch(gs, 3)
    for s, g, o in zip(specs, gs, os_):
        o.sweeps(3)
        _assert_same(g, o, f"after 3 sweeps L={s.L}")
        assert g.observables().sweep == 3
        g.destroy()


def test_mid_config_parity_first_sweeps():
    """MID (L=1024, int8): bit-exact state and observables for the first sweeps."""
    _run_parity(workloads.MID, [1, 2, 3])


def test_large_config_parity_first_sweeps():
    """LARGE (L=8192, 2-bit) in the launch configuration the benchmark times:
    the full state after one and after three sweeps (twelve phase launches,
    each sweep with its own schedule), bit-exact."""
    _run_parity(workloads.LARGE, [1, 3])


def test_large_config_invariants():
    """LARGE over 100 sweeps: charge exact and tracker == recomputed energy."""
    spec = workloads.LARGE
    _say("case LARGE invariants")
    g = lat.Lattice(spec.L, spec.n, spec.Delta, spec.V, spec.J, spec.T, spec.seed, encoding=spec.encoding)
    Q, Nc = lat.charge_target(spec.L, spec.n)
    o0 = g.observables()
    assert o0.sum_S == Q and o0.n_charged == Nc
    for _ in range(4):
        g.sweep(25)
        o = g.observables()
        assert o.sum_S == Q
        assert o.track_nD == o.n_charged - o0.n_charged
        assert o.track_nV == o.bond_SS - o0.bond_SS
        assert o.track_nJ == o.bond_ss - o0.bond_ss


# ---------------------------------------------------------------- both kernel paths, batches
@pytest.mark.parametrize("spec", [
    SMALL.with_(L=12, n=0.2, seed=61),
    SMALL.with_(L=32, seed=62),
    SMALL.with_(L=128, seed=67),                                # int8 on its packed 2-bit copy
    SMALL.with_(L=100, Delta=-0.7, V=-0.3, T=1.7, seed=63),
    SMALL.with_(L=64, encoding=1, seed=64),
    SMALL.with_(L=192, encoding=1, T=0.5, seed=65),
], ids=lambda s: f"enc{s.encoding}-L{s.L}")
def test_phase_kernel_path_matches_oracle(spec, monkeypatch):
    """Lattices with L <= 512 normally run resident in LDS; force the
    one-launch-per-phase kernels so both paths stay checked at small sizes."""
    monkeypatch.setenv("LATTICE_FORCE_PHASE_KERNELS", "1")
    _run_parity(spec, [1, 3, 10])


@pytest.mark.parametrize("spec", [
    SMALL.with_(L=64, encoding=1, seed=71),
    SMALL.with_(L=128, encoding=0, n=-0.2, seed=72),                      # int8, swept on its 2-bit copy
    SMALL.with_(L=192, encoding=1, Delta=0.9, V=-0.8, T=2.2, seed=73),    # 3 words per class row
    SMALL.with_(L=576, encoding=0, T=0.6, seed=74),                       # int8, 9 words per class row
    SMALL.with_(L=512, encoding=1, T=1.2, seed=75),
    SMALL.with_(L=1024, encoding=1, n=0.3, T=0.4, seed=76),
    SMALL.with_(L=2048, encoding=1, T=1.7, seed=77),
], ids=lambda s: f"enc{s.encoding}-L{s.L}")
@pytest.mark.parametrize("persistent,block", [("1", "256"), ("0", "256"), ("0", "1024")],
                         ids=["persistent", "per-phase", "per-phase-1024"])
def test_word_path_matches_oracle(spec, persistent, block, monkeypatch):
    """The multi-block word kernel (Q lanes per a-word, schedules computed on
    the device, several blocks per lattice) at every size it takes, both
    encodings, as one persistent launch per call (device-wide barriers
    between phases) and as one launch per phase (blocks of 256 or 1024
    threads): the same chain as the oracle, bit for bit."""
    monkeypatch.setenv("LATTICE_PATH", "words")
    monkeypatch.setenv("LATTICE_WORDS_PERSISTENT", persistent)
    monkeypatch.setenv("LATTICE_WORDS_BLOCK", block)
    _run_parity(spec, [1, 3, 10] if spec.L <= 1024 else [1, 2])


@pytest.mark.parametrize("lanes", ["1", "8"])
def test_word_path_per_phase_lane_counts_match_oracle(lanes, monkeypatch):
    """The per-phase word kernel with 1 and 8 lanes per a-word (the defaults
    are 4 up to L = 1024 and 2 above; LATTICE_WORDS_PHASE_LANES selects
    others): bit-exact against the oracle, both encodings, 5 and 9 words per
    class row."""
    monkeypatch.setenv("LATTICE_PATH", "words")
    monkeypatch.setenv("LATTICE_WORDS_PERSISTENT", "0")
    monkeypatch.setenv("LATTICE_WORDS_PHASE_LANES", lanes)
    for spec in (SMALL.with_(L=320, encoding=0, seed=1700), SMALL.with_(L=576, encoding=1, T=0.6, seed=1701)):
        _say(f"case per-phase lanes={lanes} L={spec.L}")
        _run_parity(spec, [1, 3])


@pytest.mark.parametrize("spec", [
    SMALL.with_(L=64, encoding=0, seed=78),
    SMALL.with_(L=4096, encoding=0, T=1.1, seed=79),
], ids=lambda s: f"L{s.L}")
def test_packed_int8_on_the_phase_kernel_matches_oracle(spec, monkeypatch):
    """Int8 lattices on the one-thread-per-word phase kernel run on a 2-bit
    copy packed before and unpacked after each call (L = 4096 takes that path
    by default)."""
    if spec.L <= 1024:
        monkeypatch.setenv("LATTICE_PATH", "phase")
    _run_parity(spec, [1, 3] if spec.L > 1024 else [1, 3, 10])


@pytest.mark.parametrize("persistent", ["1", "0"], ids=["persistent", "per-phase"])
def test_mixed_paths_in_one_batch_match_oracle(persistent, monkeypatch):
    """One lattice_sweep_batch over lattices on all three paths (on-chip,
    multi-block word kernel -- one persistent launch for all its lattices, or
    one launch per phase --, phase kernel): every lattice bit-exact against
    its own oracle run."""
    monkeypatch.setenv("LATTICE_WORDS_PERSISTENT", persistent)
    _say(f"case mixed paths, persistent={persistent}")
    rng = np.random.default_rng(9)
    specs = []
    for i, (L, enc) in enumerate([(64, 1), (100, 0), (320, 1), (512, 0), (576, 1), (1024, 1), (516, 0)]):
        specs.append(SMALL.with_(L=L, encoding=enc, seed=1500 + i, n=float(rng.uniform(-0.3, 0.3)),
                                 Delta=float(rng.uniform(-1, 1)), V=float(rng.uniform(-1, 1)),
                                 T=float(rng.uniform(0.2, 2.5))))
    gs = [_make(s) for s in specs]
    os_ = [_oracle(s) for s in specs]
    obs = lat.BatchObservables(len(gs))
    for k in (4, 3):
        lat.sweep_batch(gs, k)
        for o in os_:
            o.sweeps(k)
        got = obs(gs)
        for s, g, o, go in zip(specs, gs, os_, got):
            assert np.array_equal(g.read_state(), o.codes), f"L={s.L} enc={s.encoding}"
            assert go.ints() == o.observables().tolist()
            assert [go.track_nD, go.track_nV, go.track_nJ] == o.track.tolist()


@pytest.mark.parametrize("block", ["64", "128"])
def test_persistent_word_kernel_small_blocks_match_oracle(block, monkeypatch):
    """The persistent word kernel in blocks of 64 or 128 threads: the mid
    lattice's observation series (records from the tracked moves), with 64
    threads also an L = 2048 series whose threads hold several word tasks a
    phase, and one call for four L = 2048 lattices that share the resident
    blocks, so that a thread holds two word tasks a phase (draws made in
    place) -- bit-exact against the oracle."""
    monkeypatch.setenv("LATTICE_WORDS_PERSISTENT", "1")
    monkeypatch.setenv("LATTICE_WORDS_SERIES_BLOCK", block)
    _say(f"case persistent series block={block} L=1024")
    g, o = _pair(workloads.MID)
    recs = g.sweep_series(5, 1)
    for k, r in enumerate(recs):
        o.sweeps(1)
        assert r.ints() == o.observables().tolist(), k
        assert [r.track_nD, r.track_nV, r.track_nJ] == o.track.tolist(), k
    _assert_same(g, o, "after the series")
    g.destroy()
    if block == "64":
        # 8 lanes a word at L = 2048 need 4096 blocks of 64 threads; at most
        # 1024 take part, so a thread holds four tasks a phase while the
        # records are taken from the tracked moves
        monkeypatch.setenv("LATTICE_WORDS_LANES", "8")
        _say("case persistent series, several tasks a thread, L=2048")
        spec = SMALL.with_(L=2048, encoding=1, T=0.9, seed=97)
        g, o = _pair(spec)
        recs = g.sweep_series(2, 1)
        for k, r in enumerate(recs):
            o.sweeps(1)
            assert r.ints() == o.observables().tolist(), k
            assert [r.track_nD, r.track_nV, r.track_nJ] == o.track.tolist(), k
        _assert_same(g, o, "after the L=2048 series")
        g.destroy()
        monkeypatch.delenv("LATTICE_WORDS_LANES")
    _say(f"case persistent batch block={block} 4 x L=2048")
    specs = [SMALL.with_(L=2048, encoding=1, seed=1600 + i, T=0.8 + 0.3 * i) for i in range(4)]
    gs = [_make(s) for s in specs]
    os_ = [_oracle(s) for s in specs]
    lat.sweep_batch(gs, 2)
    for s, g, o in zip(specs, gs, os_):
        o.sweeps(2)
        _assert_same(g, o, f"L={s.L} seed={s.seed}")
        g.destroy()


@pytest.mark.parametrize("rows,bpc", [(1, 1), (2, 4), (32, 1), (8, 2)])
def test_phase_kernel_launch_shapes_match_oracle(rows, bpc, monkeypatch):
    """The 2-bit phase kernel under other launch shapes (rows of the a-class
    per block, blocks per compute unit) than the default: the same chain."""
    monkeypatch.setenv("LATTICE_FORCE_PHASE_KERNELS", "1")
    monkeypatch.setenv("LATTICE_2BIT_ROWS", str(rows))
    monkeypatch.setenv("LATTICE_2BIT_BLOCKS_PER_CU", str(bpc))
    _run_parity(SMALL.with_(L=256, encoding=1, T=0.8, n=-0.2, seed=66), [1, 4])


def _make(spec):
    return lat.Lattice(spec.L, spec.n, spec.Delta, spec.V, spec.J, spec.T, spec.seed, encoding=spec.encoding,
                       n_charged=spec.n_charged)


def _oracle(spec):
    return oracle.OracleLattice(spec.L, spec.n, spec.Delta, spec.V, spec.J, spec.T, spec.seed,
                                n_charged=spec.n_charged)


def test_mixed_batch_matches_oracle():
    """One batched launch over lattices of different L, encodings and
    parameters: every lattice bit-exact against its own oracle run."""
    _say("case mixed batch")
    rng = np.random.default_rng(5)
    specs = []
    for i, (L, enc) in enumerate([(4, 0), (8, 0), (12, 0), (32, 0), (64, 1), (100, 0), (128, 1), (192, 1),
                                  (256, 0), (256, 1), (512, 1), (64, 0)]):
        specs.append(SMALL.with_(L=L, encoding=enc, seed=700 + i, n=float(rng.uniform(-0.3, 0.3)),
                                 Delta=float(rng.uniform(-1, 1)), V=float(rng.uniform(-1, 1)),
                                 T=float(rng.uniform(0.2, 2.5))))
    gs = [_make(s) for s in specs]
    os_ = [_oracle(s) for s in specs]
    obs = lat.BatchObservables(len(gs))
    for k in (7, 4):
        lat.sweep_batch(gs, k)
        for o in os_:
            o.sweeps(k)
        got = obs(gs)
        for s, g, o, go in zip(specs, gs, os_, got):
            assert np.array_equal(g.read_state(), o.codes), f"L={s.L} enc={s.encoding}"
            assert go.ints() == o.observables().tolist()
            assert [go.track_nD, go.track_nV, go.track_nJ] == o.track.tolist()
            assert go.E == o.energy()


def test_batched_config_subset_matches_oracle():
    """The batched workload (L=128, 2-bit, 32 temperatures x 8 densities):
    every 16th lattice, bit-exact after 60 sweeps done in one batched launch."""
    _say("case batched subset")
    specs = workloads.batched_specs()[::16]
    gs = [_make(s) for s in specs]
    lat.sweep_batch(gs, 60)
    for s, g in zip(specs, gs):
        o = _oracle(s)
        o.sweeps(60)
        assert np.array_equal(g.read_state(), o.codes), f"seed {s.seed}"


def test_batched_config_invariants():
    """All 256 lattices of the batched workload: charge exact and tracker equal
    to the recomputed energy after 200 sweeps."""
    _say("case batched invariants")
    specs = workloads.batched_specs()
    gs = [_make(s) for s in specs]
    obs = lat.BatchObservables(len(gs))
    first = obs(gs)
    for _ in range(2):
        lat.sweep_batch(gs, 100)
        now = obs(gs)
        for s, a, b in zip(specs, first, now):
            Q, Nc = lat.charge_target(s.L, s.n)
            assert b.sum_S == Q
            assert b.track_nD == b.n_charged - a.n_charged
            assert b.track_nV == b.bond_SS - a.bond_SS
            assert b.track_nJ == b.bond_ss - a.bond_ss


def test_batched_config_graph_in_the_timed_launch_shape(monkeypatch):
    """The batched workload in the launch configuration bench.py times: all
    256 lattices in one HIP graph of observation intervals (50 sweeps each)
    with 512-thread blocks, as the autotuner picks for this shape.  Every
    16th lattice is compared with the oracle bit for bit (state and every
    interval's records); every lattice's records hold the exact charge and a
    tracker equal to the recomputed sums' changes."""
    monkeypatch.setenv("LATTICE_BATCH_THREADS", "512")
    _say("case batched config as one graph, 512 threads")
    specs = workloads.batched_specs()
    every, intervals = specs[0].every, 3
    gs = [_make(s) for s in specs]
    first = lat.BatchObservables(len(gs))(gs)
    graph = lat.BatchGraph(gs, every, intervals)
    graph.launch(1)
    recs = graph.read_array()  # (intervals, lattices)
    graph.destroy()
    for i, (s, a) in enumerate(zip(specs, first)):
        Q, _ = lat.charge_target(s.L, s.n)
        r = recs[:, i]
        assert (r["sum_S"] == Q).all(), f"seed {s.seed}"
        assert (r["track_nD"] == r["n_charged"] - a.n_charged).all(), f"seed {s.seed}"
        assert (r["track_nV"] == r["bond_SS"] - a.bond_SS).all(), f"seed {s.seed}"
        assert (r["track_nJ"] == r["bond_ss"] - a.bond_ss).all(), f"seed {s.seed}"
    for i in range(0, len(specs), 16):
        s, g = specs[i], gs[i]
        o = _oracle(s)
        for k in range(intervals):
            o.sweeps(every)
            r = recs[k, i]
            assert [int(r[f]) for f in ("sum_S", "n_charged", "bond_SS", "bond_ss", "M", "M_stag", "C_stag")] \
                == o.observables().tolist(), f"seed {s.seed} interval {k}"
            assert [int(r["track_nD"]), int(r["track_nV"]), int(r["track_nJ"])] == o.track.tolist()
        assert np.array_equal(g.read_state(), o.codes), f"seed {s.seed}"
    for g in gs:
        g.destroy()


# ---------------------------------------------------------------- serving
def test_served_results_equal_alone_and_oracle():
    """Requests served in a mix (continuous batching, small pool so requests
    queue) give the same final state and observables as each run alone, and
    as the oracle."""
    _say("case serving")
    from paper_2301_11735_amd import serve as serve_mod

    reqs = workloads.request_stream(rate_per_s=60.0, duration_s=1.5, seed=11, sizes=(64, 128),
                                    sweep_range=(20, 120))
    assert len(reqs) > 40
    pool = 1 << 20   # about 12 resident L=128 lattices: admission has to queue
    done, wall, st = serve_mod.serve(reqs, pool, slots=16, quantum=1 << 16, keep_state=True, progress=False)
    assert len(done) == len(reqs)
    rng = np.random.default_rng(3)
    for k in rng.choice(len(reqs), size=8, replace=False):
        r = reqs[int(k)]
        s = r.spec
        g = lat.Lattice(s.L, s.n, s.Delta, s.V, s.J, s.T, s.seed, encoding=s.encoding)
        g.sweep(s.sweeps)
        assert np.array_equal(g.read_state(), done[r.index]["codes"]), r.index
        assert g.observables().as_dict()["E"] == done[r.index]["obs"]["E"]
    for k in rng.choice(len(reqs), size=3, replace=False):
        r = reqs[int(k)]
        s = r.spec
        o = _oracle(s)
        o.sweeps(s.sweeps)
        assert np.array_equal(o.codes, done[r.index]["codes"]), r.index
        ob = done[r.index]["obs"]
        assert [ob["sum_S"], ob["n_charged"], ob["bond_SS"], ob["bond_ss"], ob["M"], ob["M_stag"],
                ob["C_stag"]] == o.observables().tolist()
        assert [ob["track_nD"], ob["track_nV"], ob["track_nJ"]] == o.track.tolist()


def test_served_config_sizes_equal_alone_and_oracle():
    """The served configuration's sizes and sweep counts: L in {64, 128, 256,
    512}, 500-800 sweeps, the full parameter ranges.  The L = 512 requests
    advance on the multi-block word kernel on the server's second stream
    while the others share the on-chip launch; every request's result equals
    the same request run alone, and two of L = 512 and two of L = 256 equal
    the oracle."""
    _say("case serving, served sizes")
    from concurrent.futures import ThreadPoolExecutor

    from paper_2301_11735_amd import serve as serve_mod

    reqs = workloads.request_stream(rate_per_s=40.0, duration_s=1.0, seed=12, sweep_range=(500, 800))
    assert len(reqs) > 20 and {r.spec.L for r in reqs} == {64, 128, 256, 512}
    done, wall, st = serve_mod.serve(reqs, 8 << 20, slots=32, quantum=1 << 22, keep_state=True, progress=False)
    assert len(done) == len(reqs)
    for r in reqs:
        s = r.spec
        g = lat.Lattice(s.L, s.n, s.Delta, s.V, s.J, s.T, s.seed, encoding=s.encoding)
        g.sweep(s.sweeps)
        assert np.array_equal(g.read_state(), done[r.index]["codes"]), r.index
        assert g.observables().as_dict() == done[r.index]["obs"], r.index
        g.destroy()
    picks = [r for r in reqs if r.spec.L == 512][:2] + [r for r in reqs if r.spec.L == 256][:2]

    def run_oracle(r):
        o = _oracle(r.spec)
        o.sweeps(r.spec.sweeps)
        return o

    with ThreadPoolExecutor(max_workers=4) as ex:
        oracles = list(ex.map(run_oracle, picks))
    for r, o in zip(picks, oracles):
        assert np.array_equal(o.codes, done[r.index]["codes"]), r.index
        ob = done[r.index]["obs"]
        assert [ob["sum_S"], ob["n_charged"], ob["bond_SS"], ob["bond_ss"], ob["M"], ob["M_stag"],
                ob["C_stag"]] == o.observables().tolist()
        assert [ob["track_nD"], ob["track_nV"], ob["track_nJ"]] == o.track.tolist()


@pytest.mark.parametrize("spec", [
    SMALL.with_(L=576, encoding=1, seed=81),                     # 9 words per class row
    SMALL.with_(L=1024, encoding=1, T=0.6, n=-0.15, seed=82),
], ids=lambda s: f"L{s.L}")
def test_persistent_path_matches_oracle(spec, monkeypatch):
    """2-bit lattices above the LDS size with all sweeps of a call in one
    cooperative launch (device-wide barrier between phases)."""
    monkeypatch.setenv("LATTICE_PERSISTENT", "1")
    _run_parity(spec, [1, 3, 8])


def test_autotuned_batch_launch_shapes_match_oracle():
    """The first calls for a new batch shape each try another block size
    (1024, 512, 256, 128 threads per lattice) before the fastest is kept;
    every call must leave every lattice bit-exact."""
    _say("case autotuned batch shapes")
    specs = [SMALL.with_(L=L, encoding=1, seed=900 + i, T=0.4 + 0.2 * i) for i, L in enumerate([192, 192, 128, 64, 192])]
    gs = [_make(s) for s in specs]
    os_ = [_oracle(s) for s in specs]
    for call, k in enumerate([3, 2, 4, 3, 2]):
        lat.sweep_batch(gs, k)
        for s, g, o in zip(specs, gs, os_):
            o.sweeps(k)
            assert np.array_equal(g.read_state(), o.codes), f"call {call} L={s.L}"
    # A new shape (three lattices) called back to back with no read between:
    # the timed launches of several candidates are in flight at once, and no
    # call waits for them.
    _say("case autotuned batch shapes, calls back to back")
    specs = [SMALL.with_(L=128, encoding=1, seed=950 + i, T=0.5 + 0.4 * i) for i in range(3)]
    gs = [_make(s) for s in specs]
    os_ = [_oracle(s) for s in specs]
    ks = [2, 3, 1, 2, 3, 2, 1]
    for k in ks:
        lat.sweep_batch(gs, k)
    for s, g, o in zip(specs, gs, os_):
        o.sweeps(sum(ks))
        assert np.array_equal(g.read_state(), o.codes), f"L={s.L} seed={s.seed}"


def _word_batch_specs():
    rng = np.random.default_rng(17)
    out = []
    for i, (L, enc) in enumerate([(64, 0), (64, 1), (128, 1), (192, 1), (256, 0), (320, 1), (512, 1)]):
        out.append(SMALL.with_(L=L, encoding=enc, seed=1300 + i, n=float(rng.uniform(-0.3, 0.3)),
                               Delta=float(rng.uniform(-1, 1)), V=float(rng.uniform(-1, 1)),
                               T=float(rng.uniform(0.2, 2.5))))
    return out


@pytest.mark.parametrize("threads", [128, 256, 512, 1024])
def test_word_batch_every_block_size_matches_oracle(threads, monkeypatch):
    """Batches whose lattices all have L % 64 == 0 take the word-parallel LDS
    kernel; the block size sets how many threads share an a-word (1 to 8),
    per lattice.  Every split must give the oracle's chain bit for bit,
    including int8 lattices and class rows of 1, 2, 3, 4, 5 and 8 words."""
    monkeypatch.setenv("LATTICE_BATCH_THREADS", str(threads))
    _say(f"case word batch threads={threads}")
    specs = _word_batch_specs()
    gs = [_make(s) for s in specs]
    os_ = [_oracle(s) for s in specs]
    obs = lat.BatchObservables(len(gs))
    for k in (3, 2):
        lat.sweep_batch(gs, k)
        for o in os_:
            o.sweeps(k)
        got = obs(gs)
        for s, g, o, go in zip(specs, gs, os_, got):
            assert np.array_equal(g.read_state(), o.codes), f"threads={threads} L={s.L} enc={s.encoding}"
            assert go.ints() == o.observables().tolist()
            assert [go.track_nD, go.track_nV, go.track_nJ] == o.track.tolist()
    for g in gs:
        g.destroy()


def test_word_and_site_batch_forms_agree(monkeypatch):
    """The per-site LDS kernel (forced) and the word-parallel one give the
    same states and trackers over 40 sweeps."""
    _say("case word vs site forms")
    specs = _word_batch_specs()
    monkeypatch.setenv("LATTICE_LDS_SITE", "1")
    site = [_make(s) for s in specs]
    lat.sweep_batch(site, 40)
    site_obs = lat.BatchObservables(len(site))(site)
    monkeypatch.delenv("LATTICE_LDS_SITE")
    word = [_make(s) for s in specs]
    lat.sweep_batch(word, 40)
    word_obs = lat.BatchObservables(len(word))(word)
    for s, a, b, oa, ob in zip(specs, site, word, site_obs, word_obs):
        assert np.array_equal(a.read_state(), b.read_state()), f"L={s.L}"
        assert oa.as_dict() == ob.as_dict()


@pytest.mark.parametrize("kind,threads", [("word", 0), ("word", 512), ("word", 1024), ("site", 0),
                                          ("onchip", 0), ("onchip", 512)],
                         ids=["word-auto", "word-512", "word-1024", "site", "onchip-auto", "onchip-512"])
def test_batch_graph_replays_match_eager_and_oracle(kind, threads, monkeypatch):
    """Observation intervals captured into a HIP graph: every replay (with
    eager batched work and synchronisation in between) leaves the lattices and
    every interval's observables exactly where the same eager calls do, and
    where the oracle does.  512-thread word blocks reduce the observables in
    the sweep kernel, 1024-thread ones in a separate launch: both covered,
    also for a batch whose lattices are all on the on-chip path (onchip-512;
    onchip-auto takes 1024 threads at L = 256)."""
    if threads:
        monkeypatch.setenv("LATTICE_BATCH_THREADS", str(threads))
    _say(f"case batch graph {kind} threads={threads}")
    if kind == "onchip":
        specs = [SMALL.with_(L=L, encoding=enc, seed=1450 + i, T=0.4 + 0.35 * i)
                 for i, (L, enc) in enumerate([(64, 0), (64, 1), (128, 1), (192, 1), (256, 0)])]
    elif kind == "word":
        specs = _word_batch_specs()
    else:
        specs = [SMALL.with_(L=L, encoding=enc, seed=1400 + i, T=0.3 + 0.4 * i)
                 for i, (L, enc) in enumerate([(12, 0), (64, 1), (100, 0), (128, 1)])]
    every, intervals = 4, 3
    glats = [_make(s) for s in specs]
    elats = [_make(s) for s in specs]
    os_ = [_oracle(s) for s in specs]
    obs = lat.BatchObservables(len(elats))
    graph = lat.BatchGraph(glats, every, intervals)
    total = 0
    for rep, times in enumerate([1, 1, 2, 1]):
        graph.launch(times)
        got = graph.read()
        exp = []
        for _ in range(times):
            exp = []
            for k in range(intervals):
                lat.sweep_batch(elats, every)
                exp.append(obs(elats))
        total += every * intervals * times
        for k in range(intervals):
            for s, a, b in zip(specs, got[k], exp[k]):
                assert a.as_dict() == b.as_dict(), f"replay {rep} interval {k} L={s.L}"
                assert a.sweep == total - every * (intervals - 1 - k)
        for s, g, e, o, a in zip(specs, glats, elats, os_, got[-1]):
            o.sweeps(every * intervals * times)
            assert np.array_equal(g.read_state(), e.read_state()), f"replay {rep} L={s.L}"
            assert np.array_equal(g.read_state(), o.codes), f"replay {rep} L={s.L}"
            assert a.ints() == o.observables().tolist()
            assert [a.track_nD, a.track_nV, a.track_nJ] == o.track.tolist()
    graph.destroy()
    # the lattices carry on eagerly from where the graph left them
    lat.sweep_batch(glats, 3)
    for g, o in zip(glats, os_):
        o.sweeps(3)
        assert np.array_equal(g.read_state(), o.codes)


def test_mid_series_per_phase_launches_match_oracle(monkeypatch):
    """The mid lattice's observation series through one launch per phase (the
    persistent form switched off): the same records as the oracle."""
    monkeypatch.setenv("LATTICE_WORDS_PERSISTENT", "0")
    spec = workloads.MID
    _say("case series per-phase L=1024")
    g, o = _pair(spec)
    recs = g.sweep_series(6, 1)
    for k, r in enumerate(recs):
        o.sweeps(1)
        assert r.ints() == o.observables().tolist(), k
        assert [r.track_nD, r.track_nV, r.track_nJ] == o.track.tolist(), k
        assert r.sweep == k + 1
    _assert_same(g, o, "after the series")
    g.destroy()


@pytest.mark.parametrize("spec,every,intervals", [
    (workloads.MID, 1, 12),                                        # int8 L=1024 on its 2-bit copy, every sweep
    (SMALL.with_(L=64, encoding=1, seed=91), 3, 8),                # on-chip path
    (SMALL.with_(L=4096, encoding=0, T=1.1, seed=92), 1, 3),       # phase kernel, packed int8
    (SMALL.with_(L=100, seed=93), 2, 5),                           # int8 with L % 64 != 0
    (SMALL.with_(L=576, encoding=1, seed=94), 3, 4),               # words path, 2-bit, 9 words per class row
    (SMALL.with_(L=2048, encoding=1, T=0.7, seed=95), 1, 2),       # words path, Q = 2
    (SMALL.with_(L=320, encoding=0, T=0.9, seed=96), 2, 5),        # words path, Q = 8, packed int8, 5 words a row
], ids=["mid", "lds", "phase-int8", "int8-L100", "words-L576", "words-L2048", "words-L320"])
@pytest.mark.parametrize("persistent", ["1", "0"], ids=["persistent", "per-phase"])
def test_device_observation_series_matches_oracle(spec, every, intervals, persistent, monkeypatch):
    """lattice_sweep_series keeps the observables of every interval on the
    device (no host synchronisation between intervals); each record equals the
    oracle's observables, tracker and sweep count after that interval, and
    the state after the series is the oracle's.  Lattices on the multi-block
    path run the series as persistent launches or as launches per phase."""
    monkeypatch.setenv("LATTICE_WORDS_PERSISTENT", persistent)
    _say(f"case series L={spec.L} enc={spec.encoding} every={every} intervals={intervals}")
    g, o = _pair(spec)
    g.sweep(2)
    o.sweeps(2)
    recs = g.sweep_series(intervals, every)
    for k, r in enumerate(recs):
        o.sweeps(every)
        assert r.ints() == o.observables().tolist(), k
        assert [r.track_nD, r.track_nV, r.track_nJ] == o.track.tolist(), k
        assert r.sweep == 2 + every * (k + 1)
        assert r.E == o.energy()
    _assert_same(g, o, "after the series")
    g.destroy()
