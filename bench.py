"""Benchmark of exact serial-episode counting on one MI355X.

Default (the headline line): the Large workload -- 256 event types, 50M
events over 3600 s with int64 nanosecond times (Poisson background plus 32
planted cascades of 3-8 types), 200k candidate episodes of sizes 2-8 (every
sub-episode of the planted cascades, the rest random over the interval menu
{0,5,10,20} ms offset x {5,10,20} ms width).  One step = one exact count of
all 200k candidates over the whole stream, inputs resident in HBM: the batched
engine (segment-parallel lane machines in persistent launches, one kept
hipGraph) ordered by the learned cost model (features -> MLP -> device sort ->
longest-first work items, all inside the graph).  The plain engine, round
robin and the event-count heuristic are timed beside it on the same inputs.

Metric: candidate-episode x events counted per second = m * n / step time.

Other lines: ``--mining`` (level-wise discovery of the mining preset),
``--ablation`` (presets 1, 3, 4, 5: plain vs batched schedules),
``--tracking-sweep`` (episode-length sweep of the per-event tracking
engine), ``--calibrate-copy`` (a 1 GiB device copy for the byte counters).

Prints one JSON line.  ``--gpus`` above 1 is refused: this engine runs on
one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12  # vector-ALU lane operations per second (T)
PROFILE = "k_ext_walk_mining.md"
KERNEL_SOURCES = ("epi_extend.hip",)
LARGE_PROFILE = "k_lane_persistent_large.md"
LARGE_SOURCES = ("epi_lane.hip", "epi_tiled.hip", "epi_sched.hip", "epi_sort.hip", "epi_count.h")
THRESHOLD = 100
MAX_SIZE = 6


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash(sources):
    import hashlib

    srcs = [os.path.join(ROOT, "paper_0905_2203_amd", "csrc", f) for f in sources]
    return hashlib.sha256(b"".join(open(f, "rb").read() for f in srcs)).hexdigest()[:16]


def profiled(kernel_name, key, field, profile=PROFILE, sources=KERNEL_SOURCES):
    """A per-launch figure of ``kernel_name`` (line ``key`` of the committed
    rocprofv3 counter summary), or None when the summary is for another
    kernel or the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", profile)
    try:
        h = source_hash(sources)
        for line in open(path):
            if line.startswith(key + ":"):
                rec = json.loads(line.split(":", 1)[1])
                if rec["kernel"] == kernel_name and rec["source_hash"] == h:
                    return rec[field]
    except OSError:
        pass
    return None


def profiled_traffic(kernel_name):
    """HBM bytes per launch (FETCH_SIZE and WRITE_SIZE, copy-calibrated)."""
    v = profiled(kernel_name, "traffic_bytes_per_launch", "bytes")
    return None if v is None else int(v)


def host_cpu():
    """The host CPU's model name (the CPU baseline runs on it)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def copy_gbps(stream=None):
    """Practical HBM bandwidth: a 1 GiB device-to-device copy (read + write
    bytes over its time), best of 5 after a warm-up, timed with HIP events."""
    import torch

    a = torch.empty(1 << 28, dtype=torch.int32, device="cuda").fill_(1)
    b = torch.empty_like(a)
    best = None
    with torch.cuda.stream(stream or torch.cuda.current_stream()):
        for i in range(6):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            b.copy_(a)
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            if i > 0:
                best = ms if best is None else min(best, ms)
    del a, b
    return 2 * (1 << 30) / (best / 1e3) / 1e9


def _timed(ctx, fn, reps):
    import torch

    out = []
    for _ in range(reps):
        ctx.epi_sync()
        torch.cuda.synchronize()
        a = time.perf_counter()
        fn()
        ctx.epi_sync()
        out.append(time.perf_counter() - a)
    return float(np.median(out))


ABL_LEGS = ("plain", "batched_rr", "batched_learned", "batched_heuristic", "batched_measured")
RECORDINGS_PROFILE = "k_lane_persistent_recordings.md"


def ablation(k, scale, reps, lane_engine=1, ring_classes=0, tune=False, legs=ABL_LEGS, tune_cache=None):
    """Plain engine vs the batched persistent engine under round-robin, the
    event-count heuristic and the learned cost model, on workload preset k.
    Every mode's counts are checked equal; one JSON line per preset.  With
    tune, the batched legs run autotuned (round robin tuned for itself, the
    heuristic and measured schedules with the learned schedule's setting;
    tune_cache: the autotuner's cache file, read, else written).  legs: the
    legs to time (profiling runs time one)."""
    import spikegen as sg
    from paper_0905_2203_amd import epi

    ctx = epi.Context(0)
    ctx.epi_set_option(epi.EPI_OPT_LANE_ENGINE, lane_engine)
    ctx.epi_set_option(epi.EPI_OPT_RING_CLASSES, ring_classes)
    if k == 3:
        sets = []
        for r in range(16):
            s = sg.config_stream(3, scale=scale, recording=r)
            sets.append((s, sg.config_candidates(3, s, scale=scale, recording=r)))
        train_sets = []
        for r in range(4):
            s, _ = sets[r]
            train_sets.append((r, sg.random_candidates(sg.rng_for(3, offset=3000 + r), max(int(5000 * scale), 64), 60,
                                                       2, 8, 1_000_000)))
    else:
        s = sg.config_stream(k, scale=scale)
        sets = [(s, sg.config_candidates(k, s, scale=scale))]
        if k == 4:
            train_sets = [(0, sg.config_candidates(4, s, scale=scale, training=True))]
        else:
            train_sets = [(0, sg.random_candidates(sg.rng_for(k, offset=100), max(int(50_000 * scale), 64), s["K"], 2,
                                                   8, 1_000_000))]
    log(f"ablation preset {k}: {len(sets)} sets, {sum(c['N'].size for _, c in sets)} candidates")
    sids = [ctx.epi_load_stream(s["types"], s["times"], s["K"]) for s, _ in sets]
    cids = [ctx.epi_submit_candidates(sid, c) for sid, (_, c) in zip(sids, sets)]
    units = sum(c["N"].size * s["types"].size for s, c in sets)
    res = {}

    def counts():
        return [ctx.epi_read_counts(cid, c["N"].size) for cid, (_, c) in zip(cids, sets)]

    tuned = {}
    ref = None

    def check(leg):
        nonlocal ref
        got = counts()
        if ref is None:
            ref = got
        assert all(np.array_equal(a, b) for a, b in zip(got, ref)), leg

    if "plain" in legs:
        res["plain"] = _timed(ctx, lambda: ctx.epi_count(cids, mode=epi.EPI_MODE_PLAIN), reps)
        check("plain")
    if "batched_rr" in legs:
        if tune:
            tuned["batched_rr"] = ctx.epi_autotune(cids, epi.EPI_SCHED_RR, tune_cache)
            log(f"  tuned for round robin: {tuned['batched_rr']}")
        res["batched_rr"] = _timed(ctx, lambda: ctx.epi_count(cids, mode=epi.EPI_MODE_BATCHED,
                                                              sched=epi.EPI_SCHED_RR), reps)
        check("batched_rr")
        log(f"  batched_rr: {res['batched_rr']:.3f}s")
    # learned: work log of disjoint training candidates on the same streams
    ctx.epi_set_option(epi.EPI_OPT_WORKLOG, 1)
    ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 1)  # log each episode's own work
    a = time.perf_counter()
    tids = [ctx.epi_submit_candidates(sids[r], c) for r, c in train_sets]
    ctx.epi_count(tids, mode=epi.EPI_MODE_BATCHED, sched=epi.EPI_SCHED_RR)
    losses = ctx.epi_costmodel_train(tids, epochs=40, seed=7)
    train_s = time.perf_counter() - a
    ctx.epi_set_option(epi.EPI_OPT_WORKLOG, 0)
    ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 0)
    if tune and any(x in legs for x in ("batched_learned", "batched_heuristic", "batched_measured")):
        tuned["batched_learned"] = ctx.epi_autotune(cids, epi.EPI_SCHED_LEARNED, tune_cache)
        log(f"  tuned for the learned schedule: {tuned['batched_learned']}")
    if "batched_learned" in legs:
        res["batched_learned"] = _timed(ctx, lambda: ctx.epi_count(cids, mode=epi.EPI_MODE_BATCHED,
                                                                   sched=epi.EPI_SCHED_LEARNED), reps)
        check("batched_learned")
        log(f"  learned {res['batched_learned']:.3f}s (training {train_s:.1f}s)")
    if "batched_heuristic" in legs:
        res["batched_heuristic"] = _timed(ctx, lambda: ctx.epi_count(cids, mode=epi.EPI_MODE_BATCHED,
                                                                     sched=epi.EPI_SCHED_HEURISTIC), reps)
        check("batched_heuristic")
    if "batched_measured" in legs:
        # measured: the schedule by each episode's own logged work (an exact cost model)
        ctx.epi_set_option(epi.EPI_OPT_WORKLOG, 1)
        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 1)
        ctx.epi_count(cids, mode=epi.EPI_MODE_BATCHED, sched=epi.EPI_SCHED_RR)
        ctx.epi_set_option(epi.EPI_OPT_WORKLOG, 0)
        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 0)
        res["batched_measured"] = _timed(ctx, lambda: ctx.epi_count(cids, mode=epi.EPI_MODE_BATCHED,
                                                                    sched=epi.EPI_SCHED_MEASURED), reps)
        check("batched_measured")
        log(f"  measured-cost schedule {res['batched_measured']:.3f}s")
    # parity: a seeded sample of every set's counts against the oracle, which
    # is timed on it (all host cores)
    parity = "not checked"
    cpu = None
    try:
        import oracle
        import spikegen as sg_

        rng = np.random.Generator(np.random.PCG64(11))
        bad = checked = 0
        cores = oracle.max_threads()
        cpu_units = cpu_s = 0.0
        for (s_, c_), got in zip(sets, ref):
            idx = np.sort(rng.choice(c_["N"].size, size=min(64, c_["N"].size), replace=False))
            a = time.perf_counter()
            want = oracle.count(s_, sg_.take_candidates(c_, idx), nthreads=cores)
            cpu_s += time.perf_counter() - a
            cpu_units += idx.size * s_["types"].size
            bad += int((want != got[idx]).sum())
            checked += idx.size
        parity = f"{'ok' if bad == 0 else 'MISMATCH'}: {checked} sampled counts vs the oracle, {bad} differ"
        cpu = dict(value=cpu_units / cpu_s, unit="cand*ev/s", cores=cores, kind="oracle",
                   sample=f"the {checked} parity candidates, {cpu_s:.2f}s")
        log(f"  parity {parity}")
    except Exception as exc:
        log(f"oracle leg failed: {exc!r}")
    # algorithmic bytes of the state-machine engines: each candidate reads the
    # times of its own types' events, its descriptor, and writes its count
    alg = sum(alg_bytes(s_, c_) for s_, c_ in sets)
    def ratio(a, b):
        return res[a] / res[b] if a in res and b in res else None

    roofline = None
    if "batched_learned" in res:
        # the learned count against 8 TB/s; traffic from the committed profile
        # of this preset's learned count while the engine sources match it
        ach = alg / res["batched_learned"] / 1e9
        traffic = tset = None
        if k == 3 and abs(scale - 1.0) < 1e-9 and tune:
            traffic = profiled("batched_learned_graph", "traffic_bytes_per_launch", "bytes", RECORDINGS_PROFILE,
                               LARGE_SOURCES)
            tset = profiled("batched_learned_graph", "traffic_bytes_per_launch", "setting", RECORDINGS_PROFILE,
                            LARGE_SOURCES)
        roofline = {"bound": "hbm", "kernel": "batched count graph, learned schedule", "achieved": ach,
                    "peak": 8000.0, "unit": "GB/s", "frac": ach / 8000.0,
                    "traffic": None if traffic is None else int(traffic),
                    # the (tile, launch groups, lanes, segment target) the counters were taken at
                    "traffic_setting": tset}
    line = {
        "metric": "candidate-episode x events counted/sec (exact), plain vs batched+learned-sched",
        "ablation_preset": k, "scale": scale, "unit": "cand*ev/s", "lane_engine": lane_engine,
        "ring_classes": ring_classes, "tuned": tuned,
        "value": {m: units / t for m, t in res.items()},
        "seconds": res,
        "learned_vs_rr": ratio("batched_rr", "batched_learned"),
        "learned_vs_heuristic": ratio("batched_heuristic", "batched_learned"),
        "learned_vs_plain": ratio("plain", "batched_learned"),
        "measured_vs_learned": ratio("batched_learned", "batched_measured"),
        "roofline": roofline,
        "cost_model": {"train_seconds": train_s, "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
                       "train_candidates": int(sum(c["N"].size for _, c in train_sets))},
        "counts_equal_across_modes": True,
        "parity": parity,
        "algorithmic_bytes": alg,
        "algorithmic_GBps": {m: alg / t / 1e9 for m, t in res.items()},
        "cpu_baseline": cpu,
        "candidates": int(sum(c["N"].size for _, c in sets)), "events": int(sum(s["types"].size for s, _ in sets)),
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def tracking_sweep(scale, reps, m_per_len=16):
    """Episode-length sweep (the runtime-vs-length experiment of Sec. V-C,
    on synthetic data): a few long episodes over a long stream, counted by
    per-event tracking (EPI_MODE_TRACKING) and by the one-lane-per-episode
    engine with automatic segments (EPI_MODE_PLAIN).  Stream: 64 types,
    Poisson background at 40 Hz per type over 3600 s (about 9.2M events),
    int64 nanoseconds, plus two planted 8-node cascades at 4 Hz whose gaps
    lie in (0,5], (5,10] or (10,20] ms.  Per length N = 2..8: the planted
    cascades' N-node prefixes and random N-node episodes over those
    intervals, m_per_len in all.  Counts of both modes are checked against
    the oracle; one JSON line per length."""
    import spikegen as sg
    from paper_0905_2203_amd import epi

    rng = np.random.Generator(np.random.PCG64(911))
    unit = 1_000_000
    dur = 3600.0 * scale
    s = sg.poisson_stream(rng, K=64, rate_hz=40.0, dur_s=dur, ts_kind=1, unit_per_ms=unit, cascades=[8, 8],
                          cascade_trigger_hz=[4.0, 4.0])
    n = int(s["types"].size)
    log(f"tracking sweep: n={n}")
    ctx = epi.Context(0)
    sid = ctx.epi_load_stream(s["types"], s["times"], s["K"])
    menu = [(a * unit, b * unit) for a, b in sg.MENU_MINING_MS]
    try:
        import oracle
    except ImportError:
        oracle = None
    for N in range(2, 9):
        eps = []
        for p in s["planted"]:
            eps.append(([int(x) for x in p["types"][:N]], [int(x) for x in p["lo"][: N - 1]],
                        [int(x) for x in p["hi"][: N - 1]]))
        while len(eps) < m_per_len:
            iv = [menu[int(rng.integers(len(menu)))] for _ in range(N - 1)]
            eps.append((rng.permutation(64)[:N].tolist(), [a for a, _ in iv], [b for _, b in iv]))
        c = sg.candidates_from_list(eps)
        cid = ctx.epi_submit_candidates(sid, c)
        t_track = _timed(ctx, lambda: ctx.epi_count([cid], mode=epi.EPI_MODE_TRACKING), reps)
        got_t = ctx.epi_read_counts(cid, len(eps))
        t_plain = _timed(ctx, lambda: ctx.epi_count([cid], mode=epi.EPI_MODE_PLAIN), reps)
        got_p = ctx.epi_read_counts(cid, len(eps))
        parity = "not checked"
        if oracle is not None:
            want = oracle.count(s, c)
            bad = int((want != got_t).sum() + (want != got_p).sum())
            parity = f"{'ok' if bad == 0 else 'MISMATCH'}: {len(eps)} episodes, both modes, {bad} differ"
        ctx.epi_release_set(cid)
        line = {
            "metric": "tracking_sweep", "episode_size": N, "episodes": len(eps), "events": n,
            "tracking_ms": round(1e3 * t_track, 3), "plain_ms": round(1e3 * t_plain, 3),
            "tracking_cand_ev_per_s": len(eps) * n / t_track, "plain_cand_ev_per_s": len(eps) * n / t_plain,
            "tracking_vs_plain": round(t_plain / t_track, 3), "planted_counts": [int(x) for x in got_t[:2]],
            "parity": parity, "dtype": "int64", "data": "synthetic",
        }
        print(json.dumps(line), flush=True)
    ctx.epi_release_stream(sid)
    ctx.close()


def alg_bytes(s, c):
    """Bytes the counting method must read and write for candidate set c on
    stream s: each candidate reads the times of its own types' events, its
    descriptor (128 B with int64 times, 72 B with int32) and writes a 4-B count."""
    tc = np.bincount(s["types"], minlength=s["K"]).astype(np.int64)
    tsb = 8 if s["ts_kind"] == 1 else 4
    N = c["N"].astype(np.int64)
    ty = c["types"].astype(np.int64)
    per = np.where(np.arange(8)[None, :] < N[:, None], tc[np.clip(ty, 0, None)], 0).sum(axis=1)
    return int(per.sum()) * tsb + int(N.size) * ((128 if tsb == 8 else 72) + 4)


def large_bench(args):
    """The headline line: the Large workload, batched + learned schedule."""
    import torch

    import spikegen as sg
    from paper_0905_2203_amd import epi

    t0 = time.time()
    s = sg.config_stream(5, scale=args.scale)
    c = sg.config_candidates(5, s, scale=args.scale)
    train = sg.random_candidates(sg.rng_for(5, offset=100), max(int(50_000 * args.scale), 64), s["K"], 2, 8,
                                 s["unit_per_ms"])
    n, m = int(s["types"].size), int(c["N"].size)
    log(f"large workload: n={n} K={s['K']} m={m} generated in {time.time() - t0:.1f}s")
    torch.cuda.init()
    # every count and every timing event on one stream of our own (default
    # priority): the events bracket exactly the work the counts queue
    stream = torch.cuda.Stream()
    hs = stream.cuda_stream
    d_types = torch.from_numpy(s["types"]).cuda()
    d_times = torch.from_numpy(s["times"]).cuda()
    torch.cuda.synchronize()
    assert hs != 0, "the count stream must not be the null stream"
    ctx = epi.Context(0)
    if args.ring_classes >= 0:
        ctx.epi_set_option(epi.EPI_OPT_RING_CLASSES, args.ring_classes)
    sid = ctx.epi_load_stream_device(d_types, d_times, s["K"], hip_stream=hs)
    cid = ctx.epi_submit_candidates(sid, c)
    ctx.epi_sync()

    # the cost model: trained once on the work log of a disjoint candidate set
    # (each episode's own work: no segments), or loaded from a file
    a = time.perf_counter()
    if args.costmodel_in:
        ctx.epi_costmodel_load(args.costmodel_in)
        losses = [float("nan")]
    else:
        ctx.epi_set_option(epi.EPI_OPT_WORKLOG, 1)
        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 1)
        tid = ctx.epi_submit_candidates(sid, train)
        ctx.epi_count([tid], mode=epi.EPI_MODE_BATCHED, sched=epi.EPI_SCHED_RR)
        losses = ctx.epi_costmodel_train([tid], epochs=40, seed=7)
        ctx.epi_set_option(epi.EPI_OPT_WORKLOG, 0)
        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 0)
        ctx.epi_release_set(tid)
    if args.costmodel_out:
        ctx.epi_costmodel_save(args.costmodel_out)
    train_s = time.perf_counter() - a
    log(f"cost model ready in {train_s:.1f}s (loss {losses[0]:.3f} -> {losses[-1]:.3f})")

    legs = {"batched_learned": (epi.EPI_MODE_BATCHED, epi.EPI_SCHED_LEARNED),
            "plain": (epi.EPI_MODE_PLAIN, epi.EPI_SCHED_RR),
            "batched_rr": (epi.EPI_MODE_BATCHED, epi.EPI_SCHED_RR),
            "batched_heuristic": (epi.EPI_MODE_BATCHED, epi.EPI_SCHED_HEURISTIC)}
    tuned = {}

    def tune(sched, name):
        if args.no_tune:
            return
        a = time.perf_counter()
        tuned[name] = dict(zip(("tile", "ring_classes", "lanes", "target_lanes"),
                               ctx.epi_autotune([cid], sched, args.tune_cache or None)))
        tuned[name]["seconds"] = round(time.perf_counter() - a, 1)
        log(f"  autotuned for {name}: {tuned[name]}")

    def run(mode, sched, steps, warmup, name):
        for w in range(warmup):
            ctx.epi_count([cid], mode=mode, sched=sched, hip_stream=hs)
            ctx.epi_sync()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        a = time.perf_counter()
        for e0, e1 in ev:
            e0.record(stream)
            ctx.epi_count([cid], mode=mode, sched=sched, hip_stream=hs)
            e1.record(stream)
        torch.cuda.synchronize()
        ctx.epi_sync()
        wall = time.perf_counter() - a
        ms = [e0.elapsed_time(e1) for e0, e1 in ev]
        log(f"  {name}: {np.mean(ms):.1f} ms per count (events), {1e3 * wall / steps:.1f} ms wall")
        return float(np.mean(ms)), wall

    res, counts = {}, {}
    reps = max(1, min(3, args.steps))
    # the plain engine with its defaults, then the batched engine tuned for
    # round robin, then tuned for the learned schedule (the headline leg:
    # exactly K timed steps after W warm-up steps), then the heuristic
    # schedule with the learned leg's setting
    if not args.learned_only:
        res["plain"], _ = run(*legs["plain"], reps, 1, "plain")
        counts["plain"] = ctx.epi_read_counts(cid, m)
        tune(epi.EPI_SCHED_RR, "batched_rr")
        res["batched_rr"], _ = run(*legs["batched_rr"], reps, 1, "batched_rr")
        counts["batched_rr"] = ctx.epi_read_counts(cid, m)
    tune(epi.EPI_SCHED_LEARNED, "batched_learned")
    st0 = ctx.epi_batched_stats()
    res["batched_learned"], wall_learned = run(*legs["batched_learned"], args.steps, args.warmup, "batched_learned")
    counts["batched_learned"] = ctx.epi_read_counts(cid, m)
    st1 = ctx.epi_batched_stats()
    stats = {"built": st1["built"] - st0["built"], "replays": st1["replays"] - st0["replays"]}
    if not args.learned_only:
        res["batched_heuristic"], _ = run(*legs["batched_heuristic"], reps, 1, "batched_heuristic")
        counts["batched_heuristic"] = ctx.epi_read_counts(cid, m)
    equal = all(np.array_equal(counts[k], counts["batched_learned"]) for k in counts)

    # parity: every count against the oracle-written expected counts of this
    # workload, else a seeded sample against the oracle
    parity = "not checked"
    got = counts["batched_learned"]
    try:
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from fullsize import cand_fingerprint, stream_fingerprint

        path = os.path.join(ROOT, "tests", "golden", "full_cfg5.npz")
        if args.scale == 1.0 and os.path.exists(path):
            z = np.load(path, allow_pickle=False)
            meta = json.loads(str(z["meta"]))
            if meta["stream"] == stream_fingerprint(s) and meta["candidates"] == cand_fingerprint(c):
                bad = int((z["counts"] != got).sum())
                parity = (f"{'ok' if bad == 0 and equal else 'MISMATCH'}: all {m} counts vs the oracle's "
                          f"(tests/golden/full_cfg5.npz), {bad} differ; modes agree: {equal}")
    except Exception as exc:
        log(f"golden check failed: {exc!r}")
    cpu = None
    if not args.no_cpu:
        try:
            import oracle

            k = min(args.cpu_sample, m)
            idx = np.unique(np.linspace(0, m - 1, k).astype(np.int64))
            cores = oracle.max_threads()
            a = time.perf_counter()
            want = oracle.count(s, sg.take_candidates(c, idx), nthreads=cores)
            el = time.perf_counter() - a
            bad = int((want != got[idx]).sum())
            if parity == "not checked":
                parity = f"{'ok' if bad == 0 and equal else 'MISMATCH'}: {idx.size} sampled counts vs the oracle, {bad} differ"
            cpu = dict(value=idx.size * n / el, unit="cand*ev/s", cores=cores, kind="oracle",
                       sample=f"{idx.size} of the {m} candidates (evenly spaced), all {n} events, "
                              f"decomposition oracle in {el:.1f}s", host=host_cpu())
        except Exception as exc:
            log(f"oracle leg failed: {exc!r}")

    alg = alg_bytes(s, c)
    t_step = res["batched_learned"] / 1e3
    achieved = alg / t_step / 1e9
    kname = "batched count graph (k_lane_persistent per launch class on parallel branches, scheduler, reconcile)"
    traffic = profiled("batched_learned_graph", "traffic_bytes_per_launch", "bytes", LARGE_PROFILE, LARGE_SOURCES)
    traffic_setting = profiled("batched_learned_graph", "traffic_bytes_per_launch", "setting", LARGE_PROFILE,
                               LARGE_SOURCES)
    ctx.epi_release_set(cid)
    ctx.epi_release_stream(sid)
    ctx.close()
    del d_types, d_times
    # the practical HBM peak on this GPU, beside the published 8 TB/s
    copy_bw = copy_gbps(stream)
    log(f"  1 GiB device copy: {copy_bw:.0f} GB/s (read + write)")
    value = m * n / t_step
    line = {
        "metric": "candidate-episode x events counted/sec (exact), plain vs batched+learned-sched",
        "value": value,
        "unit": "cand*ev/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["batched_learned"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {
            "workload": "Large: 256 types, 50M events over 3600 s, int64 ns, Poisson background + 32 planted "
                        "cascades (3-8 types); 200k candidates of sizes 2-8; batched persistent graph, "
                        "segment-parallel lane machines, learned cost-model schedule",
            "scale": args.scale, "events": n, "candidates": m,
            "mode": "batched + learned schedule",
        },
        "modes": {k: {"ms_per_count": v, "cand_ev_per_s": m * n / (v / 1e3)} for k, v in res.items()},
        "learned_vs_plain": res["plain"] / res["batched_learned"] if "plain" in res else None,
        "learned_vs_rr": res["batched_rr"] / res["batched_learned"] if "batched_rr" in res else None,
        "learned_vs_heuristic": res["batched_heuristic"] / res["batched_learned"] if "batched_heuristic" in res else None,
        "wall_ms_per_step": 1e3 * wall_learned / args.steps,
        # the learned leg's warm-up and timed counts: plans captured, replays
        "graph": {"plans_built": stats["built"], "replays": stats["replays"]},
        "autotuned": tuned,
        "cost_model": {"train_seconds": train_s, "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
                       "train_candidates": int(train["N"].size)},
        "roofline": {
            "bound": "hbm",
            "kernel": kname,
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": traffic,
            # the (tile, launch groups, lanes, segment target) the counters were
            # taken at; the run's own setting is under "autotuned"
            "traffic_setting": traffic_setting,
            # a 1 GiB device copy on the same GPU: the practical HBM peak
            "copy_GBps": copy_bw,
            "algorithmic_bytes": alg,
            "per_unit": "per candidate: sum over its nodes of the node type's events x 8 B + 128 B descriptor "
                        "+ 4 B count; one launch = one count of all candidates",
        },
        "cpu_baseline": cpu,
        "parity": parity,
    }
    print(json.dumps(line), flush=True)



def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="candidates timed on the CPU (default: 8000 of the Large workload; 1.5M level-3 "
                         "candidates with --mining)")
    ap.add_argument("--scale", type=float, default=1.0, help="size scale of the Large workload")
    ap.add_argument("--mining", action="store_true", help="level-wise discovery of the mining preset")
    ap.add_argument("--learned-only", action="store_true",
                    help="Large line: time only the batched + learned leg (profiling runs)")
    ap.add_argument("--no-tune", action="store_true", help="Large line: engine defaults, no autotuning")
    ap.add_argument("--tune-cache", default="",
                    help="Large line and --abl-tune: autotuner cache file (read, else written)")
    ap.add_argument("--costmodel-in", default="", help="Large line: load the cost model from this file")
    ap.add_argument("--costmodel-out", default="", help="Large line: save the trained cost model to this file")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a device-to-device copy of 1 GiB (scale reference for HBM byte counters)")
    ap.add_argument("--ablation", default="",
                    help="comma list of workload presets (1, 3, 4, 5): plain vs batched schedules, one JSON line each")
    ap.add_argument("--abl-scale", type=float, default=1.0, help="size scale of the ablation workloads")
    ap.add_argument("--abl-tune", action="store_true", help="ablation: autotune the batched legs")
    ap.add_argument("--abl-legs", default=",".join(ABL_LEGS), help="ablation: comma list of the legs to time")
    ap.add_argument("--lane-engine", type=int, default=1,
                    help="ablation: 1 = register-indexed lane machines where they apply, 0 = LDS-ring machines")
    ap.add_argument("--ring-classes", type=int, default=-1,
                    help="batched launch groups per episode size: 0 submission groups, 1 one, 2 three "
                         "(default: the engine default for the Large line, 0 for --ablation)")
    ap.add_argument("--tracking-sweep", action="store_true",
                    help="episode-length sweep: per-event tracking vs the plain engine, one JSON line per length")
    args = ap.parse_args()
    if args.tracking_sweep:
        tracking_sweep(args.abl_scale, max(1, args.steps))
        return
    if args.ablation:
        for k in [int(x) for x in args.ablation.split(",") if x]:
            ablation(k, args.abl_scale, max(1, args.steps), args.lane_engine, max(0, args.ring_classes),
                     args.abl_tune, tuple(x for x in args.abl_legs.split(",") if x), args.tune_cache or None)
        return
    if args.calibrate_copy:
        import torch

        a = torch.empty(1 << 28, dtype=torch.int32, device="cuda").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the engine has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    if args.mining:
        if args.cpu_sample <= 0:
            args.cpu_sample = 1_500_000  # about 10 s of the oracle on 16 host threads
        mining_bench(args)
        return
    if args.cpu_sample <= 0:
        args.cpu_sample = 8000  # about 11 s of the oracle on 16 host threads
    large_bench(args)


def mining_bench(args):
    """Level-wise discovery of the mining preset, one JSON line."""
    import torch

    import spikegen as sg
    from paper_0905_2203_amd import epi

    t0 = time.time()
    s = sg.config_stream(2)
    n = int(s["types"].size)
    K = int(s["K"])
    menu = [(a * 1000, b * 1000) for a, b in sg.MENU_MINING_MS]
    log(f"stream: n={n} K={K} generated in {time.time() - t0:.1f}s")
    d_types = torch.from_numpy(s["types"]).cuda()
    d_times = torch.from_numpy(s["times"]).cuda()
    torch.cuda.synchronize()

    ctx = epi.Context(0)

    def step():
        sid = ctx.epi_load_stream_device(d_types, d_times, K)
        mid = ctx.epi_mine(sid, menu, MAX_SIZE, THRESHOLD)
        return sid, mid

    def release(sid, mid):
        ctx.epi_mine_release(mid)
        ctx.epi_release_stream(sid)

    for w in range(args.warmup):
        sid, mid = step()
        release(sid, mid)
        log(f"warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    ctx.epi_sync()
    times = []
    level_info = None
    for k in range(args.steps):
        torch.cuda.synchronize()
        a = time.perf_counter()
        sid, mid = step()
        torch.cuda.synchronize()
        b = time.perf_counter()
        times.append(b - a)
        nl = ctx.epi_mine_levels(mid)
        info = [ctx.epi_mine_level_info(mid, L) for L in range(1, nl + 1)]
        if level_info is None:
            level_info = [[i] for i in info]
        else:
            for acc, i in zip(level_info, info):
                acc.append(i)
        if k == args.steps - 1:
            last = (sid, mid, nl)
        else:
            release(sid, mid)
        log(f"step {k + 1}/{args.steps}: {1e3 * (b - a):.1f} ms")
    sid, mid, nl = last
    ms_step = 1e3 * float(np.mean(times))
    cand_per_level = [lv[0][0] for lv in level_info]
    freq_per_level = [lv[0][1] for lv in level_info]
    units = sum(cand_per_level) * n
    value = units / (ms_step / 1e3)

    # dominant counting launch: the level with the largest kernel time
    kern_ms = [float(np.mean([x[2][2] for x in lv])) for lv in level_info]
    gen_ms = [float(np.mean([x[2][0] for x in lv])) for lv in level_info]
    cnt_ms = [float(np.mean([x[2][1] for x in lv])) for lv in level_info]
    dom = int(np.argmax(kern_ms)) + 1
    alg = ctx.epi_mine_level_bytes(mid, dom)
    achieved_gbs = alg / (kern_ms[dom - 1] / 1e3) / 1e9
    mp = len(menu) if len(menu) <= 4 else 8
    kname = f"k_ext_walk<int, {mp}, 0>" if dom >= 2 else "k_level1<int>"
    traffic = profiled_traffic(kname)
    valu_frac = profiled(kname, "valu_issue_per_launch", "frac")

    # parity spot check (outside the timed region): sampled counts vs the oracle
    parity = "not checked"
    cpu = None
    try:
        import oracle

        rng = np.random.Generator(np.random.PCG64(7))
        bad = 0
        checked = 0
        for L in range(1, nl + 1):
            m_l = cand_per_level[L - 1]
            idx = np.sort(rng.choice(m_l, size=min(300, m_l), replace=False))
            sub, got = ctx.epi_mine_read_at(mid, L, idx)
            want = oracle.count(s, sub)
            bad += int((want != got).sum())
            checked += idx.size
        parity = f"{'ok' if bad == 0 else 'MISMATCH'}: {checked} sampled counts over {nl} levels, {bad} differ"

        if not args.no_cpu:
            from oracle import apriori

            # the oracle's own candidates: its level 1-2 pass, then a sample of
            # its level-3 join, timed on all host cores
            lv = apriori.mine(s, menu, 2, THRESHOLD)
            c3 = apriori.join(sorted(lv[1]["frequent"]))
            step_ = max(1, len(c3) // args.cpu_sample)
            sample = c3[::step_][: args.cpu_sample]
            sc = apriori.to_candidates(sample, menu)
            cores = oracle.max_threads()
            a = time.perf_counter()
            oracle.count(s, sc, nthreads=cores)
            el = time.perf_counter() - a
            cpu = dict(value=len(sample) * n / el, unit="cand*ev/s", cores=cores, kind="oracle",
                       sample=f"{len(sample)} of the {len(c3)} level-3 candidates (1 in {step_}), "
                              f"counted by the decomposition oracle in {el:.1f}s")
    except Exception as exc:  # the benchmark line is still printed
        log(f"oracle leg failed: {exc!r}")

    release(sid, mid)
    ctx.close()

    line = {
        "metric": "candidate-episode x events counted/sec (exact), plain vs batched+learned-sched",
        "value": value,
        "unit": "cand*ev/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": "level-wise mining: 64 types x 20 Hz Poisson, 300 s, int32 us, 4 planted cascades; "
                        "sizes 1-6 over {(0,5],(5,10],(10,20]} ms, count > 100",
            "events": n,
            "candidates_per_level": cand_per_level,
            "frequent_per_level": freq_per_level,
            "mode": "plain",
            "level_ms": {"generate": gen_ms, "count_incl_transfers": cnt_ms, "kernels": kern_ms},
        },
        # the walk is bound by vector-ALU issue, not by HBM: VALU issue share
        # = wave-level VALU instructions x 4 cycles over 1024 SIMDs x 2.4 GHz
        # x the launch time (SQ counters of the committed profile); the peak
        # is 256 CUs x 64 lanes x 2.4 GHz = 39.3 T lane-ops/s
        "roofline": {
            "bound": "alu",
            "kernel": f"{kname} (level {dom}, {cand_per_level[dom - 1]} candidates)",
            "achieved": None if valu_frac is None else valu_frac * PEAK_VALU_TOPS,
            "peak": PEAK_VALU_TOPS,
            "unit": "T lane-ops/s (VALU)",
            "frac": valu_frac,
            "traffic": traffic,
            # bytes the walk must read (walked stream positions x (type + time)
            # + chain entries), over the kernel time: the walk shares one
            # stream walk among all extensions of a parent, so this is not the
            # per-candidate byte count of the state machines
            "walked_bytes": alg,
            "walked_GBps": achieved_gbs,
            "walked_frac_of_hbm_peak": achieved_gbs / PEAK_HBM_GBS,
        },
        "cpu_baseline": cpu,
        "parity": parity,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
