"""Batched persistent mode, its schedules, the work log and the learned cost
model on the GPU: counts are bit-exact against the oracle in every mode."""
import numpy as np
import pytest

import oracle
import spikegen as sg
from oracle import mlp
from paper_0905_2203_amd import epi

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-batched] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = epi.Context(0)
    yield c
    c.close()


def _recordings(n_rec=4, scale=0.02):
    """A few recordings of the bursty batched workload (different streams)."""
    recs = []
    for r in range(n_rec):
        s = sg.config_stream(3, scale=scale, recording=r)
        c = sg.config_candidates(3, s, scale=scale, recording=r)
        recs.append((s, c))
    return recs


@pytest.mark.parametrize("sched,rings", [(epi.EPI_SCHED_RR, 0), (epi.EPI_SCHED_HEURISTIC, 0),
                                         (epi.EPI_SCHED_HEURISTIC, 1), (epi.EPI_SCHED_RR, 2)])
def test_batched_multi_recording_exact(ctx, sched, rings):
    recs = _recordings()
    sids, cids = [], []
    for s, c in recs:
        sids.append(ctx.epi_load_stream(s["types"], s["times"], s["K"]))
        cids.append(ctx.epi_submit_candidates(sids[-1], c))
    say(f"sched={sched} ring classes={rings}: {[c['N'].size for _, c in recs]} candidates over {len(recs)} recordings")
    ctx.epi_set_option(epi.EPI_OPT_RING_CLASSES, rings)
    try:
        ctx.epi_count(cids, mode=epi.EPI_MODE_BATCHED, sched=sched)
        for (s, c), cid in zip(recs, cids):
            got = ctx.epi_read_counts(cid, c["N"].size)
            assert np.array_equal(got, oracle.count(s, c))
    finally:
        ctx.epi_set_option(epi.EPI_OPT_RING_CLASSES, 0)
        for cid in cids:
            ctx.epi_release_set(cid)
        for sid in sids:
            ctx.epi_release_stream(sid)


@pytest.mark.parametrize("segments", [0, 3, 17])
def test_batched_segments_exact(ctx, segments):
    s = sg.config_stream(4, scale=0.01)
    c = sg.config_candidates(4, s, scale=0.02)
    want = oracle.count(s, c)
    sid = ctx.epi_load_stream(s["types"], s["times"], s["K"])
    cid = ctx.epi_submit_candidates(sid, c)
    ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, segments)
    try:
        for sched in (epi.EPI_SCHED_RR, epi.EPI_SCHED_HEURISTIC):
            say(f"segments={segments} sched={sched}")
            ctx.epi_count([cid], mode=epi.EPI_MODE_BATCHED, sched=sched)
            assert np.array_equal(ctx.epi_read_counts(cid, c["N"].size), want)
    finally:
        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 0)
        ctx.epi_release_set(cid)
        ctx.epi_release_stream(sid)


def test_worklog_counts_pinned(ctx):
    """Without segments every event of an episode's types is visited exactly
    once, and the completions are the count."""
    s = sg.config_stream(4, scale=0.005)
    c = sg.config_candidates(4, s, scale=0.01)
    sid = ctx.epi_load_stream(s["types"], s["times"], s["K"])
    cid = ctx.epi_submit_candidates(sid, c)
    ctx.epi_set_option(epi.EPI_OPT_WORKLOG, 1)
    ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 1)
    try:
        for mode in (epi.EPI_MODE_PLAIN, epi.EPI_MODE_BATCHED):
            say(f"work log mode={mode}")
            ctx.epi_count([cid], mode=mode)
            counts = ctx.epi_read_counts(cid, c["N"].size)
            w = ctx.epi_read_worklog(cid, c["N"].size)
            cnt = np.bincount(s["types"], minlength=s["K"])
            visits = np.array([cnt[c["types"][i, :c["N"][i]]].sum() for i in range(c["N"].size)])
            np.testing.assert_array_equal(w[:, 0], visits)
            np.testing.assert_array_equal(w[:, 3], counts)
            # a completion needs a record at each of the N-1 recording nodes
            assert np.all(w[:, 1] >= (c["N"].astype(np.int64) - 1) * w[:, 3])
            assert np.all((w[:, 4] >= 1) == (w[:, 1] >= 1))
            # deepest ring within the proven bound 1 + floor(hi / (hi - lo + 1))
            live = c["hi"] > 0
            bound = np.where(live, 1 + c["hi"] // np.maximum(c["hi"] - c["lo"] + 1, 1), 0).max(axis=1)
            assert np.all(w[:, 4] <= np.maximum(bound, 1))
        cyc = ctx.epi_read_item_cycles(cid)
        assert cyc.shape[0] > 0 and np.all(cyc[:, 1] >= cyc[:, 0])
    finally:
        ctx.epi_set_option(epi.EPI_OPT_WORKLOG, 0)
        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 0)
        ctx.epi_release_set(cid)
        ctx.epi_release_stream(sid)


def test_learned_schedule_from_trained_model(ctx):
    """Train the cost model on a disjoint candidate set's work log, then count
    with the learned schedule: exact, and the model tracks the work."""
    s = sg.config_stream(4, scale=0.01)
    train = sg.config_candidates(4, s, scale=0.04, training=True)
    c = sg.config_candidates(4, s, scale=0.02)
    sid = ctx.epi_load_stream(s["types"], s["times"], s["K"])
    tid = ctx.epi_submit_candidates(sid, train)
    cid = ctx.epi_submit_candidates(sid, c)
    ctx.epi_set_option(epi.EPI_OPT_WORKLOG, 1)
    try:
        # the work of each episode alone: no time segments (whose look-back
        # re-reads depend on the schedule)
        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 1)
        ctx.epi_count([tid])
        losses = ctx.epi_costmodel_train([tid], epochs=40, seed=3)
        say(f"cost model losses {losses[0]:.3f} -> {losses[-1]:.3f}")
        assert losses[-1] < 0.2 * losses[0]
        ctx.epi_count([cid])
        w = ctx.epi_read_worklog(cid, c["N"].size)
        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 0)
        ctx.epi_count([cid], mode=epi.EPI_MODE_BATCHED, sched=epi.EPI_SCHED_LEARNED)
        assert np.array_equal(ctx.epi_read_counts(cid, c["N"].size), oracle.count(s, c))
        # the prediction is the base feature (log1p of the summed type event
        # counts) plus the standardised network: x23 + y_sd * net((x - mu) * isd) + y_mu
        m = c["N"].size
        X = ctx.epi_costmodel_features(cid, m)
        pred = ctx.epi_costmodel_predict(cid, m)
        mu, isd, y_mu, y_sd = ctx.epi_costmodel_scaling()
        assert np.all(isd >= 0) and y_sd > 0
        want = X[:, 23] + y_sd * mlp.forward(ctx.epi_mlp_get_params().astype(np.float64), (X - mu) * isd) + y_mu
        assert np.abs(pred - want).max() <= 1e-4 * np.abs(want).max()
        # predicted log-work tracks the logged work of unseen episodes, at
        # least as well as the type-count heuristic's log
        obs = np.log1p(w[:, 0] + w[:, 1] + w[:, 2])
        cnt = np.bincount(s["types"], minlength=s["K"])
        heur = np.log1p([cnt[c["types"][i, :c["N"][i]]].sum() for i in range(m)])
        r_learned = np.corrcoef(pred, obs)[0, 1]
        r_heur = np.corrcoef(heur, obs)[0, 1]
        say(f"corr(pred, work) = {r_learned:.4f}, corr(log sum n_type, work) = {r_heur:.4f}, "
            f"rmse {np.sqrt(np.mean((pred - obs) ** 2)):.3f} (sd {obs.std():.3f})")
        assert r_learned > 0.95
        # the network learns the correction of the log work relative to the
        # summed event counts of the types (the heuristic's cost): the records
        # and queries that depend on rates and windows
        assert r_learned >= r_heur
    finally:
        ctx.epi_set_option(epi.EPI_OPT_WORKLOG, 0)
        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 0)
        ctx.epi_release_set(tid)
        ctx.epi_release_set(cid)
        ctx.epi_release_stream(sid)


def test_measured_schedule_and_model_file(ctx, tmp_path):
    """The measured-cost schedule (each episode's logged work) is exact and
    needs a work log; a saved cost model loads back to the same predictions;
    malformed model files are rejected."""
    s = sg.config_stream(4, scale=0.005)
    train = sg.config_candidates(4, s, scale=0.02, training=True)
    c = sg.config_candidates(4, s, scale=0.01)
    want = oracle.count(s, c)
    sid = ctx.epi_load_stream(s["types"], s["times"], s["K"])
    tid = ctx.epi_submit_candidates(sid, train)
    cid = ctx.epi_submit_candidates(sid, c)
    m = c["N"].size
    try:
        ctx.epi_count([cid])
        with pytest.raises(epi.EpiError) as ei:
            ctx.epi_count([cid], mode=epi.EPI_MODE_BATCHED, sched=epi.EPI_SCHED_MEASURED)
        assert ei.value.code == epi.EPI_ESTATE
        ctx.epi_set_option(epi.EPI_OPT_WORKLOG, 1)
        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 1)
        ctx.epi_count([cid, tid])
        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 0)
        for rep in range(2):  # the second run schedules by the first run's log
            say(f"measured schedule, run {rep}")
            ctx.epi_count([cid], mode=epi.EPI_MODE_BATCHED, sched=epi.EPI_SCHED_MEASURED)
            assert np.array_equal(ctx.epi_read_counts(cid, m), want)
        # model file round trip
        ctx.epi_costmodel_train([tid], epochs=5, seed=11)
        pred = ctx.epi_costmodel_predict(cid, m)
        path = tmp_path / "cost.model"
        ctx.epi_costmodel_save(path)
        ctx.epi_mlp_init(24, 99)
        assert not np.array_equal(ctx.epi_costmodel_predict(cid, m), pred)
        ctx.epi_costmodel_load(path)
        assert np.array_equal(ctx.epi_costmodel_predict(cid, m), pred)
        blob = path.read_bytes()
        for bad in (blob[:-1], blob + b"\0", b"EPICM002" + blob[8:], b"nonsense"):
            path.write_bytes(bad)
            with pytest.raises(epi.EpiError) as ei:
                ctx.epi_costmodel_load(path)
            assert ei.value.code == epi.EPI_EINVAL
        assert np.array_equal(ctx.epi_costmodel_predict(cid, m), pred)  # a failed load keeps the model
    finally:
        ctx.epi_set_option(epi.EPI_OPT_WORKLOG, 0)
        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 0)
        ctx.epi_release_set(tid)
        ctx.epi_release_set(cid)
        ctx.epi_release_stream(sid)


def test_autotune_and_cache(ctx, tmp_path):
    s = sg.config_stream(4, scale=0.005)
    c = sg.config_candidates(4, s, scale=0.01)
    want = oracle.count(s, c)
    sid = ctx.epi_load_stream(s["types"], s["times"], s["K"])
    cid = ctx.epi_submit_candidates(sid, c)
    cache = tmp_path / "tune.txt"
    cache.write_text("garbage line\nts1_x 77 -3\nts1_x 4096 0 0 262144\n")  # malformed entries are ignored
    try:
        for sched in (epi.EPI_SCHED_RR, epi.EPI_SCHED_HEURISTIC):
            chosen = ctx.epi_autotune([cid], sched, cache)
            say(f"autotune sched={sched}: tile, ring classes, lanes, target = {chosen}")
            tile, rings, lanes, target = chosen
            assert tile in (4096, 2048, 1024, 512) and rings in (0, 1, 2) and lanes in (0, 64, 128)
            assert target in (131072, 262144, 524288, 1048576)
            assert np.array_equal(ctx.epi_read_counts(cid, c["N"].size), want)
            # the cache answers the second call
            assert ctx.epi_autotune([cid], sched, cache) == chosen
            ctx.epi_count([cid], mode=epi.EPI_MODE_BATCHED, sched=sched)
            assert np.array_equal(ctx.epi_read_counts(cid, c["N"].size), want)
            ctx.epi_count([cid], mode=epi.EPI_MODE_PLAIN)
            assert np.array_equal(ctx.epi_read_counts(cid, c["N"].size), want)
        assert len(cache.read_text().splitlines()) == 5
    finally:
        ctx.epi_set_option(epi.EPI_OPT_LANES, 0)
        ctx.epi_set_option(epi.EPI_OPT_RING_CLASSES, 0)
        ctx.epi_set_option(epi.EPI_OPT_TARGET_LANES, 262144)
        ctx.epi_release_set(cid)
        ctx.epi_release_stream(sid)


def test_batched_plan_reuse(ctx):
    """A repeated batched count of the same sets replays the kept graph: no
    new capture; every replay is exact and re-runs every kernel (the work
    log, cleared before each count, is complete again).  A changed option
    plans again; releasing a set drops the plans that count it."""
    recs = _recordings(n_rec=3)
    sids, cids, want = [], [], []
    for s, c in recs:
        sids.append(ctx.epi_load_stream(s["types"], s["times"], s["K"]))
        cids.append(ctx.epi_submit_candidates(sids[-1], c))
        want.append(oracle.count(s, c))
    ms = [c["N"].size for _, c in recs]
    try:
        st0 = ctx.epi_batched_stats()
        for sched in (epi.EPI_SCHED_RR, epi.EPI_SCHED_HEURISTIC):
            for rep in range(3):
                say(f"plan reuse: sched={sched} count {rep}")
                ctx.epi_count(cids, mode=epi.EPI_MODE_BATCHED, sched=sched)
                for cid, m, w in zip(cids, ms, want):
                    assert np.array_equal(ctx.epi_read_counts(cid, m), w)
                # eager work between replays
                ctx.epi_count(cids[:1], mode=epi.EPI_MODE_PLAIN)
                assert np.array_equal(ctx.epi_read_counts(cids[0], ms[0]), want[0])
        st1 = ctx.epi_batched_stats()
        assert st1["built"] - st0["built"] == 2
        assert st1["replays"] - st0["replays"] == 4
        # every replay runs the counting kernels: the work log is whole again
        ctx.epi_set_option(epi.EPI_OPT_WORKLOG, 1)
        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 1)
        logs = []
        for rep in range(2):
            ctx.epi_count(cids, mode=epi.EPI_MODE_BATCHED, sched=epi.EPI_SCHED_HEURISTIC)
            logs.append([ctx.epi_read_worklog(cid, m) for cid, m in zip(cids, ms)])
        for (s, c), w in zip(recs, logs[1]):
            cnt = np.bincount(s["types"], minlength=s["K"])
            visits = np.array([cnt[c["types"][i, :c["N"][i]]].sum() for i in range(c["N"].size)])
            np.testing.assert_array_equal(w[:, 0], visits)
        for a, b in zip(logs[0], logs[1]):
            np.testing.assert_array_equal(a, b)
        st2 = ctx.epi_batched_stats()
        assert st2["built"] - st1["built"] == 1 and st2["replays"] - st1["replays"] == 1
        ctx.epi_set_option(epi.EPI_OPT_WORKLOG, 0)
        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 0)
        kept = st2["kept"]
        ctx.epi_release_set(cids[0])
        cids = cids[1:]
        assert ctx.epi_batched_stats()["kept"] < kept
        ctx.epi_count(cids, mode=epi.EPI_MODE_BATCHED, sched=epi.EPI_SCHED_RR)
        for cid, m, w in zip(cids, ms[1:], want[1:]):
            assert np.array_equal(ctx.epi_read_counts(cid, m), w)
    finally:
        ctx.epi_set_option(epi.EPI_OPT_WORKLOG, 0)
        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 0)
        for cid in cids:
            ctx.epi_release_set(cid)
        for sid in sids:
            ctx.epi_release_stream(sid)


def _wave_efficiency(order, block, work):
    """Sum over the waves (64 lanes of a lane block) of the mean lane work
    over the sum of the maximum: 1 means no lane of a wave waits for another."""
    sel = np.flatnonzero(block >= 0)
    b = block[sel]
    first = np.zeros(b.max() + 1, np.int64)
    ub, idx = np.unique(b, return_index=True)
    first[ub] = sel[idx]
    wave = b.astype(np.int64) * 1024 + (sel - first[b]) // 64
    w = work[order[sel]].astype(np.float64)
    _, inv = np.unique(wave, return_inverse=True)
    mx = np.zeros(inv.max() + 1)
    np.maximum.at(mx, inv, w)
    return w.sum() / (mx * np.bincount(inv)).sum()


@pytest.mark.parametrize("rings", [0, 1])
def test_learned_schedule_gain(ctx, rings):
    """What the trained cost model gains over counting without it: on a slice
    of the Zipf-rate workload (128 types, rates ~ k^-1.2; 10k episodes) the
    learned lane order packs episodes of similar work into each wave, so far
    less lane time is spent waiting on the wave's slowest lane than in
    submission order (round robin).  Measured on each episode's own logged
    work (no segments), from the lane order each schedule produced; counts
    exact in every schedule.  With one launch group per episode size the order
    spans more episodes and the waves are more even still."""
    s = sg.config_stream(4, scale=0.01)
    train = sg.config_candidates(4, s, scale=0.1, training=True)
    c = sg.config_candidates(4, s, scale=0.2)
    m = c["N"].size
    want = oracle.count(s, c)
    sid = ctx.epi_load_stream(s["types"], s["times"], s["K"])
    tid = ctx.epi_submit_candidates(sid, train)
    cid = ctx.epi_submit_candidates(sid, c)
    try:
        ctx.epi_set_option(epi.EPI_OPT_WORKLOG, 1)
        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 1)
        ctx.epi_count([tid, cid])
        losses = ctx.epi_costmodel_train([tid], epochs=40, seed=3)
        w = ctx.epi_read_worklog(cid, m)
        work = w[:, 0].astype(np.int64) + w[:, 1] + w[:, 2]
        ctx.epi_set_option(epi.EPI_OPT_WORKLOG, 0)
        ctx.epi_set_option(epi.EPI_OPT_RING_CLASSES, rings)
        eff = {}
        for name, sched in (("rr", epi.EPI_SCHED_RR), ("heuristic", epi.EPI_SCHED_HEURISTIC),
                            ("learned", epi.EPI_SCHED_LEARNED)):
            ctx.epi_count([cid], mode=epi.EPI_MODE_BATCHED, sched=sched)
            assert np.array_equal(ctx.epi_read_counts(cid, m), want)
            order, block = ctx.epi_read_schedule(cid, m)
            assert np.array_equal(np.sort(order), np.arange(m))
            eff[name] = _wave_efficiency(order, block, work)
        say(f"wave efficiency (mean/max lane work): {eff}; model loss {losses[0]:.3f} -> {losses[-1]:.3f}")
        assert eff["learned"] > (2.0 if rings == 0 else 4.0) * eff["rr"]
        assert eff["learned"] >= 0.95 * eff["heuristic"]
    finally:
        ctx.epi_set_option(epi.EPI_OPT_RING_CLASSES, 0)
        ctx.epi_set_option(epi.EPI_OPT_WORKLOG, 0)
        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 0)
        ctx.epi_release_set(tid)
        ctx.epi_release_set(cid)
        ctx.epi_release_stream(sid)


def test_heuristic_schedule_is_a_stable_cost_sort(ctx):
    """The device scheduler's order, pinned exactly: with the heuristic cost
    (the summed event counts of an episode's types, an integer the host can
    compute) every launch group's lanes hold its episodes sorted by descending
    cost, equal costs in submission order (the radix sort is stable), and the
    groups stay where round robin puts them.  Two sets on two streams, so the
    global slot order spans sets."""
    recs = _recordings(n_rec=2)
    sids, cids = [], []
    for s, c in recs:
        sids.append(ctx.epi_load_stream(s["types"], s["times"], s["K"]))
        cids.append(ctx.epi_submit_candidates(sids[-1], c))
    try:
        ctx.epi_count(cids, mode=epi.EPI_MODE_BATCHED, sched=epi.EPI_SCHED_RR)
        rr = [ctx.epi_read_schedule(cid, c["N"].size) for cid, (_, c) in zip(cids, recs)]
        ctx.epi_count(cids, mode=epi.EPI_MODE_BATCHED, sched=epi.EPI_SCHED_HEURISTIC)
        for (s, c), cid, (rr_order, rr_block) in zip(recs, cids, rr):
            m = c["N"].size
            assert np.array_equal(ctx.epi_read_counts(cid, m), oracle.count(s, c))
            order, block = ctx.epi_read_schedule(cid, m)
            assert np.array_equal(block, rr_block)  # same lane blocks
            cnt = np.bincount(s["types"], minlength=s["K"])
            cost = np.array([cnt[c["types"][i, :c["N"][i]]].sum() for i in range(m)])
            # launch groups (the submission groups): episode size x class of
            # ring entries (the sum over intervals of 1 + hi // (hi - lo + 1),
            # rounded up to 1..8, 10, 12, 14, 16, 20, ..., 112); in the
            # round-robin lane order each group is a run, in submission order
            live = np.arange(7)[None, :] < (c["N"].astype(np.int64) - 1)[:, None]
            ring = np.where(live, 1 + c["hi"] // np.maximum(c["hi"] - c["lo"] + 1, 1), 0).sum(axis=1)
            caps = np.array([1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20, 24, 28, 32, 40, 48, 56, 64, 80, 96, 112])
            key = c["N"].astype(np.int64) * 64 + np.searchsorted(caps, np.maximum(ring, 1))
            k_rr = key[rr_order]
            assert np.all(np.diff(k_rr) >= 0)
            grp = np.concatenate([[0], np.cumsum(k_rr[1:] != k_rr[:-1])])
            for g in np.unique(grp):
                sl = np.flatnonzero(grp == g)
                members = rr_order[sl]  # submission order
                want = members[np.argsort(-cost[members], kind="stable")]
                assert np.array_equal(order[sl], want), f"group {g}"
        say(f"heuristic lane order equals a stable descending sort of the summed type counts in every group")
    finally:
        for cid in cids:
            ctx.epi_release_set(cid)
        for sid in sids:
            ctx.epi_release_stream(sid)
