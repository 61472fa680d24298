"""Full-size parity: every count of the five workload presets, at their full
sizes and in the launch configurations the benchmark times, equals the CPU
oracle's (the frequency of Sec. II-C computed by the decomposition of
Sec. IV-A and the greedy of Alg. 1).  The expected values were written by
``tests/golden/make_full_parity.py``, which calls only ``oracle/``; each
golden file records fingerprints of the seeded inputs it was computed from,
checked here first.

* presets 1, 3, 4, 5: every count, element by element, from the plain engine,
  the batched engine with round-robin order and the batched engine with the
  learned schedule (cost model trained here on a disjoint candidate set);
* preset 2 (level-wise discovery): per level the number of candidates and of
  frequent episodes and an order-independent digest of all (episode, count)
  rows and of the frequent ones."""
import os
import sys

import numpy as np
import pytest

import spikegen as sg
from paper_0905_2203_amd import epi

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from fullsize import MultisetDigest, cand_fingerprint, load_counts, load_json, stream_fingerprint  # noqa: E402

pytestmark = pytest.mark.gpu

MODES = [("plain", epi.EPI_MODE_PLAIN, epi.EPI_SCHED_RR), ("batched_rr", epi.EPI_MODE_BATCHED, epi.EPI_SCHED_RR),
         ("batched_learned", epi.EPI_MODE_BATCHED, epi.EPI_SCHED_LEARNED)]


def say(msg):
    print(f"[gpu-fullsize] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = epi.Context(0)
    yield c
    c.close()


def _train(ctx, sids_and_train):
    """Train the cost model on the work log of disjoint candidates (one
    episode's own work: no time segments)."""
    ctx.epi_set_option(epi.EPI_OPT_WORKLOG, 1)
    ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 1)
    tids = []
    try:
        tids = [ctx.epi_submit_candidates(sid, c) for sid, c in sids_and_train]
        ctx.epi_count(tids, mode=epi.EPI_MODE_BATCHED, sched=epi.EPI_SCHED_RR)
        losses = ctx.epi_costmodel_train(tids, epochs=20, seed=5)
        say(f"cost model trained on {sum(c['N'].size for _, c in sids_and_train)} episodes: "
            f"loss {losses[0]:.3f} -> {losses[-1]:.3f}")
    finally:
        ctx.epi_set_option(epi.EPI_OPT_WORKLOG, 0)
        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 0)
        for t in tids:
            ctx.epi_release_set(t)


def _check_modes(ctx, name, cids, sizes, wants):
    for mname, mode, sched in MODES:
        ctx.epi_count(cids, mode=mode, sched=sched)
        for i, (cid, m, want) in enumerate(zip(cids, sizes, wants)):
            got = ctx.epi_read_counts(cid, m)
            bad = np.nonzero(got != want)[0]
            assert bad.size == 0, (f"{name} {mname} set {i}: {bad.size} of {m} counts differ, first at "
                                   f"{bad[:5]}: got {got[bad[:5]]} want {want[bad[:5]]}")
        say(f"{name} {mname}: {sum(sizes)} counts equal to the oracle's")


def _single(ctx, k, train_rng_offset, train_m, train_K, train_nmin):
    meta, arrays = load_counts(f"full_cfg{k}.npz")
    s = sg.config_stream(k)
    c = sg.config_candidates(k, s)
    assert stream_fingerprint(s) == meta["stream"] and cand_fingerprint(c) == meta["candidates"], \
        f"preset {k}: the seeded inputs differ from those the expected counts were computed from"
    want = arrays["counts"]
    say(f"preset {k}: n={s['types'].size} m={c['N'].size}")
    sid = ctx.epi_load_stream(s["types"], s["times"], s["K"])
    cid = ctx.epi_submit_candidates(sid, c)
    try:
        if k == 4:
            train = sg.config_candidates(4, s, scale=train_m / 50_000, training=True)
        else:
            train = sg.random_candidates(sg.rng_for(k, offset=train_rng_offset), train_m, train_K, train_nmin, 8,
                                         s["unit_per_ms"])
        _train(ctx, [(sid, train)])
        _check_modes(ctx, f"preset {k}", [cid], [c["N"].size], [want])
    finally:
        ctx.epi_release_set(cid)
        ctx.epi_release_stream(sid)


def test_fullsize_preset1_all_pairs(ctx):
    _single(ctx, 1, 100, 2000, 32, 2)


def test_fullsize_preset4_zipf(ctx):
    _single(ctx, 4, 100, 5000, 128, 3)


def test_fullsize_preset5_large(ctx):
    _single(ctx, 5, 100, 5000, 256, 2)


def test_fullsize_preset3_sixteen_recordings(ctx):
    meta, arrays = load_counts("full_cfg3.npz")
    sids, cids, sizes, wants, train = [], [], [], [], []
    try:
        for r in range(16):
            s = sg.config_stream(3, recording=r)
            c = sg.config_candidates(3, s, recording=r)
            rm = meta["recordings"][r]
            assert stream_fingerprint(s) == rm["stream"] and cand_fingerprint(c) == rm["candidates"], \
                f"preset 3 recording {r}: the seeded inputs differ from the expected counts' inputs"
            sids.append(ctx.epi_load_stream(s["types"], s["times"], s["K"]))
            cids.append(ctx.epi_submit_candidates(sids[-1], c))
            sizes.append(c["N"].size)
            wants.append(arrays[f"counts_r{r}"])
            if r < 4:
                train.append((sids[-1], sg.random_candidates(sg.rng_for(3, offset=3000 + r), 1000, 60, 2, 8,
                                                             1_000_000)))
        say(f"preset 3: {len(sids)} recordings, {sum(sizes)} candidates")
        _train(ctx, train)
        _check_modes(ctx, "preset 3", cids, sizes, wants)
    finally:
        for c in cids:
            ctx.epi_release_set(c)
        for s in sids:
            ctx.epi_release_stream(s)


def test_fullsize_preset2_levelwise_digests(ctx):
    ref = load_json("full_cfg2.json")
    s = sg.config_stream(2)
    assert stream_fingerprint(s) == ref["stream"], "preset 2: the seeded stream differs from the expected one's"
    sid = ctx.epi_load_stream(s["types"], s["times"], s["K"])
    mid = ctx.epi_mine(sid, [tuple(x) for x in ref["menu"]], ref["max_size"], ref["threshold"])
    try:
        nl = ctx.epi_mine_levels(mid)
        assert nl == len(ref["levels"])
        for L, want in enumerate(ref["levels"], start=1):
            m, nf, _ = ctx.epi_mine_level_info(mid, L)
            assert (m, nf) == (want["candidates"], want["frequent"]), f"level {L}: sizes"
            d_all, d_freq = MultisetDigest(), MultisetDigest()
            step = 1 << 23
            for a in range(0, m, step):
                idx = np.arange(a, min(m, a + step), dtype=np.int64)
                c, cnt = ctx.epi_mine_read_at(mid, L, idx)
                d_all.add(c["N"], c["types"], c["lo"], c["hi"], cnt)
            fc, fcnt = ctx.epi_mine_read(mid, L, frequent_only=True)
            assert np.all(fcnt > ref["threshold"])
            d_freq.add(fc["N"], fc["types"], fc["lo"], fc["hi"], fcnt)
            assert d_all.as_dict() == want["all"], f"level {L}: (episode, count) rows differ from the oracle's"
            assert d_freq.as_dict() == want["frequent_rows"], f"level {L}: frequent episodes differ"
            say(f"preset 2 level {L}: {m} candidates and {nf} frequent episodes equal the oracle's")
    finally:
        ctx.epi_mine_release(mid)
        ctx.epi_release_stream(sid)
