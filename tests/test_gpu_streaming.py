"""Streaming: events appended to a loaded stream (epi_append_stream) and
counted incrementally (EPI_MODE_INCREMENTAL) give exactly the oracle's count
of the whole stream so far, whatever the first count's mode (plain with
segments, batched), with equal times across every append boundary; a set
submitted after appends is counted fully; a full recount after appends agrees;
bad appends are rejected and change nothing."""
import numpy as np
import pytest

import oracle
import spikegen as sg
from paper_0905_2203_amd import epi

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-streaming] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = epi.Context(0)
    yield c
    c.close()


def _workload(ts_kind, seed):
    unit = 1000 if ts_kind == 0 else 1_000_000
    rng = np.random.Generator(np.random.PCG64(seed))
    s = sg.poisson_stream(rng, K=8, rate_hz=20.0, dur_s=60.0, ts_kind=ts_kind, unit_per_ms=unit, cascades=[4],
                          cascade_trigger_hz=[5.0])
    n = s["types"].size
    cuts = [int(0.4 * n), int(0.75 * n)]
    t = s["times"].copy()
    for c in cuts:  # an equal time across every boundary
        t[c] = t[c - 1]
    s["times"] = t
    c = sg.concat_candidates(sg.random_candidates(rng, 150, s["K"], 2, 5, unit),
                             sg.all_pairs(s["K"], 0, 10 * unit))
    return s, c, cuts


def _prefix(s, end):
    return dict(types=s["types"][:end], times=s["times"][:end], K=s["K"], ts_kind=s["ts_kind"])


@pytest.mark.parametrize("first", ["plain_segments", "batched"])
@pytest.mark.parametrize("ts_kind", [0, 1], ids=["int32_us", "int64_ns"])
def test_streaming_matches_full_count(ctx, ts_kind, first):
    s, c, (c1, c2) = _workload(ts_kind, 71 + ts_kind)
    n = s["types"].size
    m = c["N"].size
    say(f"{ts_kind=} {first}: n={n}, cuts {c1} {c2}, {m} candidates")
    sid = ctx.epi_load_stream(s["types"][:c1], s["times"][:c1], s["K"])
    cid = ctx.epi_submit_candidates(sid, c)
    try:
        if first == "plain_segments":
            ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 3)
            ctx.epi_count([cid], mode=epi.EPI_MODE_PLAIN)
            ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 0)
        else:
            ctx.epi_count([cid], mode=epi.EPI_MODE_BATCHED, sched=epi.EPI_SCHED_RR)
        assert np.array_equal(ctx.epi_read_counts(cid, m), oracle.count(_prefix(s, c1), c))
        # second chunk
        ctx.epi_append_stream(sid, s["types"][c1:c2], s["times"][c1:c2])
        ctx.epi_count([cid], mode=epi.EPI_MODE_INCREMENTAL)
        want2 = oracle.count(_prefix(s, c2), c)
        assert np.array_equal(ctx.epi_read_counts(cid, m), want2), "after the first append"
        # an empty append, then the rest
        ctx.epi_append_stream(sid, s["types"][:0], s["times"][:0])
        ctx.epi_append_stream(sid, s["types"][c2:], s["times"][c2:])
        ctx.epi_count([cid], mode=epi.EPI_MODE_INCREMENTAL)
        want = oracle.count(s, c)
        assert np.array_equal(ctx.epi_read_counts(cid, m), want), "after the second append"
        # nothing appended since: unchanged
        ctx.epi_count([cid], mode=epi.EPI_MODE_INCREMENTAL)
        assert np.array_equal(ctx.epi_read_counts(cid, m), want)
        # a set submitted after the appends is counted fully; a full recount agrees
        cid2 = ctx.epi_submit_candidates(sid, c)
        ctx.epi_count([cid2], mode=epi.EPI_MODE_INCREMENTAL)
        assert np.array_equal(ctx.epi_read_counts(cid2, m), want)
        ctx.epi_release_set(cid2)
        ctx.epi_count([cid], mode=epi.EPI_MODE_PLAIN)
        assert np.array_equal(ctx.epi_read_counts(cid, m), want)
    finally:
        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 0)
        ctx.epi_release_set(cid)
        ctx.epi_release_stream(sid)


def test_bad_appends_change_nothing(ctx):
    s, c, (c1, _) = _workload(0, 79)
    m = c["N"].size
    sid = ctx.epi_load_stream(s["types"][:c1], s["times"][:c1], s["K"])
    cid = ctx.epi_submit_candidates(sid, c)
    try:
        ctx.epi_count([cid], mode=epi.EPI_MODE_PLAIN)
        want = oracle.count(_prefix(s, c1), c)
        with pytest.raises(epi.EpiError) as err:  # the first appended time precedes the last one
            ctx.epi_append_stream(sid, np.array([0], np.int32), np.array([s["times"][c1 - 1] - 1], np.int32))
        assert err.value.code == epi.EPI_EUNSORTED
        with pytest.raises(epi.EpiError) as err:
            ctx.epi_append_stream(sid, np.array([s["K"]], np.int32), np.array([s["times"][c1 - 1]], np.int32))
        assert err.value.code == epi.EPI_ETYPE
        n_after = ctx.epi_stream_info(sid)[0]
        assert n_after == c1
        ctx.epi_count([cid], mode=epi.EPI_MODE_INCREMENTAL)
        assert np.array_equal(ctx.epi_read_counts(cid, m), want)
    finally:
        ctx.epi_release_set(cid)
        ctx.epi_release_stream(sid)


def test_append_beyond_the_span_headroom_is_rejected(ctx):
    """An int32 stream appended to near INT32_MAX: times + the longest span of
    a set (or of a mining run) on the stream would leave the type, so the
    append is refused (EPI_EOVERFLOW) and the stream and counts are unchanged;
    an append that keeps the headroom is accepted.  Sets submitted while the
    stream was empty are checked too."""
    imax = np.iinfo(np.int32).max
    span = 30_000  # 3 nodes, (0, 10000] and (5000, 20000]
    c = sg.candidates_from_list([([0, 1, 2], [0, 5000], [10_000, 20_000]), ([1, 2], [0], [5000])])
    m = c["N"].size
    sid = ctx.epi_load_stream(np.zeros(0, np.int32), np.zeros(0, np.int32), 3)
    cid = ctx.epi_submit_candidates(sid, c)  # on the empty stream: nothing to check yet
    try:
        ok_t = np.array([imax - 1 - span - 20, imax - 1 - span - 10, imax - 1 - span], np.int32)
        ctx.epi_append_stream(sid, np.array([0, 1, 2], np.int32), ok_t)
        ctx.epi_count([cid], mode=epi.EPI_MODE_PLAIN)
        before = ctx.epi_read_counts(cid, m)
        say(f"append near INT32_MAX accepted up to {int(ok_t[-1])}")
        with pytest.raises(epi.EpiError) as err:
            ctx.epi_append_stream(sid, np.array([2], np.int32), np.array([imax - span], np.int32))
        assert err.value.code == epi.EPI_EOVERFLOW
        assert ctx.epi_stream_info(sid)[0] == 3
        ctx.epi_count([cid], mode=epi.EPI_MODE_INCREMENTAL)
        assert np.array_equal(ctx.epi_read_counts(cid, m), before)
        s_now = dict(types=np.array([0, 1, 2], np.int32), times=ok_t, K=3, ts_kind=0)
        assert np.array_equal(before, oracle.count(s_now, c))
    finally:
        ctx.epi_release_set(cid)
        ctx.epi_release_stream(sid)
