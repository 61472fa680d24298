"""The per-event tracking engine (EPI_MODE_TRACKING: Parallel Local Tracking
of Sec. IV-C, order-preserving compaction, the greedy of Alg. 1) counts
bit-exact against the oracle: long planted episodes and all their prefixes,
random episodes of sizes 1 to 8, a type with no events, equal-time events,
int32 and int64 streams, repeated types, a type with over two million events
(more than 1024 compaction blocks and 22 pointer-jumping rounds), an empty
set, incremental counting after appends that resumes from the tracking
count's last completions, and stream-order overlap (EPI_OPT_STREAM_ORDER)
against the oracle's stream-order state machine."""
import numpy as np
import pytest

import oracle
import spikegen as sg
from paper_0905_2203_amd import epi

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-tracking] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = epi.Context(0)
    yield c
    c.close()


def _planted_family(s):
    """The planted episodes, their prefixes and their suffixes."""
    eps = []
    for p in s["planted"]:
        ty, lo, hi = [int(x) for x in p["types"]], [int(x) for x in p["lo"]], [int(x) for x in p["hi"]]
        for k in range(1, len(ty) + 1):
            eps.append((ty[:k], lo[: k - 1], hi[: k - 1]))
        for k in range(1, len(ty) - 1):
            eps.append((ty[k:], lo[k:], hi[k:]))
    return eps


def _random_long(rng, m, K, unit):
    eps = []
    for _ in range(m):
        n = int(rng.integers(1, min(8, K) + 1))
        ty = rng.permutation(K)[:n].tolist()
        lo = [int(rng.integers(0, 12)) * unit for _ in range(n - 1)]
        hi = [a + int(rng.integers(1, 15)) * unit for a in lo]
        eps.append((ty, lo, hi))
    return eps


def _count_both(ctx, s, c, K=None):
    sid = ctx.epi_load_stream(s["types"], s["times"], K or s["K"])
    cid = ctx.epi_submit_candidates(sid, c)
    try:
        ctx.epi_count([cid], mode=epi.EPI_MODE_TRACKING)
        got = ctx.epi_read_counts(cid, c["N"].size)
        ctx.epi_count([cid], mode=epi.EPI_MODE_PLAIN)
        plain = ctx.epi_read_counts(cid, c["N"].size)
    finally:
        ctx.epi_release_set(cid)
        ctx.epi_release_stream(sid)
    return got, plain


@pytest.mark.parametrize("ts_kind", [0, 1], ids=["int32_us", "int64_ns"])
def test_tracking_long_episodes(ctx, ts_kind):
    unit = 1000 if ts_kind == 0 else 1_000_000
    rng = np.random.Generator(np.random.PCG64(81 + ts_kind))
    s = sg.poisson_stream(rng, K=16, rate_hz=30.0, dur_s=60.0, ts_kind=ts_kind, unit_per_ms=unit, cascades=[8, 6],
                          cascade_trigger_hz=[4.0, 6.0])
    # declared with one more type than occurs: type 16 has no events
    eps = _planted_family(s) + _random_long(rng, 60, 17, unit) + [([16], [], []), ([3, 16, 4], [0, 0], [unit, unit])]
    c = sg.candidates_from_list(eps)
    want = oracle.count(s, c)
    say(f"{ts_kind=}: n={s['types'].size}, {c['N'].size} candidates, planted counts {want[:8].tolist()}")
    assert want[7] > 100  # the planted 8-node episode occurs
    got, plain = _count_both(ctx, s, c, K=17)
    assert np.array_equal(plain, want)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} differ, e.g. #{bad[0]}: got {got[bad[0]]} want {want[bad[0]]}"


def test_tracking_equal_times(ctx):
    rng = np.random.Generator(np.random.PCG64(83))
    s = sg.poisson_stream(rng, K=6, rate_hz=40.0, dur_s=40.0, ts_kind=0, unit_per_ms=1000, cascades=[5],
                          cascade_trigger_hz=[5.0])
    s["times"] = np.ascontiguousarray(s["times"] // 2000 * 2000, dtype=np.int32)  # a 2 ms grid
    eps = _planted_family(s) + _random_long(rng, 80, 6, 1000)
    eps += [([a, b], [0], [2000]) for a in range(6) for b in range(6) if a != b]
    c = sg.candidates_from_list(eps)
    want = oracle.count(s, c)
    got, plain = _count_both(ctx, s, c)
    assert np.array_equal(plain, want)
    assert np.array_equal(got, want)


def test_tracking_repeated_types(ctx):
    rng = np.random.Generator(np.random.PCG64(84))
    s = sg.poisson_stream(rng, K=4, rate_hz=25.0, dur_s=40.0, ts_kind=1, unit_per_ms=1_000_000)
    ms = 1_000_000
    eps = [([0, 0], [0], [5 * ms]), ([1, 1, 1], [0, 0], [3 * ms, 3 * ms]), ([2, 0, 2, 0], [ms, 0, ms],
                                                                             [6 * ms, 4 * ms, 6 * ms])]
    for _ in range(60):
        n = int(rng.integers(2, 8))
        ty = [int(x) for x in rng.integers(0, 4, size=n)]
        lo = [int(rng.integers(0, 10)) * ms for _ in range(n - 1)]
        eps.append((ty, lo, [a + int(rng.integers(2, 12)) * ms for a in lo]))
    c = sg.candidates_from_list(eps)
    want = oracle.count(s, c)
    assert want.sum() > 0
    ctx.epi_set_option(epi.EPI_OPT_ALLOW_REPEATS, 1)
    try:
        got, plain = _count_both(ctx, s, c)
    finally:
        ctx.epi_set_option(epi.EPI_OPT_ALLOW_REPEATS, 0)
    assert np.array_equal(plain, want)
    assert np.array_equal(got, want)


def test_tracking_heavy_type_and_empty_set(ctx):
    # type 0 alone has about 2.4 million events
    rng = np.random.Generator(np.random.PCG64(85))
    s = sg.poisson_stream(rng, K=3, rate_hz=[20000.0, 3000.0, 800.0], dur_s=120.0, ts_kind=0, unit_per_ms=1000)
    n0 = int((s["types"] == 0).sum())
    say(f"n={s['types'].size}, type 0: {n0}")
    assert n0 > 2 * 1024 * 2048 // 2
    eps = [([0], [], []), ([0, 0], [0], [40]), ([1, 0], [0], [30]), ([0, 1, 0], [0, 0], [200, 50]),
           ([2, 0, 1, 0, 0], [0, 10, 0, 0], [300, 100, 200, 30]), ([0, 2], [100, ], [2000])]
    c = sg.candidates_from_list(eps)
    want = oracle.count(s, c)
    say(f"counts {want.tolist()}")
    ctx.epi_set_option(epi.EPI_OPT_ALLOW_REPEATS, 1)
    try:
        got, plain = _count_both(ctx, s, c)
        sid = ctx.epi_load_stream(s["types"], s["times"], s["K"])
        cid = ctx.epi_submit_candidates(sid, sg.empty_candidates(0))
        ctx.epi_count([cid], mode=epi.EPI_MODE_TRACKING)
        ctx.epi_release_set(cid)
        ctx.epi_release_stream(sid)
    finally:
        ctx.epi_set_option(epi.EPI_OPT_ALLOW_REPEATS, 0)
    assert np.array_equal(plain, want)
    assert np.array_equal(got, want)


def test_tracking_then_incremental(ctx):
    rng = np.random.Generator(np.random.PCG64(86))
    s = sg.poisson_stream(rng, K=8, rate_hz=20.0, dur_s=60.0, ts_kind=1, unit_per_ms=1_000_000, cascades=[6],
                          cascade_trigger_hz=[5.0])
    n = s["types"].size
    cut = int(0.55 * n)
    t = s["times"].copy()
    t[cut] = t[cut - 1]  # an equal time across the boundary
    s["times"] = t
    c = sg.candidates_from_list(_planted_family(s) + _random_long(rng, 60, 8, 1_000_000))
    pre = dict(types=s["types"][:cut], times=s["times"][:cut], K=s["K"], ts_kind=1)
    sid = ctx.epi_load_stream(pre["types"], pre["times"], s["K"])
    cid = ctx.epi_submit_candidates(sid, c)
    try:
        ctx.epi_count([cid], mode=epi.EPI_MODE_TRACKING)
        assert np.array_equal(ctx.epi_read_counts(cid, c["N"].size), oracle.count(pre, c))
        ctx.epi_append_stream(sid, s["types"][cut:], s["times"][cut:])
        ctx.epi_count([cid], mode=epi.EPI_MODE_INCREMENTAL)
        assert np.array_equal(ctx.epi_read_counts(cid, c["N"].size), oracle.count(s, c))
    finally:
        ctx.epi_release_set(cid)
        ctx.epi_release_stream(sid)


@pytest.mark.parametrize("ts_kind", [0, 1], ids=["int32_us", "int64_ns"])
def test_tracking_stream_order(ctx, ts_kind):
    # dense equal times (a 2 ms grid), so that stream-order and time overlap
    # differ; one-node episodes, long planted ones, repeated types
    unit = 1000 if ts_kind == 0 else 1_000_000
    rng = np.random.Generator(np.random.PCG64(87 + ts_kind))
    s = sg.poisson_stream(rng, K=12, rate_hz=40.0, dur_s=40.0, ts_kind=ts_kind, unit_per_ms=unit, cascades=[6],
                          cascade_trigger_hz=[6.0])
    s["times"] = np.ascontiguousarray(s["times"] // (2 * unit) * (2 * unit), dtype=s["times"].dtype)
    eps = _planted_family(s) + _random_long(rng, 60, 12, unit)
    eps += [([a, b], [0], [2 * unit]) for a in range(4) for b in range(4)]  # includes a == b
    eps += [([0, 1, 0], [0, 0], [4 * unit, 4 * unit]), ([2, 2, 2], [0, 0], [2 * unit, 6 * unit])]
    c = sg.candidates_from_list(eps)
    want = oracle.count(s, c, "fsm_stream")
    timewise = oracle.count(s, c, "decomp")
    say(f"{ts_kind=}: n={s['types'].size}, {c['N'].size} candidates, {(want != timewise).sum()} differ by semantics")
    assert (want != timewise).sum() > 10
    sid = ctx.epi_load_stream(s["types"], s["times"], s["K"])
    ctx.epi_set_option(epi.EPI_OPT_ALLOW_REPEATS, 1)
    ctx.epi_set_option(epi.EPI_OPT_STREAM_ORDER, 1)
    try:
        cid = ctx.epi_submit_candidates(sid, c)
    finally:
        ctx.epi_set_option(epi.EPI_OPT_STREAM_ORDER, 0)
        ctx.epi_set_option(epi.EPI_OPT_ALLOW_REPEATS, 0)
    try:
        ctx.epi_count([cid], mode=epi.EPI_MODE_TRACKING)
        got = ctx.epi_read_counts(cid, c["N"].size)
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, f"{bad.size} differ, e.g. #{bad[0]} {eps[bad[0]]}: got {got[bad[0]]} want {want[bad[0]]}"
        with pytest.raises(epi.EpiError) as err:  # the state-machine engines decide overlap on times
            ctx.epi_count([cid], mode=epi.EPI_MODE_PLAIN)
        assert err.value.code == epi.EPI_EINVAL
    finally:
        ctx.epi_release_set(cid)
        ctx.epi_release_stream(sid)
