"""The register-indexed lane machines (EPI_OPT_LANE_ENGINE = 1, the default)
against the CPU oracle and against the LDS-ring machines, on streams that
take each key form: int32 microsecond streams and int64 nanosecond streams
whose tiles fit relative times below 2^29 - 1 (packed (time, node) keys,
unsigned: one stream's tiles span between 2^28 and 2^29 ns, where a signed
key would wrap), bursty nanosecond streams that need smaller tiles or fit
only 30 bits (separate keys); every episode size 1..8, per-node ring depths from 1 to the limit,
forced segment counts, plain and batched modes.  Episodes with an interval
deeper than the rings (bound > 15) are counted by the per-event tracking
engine in every mode; they are legal (Sec. II-C admits any 0 <= lo < hi)
and checked here too."""
import numpy as np
import pytest

import oracle
import spikegen as sg
from paper_0905_2203_amd import epi

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-lane] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = epi.Context(0)
    yield c
    c.close()


def _streams():
    rng = np.random.Generator(np.random.PCG64(501))
    yield "int32_us", sg.poisson_stream(rng, K=12, rate_hz=30.0, dur_s=40.0, ts_kind=0, unit_per_ms=1000,
                                        cascades=[5], cascade_trigger_hz=[6.0])
    yield "int64_ns_dense", sg.poisson_stream(rng, K=16, rate_hz=60.0, dur_s=20.0, ts_kind=1, unit_per_ms=1_000_000,
                                              cascades=[6], cascade_trigger_hz=[8.0])
    yield "int64_ns_bursty", sg.bursty_stream(rng, K=10, dur_s=120.0, shape=2.0, scale_hz=3.0)
    yield "int64_ns_sparse", sg.poisson_stream(rng, K=8, rate_hz=2.0, dur_s=900.0, ts_kind=1, unit_per_ms=1_000_000)
    yield "int64_ns_29bit", sg.poisson_stream(rng, K=8, rate_hz=80.0, dur_s=20.0, ts_kind=1, unit_per_ms=1_000_000)


def _longest_tile(times, T):
    """Longest time span of the T-event tiles of a stream (the library's tile
    choice takes the largest power-of-two tile whose spans fit the keys)."""
    n = times.size
    last = np.minimum(np.arange(T - 1, n + T - 1, T), n - 1)
    return int((times[last] - times[::T]).max())


def _episodes(rng, K, unit, m):
    c = sg.random_candidates(rng, m, K, 1, min(8, K), unit)
    # per-node ring bounds from 1 to 15: lo = a * w for w = (hi - lo)
    deep = []
    for i in range(8):
        n = int(rng.integers(2, min(8, K) + 1))
        ty = rng.permutation(K)[:n].tolist()
        lo, hi = [], []
        for _ in range(n - 1):
            w = int(rng.integers(1, 6)) * unit
            a = int(rng.integers(0, 14))
            lo.append(a * w)
            hi.append(a * w + w)
        deep.append((ty, lo, hi))
    return sg.concat_candidates(c, sg.candidates_from_list(deep))


def _deep(rng, K, unit):
    """Episodes with an interval beyond the rings: (95, 100] and (190, 200] ms."""
    eps = []
    for i in range(12):
        n = int(rng.integers(2, min(5, K) + 1))
        ty = rng.permutation(K)[:n].tolist()
        ivs = [[(0, 10), (95, 100), (190, 200), (5, 10)][int(rng.integers(0, 4))] for _ in range(n - 1)]
        ivs[int(rng.integers(0, n - 1))] = (95, 100) if i % 2 else (190, 200)
        eps.append((ty, [a * unit for a, _ in ivs], [b * unit for _, b in ivs]))
    return sg.candidates_from_list(eps)


def _count(ctx, cid, m, mode=epi.EPI_MODE_PLAIN, sched=epi.EPI_SCHED_RR):
    ctx.epi_count([cid], mode=mode, sched=sched)
    return ctx.epi_read_counts(cid, m)


@pytest.mark.parametrize("name", ["int32_us", "int64_ns_dense", "int64_ns_bursty", "int64_ns_sparse", "int64_ns_29bit"])
def test_lane_machines_equal_oracle(ctx, name):
    s = dict(_streams())[name]
    unit = s["unit_per_ms"]
    if name == "int64_ns_29bit":
        # the premise: 512-event tiles are too long for the packed keys, 256-event
        # tiles fit them with relative times of 2^28 ns or more
        assert _longest_tile(s["times"], 512) >= (1 << 29) - 1
        assert (1 << 28) <= _longest_tile(s["times"], 256) < (1 << 29) - 1
    seed = {"int32_us": 11, "int64_ns_dense": 12, "int64_ns_bursty": 13, "int64_ns_sparse": 14,
            "int64_ns_29bit": 15}[name]
    rng = np.random.Generator(np.random.PCG64(seed))
    c = sg.concat_candidates(_episodes(rng, s["K"], unit, 600), _deep(rng, s["K"], unit))
    m = c["N"].size
    want = oracle.count(s, c)
    say(f"{name}: n={s['types'].size} m={m} max count {int(want.max())}")
    sid = ctx.epi_load_stream(s["types"], s["times"], s["K"])
    cid = ctx.epi_submit_candidates(sid, c)
    try:
        for lane in (1, 0):
            ctx.epi_set_option(epi.EPI_OPT_LANE_ENGINE, lane)
            for seg in (1, 3, 17, 0):
                ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, seg)
                got = _count(ctx, cid, m)
                bad = np.nonzero(got != want)[0]
                assert bad.size == 0, f"lane={lane} seg={seg}: {bad.size} differ, e.g. {bad[:4]} {got[bad[:4]]} {want[bad[:4]]}"
            ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 0)
            for sched in (epi.EPI_SCHED_RR, epi.EPI_SCHED_HEURISTIC):
                got = _count(ctx, cid, m, epi.EPI_MODE_BATCHED, sched)
                assert np.array_equal(got, want), f"lane={lane} batched sched={sched}"
            say(f"{name}: lane={lane} plain (segments 1, 3, 17, auto) and batched equal the oracle")
    finally:
        ctx.epi_set_option(epi.EPI_OPT_LANE_ENGINE, 1)
        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 0)
        ctx.epi_release_set(cid)
        ctx.epi_release_stream(sid)


def test_deep_intervals_every_mode(ctx):
    """(95, 100] and (190, 200] ms intervals: bounds 20 and 19; the tracking
    engine counts them inside plain, batched and incremental counts."""
    rng = np.random.Generator(np.random.PCG64(507))
    s = sg.poisson_stream(rng, K=6, rate_hz=25.0, dur_s=60.0, ts_kind=1, unit_per_ms=1_000_000)
    c = sg.concat_candidates(_deep(rng, 6, 1_000_000), sg.random_candidates(rng, 40, 6, 2, 5, 1_000_000))
    m = c["N"].size
    n = s["types"].size
    cut = n // 2
    pre = dict(types=s["types"][:cut], times=s["times"][:cut], K=6, ts_kind=1)
    sid = ctx.epi_load_stream(pre["types"], pre["times"], 6)
    cid = ctx.epi_submit_candidates(sid, c)
    try:
        assert np.array_equal(_count(ctx, cid, m), oracle.count(pre, c))
        assert np.array_equal(_count(ctx, cid, m, epi.EPI_MODE_BATCHED, epi.EPI_SCHED_HEURISTIC), oracle.count(pre, c))
        ctx.epi_append_stream(sid, s["types"][cut:], s["times"][cut:])
        want = oracle.count(s, c)
        assert np.array_equal(_count(ctx, cid, m, epi.EPI_MODE_INCREMENTAL), want)
        assert np.array_equal(_count(ctx, cid, m, epi.EPI_MODE_TRACKING), want)
        say(f"deep intervals: {m} episodes, max count {int(want.max())}, every mode equals the oracle")
    finally:
        ctx.epi_release_set(cid)
        ctx.epi_release_stream(sid)
