"""The state-machine engine's int32 relative-time machines (int64 streams whose
longest tile plus twice the longest episode span stays below 2^31 - 64) and
the int64 machines just beyond that bound: counts are bit-exact against the
oracle in plain and batched modes, with and without segments, and in
level-wise discovery through the state-machine engine.

The streams are dense bursts separated by long gaps placed inside the tiles,
so that every tile spans close to the bound while the tile boundaries fall in
dense stretches: partial occurrences are alive across every rebase."""
import numpy as np
import pytest

import oracle
import spikegen as sg
from oracle import apriori
from paper_0905_2203_amd import epi

pytestmark = pytest.mark.gpu

TILE = 2048          # events per stream tile
BOUND = (1 << 31) - 64


def say(msg):
    print(f"[gpu-rel] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = epi.Context(0)
    yield c
    c.close()


def _stream(seed, gap_ns, K=6, n=3 * TILE + 700):
    """Exponential gaps of mean 100 us, equal times now and then, and one gap
    of gap_ns in the middle of every tile."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = rng.exponential(1e5, size=n).astype(np.int64)
    d[rng.random(n) < 0.05] = 0  # ties
    d[TILE // 2::TILE] += gap_ns
    times = np.cumsum(d) + 1_000_000
    types = rng.integers(0, K, size=n).astype(np.int32)
    return dict(types=types, times=times.astype(np.int64), K=K, ts_kind=1, unit_per_ms=1_000_000)


def _max_tile_span(s):
    t = s["times"]
    starts = t[::TILE]
    ends = np.append(starts[1:], t[-1])
    return int((ends - starts).max())


def _candidates(seed, K, hmax):
    rng = np.random.Generator(np.random.PCG64(seed))
    eps = []
    for _ in range(160):
        n = int(rng.integers(2, 4))
        ty = rng.permutation(K)[:n].tolist()
        lo, hi = [], []
        for _ in range(n - 1):
            # width at least lo / 14: the interval's ring bound 1 + hi / (hi - lo + 1) stays within 16
            a = int(rng.integers(0, hmax // 2))
            b = int(rng.integers(a + a // 14 + 1, hmax + 1))
            lo.append(a)
            hi.append(b)
        eps.append((ty, lo, hi))
    for a in range(K):
        for b in range(K):
            if a != b:
                eps.append(([a, b], [0], [hmax]))
    return sg.candidates_from_list(eps)


def _hspan(c):
    return int(c["hi"].sum(axis=1).max())


def _check_all_modes(ctx, s, c, name):
    want = oracle.count(s, c)
    assert want.sum() > 0
    sid = ctx.epi_load_stream(s["types"], s["times"], s["K"])
    cid = ctx.epi_submit_candidates(sid, c)
    try:
        for segments in (0, 1, 3):
            ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, segments)
            say(f"{name}: plain, segments {segments}")
            ctx.epi_count([cid], mode=epi.EPI_MODE_PLAIN)
            assert np.array_equal(ctx.epi_read_counts(cid, c["N"].size), want), f"{name} plain segments={segments}"
            for sched in (epi.EPI_SCHED_RR, epi.EPI_SCHED_HEURISTIC):
                say(f"{name}: batched sched {sched}, segments {segments}")
                ctx.epi_count([cid], mode=epi.EPI_MODE_BATCHED, sched=sched)
                got = ctx.epi_read_counts(cid, c["N"].size)
                assert np.array_equal(got, want), f"{name} batched sched={sched} segments={segments}"
    finally:
        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 0)
        ctx.epi_release_set(cid)
        ctx.epi_release_stream(sid)


def test_relative_times_at_the_bound(ctx):
    hmax = 30_000_000  # 30 ms in ns
    s = _stream(41, gap_ns=1_760_000_000)
    c = _candidates(42, s["K"], hmax)
    span = _max_tile_span(s)
    say(f"max tile span {span}, hspan {_hspan(c)}")
    assert span + 2 * _hspan(c) < BOUND  # the relative-time machines count this stream
    assert span + 2 * _hspan(c) > BOUND - 200_000_000  # and it is close to their bound
    _check_all_modes(ctx, s, c, "at bound")


def test_int64_machines_beyond_the_bound(ctx):
    hmax = 30_000_000
    s = _stream(43, gap_ns=2_100_000_000)
    c = _candidates(44, s["K"], hmax)
    span = _max_tile_span(s)
    say(f"max tile span {span}, hspan {_hspan(c)}")
    assert span + 2 * _hspan(c) >= BOUND  # beyond: the int64 machines count it
    _check_all_modes(ctx, s, c, "beyond bound")


def test_levelwise_state_machines_relative_times(ctx):
    # level-wise discovery through the state-machine engine (a menu of more
    # than 8 intervals) on an int64 stream within the bound
    s = _stream(45, gap_ns=1_500_000_000, K=5)
    menu = [(i * 2_000_000, i * 2_000_000 + 3_000_000) for i in range(9)]
    say(f"max tile span {_max_tile_span(s)}")
    ref = apriori.mine(s, menu, 3, 40)
    sid = ctx.epi_load_stream(s["types"], s["times"], s["K"])
    mid = ctx.epi_mine(sid, menu, 3, 40)
    try:
        assert ctx.epi_mine_levels(mid) == len(ref)
        for L in range(1, len(ref) + 1):
            cands, counts = ctx.epi_mine_read(mid, L)
            got = {}
            for i in range(cands["N"].size):
                N = int(cands["N"][i])
                got[(tuple(int(x) for x in cands["types"][i, :N]), tuple(int(x) for x in cands["lo"][i, : N - 1]),
                     tuple(int(x) for x in cands["hi"][i, : N - 1]))] = int(counts[i])
            want = {}
            for (ty, iv), cnt in ref[L - 1]["counts"].items():
                want[(ty, tuple(menu[v][0] for v in iv), tuple(menu[v][1] for v in iv))] = cnt
            assert got == want, f"level {L}"
        assert len(ref) >= 2 and len(ref[1]["frequent"]) > 0
    finally:
        ctx.epi_mine_release(mid)
        ctx.epi_release_stream(sid)
