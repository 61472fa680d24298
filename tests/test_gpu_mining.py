"""GPU parity of level-wise discovery (through the C ABI): every level's
candidates, counts and frequent sets equal the oracle's level-wise run, on
inputs that reach the corners of the extension engine's window walk: more
extension types per episode than lanes in a wave (several rounds), int64
nanosecond times, menus of up to 8 overlapping intervals, a menu longer
than the walk takes (the state-machine engine then counts), equal-time events,
and a negative threshold (every candidate frequent, so empty chain lists are
written and extended)."""
import sys

import numpy as np
import pytest

import spikegen as sg
from oracle import apriori
from paper_0905_2203_amd import epi

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-mining] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = epi.Context(0)
    yield c
    c.close()


def _key(c, i):
    N = int(c["N"][i])
    return (tuple(int(x) for x in c["types"][i, :N]), tuple(int(x) for x in c["lo"][i, : N - 1]),
            tuple(int(x) for x in c["hi"][i, : N - 1]))


def compare_mining(ctx, name, s, menu, max_size, theta):
    say(f"{name}: n={s['types'].size} K={s['K']} ts_kind={s['ts_kind']} menu={len(menu)} theta={theta}")
    ref = apriori.mine(s, menu, max_size, theta)
    say(f"{name}: oracle levels {[(len(r['counts']), len(r['frequent'])) for r in ref]}")
    sid = ctx.epi_load_stream(s["types"], s["times"], s["K"])
    mid = ctx.epi_mine(sid, menu, max_size, theta)
    nl = ctx.epi_mine_levels(mid)
    assert nl == len(ref)
    for L in range(1, nl + 1):
        c, counts = ctx.epi_mine_read(mid, L)
        got = {_key(c, i): int(counts[i]) for i in range(c["N"].size)}
        want = {}
        for (ty, iv), cnt in ref[L - 1]["counts"].items():
            want[(ty, tuple(menu[v][0] for v in iv), tuple(menu[v][1] for v in iv))] = cnt
        assert len(got) == len(want), f"{name} level {L}: {len(got)} candidates, oracle {len(want)}"
        bad = [k for k, v in want.items() if got.get(k) != v]
        assert not bad, f"{name} level {L}: {len(bad)} differ, e.g. {bad[0]} got {got.get(bad[0])} want {want[bad[0]]}"
        fc, fcounts = ctx.epi_mine_read(mid, L, frequent_only=True)
        assert fc["N"].size == len(ref[L - 1]["frequent"])
        assert all(want[_key(fc, i)] == int(fcounts[i]) and fcounts[i] > theta for i in range(fc["N"].size))
    ctx.epi_mine_release(mid)
    ctx.epi_release_stream(sid)
    return ref


@pytest.mark.parametrize("list_bytes,list_alphas", [(8 << 30, 65536), (0, 65536), (8 << 30, 0)],
                         ids=["lists", "walks", "pieced_writes"])
def test_more_extension_types_than_lanes(ctx, list_bytes, list_alphas):
    # 80 types: an episode has up to 79 (level 2) or 77 (level 3) extension
    # types, more than the 64 lanes of one walk round; every level from the
    # end-event lists (walks cut into pieces), by count walks and one write
    # walk per parent, and by count walks and chain lists written in pieces
    rng = np.random.Generator(np.random.PCG64(31))
    s = sg.poisson_stream(rng, K=80, rate_hz=6.0, dur_s=60.0, ts_kind=0, unit_per_ms=1000, cascades=[4],
                          cascade_trigger_hz=[5.0])
    ctx.epi_set_option(epi.EPI_OPT_MINE_LIST_BYTES, list_bytes)
    ctx.epi_set_option(epi.EPI_OPT_MINE_LIST_ALPHAS, list_alphas)
    try:
        ref = compare_mining(ctx, "K80", s, [(a * 1000, b * 1000) for a, b in sg.MENU_MINING_MS], 4, 17)
    finally:
        ctx.epi_set_option(epi.EPI_OPT_MINE_LIST_BYTES, 8 << 30)
        ctx.epi_set_option(epi.EPI_OPT_MINE_LIST_ALPHAS, 65536)
    assert len(ref[1]["frequent"]) > 0 and len(ref[2]["frequent"]) > 0


@pytest.mark.parametrize("list_alphas", [65536, 0], ids=["lists", "pieced_writes"])
def test_int64_nanoseconds(ctx, list_alphas):
    rng = np.random.Generator(np.random.PCG64(32))
    s = sg.poisson_stream(rng, K=12, rate_hz=15.0, dur_s=60.0, ts_kind=1, unit_per_ms=1_000_000, cascades=[4],
                          cascade_trigger_hz=[5.0])
    ctx.epi_set_option(epi.EPI_OPT_MINE_LIST_ALPHAS, list_alphas)
    try:
        compare_mining(ctx, "int64", s, [(a * 1_000_000, b * 1_000_000) for a, b in sg.MENU_MINING_MS], 5, 40)
    finally:
        ctx.epi_set_option(epi.EPI_OPT_MINE_LIST_ALPHAS, 65536)


def test_menu_of_six_overlapping_intervals(ctx):
    rng = np.random.Generator(np.random.PCG64(33))
    s = sg.poisson_stream(rng, K=10, rate_hz=15.0, dur_s=60.0, ts_kind=0, unit_per_ms=1000, cascades=[4],
                          cascade_trigger_hz=[5.0])
    menu = [(0, 3000), (2000, 7000), (5000, 10000), (0, 10000), (10000, 20000), (15000, 30000)]
    compare_mining(ctx, "menu6", s, menu, 4, 40)


def test_menu_of_eight_and_of_nine(ctx):
    # 8 intervals: the widest walk; 9: the state-machine engine takes over
    rng = np.random.Generator(np.random.PCG64(35))
    s = sg.poisson_stream(rng, K=6, rate_hz=15.0, dur_s=40.0, ts_kind=0, unit_per_ms=1000)
    menu = [(i * 2000, i * 2000 + 3000) for i in range(8)]
    compare_mining(ctx, "menu8", s, menu, 3, 15)
    compare_mining(ctx, "menu9", s, menu + [(0, 25000)], 3, 15)


def test_equal_times(ctx):
    # times on a 4 ms grid: many equal-time events of different types
    rng = np.random.Generator(np.random.PCG64(34))
    s = sg.poisson_stream(rng, K=8, rate_hz=20.0, dur_s=30.0, ts_kind=0, unit_per_ms=1000)
    s["times"] = np.ascontiguousarray(s["times"] // 4000 * 4000, dtype=np.int32)
    compare_mining(ctx, "ties", s, [(0, 4000), (4000, 8000), (0, 12000)], 4, 20)


def test_negative_threshold_every_candidate_frequent(ctx):
    rng = np.random.Generator(np.random.PCG64(36))
    s = sg.poisson_stream(rng, K=5, rate_hz=4.0, dur_s=20.0, ts_kind=0, unit_per_ms=1000)
    ref = compare_mining(ctx, "theta-1", s, [(0, 5000), (5000, 20000)], 4, -1)
    assert any(v == 0 for v in ref[-1]["counts"].values())


def test_runs_of_different_sizes_share_the_context_cache(ctx):
    # the context keeps the blocks of each run for the next: runs of growing
    # and shrinking size, two mines alive at once and released out of order,
    # one run ordered after a caller's stream; every one equals the oracle
    import torch

    rng = np.random.Generator(np.random.PCG64(37))
    small = sg.poisson_stream(rng, K=6, rate_hz=10.0, dur_s=30.0, ts_kind=0, unit_per_ms=1000)
    big = sg.poisson_stream(rng, K=16, rate_hz=12.0, dur_s=60.0, ts_kind=0, unit_per_ms=1000, cascades=[4],
                            cascade_trigger_hz=[5.0])
    menu = [(a * 1000, b * 1000) for a, b in sg.MENU_MINING_MS]
    runs = [(small, 3, 10), (big, 4, 30), (small, 4, 5)]
    mids, sids, refs = [], [], []
    side = torch.cuda.Stream()
    for i, (s, size, theta) in enumerate(runs):
        say(f"run {i}: n={s['types'].size} K={s['K']} size {size} theta {theta}")
        refs.append(apriori.mine(s, menu, size, theta))
        sid = ctx.epi_load_stream(s["types"], s["times"], s["K"])
        hs = side.cuda_stream if i == 2 else None
        mids.append(ctx.epi_mine(sid, menu, size, theta, hip_stream=hs))
        sids.append(sid)
    for i in (1, 0, 2):  # out of order
        mid, ref = mids[i], refs[i]
        assert ctx.epi_mine_levels(mid) == len(ref)
        for L in range(1, len(ref) + 1):
            c, counts = ctx.epi_mine_read(mid, L)
            got = {_key(c, j): int(counts[j]) for j in range(c["N"].size)}
            want = {(ty, tuple(menu[v][0] for v in iv), tuple(menu[v][1] for v in iv)): cnt
                    for (ty, iv), cnt in ref[L - 1]["counts"].items()}
            assert got == want, f"run {i} level {L}"
        ctx.epi_mine_release(mid)
    for sid in sids:
        ctx.epi_release_stream(sid)
