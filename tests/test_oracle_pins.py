"""Pins of the CPU oracle against what the paper and the mathematics fix.

* hand-worked golden cases (constraint inequalities of Sec. II-C, Alg. 1);
* brute force on tiny random streams: every occurrence enumerated from the
  inequalities, then an exhaustive and a dynamic-programming maximum
  non-overlapped subset (neither is the greedy);
* special cases that reduce to library routines (1-node = numpy.unique;
  2-node = an independent bisect-based greedy);
* invariants of the frequency measure (anti-monotonicity of Sec. II-C and
  others), and planted-cascade recovery;
* the two oracle formulations (decomposition of Sec. IV-A + Alg. 1, and the
  serial state machine of Sec. III-A) agree.
"""
import bisect
import json
import os

import numpy as np
import pytest

import oracle
import spikegen as sg
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")


def stream_from_events(events, K=3):
    ev = sorted(events, key=lambda e: e[1])  # stable: keeps the listed order of equal times
    return dict(types=np.array([e[0] for e in ev], np.int32),
                times=np.array([e[1] for e in ev], np.int64), K=K, ts_kind=1)


def one_candidate(ep, lo, hi):
    return sg.candidates_from_list([(list(ep), list(lo), list(hi))])


def golden_cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", golden_cases(), ids=lambda c: c["name"].split()[0])
@pytest.mark.parametrize("method", ["decomp", "fsm"])
def test_golden_worked_examples(case, method):
    # keep the listed event order (W3 lists (B,5) before (A,5))
    s = dict(types=np.array([e[0] for e in case["events"]], np.int32),
             times=np.array([e[1] for e in case["events"]], np.int64), K=3, ts_kind=1)
    assert np.all(np.diff(s["times"]) >= 0)
    c = one_candidate(case["episode"], case["lo"], case["hi"])
    assert oracle.count(s, c, method)[0] == case["count"]
    occ = brute.occurrences(s["types"], s["times"], case["episode"], case["lo"], case["hi"])
    assert sorted(occ) == sorted(tuple(o) for o in case["occurrences"])
    assert brute.max_nonoverlapped_exhaustive(occ) == case["count"]
    assert brute.max_nonoverlapped_dp(occ) == case["count"]


def test_paper_literal_initialisation_would_lose_time_zero():
    """Alg. 1 as printed starts the previous end at 0; a start at time 0 is then
    never strictly after it.  The oracle starts at minus infinity instead."""
    s = stream_from_events([(0, 0), (1, 6)])
    assert oracle.count(s, one_candidate([0, 1], [5], [10]))[0] == 1
    spans = [(0, 6)]
    prev_e, literal = 0, 0
    for st, en in spans:
        if prev_e < st:
            prev_e, literal = en, literal + 1
    assert literal == 0


def _tiny_cases(seed, ncase, n, K, tmax, nmax, gap):
    rng = np.random.Generator(np.random.PCG64(seed))
    for _ in range(ncase):
        s = sg.tiny_stream(rng, int(rng.integers(1, n + 1)), K, tmax)
        c = sg.tiny_candidates(rng, 6, K, nmax, gap)
        yield s, c


@pytest.mark.parametrize("seed", range(6))
def test_bruteforce_tiny_streams(seed):
    """P1: definition by enumeration == both oracle formulations, on tiny
    streams with many equal timestamps."""
    for s, c in _tiny_cases(100 + seed, 40, 24, 4, 30, 4, 12):
        got_d = oracle.count(s, c, "decomp")
        got_f = oracle.count(s, c, "fsm")
        for i in range(c["N"].size):
            N = int(c["N"][i])
            ep = list(c["types"][i, :N])
            lo = list(c["lo"][i, : N - 1])
            hi = list(c["hi"][i, : N - 1])
            spans = brute.occurrences(s["types"], s["times"], ep, lo, hi)
            want = brute.max_nonoverlapped_dp(spans)
            if len(set(spans)) <= 14:
                assert brute.max_nonoverlapped_exhaustive(spans) == want
            assert got_d[i] == want, (ep, lo, hi)
            assert got_f[i] == want, (ep, lo, hi)


@pytest.mark.parametrize("seed", range(4))
def test_bruteforce_repeated_types(seed):
    """Episodes with a type at several nodes (drawn with replacement from 2-3
    types): definition by enumeration == both oracle formulations."""
    rng = np.random.Generator(np.random.PCG64(500 + seed))
    for _ in range(40):
        K = int(rng.integers(2, 4))
        s = sg.tiny_stream(rng, int(rng.integers(1, 25)), K, 30)
        eps = []
        for _ in range(6):
            n = int(rng.integers(2, 5))
            ty = [int(x) for x in rng.integers(0, K, size=n)]
            lo = [int(rng.integers(0, 6)) for _ in range(n - 1)]
            hi = [a + int(rng.integers(1, 8)) for a in lo]
            eps.append((ty, lo, hi))
        c = sg.candidates_from_list(eps)
        got_d = oracle.count(s, c, "decomp")
        got_f = oracle.count(s, c, "fsm")
        for i, (ty, lo, hi) in enumerate(eps):
            spans = brute.occurrences(s["types"], s["times"], ty, lo, hi)
            want = brute.max_nonoverlapped_dp(spans)
            assert got_d[i] == want, (ty, lo, hi)
            assert got_f[i] == want, (ty, lo, hi)


def test_bruteforce_dense_ties():
    """Streams where most events share timestamps (times in 0..6)."""
    for s, c in _tiny_cases(7, 200, 16, 3, 6, 3, 4):
        got = oracle.count(s, c, "fsm")
        for i in range(c["N"].size):
            N = int(c["N"][i])
            spans = brute.occurrences(s["types"], s["times"], list(c["types"][i, :N]),
                                      list(c["lo"][i, : N - 1]), list(c["hi"][i, : N - 1]))
            assert got[i] == brute.max_nonoverlapped_dp(spans)


def _medium_stream(seed, K=6, rate=40.0, dur=20.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    return sg.poisson_stream(rng, K=K, rate_hz=rate, dur_s=dur, ts_kind=1, unit_per_ms=1)


def _medium_cands(seed, K=6, m=300, nmin=1, nmax=5):
    rng = np.random.Generator(np.random.PCG64(seed))
    return sg.random_candidates(rng, m, K, nmin, nmax, 1, low_ms=(0, 1, 3, 8), width_ms=(1, 4, 10, 30))


def test_one_node_equals_unique():
    """P5: a 1-node episode counts the distinct timestamps of its type."""
    s = _medium_stream(1)
    c = sg.candidates_from_list([([k], [], []) for k in range(s["K"])])
    got = oracle.count(s, c, "decomp")
    got_f = oracle.count(s, c, "fsm")
    for k in range(s["K"]):
        want = np.unique(s["times"][s["types"] == k]).size
        assert got[k] == want and got_f[k] == want


def _two_node_greedy(times_a, times_b, lo, hi):
    """Independent 2-node greedy: walk B in time order; take the latest A
    with t_a < t_b - lo (bisect); accept if it is >= t_b - hi and starts
    after the previously accepted end."""
    count, prev_e = 0, None
    for tb in times_b:
        k = bisect.bisect_left(times_a, tb - lo) - 1
        if k < 0:
            continue
        ta = times_a[k]
        if ta < tb - hi:
            continue
        if prev_e is None or ta > prev_e:
            count += 1
            prev_e = tb
    return count


def test_two_node_equals_bisect_greedy():
    s = _medium_stream(2)
    rng = np.random.Generator(np.random.PCG64(3))
    eps = []
    for _ in range(120):
        a, b = rng.permutation(s["K"])[:2]
        lo = int(rng.integers(0, 20))
        hi = lo + int(rng.integers(1, 40))
        eps.append(([a, b], [lo], [hi]))
    c = sg.candidates_from_list(eps)
    got = oracle.count(s, c)
    for i, (ep, lo, hi) in enumerate(eps):
        ta = list(s["times"][s["types"] == ep[0]])
        tb = list(s["times"][s["types"] == ep[1]])
        assert got[i] == _two_node_greedy(ta, tb, lo[0], hi[0])


def test_formulations_agree_medium():
    """P6: decomposition (latest start per end + Alg. 1) == state machine."""
    for seed in range(3):
        s = _medium_stream(10 + seed, rate=60.0)
        c = _medium_cands(20 + seed, m=400, nmax=8)
        np.testing.assert_array_equal(oracle.count(s, c, "decomp"), oracle.count(s, c, "fsm"))


def _sub(c, i, a, b):
    """Sub-episode of candidate i made of nodes a..b-1."""
    ep = list(c["types"][i, a:b])
    return (ep, list(c["lo"][i, a:b - 1]), list(c["hi"][i, a:b - 1]))


def test_invariant_prefix_suffix_and_rarest():
    """Anti-monotonicity (Sec. II-C): a count never exceeds that of its prefix
    or suffix sub-episode, nor the distinct timestamps of its rarest type."""
    s = _medium_stream(4, rate=60.0)
    c = _medium_cands(5, m=300, nmin=2, nmax=6)
    full = oracle.count(s, c)
    pre, suf = [], []
    for i in range(c["N"].size):
        N = int(c["N"][i])
        pre.append(_sub(c, i, 0, N - 1))
        suf.append(_sub(c, i, 1, N))
    cp = oracle.count(s, sg.candidates_from_list(pre))
    cs = oracle.count(s, sg.candidates_from_list(suf))
    assert np.all(full <= cp) and np.all(full <= cs)
    for i in range(c["N"].size):
        N = int(c["N"][i])
        for k in c["types"][i, :N]:
            assert full[i] <= np.unique(s["times"][s["types"] == k]).size
    assert full.max() > 0  # not vacuous


def test_invariant_widening_never_decreases():
    s = _medium_stream(6, rate=60.0)
    c = _medium_cands(7, m=300, nmin=2, nmax=5)
    base = oracle.count(s, c)
    w = {k: v.copy() for k, v in c.items()}
    live = np.arange(7)[None, :] < (c["N"][:, None].astype(int) - 1)
    w["lo"] = np.where(live, np.maximum(c["lo"] - 1, 0), 0)
    w["hi"] = np.where(live, c["hi"] + 2, 0)
    assert np.all(oracle.count(s, w) >= base)


def test_invariant_time_shift_units_and_relabel():
    s = _medium_stream(8, rate=50.0)
    c = _medium_cands(9, m=250, nmax=6)
    base = oracle.count(s, c)
    shifted = dict(s, times=s["times"] + 123456789)
    np.testing.assert_array_equal(oracle.count(shifted, c), base)
    scaled = dict(s, times=s["times"] * 1000)
    cs = dict(c, lo=c["lo"] * 1000, hi=c["hi"] * 1000)
    np.testing.assert_array_equal(oracle.count(scaled, cs), base)
    perm = np.random.Generator(np.random.PCG64(1)).permutation(s["K"]).astype(np.int32)
    rel = dict(s, types=perm[s["types"]])
    cr = dict(c, types=np.where(c["types"] >= 0, perm[np.maximum(c["types"], 0)], -1))
    np.testing.assert_array_equal(oracle.count(rel, cr), base)


def test_invariant_equal_time_permutation():
    """The count does not depend on the order of events with equal times."""
    rng = np.random.Generator(np.random.PCG64(11))
    for _ in range(5):
        s = sg.tiny_stream(rng, 400, 4, 120)  # about 3 events per timestamp
        c = sg.tiny_candidates(rng, 80, 4, 4, 10)
        base = oracle.count(s, c, "fsm")
        key = rng.random(s["times"].size)
        order = np.lexsort((key, s["times"]))
        ps = dict(s, types=s["types"][order], times=s["times"][order])
        np.testing.assert_array_equal(oracle.count(ps, c, "fsm"), base)
        np.testing.assert_array_equal(oracle.count(ps, c, "decomp"), base)


def test_invariant_concatenation_adds():
    """Two streams separated by a gap larger than every episode span: counts add."""
    a = _medium_stream(12, dur=5.0)
    b = _medium_stream(13, dur=5.0)
    c = _medium_cands(14, m=200, nmax=6)
    gap = int(a["times"].max()) + 7 * 40 + 1
    cat = dict(types=np.concatenate([a["types"], b["types"]]),
               times=np.concatenate([a["times"], b["times"] + gap]), K=a["K"], ts_kind=1)
    np.testing.assert_array_equal(oracle.count(cat, c), oracle.count(a, c) + oracle.count(b, c))


def test_planted_cascade_recovery():
    """P4: each planted instance is a valid occurrence by construction, so the
    count of the planted episode is at least the largest non-overlapped subset
    of the planted instances."""
    s = sg.config_stream(1)
    for p in s["planted"]:
        inst = p["instances"]
        spans = [(int(r[0]), int(r[-1])) for r in inst]
        c = one_candidate(p["types"], p["lo"], p["hi"])
        assert oracle.count(s, c)[0] >= brute.max_nonoverlapped_dp(spans) > 100
    s2 = sg.config_stream(2, scale=0.2)
    for p in s2["planted"]:
        spans = [(int(r[0]), int(r[-1])) for r in p["instances"]]
        c = one_candidate(p["types"], p["lo"], p["hi"])
        assert oracle.count(s2, c)[0] >= brute.max_nonoverlapped_dp(spans) > 0


def test_oracle_rejects_bad_input():
    s = stream_from_events([(0, 1), (5, 2)], K=3)
    with pytest.raises(ValueError):
        oracle.count(s, one_candidate([0, 1], [0], [5]))


def test_levelwise_discovery_finds_every_frequent_episode():
    """The level-wise procedure (Sec. II-C) returns exactly the episodes, among
    all episodes over the types and the interval menu, whose count exceeds
    the threshold: checked against exhaustive enumeration up to size 3."""
    import itertools

    from oracle import apriori

    rng = np.random.Generator(np.random.PCG64(31))
    s = sg.poisson_stream(rng, K=5, rate_hz=40.0, dur_s=30.0, ts_kind=1, unit_per_ms=1)
    menu = [(0, 10), (10, 30)]
    theta = 25
    levels = apriori.mine(s, menu, 3, theta)
    K = s["K"]
    for N in (1, 2, 3):
        eps = [(ty, iv) for ty in itertools.permutations(range(K), N)
               for iv in itertools.product(range(len(menu)), repeat=N - 1)]
        counts = oracle.count(s, apriori.to_candidates(eps, menu))
        want = {ep for ep, c in zip(eps, counts) if c > theta}
        got = levels[N - 1]["frequent"] if N <= len(levels) else set()
        assert got == want, N
        assert len(want) > 0
        # every candidate the procedure counted has the exhaustive count
        for ep, c in levels[N - 1]["counts"].items():
            assert c == counts[eps.index(ep)]


def test_levelwise_recovers_planted_cascades():
    """P4 on the mining workload: every planted cascade is frequent at its size."""
    from oracle import apriori

    s = sg.config_stream(2, scale=0.05)  # 15 s of the 300 s stream
    menu = [(a * 1000, b * 1000) for a, b in sg.MENU_MINING_MS]
    theta = 30
    # restrict the stream to the planted types to keep the search small
    keep = np.zeros(s["K"], bool)
    for p in s["planted"]:
        keep[p["types"]] = True
    ids = np.nonzero(keep)[0]
    remap = -np.ones(s["K"], np.int64)
    remap[ids] = np.arange(ids.size)
    sel = keep[s["types"]]
    sub = dict(types=remap[s["types"][sel]].astype(np.int32), times=s["times"][sel], K=int(ids.size), ts_kind=0)
    levels = apriori.mine(sub, menu, 6, theta)
    for p in s["planted"]:
        spans = [(int(r[0]), int(r[-1])) for r in p["instances"]]
        if brute.max_nonoverlapped_dp(spans) <= theta:
            continue
        ty = tuple(int(x) for x in remap[p["types"]])
        iv = tuple(menu.index((int(a), int(b))) for a, b in zip(p["lo"], p["hi"]))
        assert (ty, iv) in levels[len(ty) - 1]["frequent"]


# ---- stream-order overlap (the listing's reset of Sec. III-A taken in stream order) ----

def _golden(name_prefix):
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")))
    items = d["cases"] if isinstance(d, dict) and "cases" in d else d
    items = items if isinstance(items, list) else list(items.values())
    return [x for x in items if x["name"].startswith(name_prefix)]


def _golden_case(x):
    ev = np.array(x["events"], dtype=np.int64).reshape(-1, 2)
    s = dict(types=ev[:, 0].astype(np.int32), times=ev[:, 1], K=int(ev[:, 0].max()) + 1 if ev.size else 1, ts_kind=1)
    c = sg.candidates_from_list([(x["episode"], x["lo"], x["hi"])])
    return s, c


def test_stream_order_worked_examples():
    """Hand-derived from the state machine of Sec. III-A with its reset in
    stream order.  W3: (A,0),(B,5) completes at the second event; (A,5) comes
    later in the stream, so it starts again and (B,10) (gap 5 <= 5) completes:
    2 (time semantics: 1).  W6: every event of a one-node episode is an
    occurrence: 3 (time semantics: 2 distinct timestamps)."""
    for prefix, want in (("W3 ", 2), ("W6 ", 3)):
        (x,) = _golden(prefix)
        s, c = _golden_case(x)
        assert oracle.count(s, c, "fsm_stream")[0] == want
        assert oracle.count(s, c, "fsm")[0] == x["count"]
        assert brute.count_stream_order(s["types"], s["times"], x["episode"], x["lo"], x["hi"]) == want


def test_stream_order_equals_time_semantics_without_ties():
    """With every timestamp distinct, stream order is time order."""
    rng = np.random.Generator(np.random.PCG64(610))
    for _ in range(30):
        n = int(rng.integers(1, 400))
        times = np.sort(rng.choice(10 * n + 10, size=n, replace=False)).astype(np.int64)
        K = int(rng.integers(2, 6))
        s = dict(types=rng.integers(0, K, size=n).astype(np.int32), times=times, K=K, ts_kind=1)
        c = sg.tiny_candidates(rng, 20, K, 4, 30)
        assert np.array_equal(oracle.count(s, c, "fsm_stream"), oracle.count(s, c, "decomp"))


@pytest.mark.parametrize("seed", range(3))
def test_stream_order_bruteforce_with_ties(seed):
    """Dense ties and repeated types: the stream-order state machine equals
    the maximum number of occurrences that pairwise do not share stream
    positions in overlapping order (enumeration + interval-scheduling DP over
    positions)."""
    rng = np.random.Generator(np.random.PCG64(620 + seed))
    for _ in range(40):
        K = int(rng.integers(2, 4))
        s = sg.tiny_stream(rng, int(rng.integers(1, 22)), K, 8)
        eps = []
        for _ in range(6):
            n = int(rng.integers(1, 5))
            ty = [int(x) for x in rng.integers(0, K, size=n)]
            lo = [int(rng.integers(0, 3)) for _ in range(n - 1)]
            hi = [a + int(rng.integers(1, 5)) for a in lo]
            eps.append((ty, lo, hi))
        c = sg.candidates_from_list(eps)
        got = oracle.count(s, c, "fsm_stream")
        for i, (ty, lo, hi) in enumerate(eps):
            assert got[i] == brute.count_stream_order(s["types"], s["times"], ty, lo, hi), (ty, lo, hi)


def test_array_levelwise_equals_tuple_levelwise():
    """The array form of the level-wise procedure (used for levels of 1e8
    candidates) generates the same candidates, in the same order, with the same
    counts and frequent sets as the tuple form."""
    from oracle import apriori

    rng = np.random.Generator(np.random.PCG64(41))
    s = sg.poisson_stream(rng, K=12, rate_hz=15.0, dur_s=60.0, ts_kind=0, unit_per_ms=1000, cascades=[4],
                          cascade_trigger_hz=[5.0])
    menu = [(a * 1000, b * 1000) for a, b in sg.MENU_MINING_MS]
    ref = apriori.mine(s, menu, 5, 20)
    arr = apriori.mine_arrays(s, menu, 5, 20, chunk=777)
    assert len(ref) == len(arr) == 5
    for L, (r, a) in enumerate(zip(ref, arr), start=1):
        eps = [(tuple(int(x) for x in a["types"][i]), tuple(int(x) for x in a["ivs"][i]))
               for i in range(a["counts"].size)]
        assert {ep: int(c) for ep, c in zip(eps, a["counts"])} == r["counts"]
        assert {ep for ep, f in zip(eps, a["frequent"]) if f} == r["frequent"]
        if L >= 3:
            assert eps == apriori.join(sorted(ref[L - 2]["frequent"]))
