"""Pins of the oracle's segment-parallel counting with exact reconciliation
(``oracle/segmented.py``, the joining rule of the segment idea of Sec. III-B
stated exactly): for any boundaries -- segments shorter than the episode span,
empty segments, boundaries before the first or after the last event, equal
times across a boundary -- its counts equal the unsegmented count of the C
oracle, which is itself pinned by brute force; and plausible mistakes planted
into a copy of the rule are caught."""
import types as _types

import numpy as np
import pytest

import oracle
import spikegen as sg
from oracle import brute, segmented


def _cases(seed, n_iter):
    rng = np.random.Generator(np.random.PCG64(seed))
    for _ in range(n_iter):
        s = sg.tiny_stream(rng, int(rng.integers(1, 60)), 4, 80, ts_kind=int(rng.integers(0, 2)))
        c = sg.tiny_candidates(rng, 8, 4, 4, 12)
        P = int(rng.integers(1, 10))
        bounds = sorted(set(int(x) for x in rng.integers(-5, 90, size=P)))
        yield s, c, bounds


@pytest.mark.parametrize("q", [1, 2, 4])
def test_segmented_equals_unsegmented(q):
    for s, c, bounds in _cases(21 + q, 120):
        want = oracle.count(s, c, "fsm")
        got = np.array(segmented.count(s, c, bounds, q))
        assert np.array_equal(got, want), (bounds, got, want)


def test_segmented_equals_brute_force_with_dense_boundaries():
    # a boundary at every other time value: segments shorter than any span
    rng = np.random.Generator(np.random.PCG64(29))
    for _ in range(60):
        s = sg.tiny_stream(rng, int(rng.integers(2, 30)), 3, 30)
        c = sg.tiny_candidates(rng, 5, 3, 3, 8)
        bounds = list(range(1, 31, 2))
        got = segmented.count(s, c, bounds, 2)
        for i in range(c["N"].size):
            N = int(c["N"][i])
            spans = brute.occurrences(s["types"], s["times"], list(c["types"][i, :N]),
                                      list(c["lo"][i, :N - 1]), list(c["hi"][i, :N - 1]))
            assert got[i] == brute.max_nonoverlapped_dp(spans)


def test_segmented_planted_workload_slice():
    # a slice of the 32-type workload: real rates and the planted cascades
    s = sg.config_stream(1, scale=0.05)
    c = sg.config_candidates(1)
    idx = np.arange(0, c["N"].size, 31)
    sub = sg.take_candidates(c, idx)
    t = s["times"]
    bounds = [int(x) for x in np.linspace(t[0], t[-1], 7)[1:-1]]
    assert np.array_equal(np.array(segmented.count(s, sub, bounds, 4)), oracle.count(s, sub, "fsm"))


MUTANTS = [
    ("speculation starts at the boundary", "i0, e0 = bisect.bisect_left(times, B[p] - H), B[p] - H - 1",
     "i0, e0 = bisect.bisect_left(times, B[p]), B[p] - 1"),
    ("free state tested against the boundary", "if p == 0 or tau < B[p] - H:", "if p == 0 or tau < B[p]:"),
    ("meeting counts the shared completion twice", "total += len(comp) + (c - k - 1)",
     "total += len(comp) + (c - k)"),
    ("re-run starts at the boundary", "i0 = bisect.bisect_right(times, tau)", "i0 = bisect.bisect_left(times, B[p])"),
    ("speculative machine admits a start at its first time", "B[p] - H - 1\n", "B[p] - H\n"),
]


@pytest.mark.parametrize("mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(mut):
    name, old, new = mut
    src = open(segmented.__file__).read()
    assert src.count(old) >= 1, f"mutation site for {name!r} not found"
    mod = _types.ModuleType("segmented_mutant")
    exec(compile(src.replace(old, new), "segmented_mutant", "exec"), mod.__dict__)
    caught = False
    for s, c, bounds in _cases(77, 200):
        if not np.array_equal(np.array(mod.count(s, c, bounds, 2)), oracle.count(s, c, "fsm")):
            caught = True
            break
    assert caught, f"mutant {name!r} survived"
