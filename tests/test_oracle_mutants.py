"""The pins are strong enough: each plausible mistake planted into a copy of the
oracle (on the CPU; the real oracle is untouched) makes the brute-force /
golden comparison fail."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import spikegen as sg
from oracle import brute

# (name, exact source text, replacement)
MUTANTS = [
    ("alg1 init at 0", "int64_t count = 0, prev_e = NONE;", "int64_t count = 0, prev_e = 0;"),
    ("alg1 non-strict", "if (prev_e < prev[x]) {", "if (prev_e <= prev[x]) {"),
    ("alg1 keeps start", "prev_e = t[pprev[x]];", "prev_e = prev[x];"),
    ("decomp lower bound inclusive", "if (d <= lo[k - 1]) break;", "if (d < lo[k - 1]) break;"),
    ("decomp upper bound exclusive", "while (a < nprev && t[pprev[a]] < tx - hi[k - 1]) a++;",
     "while (a < nprev && t[pprev[a]] <= tx - hi[k - 1]) a++;"),
    ("decomp earliest start", "if (prev[y] != NONE && prev[y] > best) best = prev[y];",
     "if (prev[y] != NONE && (best == NONE || prev[y] < best)) best = prev[y];"),
    ("fsm admits ties", "stream_order ? i > pe : t[i] > e", "stream_order ? i > pe : t[i] >= e"),
    ("stream order admits the completing event", "stream_order ? i > pe : t[i] > e",
     "stream_order ? i >= pe : t[i] > e"),
    ("stream order keeps time admission", "stream_order ? i > pe : t[i] > e", "t[i] > e"),
    ("fsm lower bound inclusive", "if (lo[j - 1] < d && d <= hi[j - 1]) {", "if (lo[j - 1] <= d && d <= hi[j - 1]) {"),
    ("fsm completion one node early", "if (j == N - 1) {", "if (j == N - 2) {"),
    ("fsm prune inclusive", "pl->v[pl->head] < t[i] - hi[j - 1]", "pl->v[pl->head] <= t[i] - hi[j - 1]"),
    ("fsm no clear", "for (int k = 0; k < N; k++) s[k].head = s[k].len = 0;", ";"),
    ("fsm wrong interval index", "int64_t d = t[i] - pl->v[q];\n                    if (lo[j - 1] < d && d <= hi[j - 1]) {",
     "int64_t d = t[i] - pl->v[q];\n                    if (lo[0] < d && d <= hi[0]) {"),
]


def _build_mutant(tmp_path, name, old, new):
    src = open(oracle.SRC_PATH).read()
    assert src.count(old) >= 1, f"mutation site for {name!r} not found"
    mut = src.replace(old, new)
    d = tmp_path / name.replace(" ", "_")
    d.mkdir()
    c = d / "m.c"
    so = d / "m.so"
    c.write_text(mut)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", str(so), str(c)])
    L = ctypes.CDLL(str(so))
    P = ctypes.c_void_p
    L.oracle_count_batch.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                     P, P, P, P, ctypes.c_int, ctypes.c_int, P]
    return L


def _count_with(L, s, c, method):
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    types = np.ascontiguousarray(s["types"], np.int32)
    times = np.ascontiguousarray(s["times"], np.int64)
    N = np.ascontiguousarray(c["N"], np.int32)
    ty = np.ascontiguousarray(c["types"], np.int32)
    lo = np.ascontiguousarray(c["lo"], np.int64)
    hi = np.ascontiguousarray(c["hi"], np.int64)
    out = np.zeros(N.size, np.int64)
    L.oracle_count_batch(p(types), p(times), types.size, s["K"], N.size, p(N), p(ty), p(lo), p(hi),
                         oracle.METHODS[method], 1, p(out))
    return out


def _stream_pins_detect(L):
    # tiny streams with dense ties and episodes with repeated types, against
    # the enumeration over stream positions
    rng = np.random.Generator(np.random.PCG64(6))
    for _ in range(150):
        s = sg.tiny_stream(rng, int(rng.integers(2, 20)), 3, 8)
        eps = []
        for _ in range(6):
            n = int(rng.integers(1, 4))
            ty = [int(x) for x in rng.integers(0, 3, size=n)]
            lo = [int(rng.integers(0, 3)) for _ in range(n - 1)]
            eps.append((ty, lo, [a + int(rng.integers(1, 5)) for a in lo]))
        c = sg.candidates_from_list(eps)
        got = _count_with(L, s, c, "fsm_stream")
        for i, (ty, lo, hi) in enumerate(eps):
            if got[i] != brute.count_stream_order(s["types"], s["times"], ty, lo, hi):
                return True
    return False


def _pins_detect(L, method):
    if method == "fsm_stream":
        return _stream_pins_detect(L)
    rng = np.random.Generator(np.random.PCG64(5))
    for _ in range(150):
        s = sg.tiny_stream(rng, int(rng.integers(2, 24)), 4, 30)
        c = sg.tiny_candidates(rng, 6, 4, 4, 12)
        got = _count_with(L, s, c, method)
        for i in range(c["N"].size):
            N = int(c["N"][i])
            spans = brute.occurrences(s["types"], s["times"], list(c["types"][i, :N]),
                                      list(c["lo"][i, : N - 1]), list(c["hi"][i, : N - 1]))
            if got[i] != brute.max_nonoverlapped_dp(spans):
                return True
    return False


@pytest.mark.parametrize("mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, mut):
    if shutil.which("gcc") is None:
        pytest.skip("gcc missing")
    name, old, new = mut
    L = _build_mutant(tmp_path, name, old, new)
    method = "fsm_stream" if name.startswith("stream") else "fsm" if name.startswith("fsm") else "decomp"
    assert _pins_detect(L, method), f"mutant {name!r} survived the brute-force pins"
