"""Helpers of the full-size parity tests and of the script that writes their
expected values (``tests/golden/make_full_parity.py``).

Nothing here counts anything: the expected counts come from ``oracle/`` (run
by the script, on the CPU), the observed ones from the HIP engine (run by the
GPU tests).  This module only fingerprints inputs (so a test can tell that
the seeded generator still draws the inputs the expected values were
computed from) and digests large result sets whose order may differ between
the two sides (an order-independent multiset hash of (episode, count) rows).
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_U = np.uint64


def input_fingerprint(*arrays) -> str:
    """sha256 (first 16 hex) over the raw bytes of the given arrays."""
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()[:16]


def stream_fingerprint(s) -> str:
    return input_fingerprint(s["types"], s["times"], np.int64(s["K"]))


def cand_fingerprint(c) -> str:
    return input_fingerprint(c["N"], c["types"], c["lo"], c["hi"])


def _mix(x):
    # SplitMix64 finaliser (wrapping uint64 arithmetic)
    with np.errstate(over="ignore"):
        x = (x ^ (x >> _U(30))) * _U(0xBF58476D1CE4E5B9)
        x = (x ^ (x >> _U(27))) * _U(0x94D049BB133111EB)
        return x ^ (x >> _U(31))


def row_hashes(N, types, lo, hi, counts):
    """One uint64 per row of (N, the N types, the N-1 (lo, hi] bounds, count);
    slots beyond N are ignored."""
    N = np.asarray(N, np.int64)
    m = N.size
    h = np.full(m, _U(0x243F6A8885A308D3), dtype=np.uint64)
    h = _mix(h ^ N.astype(np.uint64))
    for j in range(8):
        live = j < N
        h = np.where(live, _mix(h ^ np.asarray(types[:, j], np.int64).astype(np.uint64)), h) if j < types.shape[1] else h
    for j in range(7):
        if j >= lo.shape[1]:
            break
        live = j < N - 1
        h = np.where(live, _mix(h ^ np.asarray(lo[:, j], np.int64).astype(np.uint64)), h)
        h = np.where(live, _mix(h ^ np.asarray(hi[:, j], np.int64).astype(np.uint64)), h)
    return _mix(h ^ np.asarray(counts, np.int64).astype(np.uint64))


class MultisetDigest:
    """Order-independent digest of a multiset of rows: two wrapping sums of
    differently mixed row hashes, plus the row count and the sum of counts."""

    def __init__(self):
        self.s1 = 0
        self.s2 = 0
        self.rows = 0
        self.count_sum = 0

    def add(self, N, types, lo, hi, counts):
        h = row_hashes(N, types, lo, hi, counts)
        with np.errstate(over="ignore"):
            self.s1 = (self.s1 + int(h.sum(dtype=np.uint64))) % (1 << 64)
            self.s2 = (self.s2 + int(_mix(h ^ _U(0x5851F42D4C957F2D)).sum(dtype=np.uint64))) % (1 << 64)
        self.rows += int(np.asarray(N).size)
        self.count_sum += int(np.asarray(counts, np.int64).sum())

    def as_dict(self):
        return {"rows": self.rows, "count_sum": self.count_sum, "h1": f"{self.s1:016x}", "h2": f"{self.s2:016x}"}


def _need(path):
    if not os.path.exists(path):
        import pytest

        pytest.skip(f"expected values {os.path.basename(path)} not written yet (tests/golden/make_full_parity.py)")


def load_counts(name):
    """Expected counts of a full-size workload: (meta dict, {key: int32 array})."""
    path = os.path.join(GOLDEN, name)
    _need(path)
    z = np.load(path, allow_pickle=False)
    meta = json.loads(str(z["meta"]))
    return meta, {k: z[k] for k in z.files if k != "meta"}


def load_json(name):
    _need(os.path.join(GOLDEN, name))
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)
