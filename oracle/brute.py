"""Brute force for tiny inputs -- TEST INFRASTRUCTURE (part of the oracle).

Straight from the definitions of Sec. II-C: every index tuple whose events have
the episode's types in order and meet each inter-event constraint
lo_j < t_{j+1} - t_j <= hi_j is an occurrence; the frequency is the largest
number of pairwise non-overlapped occurrences, where two occurrences are
non-overlapped iff one ends strictly before the other starts.

Two independent maximisations are given, neither of which is the greedy of
Alg. 1: an exhaustive search over subsets of distinct spans, and the textbook
dynamic programme for (unit-weight) weighted interval scheduling.
"""
from __future__ import annotations

import bisect


def occurrences(types, times, ep, lo, hi):
    """All occurrences as (start, end) spans, with multiplicity."""
    n = len(types)
    N = len(ep)
    out = []

    def rec(k, prev_idx, start):
        for i in range(n):
            if types[i] != ep[k]:
                continue
            if k > 0:
                d = int(times[i]) - int(times[prev_idx])
                if not (lo[k - 1] < d <= hi[k - 1]):
                    continue
            s = int(times[i]) if k == 0 else start
            if k == N - 1:
                out.append((s, int(times[i])))
            else:
                rec(k + 1, i, s)

    rec(0, -1, 0)
    return out


def _compatible(a, b):
    return a[1] < b[0] or b[1] < a[0]


def max_nonoverlapped_exhaustive(spans, limit=18):
    """Largest pairwise non-overlapped subset, by exhaustive search."""
    spans = sorted(set(spans))  # equal spans always overlap each other
    m = len(spans)
    if m > limit:
        raise ValueError(f"{m} distinct spans: too many for exhaustive search")
    compat = [0] * m
    for i in range(m):
        for j in range(m):
            if i != j and _compatible(spans[i], spans[j]):
                compat[i] |= 1 << j
    best = 0
    for mask in range(1 << m):
        ok = True
        mm = mask
        size = 0
        while mm:
            low = mm & -mm
            i = low.bit_length() - 1
            if (mask & ~compat[i]) & ~low:
                ok = False
                break
            size += 1
            mm ^= low
        if ok and size > best:
            best = size
    return best


def max_nonoverlapped_dp(spans):
    """Weighted interval scheduling DP with unit weights:
    opt(j) = max(opt(j-1), 1 + opt(p(j))), p(j) = last span ending before s_j."""
    spans = sorted(spans, key=lambda se: (se[1], se[0]))
    ends = [e for _, e in spans]
    opt = [0] * (len(spans) + 1)
    for j, (s, e) in enumerate(spans, start=1):
        p = bisect.bisect_left(ends, s)  # spans with end < s
        opt[j] = max(opt[j - 1], 1 + opt[p])
    return opt[-1]


def count(types, times, ep, lo, hi, method="dp"):
    spans = occurrences(types, times, ep, lo, hi)
    if method == "exhaustive":
        return max_nonoverlapped_exhaustive(spans)
    return max_nonoverlapped_dp(spans)


def occurrences_positions(types, times, ep, lo, hi):
    """All occurrences as (first event index, last event index) spans."""
    n = len(types)
    N = len(ep)
    out = []

    def rec(k, prev_idx, first):
        for i in range(n):
            if types[i] != ep[k]:
                continue
            if k > 0:
                d = int(times[i]) - int(times[prev_idx])
                if not (lo[k - 1] < d <= hi[k - 1]):
                    continue
            f = i if k == 0 else first
            if k == N - 1:
                out.append((f, i))
            else:
                rec(k + 1, i, f)

    rec(0, -1, 0)
    return out


def count_stream_order(types, times, ep, lo, hi):
    """Frequency with overlap decided in stream order (the reset of the state
    machine of Sec. III-A taken literally): two occurrences are non-overlapped
    iff one's last event comes before the other's first event in the stream.
    The same interval-scheduling DP, over stream positions."""
    return max_nonoverlapped_dp(occurrences_positions(types, times, ep, lo, hi))
