"""Segment-parallel counting with exact boundary reconciliation -- TEST
INFRASTRUCTURE (pure Python; small inputs only).

Sec. III-B splits the stream into segments counted independently and joins
the segments' results afterwards (MapConcat; the figures that give its joining
rule are missing from the paper).  This module states an exact joining rule
and implements it from scratch, without the HIP engine, so the rule itself is
pinned: its counts must equal the unsegmented count of ``oracle.count`` for
any boundaries (tests/test_oracle_pins.py).

Segments are cut at timestamp values B_1 < ... < B_{P-1}; segment p holds the
events with B_p <= t < B_{p+1} (B_0 = -inf, B_P = +inf).  H = sum of the upper
bounds is the longest span of an occurrence, so every occurrence ending at or
after B_p starts at or after B_p - H.

1. Speculate (independent per segment): run the time-semantic state machine
   (Sec. III-A; a start is admitted only strictly after the last completion,
   which makes its completions the greedy picks of Alg. 1) over the events
   from time B_p - H on, as if the last completion were B_p - H - 1; keep the
   completions at t >= B_p: their number c_p, the first ``q`` of them and the
   last.
2. Reconcile (in segment order, carrying tau = the last true completion before
   B_p, -inf at first):
   * tau < B_p - H: partial occurrences the true machine holds at B_p - H began
     after tau and could only complete before B_p, which would contradict tau;
     so from B_p on it completes exactly where the speculative machine does:
     take c_p (and its last completion as the new tau);
   * otherwise re-run the machine from the state right after the completion
     at tau (last completion tau, no partial occurrence) over the events after
     tau.  Right after any completion time both machines share, they are in
     the same state; so when the re-run completes at one of the speculative
     first ``q`` completions, the rest of c_p is taken as is.  If it meets none
     of them it runs to the end of the segment.
"""
from __future__ import annotations

import bisect

NEG_INF = float("-inf")


def fsm_completions(types, times, i0, i1, ep, lo, hi, e0, meet=None):
    """Completion times of the time-semantic state machine of Sec. III-A over
    stream positions [i0, i1), started with last completion e0 and empty
    per-node lists.  With ``meet`` (a list of times), stops right after the
    first completion that is in it and returns (completions, index in meet);
    otherwise returns (completions, None)."""
    N = len(ep)
    lists = [[] for _ in range(N)]
    e = e0
    out = []
    for i in range(i0, i1):
        E, t = int(types[i]), int(times[i])
        for j in range(N - 1, -1, -1):  # a type at several nodes: last node first
            if E != ep[j]:
                continue
            if j == 0:
                if t > e:
                    if N == 1:
                        e = t
                        out.append(t)
                    else:
                        lists[0].append(t)
            else:
                ok = any(lo[j - 1] < t - tp <= hi[j - 1] for tp in lists[j - 1])
                if ok:
                    if j == N - 1:
                        e = t
                        out.append(t)
                        lists = [[] for _ in range(N)]
                    else:
                        lists[j].append(t)
            if meet is not None and out and out[-1] == t and t in meet:
                return out, meet.index(t)
    return out, None


def count_segmented(stream, ep, lo, hi, bounds, q=4):
    """Count of one episode (types ep, intervals (lo[j], hi[j]]) by segments
    cut at the timestamp values ``bounds`` (strictly increasing), joined by
    exact reconciliation.  Returns (count, last completion or -inf)."""
    types, times = stream["types"], [int(x) for x in stream["times"]]
    n = len(times)
    H = sum(int(x) for x in hi)
    B = [NEG_INF] + [int(b) for b in bounds]
    P = len(B)
    seg_end = [bisect.bisect_left(times, B[p + 1]) if p + 1 < P else n for p in range(P)]
    # 1. speculation per segment
    spec = []
    for p in range(P):
        if p == 0:
            i0, e0 = 0, NEG_INF
        else:
            i0, e0 = bisect.bisect_left(times, B[p] - H), B[p] - H - 1
        comp, _ = fsm_completions(types, times, i0, seg_end[p], ep, lo, hi, e0)
        own = [x for x in comp if p == 0 or x >= B[p]]
        spec.append((len(own), own[:q], own[-1] if own else None))
    # 2. reconciliation in segment order
    tau = NEG_INF
    total = 0
    for p in range(P):
        c, first, last = spec[p]
        if p == 0 or tau < B[p] - H:
            total += c
            if c:
                tau = last
            continue
        i0 = bisect.bisect_right(times, tau)
        comp, k = fsm_completions(types, times, i0, seg_end[p], ep, lo, hi, tau, meet=first)
        if k is not None:
            total += len(comp) + (c - k - 1)
            tau = last
        else:
            total += len(comp)
            if comp:
                tau = comp[-1]
    return total, tau


def count(stream, cands, bounds, q=4):
    """Counts of every candidate of a candidate dict (see ``oracle.count``)."""
    out = []
    for i in range(len(cands["N"])):
        N = int(cands["N"][i])
        ep = [int(x) for x in cands["types"][i, :N]]
        lo = [int(x) for x in cands["lo"][i, :N - 1]]
        hi = [int(x) for x in cands["hi"][i, :N - 1]]
        out.append(count_segmented(stream, ep, lo, hi, bounds, q)[0])
    return out
