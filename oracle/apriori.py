"""Level-wise discovery of frequent serial episodes -- TEST INFRASTRUCTURE.

Sec. II-C: candidates of size N are generated from the frequent episodes of
size N-1, their counts are obtained in one pass over the stream, and the
episodes whose count is greater than the threshold are kept.  Generation:
level 1 takes every type; level 2 pairs distinct frequent types with every
interval of the menu; level N+1 extends a frequent alpha by the last node of
a frequent beta whose first N-1 nodes (types and intervals) equal alpha's
last N-1 nodes, when the new type does not repeat alpha's first type.

Episodes are tuples (types, interval ids); counts come from ``oracle.count``.
"""
from __future__ import annotations

from collections import defaultdict

import numpy as np

from . import count as oracle_count


def to_candidates(eps, menu):
    """Episode tuples -> candidate dict (types, lo, hi) for oracle.count."""
    m = len(eps)
    c = dict(N=np.zeros(m, np.uint8), types=np.full((m, 8), -1, np.int32), lo=np.zeros((m, 7), np.int64),
             hi=np.zeros((m, 7), np.int64))
    for i, (ty, iv) in enumerate(eps):
        n = len(ty)
        c["N"][i] = n
        c["types"][i, :n] = ty
        for k, v in enumerate(iv):
            c["lo"][i, k], c["hi"][i, k] = menu[v]
    return c


def join(frequent):
    """Candidates of the next level from the frequent episodes of this one."""
    if not frequent:
        return []
    n = len(frequent[0][0])
    by_prefix = defaultdict(list)
    for ty, iv in frequent:
        by_prefix[(ty[:-1], iv[:-1] if n > 1 else ())].append((ty, iv))
    out = []
    for ty, iv in frequent:
        key = (ty[1:], iv[1:])
        for ty2, iv2 in by_prefix.get(key, []):
            if ty2[-1] == ty[0]:
                continue
            out.append((ty + (ty2[-1],), iv + (iv2[-1],)))
    return out


def mine(stream, menu, max_size, threshold, method="decomp"):
    """Returns a list of levels; each level is a dict episode -> count (all
    candidates) and the set of frequent episodes."""
    K = stream["K"]
    levels = []
    for N in range(1, max_size + 1):
        if N == 1:
            cands = [((k,), ()) for k in range(K)]
        elif N == 2:
            f1 = sorted(ep[0][0] for ep in levels[-1]["frequent"])
            cands = [((a, b), (i,)) for a in f1 for b in f1 if a != b for i in range(len(menu))]
        else:
            cands = join(sorted(levels[-1]["frequent"]))
        if not cands:
            break
        counts = oracle_count(stream, to_candidates(cands, menu), method)
        lv = dict(counts={ep: int(c) for ep, c in zip(cands, counts)},
                  frequent={ep for ep, c in zip(cands, counts) if c > threshold})
        levels.append(lv)
        if not lv["frequent"]:
            break
    return levels
