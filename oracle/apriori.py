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


# ---------------------------------------------------------------------------
# The same procedure on arrays, for levels of 1e8 candidates (the tuple form
# above needs hundreds of bytes per episode).  A level is (types[m, N],
# ivs[m, N-1]) with int32 entries; candidates are generated with the join rule
# above (alpha + the last node of beta, beta's first N-1 nodes equal alpha's
# last N-1 nodes, new type != alpha's first type) and counted in chunks by
# ``oracle.count``.  The candidate order is alpha-major over the frequent
# episodes in lexicographic (types, ivs) order, then beta in that order -- the
# order of ``join(sorted(frequent))``.
# ---------------------------------------------------------------------------
def _lex_order(types, ivs):
    """Permutation sorting episodes by (types..., ivs...) like sorted() on tuples."""
    keys = [ivs[:, j] for j in range(ivs.shape[1] - 1, -1, -1)] + \
           [types[:, j] for j in range(types.shape[1] - 1, -1, -1)]
    return np.lexsort(keys) if keys else np.arange(types.shape[0])


def _row_keys(cols):
    """Equal rows -> equal keys (consecutive integers from np.unique over rows)."""
    if not cols:
        return np.zeros(0, np.int64)
    a = np.ascontiguousarray(np.stack(cols, axis=1).astype(np.int64))
    _, inv = np.unique(a, axis=0, return_inverse=True)
    return inv.reshape(-1).astype(np.int64)


def join_arrays(ftypes, fivs):
    """Candidates of the next level from frequent episodes given as arrays
    (same set and order as ``join(sorted(frequent))``)."""
    f, n = ftypes.shape
    if f == 0:
        return np.zeros((0, n + 1), np.int32), np.zeros((0, n), np.int32)
    o = _lex_order(ftypes, fivs)
    ty, iv = ftypes[o], fivs[o]
    # key of alpha's suffix and of beta's prefix, from one common numbering
    suf_cols = [ty[:, j] for j in range(1, n)] + [iv[:, j] for j in range(1, n - 1)]
    pre_cols = [ty[:, j] for j in range(0, n - 1)] + [iv[:, j] for j in range(0, n - 2)]
    both = _row_keys([np.concatenate([a, b]) for a, b in zip(suf_cols, pre_cols)])
    ksuf, kpre = both[:f], both[f:]
    # betas grouped by prefix key, in sorted order within a group
    bo = np.argsort(kpre, kind="stable")
    kpre_s = kpre[bo]
    lo = np.searchsorted(kpre_s, ksuf, side="left")
    hi = np.searchsorted(kpre_s, ksuf, side="right")
    cnt = hi - lo
    alpha = np.repeat(np.arange(f), cnt)
    start = np.repeat(lo - np.concatenate([[0], np.cumsum(cnt)[:-1]]), cnt)
    beta = bo[start + np.arange(alpha.size)]
    keep = ty[beta, n - 1] != ty[alpha, 0]
    alpha, beta = alpha[keep], beta[keep]
    ct = np.concatenate([ty[alpha], ty[beta, n - 1:n]], axis=1).astype(np.int32)
    ci = np.concatenate([iv[alpha], iv[beta, n - 2:n - 1]], axis=1).astype(np.int32)
    return ct, ci


def arrays_to_candidates(types, ivs, menu):
    """(types[m, N], ivs[m, N-1]) -> candidate dict for ``oracle.count``."""
    m, n = types.shape
    lo_m = np.array([a for a, _ in menu], np.int64)
    hi_m = np.array([b for _, b in menu], np.int64)
    c = dict(N=np.full(m, n, np.uint8), types=np.full((m, 8), -1, np.int32), lo=np.zeros((m, 7), np.int64),
             hi=np.zeros((m, 7), np.int64))
    c["types"][:, :n] = types
    if n > 1:
        c["lo"][:, :n - 1] = lo_m[ivs]
        c["hi"][:, :n - 1] = hi_m[ivs]
    return c


def mine_arrays(stream, menu, max_size, threshold, chunk=1 << 20, nthreads=0, log=None):
    """``mine`` on arrays: a list of levels, each a dict with ``types``
    (int32[m, N]), ``ivs`` (int32[m, N-1]), ``counts`` (int64[m]) and
    ``frequent`` (bool[m], count > threshold)."""
    K = int(stream["K"])
    levels = []
    for N in range(1, max_size + 1):
        if N == 1:
            ct = np.arange(K, dtype=np.int32)[:, None]
            ci = np.zeros((K, 0), np.int32)
        elif N == 2:
            f1 = np.sort(levels[-1]["types"][levels[-1]["frequent"], 0])
            a, b, i = np.meshgrid(f1, f1, np.arange(len(menu)), indexing="ij")
            keep = (a != b).reshape(-1)
            ct = np.stack([a.reshape(-1), b.reshape(-1)], axis=1)[keep].astype(np.int32)
            ci = i.reshape(-1, 1)[keep].astype(np.int32)
        else:
            prev = levels[-1]
            ct, ci = join_arrays(prev["types"][prev["frequent"]], prev["ivs"][prev["frequent"]])
        m = ct.shape[0]
        if m == 0:
            break
        counts = np.empty(m, np.int64)
        for a in range(0, m, chunk):
            b = min(m, a + chunk)
            counts[a:b] = oracle_count(stream, arrays_to_candidates(ct[a:b], ci[a:b], menu), "decomp", nthreads)
            if log:
                log(f"level {N}: {b}/{m} counted")
        lv = dict(types=ct, ivs=ci, counts=counts, frequent=counts > threshold)
        levels.append(lv)
        if not lv["frequent"].any():
            break
    return levels
