"""Seeded synthetic spike-train streams and candidate serial-episode sets.

This module only draws inputs: event times, event types and candidate episode
descriptions.  It holds none of the counting arithmetic, so both the CPU oracle
(test infrastructure) and the HIP engine can be fed from it without sharing any
of the method.

Streams follow Def. 1 of the paper (events (E_i, t_i) with non-decreasing
integer times); the spike-train datasets of Sec. V-A (Table II) came from a
network simulator that is not available, so the workloads here are Poisson
spike trains with planted cascades of the shapes listed in the five workload
presets below (``config_stream`` / ``config_candidates``).

Conventions
-----------
* A stream is a dict with ``types`` (int32[n]), ``times`` (int32[n] for
  microsecond streams, int64[n] for nanosecond streams), ``K`` (number of event
  types), ``ts_kind`` (0 = int32, 1 = int64), ``unit_per_ms`` and ``planted``
  (list of planted cascades: ``types``, ``lo``, ``hi`` and ``instances``).
* A candidate set is a dict with ``N`` (uint8[m]), ``types`` (int32[m, 8],
  padded with -1), ``lo`` and ``hi`` (int64[m, 7], padded with 0).  Interval j
  of a candidate is the open-closed (lo[j], hi[j]] between nodes j and j+1.
* Events are merged and sorted by (time, type); equal times are kept.
"""
from __future__ import annotations

import numpy as np

MAXN = 8  # largest episode size held by a candidate record
SEED_BASE = 9052203

# Interval menu used for planted cascades and level-wise mining, in ms.
MENU_MINING_MS = ((0, 5), (5, 10), (10, 20))
# Random-candidate menu: lower bound l and width w, in ms.
MENU_LOW_MS = (0, 5, 10, 20)
MENU_WIDTH_MS = (5, 10, 20)


def rng_for(k: int, offset: int = 0) -> np.random.Generator:
    """PCG64 generator for workload preset k (1-based) plus an optional offset."""
    return np.random.Generator(np.random.PCG64(SEED_BASE + k + offset))


# ----------------------------------------------------------------------------
# stream pieces
# ----------------------------------------------------------------------------
def _poisson_seconds(rng, rate_hz: float, dur_s: float) -> np.ndarray:
    cnt = rng.poisson(rate_hz * dur_s)
    return rng.uniform(0.0, dur_s, size=cnt)


def _merge(parts_types, parts_times, ts_kind: int):
    types = np.concatenate(parts_types).astype(np.int32)
    times = np.concatenate(parts_times).astype(np.int64)
    order = np.lexsort((types, times))
    types = types[order]
    times = times[order]
    if ts_kind == 0:
        assert times.max(initial=0) < 2**31 - 1
        times = times.astype(np.int32)
    return np.ascontiguousarray(types), np.ascontiguousarray(times)


def _plant_cascades(rng, sizes, type_pool, dur_units, unit_per_ms, trigger_hz,
                    dur_s, link_menu_ms):
    """Planted cascades whose inter-event gaps are integers drawn uniformly in
    (l, h] of a per-link interval from ``link_menu_ms``; every instance is a
    valid constrained occurrence by construction."""
    planted = []
    used = 0
    for size in sizes:
        ctypes_ = np.array(type_pool[used:used + size], dtype=np.int32)
        used += size
        links = [link_menu_ms[rng.integers(len(link_menu_ms))] for _ in range(size - 1)]
        lo = np.array([a * unit_per_ms for a, _ in links], dtype=np.int64)
        hi = np.array([b * unit_per_ms for _, b in links], dtype=np.int64)
        rate = trigger_hz[len(planted)] if np.ndim(trigger_hz) else trigger_hz
        starts = np.floor(_poisson_seconds(rng, rate, dur_s) * 1000.0 * unit_per_ms).astype(np.int64)
        starts.sort()
        inst = np.empty((starts.size, size), dtype=np.int64)
        inst[:, 0] = starts
        for j in range(size - 1):
            inst[:, j + 1] = inst[:, j] + rng.integers(lo[j] + 1, hi[j] + 1, size=starts.size)
        inst = inst[inst[:, -1] < dur_units]
        planted.append(dict(types=ctypes_, lo=lo, hi=hi, instances=inst))
    return planted


def _stream_from(parts_types, parts_times, planted, K, ts_kind, unit_per_ms):
    for p in planted:
        parts_types.append(np.repeat(p["types"][None, :], p["instances"].shape[0], 0).ravel())
        parts_times.append(p["instances"].ravel())
    types, times = _merge(parts_types, parts_times, ts_kind)
    return dict(types=types, times=times, K=int(K), ts_kind=int(ts_kind),
                unit_per_ms=int(unit_per_ms), planted=planted)


def poisson_stream(rng, K: int, rate_hz, dur_s: float, ts_kind: int,
                   unit_per_ms: int, cascades=None, cascade_trigger_hz=5.0,
                   link_menu_ms=MENU_MINING_MS):
    """Independent homogeneous Poisson spike trains (one per type) plus planted
    cascades.  ``rate_hz`` is a scalar or a per-type array; ``cascades`` is a
    list of cascade sizes (types are drawn distinct across all cascades)."""
    rates = np.broadcast_to(np.asarray(rate_hz, dtype=np.float64), (K,))
    per_s = 1000.0 * unit_per_ms
    pt, ptm = [], []
    for k in range(K):
        s = _poisson_seconds(rng, rates[k], dur_s)
        pt.append(np.full(s.size, k, dtype=np.int32))
        ptm.append(np.floor(s * per_s).astype(np.int64))
    planted = []
    if cascades:
        pool = rng.permutation(K)[: sum(cascades)]
        planted = _plant_cascades(rng, cascades, pool, int(dur_s * per_s), unit_per_ms,
                                  cascade_trigger_hz, dur_s, link_menu_ms)
    return _stream_from(pt, ptm, planted, K, ts_kind, unit_per_ms)


def bursty_stream(rng, K: int, dur_s: float, shape: float, scale_hz: float,
                  window_s: float = 1.0, ts_kind: int = 1, unit_per_ms: int = 1_000_000):
    """Poisson spike trains whose rate is redrawn per type per window from a
    Gamma(shape, scale) distribution (gamma-modulated, bursty)."""
    per_s = 1000.0 * unit_per_ms
    nwin = int(np.ceil(dur_s / window_s))
    rates = rng.gamma(shape, scale_hz, size=(K, nwin))
    counts = rng.poisson(rates * window_s)
    pt, ptm = [], []
    for k in range(K):
        c = counts[k]
        tot = int(c.sum())
        win = np.repeat(np.arange(nwin), c)
        s = (win + rng.uniform(0.0, 1.0, size=tot)) * window_s
        s = s[s < dur_s]
        pt.append(np.full(s.size, k, dtype=np.int32))
        ptm.append(np.floor(s * per_s).astype(np.int64))
    return _stream_from(pt, ptm, [], K, ts_kind, unit_per_ms)


def jitter_cascade_stream(rng, K, rate_hz, dur_s, n_cascades, size, trigger_hz,
                          delay_ms=(5.0, 10.0), jitter_ms=1.0, ts_kind=0, unit_per_ms=1000):
    """Poisson background plus cascades with a fixed per-link delay drawn once
    from U(delay_ms) and a per-instance jitter U[-jitter_ms, +jitter_ms]."""
    per_s = 1000.0 * unit_per_ms
    pt, ptm = [], []
    for k in range(K):
        s = _poisson_seconds(rng, rate_hz, dur_s)
        pt.append(np.full(s.size, k, dtype=np.int32))
        ptm.append(np.floor(s * per_s).astype(np.int64))
    pool = rng.permutation(K)[: n_cascades * size]
    planted = []
    for c in range(n_cascades):
        ctypes_ = pool[c * size:(c + 1) * size].astype(np.int32)
        # U(a, b]: 1 - U[0,1) lies in (0, 1]
        delays = delay_ms[0] + (delay_ms[1] - delay_ms[0]) * (1.0 - rng.uniform(size=size - 1))
        trig = np.sort(_poisson_seconds(rng, trigger_hz, dur_s))
        inst_s = np.empty((trig.size, size))
        inst_s[:, 0] = trig
        for j in range(size - 1):
            jit = rng.uniform(-jitter_ms, jitter_ms, size=trig.size)
            inst_s[:, j + 1] = inst_s[:, j] + (delays[j] + jit) / 1000.0
        inst_s = inst_s[inst_s[:, -1] < dur_s]
        inst = np.floor(inst_s * per_s).astype(np.int64)
        planted.append(dict(types=ctypes_, delays_ms=delays, instances=inst,
                            lo=np.array([int((d - jitter_ms - 1) * unit_per_ms) for d in delays]),
                            hi=np.array([int((d + jitter_ms + 1) * unit_per_ms) for d in delays])))
    return _stream_from(pt, ptm, planted, K, ts_kind, unit_per_ms)


def tiny_stream(rng, n: int, K: int, tmax: int, ts_kind: int = 1):
    """Tiny random stream with integer times in [0, tmax] (many equal times)."""
    types = rng.integers(0, K, size=n).astype(np.int32)
    times = rng.integers(0, tmax + 1, size=n).astype(np.int64)
    types, times = _merge([types], [times], ts_kind)
    return dict(types=types, times=times, K=int(K), ts_kind=int(ts_kind),
                unit_per_ms=1, planted=[])


# ----------------------------------------------------------------------------
# candidate sets
# ----------------------------------------------------------------------------
def empty_candidates(m: int):
    return dict(N=np.zeros(m, np.uint8), types=np.full((m, MAXN), -1, np.int32),
                lo=np.zeros((m, MAXN - 1), np.int64), hi=np.zeros((m, MAXN - 1), np.int64))


def candidates_from_list(eps):
    """``eps`` is a list of (types, lo, hi) tuples."""
    c = empty_candidates(len(eps))
    for i, (ty, lo, hi) in enumerate(eps):
        n = len(ty)
        c["N"][i] = n
        c["types"][i, :n] = ty
        c["lo"][i, : n - 1] = lo
        c["hi"][i, : n - 1] = hi
    return c


def concat_candidates(a, b):
    return {k: np.concatenate([a[k], b[k]]) for k in ("N", "types", "lo", "hi")}


def take_candidates(c, idx):
    return {k: np.ascontiguousarray(c[k][idx]) for k in ("N", "types", "lo", "hi")}


def all_pairs(K: int, lo: int, hi: int):
    """Every ordered pair A->B with A != B, lexicographic, one interval (lo, hi]."""
    a, b = np.meshgrid(np.arange(K), np.arange(K), indexing="ij")
    mask = a != b
    a, b = a[mask], b[mask]
    c = empty_candidates(a.size)
    c["N"][:] = 2
    c["types"][:, 0] = a
    c["types"][:, 1] = b
    c["lo"][:, 0] = lo
    c["hi"][:, 0] = hi
    return c


def random_candidates(rng, m: int, K: int, nmin: int, nmax: int, unit_per_ms: int,
                      low_ms=MENU_LOW_MS, width_ms=MENU_WIDTH_MS):
    """Random episodes: N ~ U{nmin..nmax}, distinct uniform types, per link
    l ~ U(low_ms) and w ~ U(width_ms), interval (l, l+w]."""
    c = empty_candidates(m)
    nmax = min(nmax, K)
    N = rng.integers(nmin, nmax + 1, size=m)
    c["N"][:] = N
    # distinct types: first N entries of a random permutation per candidate
    keys = rng.random((m, K))
    perm = np.full((m, MAXN), -1, np.int32)
    take = min(K, MAXN)
    perm[:, :take] = np.argsort(keys, axis=1)[:, :take]
    col = np.arange(MAXN)[None, :]
    c["types"][:] = np.where(col < N[:, None], perm, -1)
    lows = np.asarray(low_ms, np.int64)[rng.integers(0, len(low_ms), size=(m, MAXN - 1))]
    wids = np.asarray(width_ms, np.int64)[rng.integers(0, len(width_ms), size=(m, MAXN - 1))]
    live = np.arange(MAXN - 1)[None, :] < (N[:, None] - 1)
    c["lo"][:] = np.where(live, lows * unit_per_ms, 0)
    c["hi"][:] = np.where(live, (lows + wids) * unit_per_ms, 0)
    return c


def tiny_candidates(rng, m: int, K: int, nmax: int, tmax_gap: int):
    """Tiny random episodes for brute-force checks: N ~ U{1..nmax} distinct
    types, 0 <= lo < hi <= tmax_gap."""
    c = empty_candidates(m)
    for i in range(m):
        n = int(rng.integers(1, min(nmax, K) + 1))
        c["N"][i] = n
        c["types"][i, :n] = rng.permutation(K)[:n]
        for j in range(n - 1):
            lo = int(rng.integers(0, tmax_gap))
            hi = int(rng.integers(lo + 1, tmax_gap + 1))
            c["lo"][i, j] = lo
            c["hi"][i, j] = hi
    return c


def planted_subepisodes(planted):
    """Every full, prefix and suffix sub-episode (size >= 2) of each planted cascade."""
    eps = []
    seen = set()
    for p in planted:
        ty, lo, hi = list(p["types"]), list(p["lo"]), list(p["hi"])
        n = len(ty)
        for a in range(n):
            for b in range(a + 2, n + 1):
                if a != 0 and b != n:
                    continue
                key = (tuple(ty[a:b]), tuple(lo[a:b - 1]), tuple(hi[a:b - 1]))
                if key not in seen:
                    seen.add(key)
                    eps.append((ty[a:b], lo[a:b - 1], hi[a:b - 1]))
    return eps


# ----------------------------------------------------------------------------
# workload presets (1..5); ``scale`` < 1 shrinks them for quick tests
# ----------------------------------------------------------------------------
def config_stream(k: int, scale: float = 1.0, recording: int | None = None):
    """Stream of workload preset k.  For preset 3 pass ``recording`` in 0..15."""
    rng = rng_for(k)
    if k == 1:
        return jitter_cascade_stream(rng, K=32, rate_hz=10.0, dur_s=30.0 * scale, n_cascades=2,
                                     size=3, trigger_hz=5.0, ts_kind=0, unit_per_ms=1000)
    if k == 2:
        sizes = list(rng.integers(4, 7, size=4))
        trig = rng.uniform(2.0, 8.0, size=4)
        return poisson_stream(rng, K=64, rate_hz=20.0, dur_s=300.0 * scale, ts_kind=0,
                              unit_per_ms=1000, cascades=sizes, cascade_trigger_hz=trig)
    if k == 3:
        sizes = recording_sizes(scale)
        r = 0 if recording is None else int(recording)
        rr = rng_for(3, offset=1000 + r)
        n_r = sizes[r]
        return bursty_stream(rr, K=60, dur_s=n_r / 900.0, shape=2.0, scale_hz=7.5)
    if k == 4:
        kk = np.arange(1, 129, dtype=np.float64)
        w = kk ** -1.2
        dur = 3600.0 * scale
        rates = w / w.sum() * (10_000_000 / 3600.0)
        return poisson_stream(rng, K=128, rate_hz=rates, dur_s=dur, ts_kind=1, unit_per_ms=1_000_000)
    if k == 5:
        sizes = list(rng.integers(3, 9, size=32))
        trig = rng.uniform(2.0, 8.0, size=32)
        dur = 3600.0 * scale
        planted_events = float(np.sum(np.asarray(sizes) * trig)) * dur
        bg = (50_000_000 * scale - planted_events) / (256 * dur)
        return poisson_stream(rng, K=256, rate_hz=bg, dur_s=dur, ts_kind=1, unit_per_ms=1_000_000,
                              cascades=sizes, cascade_trigger_hz=trig)
    raise ValueError(f"no workload preset {k}")


def recording_sizes(scale: float = 1.0):
    """Event counts of the 16 recordings of preset 3 (log-uniform in [5e4, 2e6])."""
    rng = rng_for(3, offset=500)
    n = np.exp(rng.uniform(np.log(5e4), np.log(2e6), size=16))
    return np.maximum((n * scale).astype(np.int64), 100)


def recording_cand_counts(scale: float = 1.0):
    rng = rng_for(3, offset=600)
    m = np.exp(rng.uniform(np.log(1e3), np.log(6e4), size=16))
    return np.maximum((m * scale).astype(np.int64), 8)


def config_candidates(k: int, stream=None, scale: float = 1.0, recording: int | None = None,
                      training: bool = False):
    """Candidate set of workload preset k (preset 2 mines level-wise and has none)."""
    if k == 1:
        return all_pairs(32, 0, 10 * 1000)
    if k == 3:
        r = 0 if recording is None else int(recording)
        m = int(recording_cand_counts(scale)[r])
        return random_candidates(rng_for(3, offset=2000 + r), m, 60, 2, 8, 1_000_000)
    if k == 4:
        rng = rng_for(4, offset=100 if training else 1)
        return random_candidates(rng, max(int(50_000 * scale), 64), 128, 3, 8, 1_000_000)
    if k == 5:
        rng = rng_for(5, offset=1)
        sub = candidates_from_list(planted_subepisodes(stream["planted"])) if stream else empty_candidates(0)
        m = max(int(200_000 * scale), 64)
        rest = random_candidates(rng, max(m - sub["N"].size, 0), 256, 2, 8, 1_000_000)
        return concat_candidates(sub, rest)
    raise ValueError(f"preset {k} has no fixed candidate set")
