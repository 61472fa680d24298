"""Write the expected counts of the five workload presets at full size.

Every expected value is computed by the CPU oracle (``oracle.count``, the
decomposition of Sec. IV-A with the greedy of Alg. 1; ``oracle.apriori`` for
the level-wise run of Sec. II-C) on the seeded inputs of ``spikegen``; nothing
here comes from the HIP engine.  Outputs (in this folder):

  full_cfg1.npz   every count of preset 1 (992 pairs)
  full_cfg3.npz   every count of preset 3 (16 recordings, counts_r0..counts_r15)
  full_cfg4.npz   every count of preset 4 (50k episodes)
  full_cfg5.npz   every count of preset 5 (200k episodes)
  full_cfg2.json  preset 2, level-wise discovery: per level the number of
                  candidates and of frequent episodes and an order-independent
                  digest of the (episode, count) rows of all candidates and of
                  the frequent ones (``tests/fullsize.py``)

Each file records fingerprints of the inputs it was computed from.  Usage:
    python tests/golden/make_full_parity.py 1 3 4 5 2 [--threads T]
Preset 5 takes about 70 min and preset 2 several hours on 8 cores; partial
results of both are kept in a resume file under /tmp.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
import spikegen as sg  # noqa: E402
from fullsize import MultisetDigest, cand_fingerprint, stream_fingerprint  # noqa: E402
from oracle import apriori  # noqa: E402


def log(msg):
    print(f"[golden] {time.strftime('%H:%M:%S')} {msg}", flush=True)


def save_npz(name, meta, arrays):
    path = os.path.join(HERE, name)
    tmp = path + ".tmp.npz"
    np.savez_compressed(tmp, meta=np.array(json.dumps(meta)), **arrays)
    os.replace(tmp, path)
    log(f"wrote {path} ({os.path.getsize(path)} bytes)")


def count_resumable(s, c, tag, threads, chunk=4096):
    """oracle.count in chunks, resuming from /tmp/<tag>.partial.npy."""
    m = c["N"].size
    part = f"/tmp/golden_{tag}.partial.npy"
    out = np.full(m, -1, np.int64)
    if os.path.exists(part):
        prev = np.load(part, allow_pickle=False)
        if prev.size == m:
            out = prev
    t0 = time.time()
    done0 = int((out >= 0).sum())
    for a in range(0, m, chunk):
        b = min(m, a + chunk)
        if (out[a:b] >= 0).all():
            continue
        out[a:b] = oracle.count(s, sg.take_candidates(c, np.arange(a, b)), "decomp", threads)
        np.save(part, out)
        el = time.time() - t0
        done = int((out >= 0).sum())
        log(f"{tag}: {done}/{m} counted ({el:.0f}s, eta {el / max(done - done0, 1) * (m - done):.0f}s)")
    os.remove(part)
    return out


def meta_of(s, c, extra=None):
    meta = {"stream": stream_fingerprint(s), "candidates": cand_fingerprint(c), "events": int(s["types"].size),
            "m": int(c["N"].size), "oracle": "decomp", "numpy": np.__version__}
    meta.update(extra or {})
    return meta


def cfg_single(k, threads):
    s = sg.config_stream(k)
    c = sg.config_candidates(k, s)
    log(f"preset {k}: n={s['types'].size} m={c['N'].size}")
    counts = count_resumable(s, c, f"cfg{k}", threads)
    assert counts.max(initial=0) < 2**31
    save_npz(f"full_cfg{k}.npz", meta_of(s, c), {"counts": counts.astype(np.int32)})


def cfg3(threads):
    metas, arrays = [], {}
    for r in range(16):
        s = sg.config_stream(3, recording=r)
        c = sg.config_candidates(3, s, recording=r)
        t = time.time()
        arrays[f"counts_r{r}"] = oracle.count(s, c, "decomp", threads).astype(np.int32)
        metas.append(meta_of(s, c))
        log(f"preset 3 recording {r}: n={s['types'].size} m={c['N'].size} ({time.time() - t:.1f}s)")
    save_npz("full_cfg3.npz", {"recordings": metas}, arrays)


def cfg2(threads):
    s = sg.config_stream(2)
    menu = [(a * 1000, b * 1000) for a, b in sg.MENU_MINING_MS]
    log(f"preset 2: n={s['types'].size}")
    levels = apriori.mine_arrays(s, menu, 6, 100, chunk=1 << 20, nthreads=threads, log=log)
    out = {"stream": stream_fingerprint(s), "events": int(s["types"].size), "menu": menu, "threshold": 100,
           "max_size": 6, "oracle": "decomp", "levels": []}
    lo_m = np.array([a for a, _ in menu], np.int64)
    hi_m = np.array([b for _, b in menu], np.int64)
    for L, lv in enumerate(levels, start=1):
        m = lv["counts"].size
        d_all, d_freq = MultisetDigest(), MultisetDigest()
        step = 1 << 22
        for a in range(0, m, step):
            b = min(m, a + step)
            ty = lv["types"][a:b]
            iv = lv["ivs"][a:b]
            N = np.full(b - a, L, np.int64)
            lo = lo_m[iv] if L > 1 else np.zeros((b - a, 0), np.int64)
            hi = hi_m[iv] if L > 1 else np.zeros((b - a, 0), np.int64)
            cnt = lv["counts"][a:b]
            d_all.add(N, ty, lo, hi, cnt)
            f = lv["frequent"][a:b]
            d_freq.add(N[f], ty[f], lo[f], hi[f], cnt[f])
        out["levels"].append({"level": L, "candidates": int(m), "frequent": int(lv["frequent"].sum()),
                              "all": d_all.as_dict(), "frequent_rows": d_freq.as_dict()})
        log(f"level {L}: {m} candidates, {int(lv['frequent'].sum())} frequent")
    path = os.path.join(HERE, "full_cfg2.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    log(f"wrote {path}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("presets", nargs="+", type=int)
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    for k in a.presets:
        if k == 3:
            cfg3(a.threads)
        elif k == 2:
            cfg2(a.threads)
        else:
            cfg_single(k, a.threads)


if __name__ == "__main__":
    main()
