"""CPU oracle for exact non-overlapped serial-episode counting -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP engine (``paper_0905_2203_amd``)
never imports it and shares no code with it.

* ``count(stream, cands, method)``: the C oracle (``episode_oracle.c``), either
  the decomposition of Sec. IV-A with Alg. 1 (``"decomp"``, the definition) or
  the serial state machine of Sec. III-A (``"fsm"``).
* ``brute``: tiny-input enumeration of every constrained occurrence followed by
  an exhaustive / dynamic-programming maximum non-overlapped subset.
* ``apriori``: the level-wise discovery procedure of Sec. II-C on top of
  ``count`` (tuples for small runs, arrays for levels of 1e8 candidates).
* ``segmented``: segment-parallel counting with an exact joining rule for the
  segments (the segment idea of Sec. III-B), pure Python, pinned against the
  unsegmented count.
* ``mlp``: the scheduler's cost model in FP64 (forward, back-propagation, Adam).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "episode_oracle.c")

METHODS = {"decomp": 0, "fsm": 1, "fsm_stream": 2}


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP over candidates)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, SRC_PATH])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.oracle_count_batch.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                         P, P, P, P, ctypes.c_int, ctypes.c_int, P]
        L.oracle_count_batch.restype = ctypes.c_int
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def count(stream, cands, method: str = "decomp", nthreads: int = 0) -> np.ndarray:
    """int64 counts of every candidate of ``cands`` in ``stream``."""
    types = np.ascontiguousarray(stream["types"], dtype=np.int32)
    times = np.ascontiguousarray(stream["times"], dtype=np.int64)
    N = np.ascontiguousarray(cands["N"], dtype=np.int32)
    ty = np.ascontiguousarray(cands["types"], dtype=np.int32)
    lo = np.ascontiguousarray(cands["lo"], dtype=np.int64)
    hi = np.ascontiguousarray(cands["hi"], dtype=np.int64)
    m = N.size
    assert ty.shape == (m, 8) and lo.shape == (m, 7) and hi.shape == (m, 7)
    out = np.zeros(m, dtype=np.int64)
    rc = lib().oracle_count_batch(_p(types), _p(times), types.size, int(stream["K"]), m, _p(N),
                                  _p(ty), _p(lo), _p(hi), METHODS[method], int(nthreads), _p(out))
    if rc != 0:
        raise ValueError("oracle rejected its input")
    return out
