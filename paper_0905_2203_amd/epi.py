"""Thin ctypes binding of ``libepi.so`` (the C ABI declared in include/epi.h).

Every function here only marshals arguments: host arrays are numpy arrays,
device arrays are torch tensors on the ROCm device (torch supplies device
memory and streams), and every count is computed by the library's HIP
kernels.  A missing library is an error, never a fallback.

Status codes other than EPI_OK raise ``EpiError`` carrying the code and the
context's last error message.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libepi.so")

EPI_OK = 0
EPI_EINVAL = -1
EPI_EUNSORTED = -2
EPI_ETYPE = -3
EPI_EINTERVAL = -4
EPI_ESIZE = -5
EPI_EREPEAT = -6
EPI_EOVERFLOW = -7
EPI_ENOMEM = -8
EPI_EDEVICE = -9
EPI_ESTATE = -10
EPI_TS_I32 = 0
EPI_TS_I64 = 1
EPI_MODE_PLAIN = 0
EPI_MODE_BATCHED = 1
EPI_MODE_INCREMENTAL = 2
EPI_MODE_TRACKING = 3
EPI_SCHED_RR = 0
EPI_SCHED_LEARNED = 1
EPI_SCHED_HEURISTIC = 2
EPI_SCHED_MEASURED = 3

EXPORTS = [
    "epi_create", "epi_destroy", "epi_last_error", "epi_status_string",
    "epi_validate_stream", "epi_validate_candidates",
    "epi_load_stream", "epi_load_stream_device", "epi_stream_info", "epi_read_type_index",
    "epi_release_stream", "epi_append_stream", "epi_submit_candidates", "epi_release_set",
    "epi_count", "epi_set_option", "epi_sync", "epi_read_counts", "epi_counts_device", "epi_batched_stats",
    "epi_read_schedule", "epi_count_noalloc",
    "epi_mine", "epi_mine_levels", "epi_mine_level_info", "epi_mine_read", "epi_mine_read_at",
    "epi_mine_level_bytes", "epi_mine_release",
    "epi_mlp_init", "epi_mlp_params", "epi_mlp_get_params", "epi_mlp_set_params", "epi_mlp_forward",
    "epi_mlp_grad", "epi_mlp_adam_step", "epi_mlp_train", "epi_costmodel_features",
    "epi_read_worklog", "epi_read_item_cycles", "epi_costmodel_train", "epi_costmodel_scaling",
    "epi_costmodel_predict", "epi_costmodel_save", "epi_costmodel_load", "epi_autotune",
]
EPI_OPT_SEGMENTS = 1
EPI_OPT_LANES = 2
EPI_OPT_TARGET_LANES = 3
EPI_OPT_PAIR_FILTER = 4
EPI_OPT_MINE_ENGINE = 5
EPI_OPT_WORKLOG = 6
EPI_OPT_TARGET_ITEMS = 7
EPI_OPT_MINE_LIST_BYTES = 8
EPI_OPT_ALLOW_REPEATS = 9
EPI_OPT_MINE_LIST_ALPHAS = 10
EPI_OPT_STREAM_ORDER = 11
EPI_OPT_LANE_ENGINE = 12
EPI_OPT_RING_CLASSES = 13


class EpiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{status_string(code)} ({code}): {msg}")
        self.code = code


_lib = None
P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
INT = ctypes.c_int


def lib():
    """Load libepi.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_0905_2203_amd/build.py")
        # torch bundles its own libamdhip64 (same soname as the system one).
        # Loading torch first makes libepi bind to that copy, so the process
        # holds a single HIP runtime and device pointers are shared with torch.
        import torch  # noqa: F401

        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "epi_create": ([INT, ctypes.POINTER(P)], I32),
            "epi_destroy": ([P], None),
            "epi_last_error": ([P], ctypes.c_char_p),
            "epi_status_string": ([I32], ctypes.c_char_p),
            "epi_validate_stream": ([P, P, I64, INT, I32], I32),
            "epi_validate_candidates": ([I64, P, P, P, P, I32, INT], I32),
            "epi_load_stream": ([P, P, P, I64, INT, I32, ctypes.POINTER(I32)], I32),
            "epi_load_stream_device": ([P, P, P, I64, INT, I32, P, ctypes.POINTER(I32)], I32),
            "epi_stream_info": ([P, I32, ctypes.POINTER(I64), ctypes.POINTER(I32), ctypes.POINTER(INT)], I32),
            "epi_read_type_index": ([P, I32, P, P], I32),
            "epi_release_stream": ([P, I32], I32),
            "epi_append_stream": ([P, I32, P, P, I64], I32),
            "epi_submit_candidates": ([P, I32, I64, P, P, P, P, ctypes.POINTER(I32)], I32),
            "epi_release_set": ([P, I32], I32),
            "epi_count": ([P, P, I32, INT, INT, P], I32),
            "epi_sync": ([P], I32),
            "epi_set_option": ([P, INT, I64], I32),
            "epi_read_counts": ([P, I32, P, I64], I32),
            "epi_counts_device": ([P, I32, ctypes.POINTER(P)], I32),
            "epi_batched_stats": ([P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I64)], I32),
            "epi_read_schedule": ([P, I32, P, P, I64], I32),
            "epi_count_noalloc": ([P, I32, I64, P], I32),
            "epi_mine": ([P, I32, I32, P, P, I32, I64, P, ctypes.POINTER(I32)], I32),
            "epi_mine_levels": ([P, I32, ctypes.POINTER(I32)], I32),
            "epi_mine_level_info": ([P, I32, I32, ctypes.POINTER(I64), ctypes.POINTER(I64), P], I32),
            "epi_mine_read": ([P, I32, I32, INT, I64, P, P, P, P, P], I32),
            "epi_mine_release": ([P, I32], I32),
            "epi_mine_read_at": ([P, I32, I32, I64, P, P, P, P, P, P], I32),
            "epi_mine_level_bytes": ([P, I32, I32, ctypes.POINTER(I64)], I32),
            "epi_mlp_init": ([P, I32, ctypes.c_uint64], I32),
            "epi_mlp_params": ([P, ctypes.POINTER(I32), ctypes.POINTER(I64)], I32),
            "epi_mlp_get_params": ([P, P, I64], I32),
            "epi_mlp_set_params": ([P, P, I64], I32),
            "epi_mlp_forward": ([P, P, I64, P], I32),
            "epi_mlp_grad": ([P, P, P, I64, ctypes.POINTER(ctypes.c_float), P], I32),
            "epi_mlp_adam_step": ([P, P, ctypes.c_float], I32),
            "epi_mlp_train": ([P, P, P, I64, I32, I32, ctypes.c_float, P], I32),
            "epi_costmodel_features": ([P, I32, P, I64], I32),
            "epi_read_worklog": ([P, I32, P, I64], I32),
            "epi_read_item_cycles": ([P, I32, P, I64, ctypes.POINTER(I64)], I32),
            "epi_costmodel_train": ([P, P, I32, I32, ctypes.c_uint64, P], I32),
            "epi_costmodel_scaling": ([P, P, P, P], I32),
            "epi_costmodel_predict": ([P, I32, P, I64], I32),
            "epi_costmodel_save": ([P, ctypes.c_char_p], I32),
            "epi_costmodel_load": ([P, ctypes.c_char_p], I32),
            "epi_autotune": ([P, P, I32, INT, ctypes.c_char_p, P], I32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def status_string(code: int) -> str:
    return lib().epi_status_string(int(code)).decode()


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(P)
    return P(a.data_ptr())  # torch tensor


def _ts_kind(times) -> int:
    dt = str(times.dtype)
    if dt.endswith("int64"):
        return EPI_TS_I64
    if dt.endswith("int32"):
        return EPI_TS_I32
    raise TypeError("times must be int32 or int64")


def epi_validate_stream(types: np.ndarray, times: np.ndarray, K: int) -> int:
    types = np.ascontiguousarray(types, np.int32)
    times = np.ascontiguousarray(times)
    return int(lib().epi_validate_stream(_ptr(types), _ptr(times), types.size, _ts_kind(times), int(K)))


def _cand_arrays(c):
    N = np.ascontiguousarray(c["N"], np.uint8)
    ty = np.ascontiguousarray(c["types"], np.int32)
    lo = np.ascontiguousarray(c["lo"], np.int64)
    hi = np.ascontiguousarray(c["hi"], np.int64)
    m = N.size
    if ty.shape != (m, 8) or lo.shape != (m, 7) or hi.shape != (m, 7):
        raise ValueError("candidate arrays must be N[m], types[m,8], lo[m,7], hi[m,7]")
    return N, ty, lo, hi


def epi_validate_candidates(cands, K: int, ts_kind: int) -> int:
    N, ty, lo, hi = _cand_arrays(cands)
    return int(lib().epi_validate_candidates(N.size, _ptr(N), _ptr(ty), _ptr(lo), _ptr(hi), int(K), int(ts_kind)))


class Context:
    """An epi_ctx bound to one HIP device.  Methods are the ABI calls."""

    def __init__(self, device: int = 0):
        h = P()
        rc = lib().epi_create(int(device), ctypes.byref(h))
        if rc != EPI_OK:
            raise EpiError(rc, lib().epi_last_error(None).decode())
        self.h = h
        self._keep = []

    def close(self):
        if self.h:
            lib().epi_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != EPI_OK:
            raise EpiError(rc, lib().epi_last_error(self.h).decode())

    def last_error(self) -> str:
        return lib().epi_last_error(self.h).decode()

    # streams -------------------------------------------------------------
    def epi_load_stream(self, types: np.ndarray, times: np.ndarray, K: int) -> int:
        types = np.ascontiguousarray(types, np.int32)
        times = np.ascontiguousarray(times)
        sid = I32()
        self._check(lib().epi_load_stream(self.h, _ptr(types), _ptr(times), types.size, _ts_kind(times),
                                          int(K), ctypes.byref(sid)))
        return sid.value

    def epi_append_stream(self, sid: int, types: np.ndarray, times: np.ndarray):
        """Append events (times not before the stream's last) to stream sid."""
        types = np.ascontiguousarray(types, np.int32)
        times = np.ascontiguousarray(times)
        self._check(lib().epi_append_stream(self.h, int(sid), _ptr(types), _ptr(times), types.size))

    def epi_load_stream_device(self, d_types, d_times, K: int, hip_stream=None) -> int:
        """d_types / d_times: contiguous torch tensors on the device."""
        sid = I32()
        st = None if hip_stream is None else P(int(hip_stream))
        self._check(lib().epi_load_stream_device(self.h, _ptr(d_types), _ptr(d_times), int(d_types.numel()),
                                                 _ts_kind(d_times), int(K), st, ctypes.byref(sid)))
        return sid.value

    def epi_stream_info(self, sid: int):
        n, K, kind = I64(), I32(), INT()
        self._check(lib().epi_stream_info(self.h, int(sid), ctypes.byref(n), ctypes.byref(K), ctypes.byref(kind)))
        return n.value, K.value, kind.value

    def epi_read_type_index(self, sid: int):
        n, K, kind = self.epi_stream_info(sid)
        off = np.zeros(K + 1, np.int32)
        ts = np.zeros(n, np.int64 if kind == EPI_TS_I64 else np.int32)
        self._check(lib().epi_read_type_index(self.h, int(sid), _ptr(off), _ptr(ts)))
        return off, ts

    def epi_release_stream(self, sid: int):
        self._check(lib().epi_release_stream(self.h, int(sid)))

    # candidates ------------------------------------------------------------
    def epi_submit_candidates(self, sid: int, cands) -> int:
        N, ty, lo, hi = _cand_arrays(cands)
        out = I32()
        self._check(lib().epi_submit_candidates(self.h, int(sid), N.size, _ptr(N), _ptr(ty), _ptr(lo), _ptr(hi),
                                                ctypes.byref(out)))
        return out.value

    def epi_release_set(self, set_id: int):
        self._check(lib().epi_release_set(self.h, int(set_id)))

    # counting ----------------------------------------------------------------
    def epi_count(self, set_ids, mode: int = EPI_MODE_PLAIN, sched: int = EPI_SCHED_RR, hip_stream=None):
        ids = np.ascontiguousarray(np.atleast_1d(np.asarray(set_ids, np.int32)))
        st = None if hip_stream is None else P(int(hip_stream))
        self._check(lib().epi_count(self.h, _ptr(ids), ids.size, int(mode), int(sched), st))

    def epi_set_option(self, option: int, value: int):
        self._check(lib().epi_set_option(self.h, int(option), int(value)))

    def epi_sync(self):
        self._check(lib().epi_sync(self.h))

    def epi_read_counts(self, set_id: int, m: int) -> np.ndarray:
        out = np.zeros(int(m), np.int32)
        self._check(lib().epi_read_counts(self.h, int(set_id), _ptr(out), int(m)))
        return out

    def epi_counts_device(self, set_id: int) -> int:
        p = P()
        self._check(lib().epi_counts_device(self.h, int(set_id), ctypes.byref(p)))
        return p.value or 0

    def epi_count_noalloc(self, set_id: int, segments: int = 0, hip_stream=None):
        st = None if hip_stream is None else P(int(hip_stream))
        self._check(lib().epi_count_noalloc(self.h, int(set_id), int(segments), st))

    def epi_batched_stats(self) -> dict:
        """Plans built, replays of kept plans and plans kept by this context."""
        b, r, k = I64(), I64(), I64()
        self._check(lib().epi_batched_stats(self.h, ctypes.byref(b), ctypes.byref(r), ctypes.byref(k)))
        return {"built": b.value, "replays": r.value, "kept": k.value}

    def epi_read_schedule(self, set_id: int, m: int):
        """(order, block): submission index and lane block of every lane slot
        of the set's last batched count."""
        order = np.zeros(int(m), np.int32)
        block = np.zeros(int(m), np.int32)
        self._check(lib().epi_read_schedule(self.h, int(set_id), _ptr(order), _ptr(block), int(m)))
        return order, block

    # level-wise discovery ------------------------------------------------------
    def epi_mine(self, sid: int, menu, max_size: int, threshold: int, hip_stream=None) -> int:
        """menu: sequence of (lo, hi) intervals."""
        lo = np.ascontiguousarray([a for a, _ in menu], np.int64)
        hi = np.ascontiguousarray([b for _, b in menu], np.int64)
        out = I32()
        st = None if hip_stream is None else P(int(hip_stream))
        self._check(lib().epi_mine(self.h, int(sid), lo.size, _ptr(lo), _ptr(hi), int(max_size), int(threshold),
                                   st, ctypes.byref(out)))
        return out.value

    def epi_mine_levels(self, mid: int) -> int:
        n = I32()
        self._check(lib().epi_mine_levels(self.h, int(mid), ctypes.byref(n)))
        return n.value

    def epi_mine_level_info(self, mid: int, level: int):
        """(n_candidates, n_frequent, (gen_ms, count_ms, kernel_ms))."""
        m, f = I64(), I64()
        t = np.zeros(3, np.float64)
        self._check(lib().epi_mine_level_info(self.h, int(mid), int(level), ctypes.byref(m), ctypes.byref(f),
                                              _ptr(t)))
        return m.value, f.value, tuple(float(x) for x in t)

    def epi_mine_read(self, mid: int, level: int, frequent_only: bool = False):
        """Candidate dict (N, types, lo, hi) plus int32 counts."""
        m, f, _ = self.epi_mine_level_info(mid, level)
        k = f if frequent_only else m
        c = dict(N=np.zeros(k, np.uint8), types=np.zeros((k, 8), np.int32), lo=np.zeros((k, 7), np.int64),
                 hi=np.zeros((k, 7), np.int64))
        counts = np.zeros(k, np.int32)
        self._check(lib().epi_mine_read(self.h, int(mid), int(level), int(bool(frequent_only)), k, _ptr(c["N"]),
                                        _ptr(c["types"]), _ptr(c["lo"]), _ptr(c["hi"]), _ptr(counts)))
        return c, counts

    def epi_mine_read_at(self, mid: int, level: int, idx):
        idx = np.ascontiguousarray(idx, np.int64)
        k = idx.size
        c = dict(N=np.zeros(k, np.uint8), types=np.zeros((k, 8), np.int32), lo=np.zeros((k, 7), np.int64),
                 hi=np.zeros((k, 7), np.int64))
        counts = np.zeros(k, np.int32)
        self._check(lib().epi_mine_read_at(self.h, int(mid), int(level), k, _ptr(idx), _ptr(c["N"]),
                                           _ptr(c["types"]), _ptr(c["lo"]), _ptr(c["hi"]), _ptr(counts)))
        return c, counts

    def epi_mine_level_bytes(self, mid: int, level: int) -> int:
        v = I64()
        self._check(lib().epi_mine_level_bytes(self.h, int(mid), int(level), ctypes.byref(v)))
        return v.value

    def epi_mine_release(self, mid: int):
        self._check(lib().epi_mine_release(self.h, int(mid)))

    # cost model ---------------------------------------------------------------
    def epi_mlp_init(self, n_features: int, seed: int):
        self._check(lib().epi_mlp_init(self.h, int(n_features), int(seed)))

    def epi_mlp_params(self):
        f, n = I32(), I64()
        self._check(lib().epi_mlp_params(self.h, ctypes.byref(f), ctypes.byref(n)))
        return f.value, n.value

    def epi_mlp_get_params(self) -> np.ndarray:
        _, n = self.epi_mlp_params()
        p = np.zeros(n, np.float32)
        self._check(lib().epi_mlp_get_params(self.h, _ptr(p), n))
        return p

    def epi_mlp_set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        self._check(lib().epi_mlp_set_params(self.h, _ptr(p), p.size))

    def epi_mlp_forward(self, X) -> np.ndarray:
        X = np.ascontiguousarray(X, np.float32)
        y = np.zeros(X.shape[0], np.float32)
        self._check(lib().epi_mlp_forward(self.h, _ptr(X), X.shape[0], _ptr(y)))
        return y

    def epi_mlp_grad(self, X, t):
        X = np.ascontiguousarray(X, np.float32)
        t = np.ascontiguousarray(t, np.float32)
        _, n = self.epi_mlp_params()
        g = np.zeros(n, np.float32)
        L = ctypes.c_float()
        self._check(lib().epi_mlp_grad(self.h, _ptr(X), _ptr(t), X.shape[0], ctypes.byref(L), _ptr(g)))
        return float(L.value), g

    def epi_mlp_adam_step(self, g, lr: float):
        g = np.ascontiguousarray(g, np.float32)
        self._check(lib().epi_mlp_adam_step(self.h, _ptr(g), float(lr)))

    def epi_mlp_train(self, X, t, epochs: int, batch: int, lr: float) -> np.ndarray:
        X = np.ascontiguousarray(X, np.float32)
        t = np.ascontiguousarray(t, np.float32)
        losses = np.zeros(int(epochs), np.float32)
        self._check(lib().epi_mlp_train(self.h, _ptr(X), _ptr(t), X.shape[0], int(epochs), int(batch), float(lr),
                                        _ptr(losses)))
        return losses

    def epi_costmodel_features(self, set_id: int, m: int) -> np.ndarray:
        X = np.zeros((int(m), 24), np.float32)
        self._check(lib().epi_costmodel_features(self.h, int(set_id), _ptr(X), int(m)))
        return X

    # work log -------------------------------------------------------------------
    def epi_read_worklog(self, set_id: int, m: int) -> np.ndarray:
        w = np.zeros((int(m), 5), np.int32)
        self._check(lib().epi_read_worklog(self.h, int(set_id), _ptr(w), int(m)))
        return w

    def epi_read_item_cycles(self, set_id: int) -> np.ndarray:
        n = I64()
        self._check(lib().epi_read_item_cycles(self.h, int(set_id), None, 0, ctypes.byref(n)))
        c = np.zeros((n.value, 2), np.int64)
        if n.value:
            self._check(lib().epi_read_item_cycles(self.h, int(set_id), _ptr(c), n.value, ctypes.byref(n)))
        return c

    def epi_costmodel_train(self, set_ids, epochs: int, seed: int) -> np.ndarray:
        ids = np.ascontiguousarray(np.atleast_1d(np.asarray(set_ids, np.int32)))
        losses = np.zeros(int(epochs), np.float32)
        self._check(lib().epi_costmodel_train(self.h, _ptr(ids), ids.size, int(epochs), int(seed), _ptr(losses)))
        return losses

    def epi_costmodel_scaling(self):
        """Returns (x_mu[F], x_isd[F], y_mu, y_sd)."""
        F, _ = self.epi_mlp_params()
        mu = np.zeros(F, np.float32)
        isd = np.zeros(F, np.float32)
        y = np.zeros(2, np.float32)
        self._check(lib().epi_costmodel_scaling(self.h, _ptr(mu), _ptr(isd), _ptr(y)))
        return mu, isd, float(y[0]), float(y[1])

    def epi_costmodel_predict(self, set_id: int, m: int) -> np.ndarray:
        y = np.zeros(int(m), np.float32)
        self._check(lib().epi_costmodel_predict(self.h, int(set_id), _ptr(y), int(m)))
        return y

    def epi_costmodel_save(self, path):
        self._check(lib().epi_costmodel_save(self.h, str(path).encode()))

    def epi_costmodel_load(self, path):
        self._check(lib().epi_costmodel_load(self.h, str(path).encode()))

    def epi_autotune(self, set_ids, sched: int = EPI_SCHED_RR, cache_path=None):
        """Returns (tile size, ring classes, lanes, segment target)."""
        ids = np.ascontiguousarray(np.atleast_1d(np.asarray(set_ids, np.int32)))
        out = np.zeros(4, np.int64)
        cp = None if cache_path is None else str(cache_path).encode()
        self._check(lib().epi_autotune(self.h, _ptr(ids), ids.size, int(sched), cp, _ptr(out)))
        return tuple(int(x) for x in out)
