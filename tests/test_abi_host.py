"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and the host-only validators return each documented code."""
import ctypes
import os
import re

import numpy as np
import pytest

import spikegen as sg
from paper_0905_2203_amd import epi

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "epi.h")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(epi_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = epi.lib()
    decl = declared_symbols()
    assert len(decl) >= 15
    for name in decl:
        assert hasattr(L, name), f"{name} declared in epi.h but not exported"
    assert set(epi.EXPORTS) == set(decl)


def test_status_strings():
    for code, name in [(0, "EPI_OK"), (-2, "EPI_EUNSORTED"), (-7, "EPI_EOVERFLOW"), (-10, "EPI_ESTATE")]:
        assert epi.status_string(code) == name


def _stream():
    return sg.config_stream(1, scale=0.1)


def test_validate_stream_codes():
    s = _stream()
    assert epi.epi_validate_stream(s["types"], s["times"], 32) == epi.EPI_OK
    t = s["times"].copy()
    t[10] = t[9] - 1
    assert epi.epi_validate_stream(s["types"], t, 32) == epi.EPI_EUNSORTED
    ty = s["types"].copy()
    ty[3] = 32
    assert epi.epi_validate_stream(ty, s["times"], 32) == epi.EPI_ETYPE
    ty[3] = -1
    assert epi.epi_validate_stream(ty, s["times"], 32) == epi.EPI_ETYPE
    t = s["times"].copy()
    t[-1] = np.iinfo(np.int32).max
    assert epi.epi_validate_stream(s["types"], t, 32) == epi.EPI_EOVERFLOW
    assert epi.epi_validate_stream(s["types"], s["times"], 0) == epi.EPI_ESIZE
    assert epi.epi_validate_stream(s["types"], s["times"], 5000) == epi.EPI_ESIZE
    # empty stream is valid
    assert epi.epi_validate_stream(np.zeros(0, np.int32), np.zeros(0, np.int64), 4) == epi.EPI_OK
    # int64 times
    assert epi.epi_validate_stream(s["types"], s["times"].astype(np.int64), 32) == epi.EPI_OK


def test_validate_stream_null_and_kind():
    L = epi.lib()
    assert L.epi_validate_stream(None, None, 5, 0, 4) == epi.EPI_EINVAL
    ty = np.zeros(3, np.int32)
    tm = np.zeros(3, np.int32)
    assert L.epi_validate_stream(ty.ctypes.data_as(ctypes.c_void_p), tm.ctypes.data_as(ctypes.c_void_p),
                                 3, 7, 4) == epi.EPI_EINVAL


def _one(ep, lo, hi):
    return sg.candidates_from_list([(ep, lo, hi)])


@pytest.mark.parametrize("case,code", [
    (([0, 1], [0], [5]), epi.EPI_OK),
    (([0], [], []), epi.EPI_OK),
    (([0, 1, 2, 3, 4, 5, 6, 7], [0] * 7, [5] * 7), epi.EPI_OK),
    (([0, 40], [0], [5]), epi.EPI_ETYPE),
    (([0, -1], [0], [5]), epi.EPI_ETYPE),
    (([0, 0], [0], [5]), epi.EPI_EREPEAT),
    (([0, 1, 0], [0, 0], [5, 5]), epi.EPI_EREPEAT),
    (([0, 1], [5], [5]), epi.EPI_EINTERVAL),
    (([0, 1], [-1], [5]), epi.EPI_EINTERVAL),
    (([0, 1], [6], [5]), epi.EPI_EINTERVAL),
])
def test_validate_candidate_codes(case, code):
    assert epi.epi_validate_candidates(_one(*case), 32, epi.EPI_TS_I32) == code


def test_validate_candidate_size_and_overflow():
    c = _one([0, 1], [0], [5])
    c["N"][0] = 9
    assert epi.epi_validate_candidates(c, 32, 0) == epi.EPI_ESIZE
    c["N"][0] = 0
    assert epi.epi_validate_candidates(c, 32, 0) == epi.EPI_ESIZE
    big = _one([0, 1, 2], [0, 0], [2**30, 2**30])
    assert epi.epi_validate_candidates(big, 32, epi.EPI_TS_I32) == epi.EPI_EOVERFLOW
    assert epi.epi_validate_candidates(big, 32, epi.EPI_TS_I64) == epi.EPI_OK
    # empty set is valid
    assert epi.epi_validate_candidates(sg.empty_candidates(0), 32, 0) == epi.EPI_OK


def test_validate_accepts_every_legal_interval():
    # Sec. II-C admits any 0 <= lo < hi: a narrow interval far from its node,
    # 1 + hi/(hi-lo+1) = 1 + 100/2 = 51 live acceptance intervals, is legal
    # (the state machines leave such episodes to the per-event tracking engine)
    assert epi.epi_validate_candidates(_one([0, 1], [99], [100]), 32, 0) == epi.EPI_OK
    assert epi.epi_validate_candidates(_one([0, 1], [95_000_000], [100_000_000]), 32, 1) == epi.EPI_OK
    assert epi.epi_validate_candidates(_one([0, 1], [20_000_000], [25_000_000]), 32, 1) == epi.EPI_OK
    # still refused: lo < 0, lo >= hi
    assert epi.epi_validate_candidates(_one([0, 1], [-1], [5]), 32, 0) == epi.EPI_EINTERVAL
    assert epi.epi_validate_candidates(_one([0, 1], [5], [5]), 32, 0) == epi.EPI_EINTERVAL


def test_generated_workloads_validate():
    for k in (1, 4, 5):
        s = sg.config_stream(k, scale=0.01)
        assert epi.epi_validate_stream(s["types"], s["times"], s["K"]) == epi.EPI_OK
        c = sg.config_candidates(k, s, scale=0.01)
        assert epi.epi_validate_candidates(c, s["K"], s["ts_kind"]) == epi.EPI_OK


def test_context_without_gpu_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(epi.EpiError) as ei:
        epi.Context(0)
    assert ei.value.code == epi.EPI_EDEVICE


def test_binding_constants_match_the_header():
    """Every mode, option, schedule, timestamp-kind and status constant the
    header declares has the same value in the binding."""
    from paper_0905_2203_amd import epi as binding

    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "epi.h")).read()
    consts = dict((k, int(v)) for k, v in re.findall(r"\b(EPI_[A-Z0-9_]+)\s*=\s*(-?\d+)", hdr))
    assert any(k.startswith("EPI_OPT_") for k in consts) and "EPI_MODE_TRACKING" in consts
    missing = [k for k in consts if not hasattr(binding, k)]
    assert not missing, missing
    wrong = {k: (v, getattr(binding, k)) for k, v in consts.items() if getattr(binding, k) != v}
    assert not wrong, wrong
