"""Host-side pieces of bench.py: the algorithmic bytes of the roofline (each
candidate reads the times of its own types' events, its descriptor and
writes its count), checked on a hand-built stream and candidate set."""
import numpy as np

import bench


def test_alg_bytes_by_hand():
    # 3 types with 4, 1 and 2 events
    types = np.array([0, 1, 0, 2, 0, 2, 0], np.int32)
    for ts_kind, tsb, desc in ((1, 8, 128), (0, 4, 72)):
        s = {"types": types, "K": 3, "ts_kind": ts_kind}
        c = {
            "N": np.array([1, 2, 3], np.uint8),
            "types": np.array([[2] + [-1] * 7, [0, 1] + [-1] * 6, [1, 2, 0] + [-1] * 5], np.int32),
        }
        # visits: 2, 4 + 1, 1 + 2 + 4
        want = (2 + 5 + 7) * tsb + 3 * (desc + 4)
        assert bench.alg_bytes(s, c) == want


def test_ablation_legs_are_the_five_modes():
    assert bench.ABL_LEGS == ("plain", "batched_rr", "batched_learned", "batched_heuristic", "batched_measured")
