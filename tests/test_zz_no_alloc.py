"""The allocation-free count (epi_count_noalloc) through the C ABI: the same
counts as epi_count in plain mode with the same segments, on two calls in a
row (the second with a smaller set, so its records lie over the first call's
in the shared static scratch), and the size limit of that scratch."""
import numpy as np
import pytest

import oracle
import spikegen as sg
from paper_0905_2203_amd import epi

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-noalloc] {msg}", flush=True)


def test_noalloc_equals_plain_count():
    s = sg.config_stream(4, scale=0.01)
    big = sg.config_candidates(4, s, scale=0.04)
    small = sg.take_candidates(big, np.arange(0, 300))
    with epi.Context(0) as ctx:
        sid = ctx.epi_load_stream(s["types"], s["times"], s["K"])
        try:
            for segments in (7, 0):
                for name, c in (("big", big), ("small", small)):
                    m = c["N"].size
                    cid = ctx.epi_submit_candidates(sid, c)
                    try:
                        say(f"segments={segments} {name}: {m} episodes")
                        ctx.epi_count_noalloc(cid, segments)
                        ctx.epi_sync()
                        got = ctx.epi_read_counts(cid, m)
                        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, segments)
                        ctx.epi_count([cid], mode=epi.EPI_MODE_PLAIN)
                        ref = ctx.epi_read_counts(cid, m)
                        assert np.array_equal(got, ref)
                        assert np.array_equal(got, oracle.count(s, c))
                    finally:
                        ctx.epi_set_option(epi.EPI_OPT_SEGMENTS, 0)
                        ctx.epi_release_set(cid)
        finally:
            ctx.epi_release_stream(sid)


def test_noalloc_rejects_records_beyond_scratch():
    s = sg.config_stream(4, scale=0.01)
    c = sg.random_candidates(sg.rng_for(4, offset=77), 30000, 128, 2, 2, 1_000_000)
    with epi.Context(0) as ctx:
        sid = ctx.epi_load_stream(s["types"], s["times"], s["K"])
        cid = ctx.epi_submit_candidates(sid, c)
        try:
            with pytest.raises(epi.EpiError) as ei:
                ctx.epi_count_noalloc(cid, 100000)
            assert ei.value.code == epi.EPI_ESIZE
            ctx.epi_count_noalloc(cid, 2)
            ctx.epi_sync()
            assert np.array_equal(ctx.epi_read_counts(cid, c["N"].size)[:200],
                                  oracle.count(s, sg.take_candidates(c, np.arange(200))))
        finally:
            ctx.epi_release_set(cid)
            ctx.epi_release_stream(sid)
