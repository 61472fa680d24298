"""MI355X (gfx950) engine for exact counting of non-overlapped occurrences of
serial episodes with inter-event constraints (HIP kernels behind a C ABI).

``paper_0905_2203_amd.epi`` is the ctypes binding of ``libepi.so``; the
library must be built (``paper_0905_2203_amd/build.py``) before use.
"""
from . import epi  # noqa: F401

__all__ = ["epi"]
