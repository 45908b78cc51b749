"""Lock-free push-relabel for MI355X (gfx950): grid max-flow / min-cut and
dense assignment by cost scaling, behind the C ABI of ``include/lpr.h``.

``paper_1110_6231_amd.lpr`` is the ctypes binding; importing this package does
not load the HIP library (that happens on the first call).
"""
from . import lpr  # noqa: F401

__all__ = ["lpr"]
