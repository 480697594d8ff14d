"""MI355X (gfx950) library for the hot path of averaged recurrence
quantification analysis (Panis, Adamek & Marwan, arXiv 2208.09136).

The compute lives in librqa.so (HIP kernels behind the C ABI of
include/rqa.h); ``rqa`` is its ctypes binding.
"""
from . import rqa  # noqa: F401
from .rqa import Context, RqaError, rqa_params  # noqa: F401
