"""MI355X-native mixed-time-slicing PIMD hot path (arXiv 2411.11988).

The compute lives in ``_lib/libmixpi.so`` (HIP kernels for gfx950 behind the
C-ABI of ``include/mixpi.h``); ``mixpi`` is its ctypes binding.
"""
from . import mixpi  # noqa: F401
