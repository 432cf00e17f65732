"""MI355X-native Dey--Mittra cut-cell cavity eigensolver.

The compute path lives in ``libdm.so`` (HIP kernels for gfx950 behind the C
ABI of ``include/dm.h``); ``dm`` is its ctypes binding.
"""
from . import dm  # noqa: F401
