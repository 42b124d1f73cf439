"""MI355X (gfx950) interior point search-direction library for radiotherapy QPs.

The compute path lives in libqpgpu.so (HIP kernels behind the C ABI of
include/qpgpu.h); ``qpgpu`` is its ctypes binding.
"""
from . import qpgpu  # noqa: F401
