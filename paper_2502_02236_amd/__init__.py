"""MI355X-native sLLG Heun step of atomistic spin dynamics (arXiv 2502.02236).

The compute path lives in libasd.so (hand-written HIP kernels for gfx950 and a
C ABI declared in include/asd.h); ``asd`` is its ctypes binding and
``bridge`` turns the workload definitions into library descriptors.
"""
from . import asd  # noqa: F401
