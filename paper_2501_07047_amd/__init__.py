"""CROSS on MI355X: BAT/MAT int8-MFMA NTT and CKKS modular matrix products.

The compute lives in ``libcross.so`` (HIP kernels for gfx950 behind the C ABI
declared in ``include/cross.h``); ``binding`` marshals torch device tensors
into it.
"""
from . import binding  # noqa: F401
from .binding import CrossError  # noqa: F401
