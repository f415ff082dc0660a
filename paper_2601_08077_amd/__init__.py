"""MI355X (gfx950) density-fitting J/K build with INT8-sliced FP64 emulation.

The compute path lives in ``libdfjk.so`` (hand-written HIP kernels behind the
C ABI of ``include/dfjk.h``); ``binding`` exposes the same entry points to
Python through ctypes, with torch supplying device memory and streams.
"""
from .binding import (DF_DENSE, DF_PACKED, DF_EHIP, DF_EINVAL, DF_ENONFINITE, DF_ENOTSPD, DF_EOVERFLOW_GUARD,
                      DF_EWORKSPACE, DF_OK, Context, DFError, load)

__all__ = ["Context", "DFError", "load", "DF_DENSE", "DF_PACKED", "DF_OK", "DF_EINVAL", "DF_EWORKSPACE",
           "DF_EHIP", "DF_ENONFINITE", "DF_ENOTSPD", "DF_EOVERFLOW_GUARD"]
