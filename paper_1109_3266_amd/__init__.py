"""MI355X (gfx950) Monte Carlo CT/CBCT imaging-dose transport.

The compute path is libctd.so (HIP kernels behind the C ABI in
include/ctd.h); ``ctd`` is its ctypes binding and ``session`` marshals a
workload description into it.  There is no CPU fallback: using the binding
without the built library raises.
"""
from . import ctd  # noqa: F401

__all__ = ["ctd"]
