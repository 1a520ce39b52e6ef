"""MI355X (gfx950) sparse approximate map construction.

Builds the sparse approximate map N_k = argmin ||A_k N - A_0||_F over a
sparsity pattern (Islam, Carr and Jacobs, Section 2) with hand-written HIP
kernels behind the C ABI of include/sam.h; this package is its Python
binding over torch device tensors.
"""
from .sam import Context, DeviceCSC, Plan, SamError, Sequence  # noqa: F401
from . import _capi  # noqa: F401

__all__ = ["Context", "DeviceCSC", "Plan", "SamError", "Sequence"]
