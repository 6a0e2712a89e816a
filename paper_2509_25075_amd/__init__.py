"""MI355X-native batched state-vector simulation of parameterised circuits.

The computation lives in libqs.so (HIP for gfx950, C ABI in include/qs.h);
``_native`` binds it with ctypes and ``sim`` wraps it for torch device
tensors (``from paper_2509_25075_amd import sim``). There is no CPU
fallback: every call fails loudly when the library or the GPU is missing.
"""

from . import _native  # noqa: F401

__all__ = ["_native", "sim"]
