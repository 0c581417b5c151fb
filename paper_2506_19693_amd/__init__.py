"""MI355X-native (gfx950) RNS-CKKS hot path of ReBoot's encrypted MLP training.

The arithmetic lives in librbk.so (HIP kernels behind the C ABI of
include/rbk.h); ``rbk`` is its ctypes binding.
"""
from . import rbk  # noqa: F401
from .rbk import Context, Graph, Mlp, RbkError, Server, load, to_device, to_host  # noqa: F401

__all__ = ["rbk", "Context", "Graph", "Mlp", "RbkError", "Server", "load", "to_device", "to_host"]
