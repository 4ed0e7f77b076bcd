"""MI355X-native learned digital backpropagation (Haeger & Pfister, arXiv 2010.14258).

The compute path lives in the gfx950 HIP library ``libldbp.so`` (C ABI in
``include/ldbp.h``); this package is its Python binding.
"""
from . import _native  # noqa: F401
from .ldbp import (LDBPFunction, ldbp_backward, ldbp_backward_workspace_size, ldbp_forward,  # noqa: F401
                   ldbp_forward_workspace_size)

__all__ = ["ldbp_forward", "ldbp_forward_workspace_size", "ldbp_backward", "ldbp_backward_workspace_size",
           "LDBPFunction"]
