"""MI355X-native discrete flow mapping on tetrahedral meshes.

The computation lives in libdfm.so (hand-written HIP for gfx950 behind the C
ABI of include/dfm.h); ``dfm`` is its thin PyTorch-facing binding.
"""
from . import _lib  # noqa: F401

__all__ = ["dfm", "build"]
