"""MI355X (gfx950) renewal tau-leap SEIR step of FlashSpread (arXiv 2604.22092).

The step runs in hand-written HIP kernels inside ``libflashspread.so``; this
package is the thin Python binding of its C ABI (``include/fs.h``).  Importing
the package does not load the library; the first call does, and raises if it
is not built.

With PyTorch in the same process, import torch before the library's first
call: the library then binds PyTorch's HIP runtime.  Loaded the other way
round, PyTorch maps a second runtime of its own, which finds no GPU.
"""
from ._capi import *  # noqa: F401,F403  (the binding's public names)
from ._capi import EXPORTS, FsError, LIB_PATH, lib

__all__ = [n for n in dir() if not n.startswith("_")]
