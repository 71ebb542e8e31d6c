"""MI355X-native tiled 2D3V electromagnetic PIC hot path.

The compute lives in ``libpic.so`` (HIP kernels for gfx950 behind the C ABI
declared in ``include/pic.h``); this package is a thin ctypes binding
(``_lib``) plus a convenience wrapper that owns torch device buffers
(``Sim``).  Nothing here computes any step of the method on the CPU.
"""
from . import _lib
from ._lib import PicError
from .sim import Batch, BatchMember, Sim, pack_cells, unpack_cells

__all__ = ["Sim", "Batch", "BatchMember", "PicError", "pack_cells", "unpack_cells", "_lib"]
