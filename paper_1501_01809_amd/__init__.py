"""MI355X-native cell-loop finite element assembler (HIP, gfx950).

The product path is the C-ABI library ``libfem.so`` (``include/fem.h``);
``paper_1501_01809_amd.fem`` is its thin ctypes binding.  Nothing here falls
back to a CPU implementation.
"""
from . import fem  # noqa: F401

__all__ = ["fem"]
