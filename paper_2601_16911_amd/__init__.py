"""Cell-vertex WENO stabilised residual on AMD Instinct MI355X (gfx950).

The compute path is the HIP library libcvw.so (C ABI in include/cvw.h);
`paper_2601_16911_amd.cvw` is its ctypes binding and
`paper_2601_16911_amd.build` compiles it.
"""
from . import cvw  # noqa: F401

__all__ = ["cvw"]
