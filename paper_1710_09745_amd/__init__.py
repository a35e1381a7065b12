"""Block CG (blockCGrQ) for the even-odd staggered normal operator on MI355X.

The solver is a HIP library for gfx950 behind a C ABI (``include/bcg.h``);
``paper_1710_09745_amd.bcg`` is its ctypes binding.  Importing this package
loads nothing; the library is loaded on first use and its absence is an error.
"""
__all__ = ["synth"]
