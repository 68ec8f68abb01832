"""MI355X-native P1-tetrahedron incompressible Navier-Stokes element assembly.

The compute path is hand-written HIP for gfx950 behind the C-ABI library ``libnsa.so``
(``include/nsa.h``); ``paper_2111_05651_amd.nsa`` is the thin ctypes binding to it.
Importing the package itself loads nothing; the library is loaded on first use and the
binding raises if it is missing (there is no CPU fallback).
"""
__all__ = ["inputs", "nsa"]
