"""CPU oracle for P1-tet incompressible Navier-Stokes assembly (plain FP64, serial).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the package smoke check and by the
benchmark's CPU-baseline leg. The product path never imports it.

The arithmetic lives in ``nsa_oracle.c`` (plain C, built with ``-O2 -ffp-contract=off``);
this module only compiles it and marshals NumPy arrays through ctypes.
"""
from .oracle import (build, load, load_omp, flops, element, element_integrals, validate, pattern, assemble,
                     assemble_rows, residual, OR_OK, OR_EINVAL, OR_ERANGE, OR_EDEGENERATE, OR_ENOMEM)

__all__ = ["build", "load", "load_omp", "flops", "element", "element_integrals", "validate", "pattern", "assemble",
           "assemble_rows", "residual", "OR_OK", "OR_EINVAL", "OR_ERANGE", "OR_EDEGENERATE", "OR_ENOMEM"]
