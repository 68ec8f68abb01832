"""CPU oracle for incompressible Navier-Stokes element assembly (plain FP64, serial): linear
tetrahedra (nsa_oracle.c) and the 2-D family of bilinear quadrilaterals (nsa_oracle_q1.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the package smoke check and by the
benchmark's CPU-baseline leg. The product path never imports it.

The arithmetic lives in ``nsa_oracle.c`` and ``nsa_oracle_q1.c`` (plain C, built with
``-O2 -ffp-contract=off``); this module only compiles them and marshals NumPy arrays through ctypes.
"""
from .oracle import (build, load, load_omp, flops, element, element_integrals, validate, pattern, assemble,
                     assemble_rows, residual, q1_element, q1_element_integrals, q1_validate, q1_assemble, OR_OK,
                     OR_EINVAL, OR_ERANGE, OR_EDEGENERATE, OR_ENOMEM)

__all__ = ["build", "load", "load_omp", "flops", "element", "element_integrals", "validate", "pattern", "assemble",
           "assemble_rows", "residual", "q1_element", "q1_element_integrals", "q1_validate", "q1_assemble", "OR_OK",
           "OR_EINVAL", "OR_ERANGE", "OR_EDEGENERATE", "OR_ENOMEM"]
