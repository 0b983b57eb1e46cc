"""CPU FP64 oracle for the matrix-free Q2 operators and their Krylov solvers.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only code allowed to import this package.  It shares
no code with the GPU library (``paper_2501_18781_amd``), and neither imports
the other.

Contents
--------
* ``mf_oracle.c`` (built into ``liboracle.so``): reference element, explicit
  per-cell matrices by full Gauss quadrature, CSR assembly, SpMV, spot rows,
  quadrature-point fields, adjoint gradient formulas, Q2 prolongation.
* ``reference.py``: Python wrappers and the Krylov / multigrid algorithms
  (CG, GMRES(m), Chebyshev smoothing, V-cycle, flexible CG, Lanczos), written
  out from their textbook definitions in numpy.
"""
from .reference import *  # noqa: F401,F403
