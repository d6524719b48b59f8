"""CPU oracle for the filtered fast direct solver (2D TE-EFIE / TE-MFIE).

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, FP64 NumPy/SciPy
implementation of what the GPU path computes. Only the tests, the smoke check
and the bench's CPU-baseline leg may import it; the product path never does.
It shares no code with the HIP library: Bessel functions come from
scipy.special, linear algebra from SciPy's LAPACK.

Module map (each function cites the passage of the paper it follows):
  special      Green's function g = (i/4) H0^(1)(kR) and its normal derivative
  geometry     straight-panel mesh of a closed curve, P1 hat basis
  quadrature   Gauss-Legendre rules, self/adjacent-panel singular integrals
  assembly     Galerkin S, N (Maue form), D; Gram G; Laplacian L; RHS moments
  formulation  normalised Calderon TE-EFIE, TE-MFIE, TE-CFIE; compact parts
  filters      Laplacian filter P = V_n V_n^T from the orthonormalised Laplacian
  rng          counter-based sketch matrix (splitmix64)
  compress     randomised range finder / subspace iteration, truncation
  woodbury     Woodbury factor and solve, iterative refinement
  solver       end-to-end pipeline and the exact references y_fil, y_full

Parity status: every function here is pinned by a CPU test in tests/ (closed
forms on the circle, Calderon identity, Gauss's lemma, brute-force mpmath
integrals, dense LU), except where a module header says "parity unpinned".
"""
from . import special, geometry, quadrature, assembly, formulation, filters, rng
from . import compress, woodbury, solver

__all__ = ["special", "geometry", "quadrature", "assembly", "formulation",
           "filters", "rng", "compress", "woodbury", "solver"]
