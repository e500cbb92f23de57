"""Plain FP64 CPU oracle for the sum-factorized interior-penalty DG operator.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import this package:
only the tests, the smoke check and the CPU-baseline leg of the benchmark use it.

What it computes, and where the paper defines it:

* Gauss-Legendre rules and the nodal Lagrange basis on [0, 1]
  (tensor-product quadrature and 1D basis matrices, Section 2.1/2.2).
* Hexahedral cells as images of the reference cube under a trilinear map
  (Section 2.1).
* Element, interior-face and boundary-face matrices of the SIPG
  diffusion-reaction form (Section 5.2, eq. diffreac_weak) and of the DG Stokes
  form (Section 5.3, eq. stokes_weak), each by full tensor quadrature: every
  3D basis function is evaluated as a product of 1D factors at every
  quadrature point; there is no sum factorization anywhere in this package.
* A block-sparse global matrix (one block row per element, at most seven
  blocks) and its products with vectors, y = A x and y = A^T x; the
  operator apply is the Jacobian action of Section 2.1, which for the linear
  problems here is A x.
* The derivative of L = g^T A(kappa) u with respect to a diffusion coefficient
  given per volume quadrature point.
* Load vectors, plain conjugate gradients and L2 errors for the
  manufactured-solution checks; the element block-Jacobi preconditioner
  (dense solves with each cell's diagonal block) and preconditioned CG.

Every routine here is pinned by the CPU tests (tests/test_oracle_*.py) to
things other than itself: library quadrature rules, closed forms, symbolic
brute force on tiny meshes, exactness on polynomials, manufactured-solution
convergence and finite differences.
"""

from .gauss import gauss_legendre
from .lagrange import lagrange_eval, lagrange_deriv
from .mesh import HexMesh
from .problem import Problem, problem_from_workload
from .blocks import BlockMatrix
from .scalar import ScalarDG
from .stokes import StokesDG
from .solve import cg, pcg, block_jacobi

__all__ = [
    "gauss_legendre", "lagrange_eval", "lagrange_deriv", "HexMesh", "Problem",
    "BlockMatrix", "ScalarDG", "StokesDG", "cg", "problem_from_workload",
]
