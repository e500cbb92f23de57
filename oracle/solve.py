"""Plain conjugate gradients and the block-Jacobi preconditioner (test
infrastructure; oracle only).

CG on a symmetric positive definite operator, used by the manufactured-solution
checks and as the reference iteration count for the library's solver; the
element block-Jacobi preconditioner (one of the matrix-free preconditioners
the paper's introduction, Section 1, points to) as the inverse of each
cell's diagonal block, by dense solves; and preconditioned CG.
"""
from __future__ import annotations

import numpy as np


def cg(apply, b: np.ndarray, x0: np.ndarray | None = None, rtol: float = 1e-10, maxit: int = 100000):
    """Solve A x = b; stops when ||b - A x||_2 <= rtol ||b||_2 (recursive residual).
    Returns (x, iterations, true relative residual)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply(x)
    p = r.copy()
    rr = float(r @ r)
    bn = float(np.sqrt(b @ b))
    it = 0
    while it < maxit and np.sqrt(rr) > rtol * bn:
        q = apply(p)
        alpha = rr / float(p @ q)
        x += alpha * p
        r -= alpha * q
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    true_res = float(np.linalg.norm(b - apply(x)) / bn)
    return x, it, true_res


def block_jacobi(A, r: np.ndarray) -> np.ndarray:
    """z with A_ee z_e = r_e for every cell e, A_ee the diagonal block of the
    block-sparse matrix A (block row e, slot 0). Cells whose diagonal blocks
    share one stored class are solved together."""
    N, E = A.bsize, A.nelem
    R = np.asarray(r, dtype=np.float64).reshape(E, N)
    Z = np.empty_like(R)
    if A.blocks is not None:
        for e in range(E):
            Z[e] = np.linalg.solve(A.blocks[e, 0], R[e])
    else:
        cl = A.cls[:, 0]
        for c in np.unique(cl):
            rows = np.nonzero(cl == c)[0]
            Z[rows] = np.linalg.solve(A.classes[c], R[rows].T).T
    return Z.reshape(-1)


def pcg(apply, precond, b: np.ndarray, x0: np.ndarray | None = None, rtol: float = 1e-10, maxit: int = 100000):
    """Preconditioned CG for A x = b with z = precond(r) (SPD): alpha = r.z / p.Ap,
    beta = r_new.z_new / r.z, p = z + beta p. Stops when ||r||_2 <= rtol ||b||_2
    (recursive residual). Returns (x, iterations, true relative residual)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply(x)
    z = precond(r)
    p = z.copy()
    rz = float(r @ z)
    bn = float(np.sqrt(b @ b))
    it = 0
    while it < maxit and np.sqrt(float(r @ r)) > rtol * bn:
        q = apply(p)
        alpha = rz / float(p @ q)
        x += alpha * p
        r -= alpha * q
        z = precond(r)
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    true_res = float(np.linalg.norm(b - apply(x)) / bn)
    return x, it, true_res
