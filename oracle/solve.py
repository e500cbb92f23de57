"""Plain conjugate gradients (test infrastructure; oracle only).

Unpreconditioned CG on a symmetric positive definite operator, used by the
manufactured-solution checks and as the reference iteration count for the
library's solver.
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
