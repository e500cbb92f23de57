"""Gauss-Legendre quadrature on [0, 1] (test infrastructure; oracle only).

The paper builds its cell rules as tensor products of 1D rules of maximal
order with m_i points per direction (Section 2.1). This is that 1D rule,
computed by Newton's method on the Legendre polynomial P_m, which is evaluated
with its three-term recurrence, in extended precision.
"""
from __future__ import annotations

import numpy as np


def _legendre_and_derivative(m: int, t: np.ndarray):
    """P_m(t) and P_m'(t) by the recurrence n P_n = (2n-1) t P_{n-1} - (n-1) P_{n-2}."""
    p_prev = np.ones_like(t)
    p = t.copy()
    for n in range(2, m + 1):
        p_prev, p = p, ((2 * n - 1) * t * p - (n - 1) * p_prev) / n
    # (1 - t^2) P_m'(t) = m (P_{m-1}(t) - t P_m(t))
    dp = m * (p_prev - t * p) / (1.0 - t * t)
    return p, dp


def gauss_legendre(m: int):
    """Nodes (ascending) and weights of the m-point Gauss-Legendre rule on [0, 1]."""
    if m < 1:
        raise ValueError("m must be >= 1")
    if m == 1:
        return np.array([0.5]), np.array([1.0])
    ld = np.longdouble
    i = np.arange(m, dtype=ld)
    t = np.cos(np.pi * (i + ld(0.75)) / (ld(m) + ld(0.5)))  # initial guesses on [-1, 1]
    for _ in range(100):
        p, dp = _legendre_and_derivative(m, t)
        step = p / dp
        t = t - step
        if np.max(np.abs(step)) < 8 * np.finfo(ld).eps:
            break
    p, dp = _legendre_and_derivative(m, t)
    w = ld(2) / ((ld(1) - t * t) * dp * dp)
    order = np.argsort(t)
    t, w = t[order], w[order]
    x = (ld(1) + t) / ld(2)
    return x.astype(np.float64), (w / ld(2)).astype(np.float64)
