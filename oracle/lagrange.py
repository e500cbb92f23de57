"""Nodal Lagrange basis on [0, 1] (test infrastructure; oracle only).

The paper leaves the local basis of P_k open (Section 2.1). Here it is the
Lagrange basis at the k+1 Gauss-Legendre nodes, evaluated pointwise by the
product formula; the 1D basis matrices A and D of Section 2.2 are these
functions and their derivatives at the quadrature points.
"""
from __future__ import annotations

import numpy as np


def lagrange_eval(nodes: np.ndarray, t) -> np.ndarray:
    """Values l_j(t) for all j; returns shape (len(t), len(nodes))."""
    nodes = np.asarray(nodes, dtype=np.float64)
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    n = len(nodes)
    out = np.ones((len(t), n))
    for j in range(n):
        for i in range(n):
            if i != j:
                out[:, j] *= (t - nodes[i]) / (nodes[j] - nodes[i])
    return out


def lagrange_deriv(nodes: np.ndarray, t) -> np.ndarray:
    """Derivatives l_j'(t) by the product rule; returns shape (len(t), len(nodes))."""
    nodes = np.asarray(nodes, dtype=np.float64)
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    n = len(nodes)
    out = np.zeros((len(t), n))
    for j in range(n):
        for k in range(n):
            if k == j:
                continue
            term = np.full(len(t), 1.0 / (nodes[j] - nodes[k]))
            for i in range(n):
                if i != j and i != k:
                    term *= (t - nodes[i]) / (nodes[j] - nodes[i])
            out[:, j] += term
    return out
