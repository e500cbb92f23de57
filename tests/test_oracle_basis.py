"""Pins of the oracle's 1D building blocks: Gauss-Legendre rules and the nodal
Lagrange basis (Section 2.1/2.2: tensor quadrature of maximal order and the
1D basis matrices A, D)."""
import math

import numpy as np
import pytest

from oracle import gauss_legendre, lagrange_eval, lagrange_deriv


@pytest.mark.parametrize("m", range(1, 11))
def test_gauss_matches_numpy_leggauss(m):
    x, w = gauss_legendre(m)
    t, wt = np.polynomial.legendre.leggauss(m)
    assert np.max(np.abs(x - (t + 1) / 2)) < 1e-15  # numpy's own rule is good to a few ulps
    assert np.max(np.abs(w - wt / 2)) < 1e-15


@pytest.mark.parametrize("m", range(1, 11))
def test_gauss_exact_up_to_degree_2m_minus_1(m):
    x, w = gauss_legendre(m)
    for a in range(2 * m):
        assert abs(np.sum(w * x ** a) - 1.0 / (a + 1)) < 1e-15
    # degree 2m: the textbook error (m!)^4 / ((2m+1) ((2m)!)^2) of the m-point rule on [0,1]
    err = 1.0 / (2 * m + 1) - np.sum(w * x ** (2 * m))
    ref = math.factorial(m) ** 4 / ((2 * m + 1) * math.factorial(2 * m) ** 2)
    assert abs(err - ref) < 1e-14 + 1e-9 * ref


@pytest.mark.parametrize("p", range(1, 9))
def test_lagrange_kronecker_delta_and_partition_of_unity(p):
    nodes, _ = gauss_legendre(p)
    L = lagrange_eval(nodes, nodes)
    assert np.array_equal(L, np.eye(p)) or np.max(np.abs(L - np.eye(p))) < 1e-15
    t = np.linspace(-0.2, 1.2, 37)
    assert np.max(np.abs(lagrange_eval(nodes, t).sum(axis=1) - 1.0)) < 1e-12
    assert np.max(np.abs(lagrange_deriv(nodes, t).sum(axis=1))) < 1e-10


@pytest.mark.parametrize("p", range(2, 9))
def test_lagrange_derivative_exact_on_polynomials(p):
    """D reproduces derivatives of every polynomial of degree <= k = p-1."""
    nodes, _ = gauss_legendre(p)
    t = np.array([0.0, 0.13, 0.5, 0.77, 1.0])
    D = lagrange_deriv(nodes, t)
    A = lagrange_eval(nodes, t)
    for a in range(p):
        vals = nodes ** a
        assert np.max(np.abs(A @ vals - t ** a)) < 1e-12
        ref = a * t ** (a - 1) if a > 0 else np.zeros_like(t)
        assert np.max(np.abs(D @ vals - ref)) < 1e-10 * max(1, a * a)


def test_collocation_matrix_is_identity_bitwise():
    """With m = p the interpolation matrix A of Section 2.2 is the identity."""
    for p in range(1, 9):
        nodes, _ = gauss_legendre(p)
        assert np.array_equal(lagrange_eval(nodes, nodes), np.eye(p))


def test_lagrange_derivative_matches_finite_difference():
    nodes, _ = gauss_legendre(5)
    t = np.array([0.2, 0.61])
    h = 1e-6
    fd = (lagrange_eval(nodes, t + h) - lagrange_eval(nodes, t - h)) / (2 * h)
    assert np.max(np.abs(fd - lagrange_deriv(nodes, t))) < 1e-7
