"""Pins of the oracle's nonlinear diffusion operator (kappa(u) = 1 + u^2):
the residual against exact polynomial integrals of the strong form, its
small-u limit against the pinned linear SIPG operator, and the Jacobian
against exact central differences of the residual."""
import numpy as np
import pytest
from numpy.polynomial import Polynomial

from oracle import Problem, ScalarDG, gauss_legendre
from oracle.nonlinear import NonlinearDG

RNG = np.random.default_rng(7)


def _rand(n):
    return RNG.uniform(-1.0, 1.0, n)


@pytest.mark.parametrize("theta,mask", [(-1.0, 0x3F), (1.0, 0x2B), (-1.0, 0x00)])
def test_small_u_limit_is_the_linear_operator(theta, mask):
    """R is odd in u (kappa is even): R(eps u) = eps A u + eps^3 C(u), so
    (8 R(eps u) - R(2 eps u)) / (6 eps) = A u with A the kappa = 1 SIPG
    operator, exactly up to rounding; and J(0) = A."""
    pr = Problem(2, 2, 1, k=2, theta=theta, mask=mask)
    op = NonlinearDG(pr)
    A = ScalarDG(Problem(2, 2, 1, k=2, theta=theta, mask=mask)).assemble("explicit")
    u = _rand(A.shape[0])
    Au = A.matvec(u)
    eps = 0.05
    lim = (8 * op.residual(eps * u) - op.residual(2 * eps * u)) / (6 * eps)
    assert np.linalg.norm(lim - Au) <= 1e-12 * np.linalg.norm(Au)
    J0 = op.jacobian(np.zeros_like(u))
    assert np.linalg.norm(J0.matvec(u) - Au) <= 1e-13 * np.linalg.norm(Au)


@pytest.mark.parametrize("k,theta,mask,shape", [(2, -1.0, 0x3F, (2, 2, 1)), (2, 1.0, 0x17, (1, 2, 2)),
                                                (3, -1.0, 0x2D, (2, 1, 1)), (1, 1.0, 0x3F, (2, 2, 2))])
def test_jacobian_is_the_derivative_of_the_residual(k, theta, mask, shape):
    """R(u0 + t z) is a cubic polynomial in t, so the central difference
    D(t) = (R(u0 + t z) - R(u0 - t z)) / 2t equals J z + t^2 C exactly and
    (4 D(t) - D(2t)) / 3 = J(u0) z up to rounding."""
    pr = Problem(*shape, k=k, theta=theta, mask=mask, c=1.5)
    op = NonlinearDG(pr)
    n = pr.nelem * (k + 1) ** 3
    u0, z = _rand(n), _rand(n)
    Jz = op.jacobian(u0).matvec(z)

    def D(t):
        return (op.residual(u0 + t * z) - op.residual(u0 - t * z)) / (2 * t)

    t = 1e-2
    fd = (4 * D(t) - D(2 * t)) / 3
    assert np.linalg.norm(fd - Jz) <= 1e-11 * np.linalg.norm(Jz)
    # the Jacobian is not symmetric once u0 varies (the kappa'(u0) z grad u0 terms)
    Jd = op.jacobian(u0)
    M = np.zeros((n, n))
    for j in range(n):
        ej = np.zeros(n)
        ej[j] = 1.0
        M[:, j] = Jd.matvec(ej)
    assert np.abs(M - M.T).max() > 1e-3 * np.abs(M).max()


def _lagrange_polys(nodes):
    out = []
    for j, xj in enumerate(nodes):
        pj = Polynomial([1.0])
        for m, xm in enumerate(nodes):
            if m != j:
                pj = pj * Polynomial([-xm, 1.0]) / (xj - xm)
        out.append(pj)
    return out


def _integral(p):
    q = p.integ()
    return q(1.0) - q(0.0)


@pytest.mark.parametrize("k", [2, 3])
def test_residual_of_a_linear_field_is_its_strong_form(k):
    """u = x is in Q_k and smooth: integrating by parts cell by cell, the
    interior-face and Dirichlet flux terms cancel the boundary terms of the
    volume integral, so R_i(u) = int (-div((1 + u^2) grad u) + c u) phi_i
    + sum over the boundary of int (theta u kappa(u) d_n phi_i + gamma u phi_i),
    with -div((1 + x^2) e_x) = -2x. All integrands are polynomials that the
    rule integrates exactly for k >= 2; the right side is integrated exactly
    here with polynomial arithmetic (no quadrature rule)."""
    n, c, theta, alpha = 2, 1.5, -1.0, 3.0
    pr = Problem(n, n, n, k=k, theta=theta, c=c, alpha=alpha, mask=0x3F)
    op = NonlinearDG(pr)
    p = k + 1
    h = 1.0 / n
    nodes, _ = gauss_legendre(p)
    ell = _lagrange_polys(nodes)
    dell = [l.deriv() for l in ell]
    gamma = alpha * k * (k + 1) / h
    E = n ** 3
    u = np.zeros(E * p ** 3)
    ref = np.zeros(E * p ** 3)
    for e in range(E):
        ex, ey, ez = e % n, (e // n) % n, e // (n * n)
        X = Polynomial([ex * h, h])  # x(xi_0) on this cell
        for i2 in range(p):
            for i1 in range(p):
                for i0 in range(p):
                    i = e * p ** 3 + i0 + p * (i1 + p * i2)
                    u[i] = (ex + nodes[i0]) * h
                    # volume: (c - 2) x phi_i, |J| = h^3
                    v = (_integral((c - 2.0) * X * ell[i0]) * _integral(ell[i1]) * _integral(ell[i2]) * h ** 3)
                    # boundary faces: theta u kappa(u) d_n phi_i + gamma u phi_i, dA = h^2
                    g = X * (1.0 + X * X)  # u kappa(u)
                    if ex == n - 1:  # x = 1, n = +e_x, u = 1
                        val = ell[i0](1.0)
                        dn = dell[i0](1.0) / h
                        v += h * h * _integral(ell[i1]) * _integral(ell[i2]) * (theta * 2.0 * dn + gamma * val)
                    for (idx, lo, hi, other) in ((i1, ey == 0, ey == n - 1, i2), (i2, ez == 0, ez == n - 1, i1)):
                        for side, on in ((0, lo), (1, hi)):
                            if not on:
                                continue
                            sgn = 1.0 if side else -1.0
                            val = ell[idx](float(side))
                            dn = sgn * dell[idx](float(side)) / h
                            v += h * h * _integral(ell[other]) * (theta * dn * _integral(g * ell[i0])
                                                                  + gamma * val * _integral(X * ell[i0]))
                    ref[i] = v
    R = op.residual(u)
    assert np.linalg.norm(R - ref) <= 1e-12 * np.linalg.norm(ref)


def test_sampled_rows_match_the_full_objects():
    """The row-sampled residual and Jacobian (used at full size) are the same
    numbers as the assembled ones."""
    pr = Problem(3, 2, 2, k=2, theta=-1.0, mask=0x1B, c=0.7)
    op = NonlinearDG(pr)
    n = pr.nelem * 27
    u0, z = _rand(n), _rand(n)
    cells = [0, 5, 11, 7]
    R = op.residual(u0).reshape(-1, 27)
    assert np.array_equal(op.residual(u0, elems=cells), R[cells])
    Jz = op.jacobian(u0).matvec(z).reshape(-1, 27)
    assert np.allclose(op.jacobian_rows(u0, z, cells), Jz[cells], rtol=1e-13, atol=1e-13)
