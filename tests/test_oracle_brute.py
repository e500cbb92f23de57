"""Brute-force pin: a separately written assembly of the SIPG form of
Section 5.2 (eq. diffreac_weak) on tiny axis-aligned meshes, by exact
integration of polynomials in physical coordinates, against the oracle's
quadrature assembly.

Basis functions are built here as coefficient tensors of polynomials in
(x, y, z) (Lagrange factors from their roots at numpy's Gauss-Legendre nodes),
products are tensor convolutions and integrals use the antiderivatives of
monomials; nothing is shared with the oracle. On axis-aligned cells every
integrand is a polynomial the (k+1)-point Gauss rule integrates exactly, so
the two must agree to rounding. theta = +1 and mixed Dirichlet/Neumann masks
make sign or side mistakes visible.
"""
import numpy as np
import pytest
from numpy.polynomial import polynomial as npoly
from scipy.signal import convolve

from oracle import Problem, ScalarDG


def _lagrange_poly(tnodes, j, x0, h):
    """l_j((x - x0)/h) as coefficients in x (low to high)."""
    roots = [x0 + h * t for i, t in enumerate(tnodes) if i != j]
    xj = x0 + h * tnodes[j]
    coef = npoly.polyfromroots(roots) if roots else np.array([1.0])
    return coef / np.prod([xj - r for r in roots]) if roots else coef


def _tensor(px, py, pz):
    return np.einsum("a,b,c->abc", px, py, pz)


def _mul(A, B):
    return convolve(A, B, method="direct")


def _der(A, d):
    return npoly.polyder(A, axis=d) if A.shape[d] > 1 else np.zeros_like(A)


def _restrict(A, d, val):
    """Evaluate the tensor polynomial at x_d = val (the axis stays, of length 1)."""
    w = val ** np.arange(A.shape[d])
    return np.expand_dims(np.tensordot(A, w, axes=([d], [0])), d)


def _integrate(A, lo, hi):
    """Integral over the box [lo, hi]; a None bound marks an axis of length 1 (a face)."""
    out = A
    for d in range(2, -1, -1):
        if lo[d] is None:
            out = out[..., 0] if out.ndim else out
            continue
        a = np.arange(out.shape[-1])
        w = (hi[d] ** (a + 1) - lo[d] ** (a + 1)) / (a + 1)
        out = out @ w
    return float(out)


def _assemble_exact(n, k, c, theta, alpha, mask):
    nx, ny, nz = n
    h = [1.0 / nx, 1.0 / ny, 1.0 / nz]
    p = k + 1
    t, _ = np.polynomial.legendre.leggauss(p)
    tn = (t + 1) / 2
    E = nx * ny * nz
    N = p ** 3
    cells = [(e % nx, (e // nx) % ny, e // (nx * ny)) for e in range(E)]

    def basis(e):
        lo = [cells[e][d] * h[d] for d in range(3)]
        L = [[_lagrange_poly(tn, j, lo[d], h[d]) for j in range(p)] for d in range(3)]
        return lo, [_tensor(L[0][i0], L[1][i1], L[2][i2])
                    for i2 in range(p) for i1 in range(p) for i0 in range(p)]

    B = [basis(e) for e in range(E)]
    vol = h[0] * h[1] * h[2]
    A = np.zeros((E * N, E * N))
    for e in range(E):
        lo, fns = B[e]
        hi = [lo[d] + h[d] for d in range(3)]
        grads = [[_der(f, d) for d in range(3)] for f in fns]
        for i in range(N):
            for j in range(N):
                val = c * _integrate(_mul(fns[i], fns[j]), lo, hi)
                for d in range(3):
                    val += _integrate(_mul(grads[i][d], grads[j][d]), lo, hi)
                A[e * N + i, e * N + j] += val
    coef = alpha * k * (k + 1)
    for e in range(E):
        lo, fns = B[e]
        for d in range(3):
            tang = [a for a in range(3) if a != d]
            gam = coef * h[tang[0]] * h[tang[1]] / vol
            flo = [lo[a] if a != d else None for a in range(3)]
            fhi = [lo[a] + h[a] if a != d else None for a in range(3)]
            for side in (0, 1):
                plane = lo[d] + side * h[d]
                nb = list(cells[e])
                nb[d] += 1 if side else -1
                if 0 <= nb[d] < n[d]:
                    if side == 0:
                        continue  # each interior face once, from its lower cell
                    e2 = nb[0] + nx * (nb[1] + ny * nb[2])
                    cl = {0: e, 1: e2}
                    tr = {s: [_restrict(f, d, plane) for f in B[cl[s]][1]] for s in (0, 1)}
                    dn = {s: [_restrict(_der(f, d), d, plane) for f in B[cl[s]][1]] for s in (0, 1)}
                    sg = {0: 1.0, 1: -1.0}   # [w] = w(T-) - w(T+), n = +e_d
                    for a in (0, 1):
                        for b in (0, 1):
                            for i in range(N):
                                for j in range(N):
                                    v = (-0.5 * sg[a] * _integrate(_mul(dn[b][j], tr[a][i]), flo, fhi)
                                         + theta * 0.5 * sg[b] * _integrate(_mul(tr[b][j], dn[a][i]), flo, fhi)
                                         + gam * sg[a] * sg[b] * _integrate(_mul(tr[a][i], tr[b][j]), flo, fhi))
                                    A[cl[a] * N + i, cl[b] * N + j] += v
                elif (mask >> (2 * d + side)) & 1:
                    ns = 1.0 if side else -1.0
                    tr = [_restrict(f, d, plane) for f in fns]
                    dn = [ns * _restrict(_der(f, d), d, plane) for f in fns]
                    for i in range(N):
                        for j in range(N):
                            A[e * N + i, e * N + j] += (
                                -_integrate(_mul(dn[j], tr[i]), flo, fhi)
                                + theta * _integrate(_mul(tr[j], dn[i]), flo, fhi)
                                + gam * _integrate(_mul(tr[i], tr[j]), flo, fhi))
    return A


@pytest.mark.parametrize("n,k,mask", [((2, 1, 1), 1, 0x3F), ((2, 2, 1), 1, 0x1B),
                                      ((1, 1, 1), 2, 0x2D), ((1, 2, 1), 2, 0x3F)])
def test_exact_polynomial_brute_force(n, k, mask):
    c, theta, alpha = 3.0, 1.0, 3.0
    ref = _assemble_exact(n, k, c, theta, alpha, mask)
    got = ScalarDG(Problem(*n, k=k, c=c, theta=theta, alpha=alpha, mask=mask)).assemble("explicit").to_dense()
    # the monomial coefficients of the reference lose a few digits to cancellation at
    # k = 2; a wrong sign, term or side would show at O(1)
    assert np.max(np.abs(got - ref)) < 1e-10 * np.max(np.abs(ref))
