"""Nonlinear SIPG diffusion operator by full quadrature (test infrastructure; oracle only).

Problem: -div(kappa(u) grad u) + c u = f with kappa(u) = 1 + u^2 and
homogeneous Dirichlet data on the sides flagged in the mask. The residual of
Section 2.1, R_i(u) = r(u_h, phi_i), uses the SIPG form of Section 5.2
(eq. diffreac_weak) with the coefficient evaluated at the solution:

  r(u, v) = sum_T (kappa(u) grad u, grad v)_T + (c u, v)_T
          + sum_F [ -({kappa(u) grad u}.n_F, [v])_F + theta ([u], {kappa(u) grad v}.n_F)_F
                    + gamma_F ([u], [v])_F ]

over interior and Dirichlet faces ([w] = {w} = w there, data 0), with kappa
on a face taken from each side's own trace of u. The source term -(f, v) is
not part of R here (it is a load vector). The Jacobian J(u0)_ij = dR_i/du_j
at a linearization point u0 (Section 2.1: its action depends on both the
linearization point and the direction) is

  (kappa(u0) grad z + kappa'(u0) z grad u0, grad v) + (c z, v)
  + sum_F [ -({kappa(u0) grad z + kappa'(u0) z grad u0}.n_F, [v])
            + theta ([z], {kappa(u0) grad v}.n_F)
            + theta ([u0], {kappa'(u0) z grad v}.n_F) + gamma_F ([z], [v]) ].

Every integral is a plain tensor Gauss-Legendre sum with every basis function
evaluated as a product of 1D Lagrange factors, as in ScalarDG; R is evaluated
directly from u at the points, J is assembled as a block matrix, and neither
is derived from the other in code.
"""
from __future__ import annotations

import numpy as np

from .blocks import BlockMatrix, NSLOT, slot
from .problem import physical_gradients
from .scalar import ScalarDG


def kappa(u):
    return 1.0 + u * u


def dkappa(u):
    return 2.0 * u


class NonlinearDG(ScalarDG):
    """The problem's kappa fields must be unset: the coefficient is kappa(u)."""

    def __init__(self, prob):
        assert prob.kappa is None and prob.kappa_tensor is None
        super().__init__(prob)

    # ---- u and its gradient at the points ---------------------------------
    def _cell(self, e, u):
        pr = self.prob
        J = pr.mesh.jacobian(e, pr.cell_xi)
        wd = pr.cell_w * np.abs(np.linalg.det(J))
        g = physical_gradients(self.grad_c, J)
        ue = u[e * self.N:(e + 1) * self.N]
        return wd, g, self.phi_c @ ue, np.einsum("pna,n->pa", g, ue)

    def _side(self, e, d, s, u):
        """Face (d, s) of cell e: area elements, basis values, basis derivatives
        along n (toward +xi_d), and the trace and normal derivative of u."""
        pr = self.prob
        xi, x, dA, n = pr.face_geometry(e, d, s)
        phi, gref = self.face_tab[(d, s)]
        g = physical_gradients(gref, pr.mesh.jacobian(e, xi))
        dn = np.einsum("pja,pa->pj", g, n)
        ue = u[e * self.N:(e + 1) * self.N]
        return x, dA, phi, dn, phi @ ue, dn @ ue

    # ---- residual -----------------------------------------------------------
    def residual_cell(self, e: int, u: np.ndarray) -> np.ndarray:
        """R restricted to the test functions of cell e (its volume and its six faces)."""
        pr = self.prob
        mesh = pr.mesh
        th = pr.theta
        wd, g, uq, gu = self._cell(e, u)
        R = np.einsum("p,pia,pa->i", wd * kappa(uq), g, gu)
        R += pr.c * np.einsum("p,pi,p->i", wd, self.phi_c, uq)
        for d in range(3):
            for s in range(2):
                nb = mesh.neighbor(e, d, s)
                if nb >= 0:
                    em, ep = (e, nb) if s == 1 else (nb, e)  # T^-, T^+ of the face
                    xm, dA, phm, dnm, um, dum = self._side(em, d, 1, u)
                    xp, _, php, dnp, up, dup = self._side(ep, d, 0, u)
                    assert np.allclose(xm, xp, rtol=0, atol=1e-13)
                    gam = self.gamma(dA.sum(), (self.cell_volume(em), self.cell_volume(ep)))
                    flux = 0.5 * (kappa(um) * dum + kappa(up) * dup)
                    ju = um - up
                    if e == em:  # [phi_i] = phi_i, {kappa(u) d_n phi_i} = kappa(u^-) d_n phi_i / 2
                        R += phm.T @ (dA * (-flux + gam * ju)) + th * dnm.T @ (dA * 0.5 * kappa(um) * ju)
                    else:  # [phi_i] = -phi_i
                        R += -php.T @ (dA * (-flux + gam * ju)) + th * dnp.T @ (dA * 0.5 * kappa(up) * ju)
                elif (pr.mask >> (2 * d + s)) & 1:
                    x, dA, ph, dn, ut, dnu = self._side(e, d, s, u)
                    if s == 0:  # outward normal
                        dn, dnu = -dn, -dnu
                    gam = self.gamma(dA.sum(), (self.cell_volume(e),))
                    R += ph.T @ (dA * (-kappa(ut) * dnu + gam * ut)) + th * dn.T @ (dA * kappa(ut) * ut)
        return R

    def residual(self, u: np.ndarray, elems=None) -> np.ndarray:
        """R(u); with `elems`, only the rows of those cells, shape (len(elems), N)."""
        if elems is not None:
            return np.stack([self.residual_cell(int(e), u) for e in elems])
        return np.concatenate([self.residual_cell(e, u) for e in range(self.prob.mesh.nelem)])

    # ---- Jacobian -----------------------------------------------------------
    def jac_volume_block(self, e, u0):
        wd, g, uq, gu = self._cell(e, u0)
        A = np.einsum("p,pia,pja->ij", wd * kappa(uq), g, g)
        A += np.einsum("p,pia,pa,pj->ij", wd * dkappa(uq), g, gu, self.phi_c)
        A += self.prob.c * np.einsum("p,pi,pj->ij", wd, self.phi_c, self.phi_c)
        return A

    def jac_interior_face_blocks(self, em, ep, d, u0):
        """B[a][b]: test side a, trial side b (0 = T^-, 1 = T^+)."""
        xm, dA, phm, dnm, um, dum = self._side(em, d, 1, u0)
        xp, _, php, dnp, up, dup = self._side(ep, d, 0, u0)
        assert np.allclose(xm, xp, rtol=0, atol=1e-13)
        gam = self.gamma(dA.sum(), (self.cell_volume(em), self.cell_volume(ep)))
        th = self.prob.theta
        ju0 = um - up
        # derivative of {kappa(u) d_n u} with respect to a trial function of side b
        fl = (0.5 * (kappa(um)[:, None] * dnm + (dkappa(um) * dum)[:, None] * phm),
              0.5 * (kappa(up)[:, None] * dnp + (dkappa(up) * dup)[:, None] * php))
        jump = (phm, -php)
        phis = (phm, php)
        tavg = (0.5 * kappa(um)[:, None] * dnm, 0.5 * kappa(up)[:, None] * dnp)
        tkap = (0.5 * dkappa(um)[:, None] * dnm, 0.5 * dkappa(up)[:, None] * dnp)
        B = [[None, None], [None, None]]
        for a in range(2):
            for b in range(2):
                B[a][b] = (-np.einsum("q,qi,qj->ij", dA, jump[a], fl[b])
                           + th * np.einsum("q,qi,qj->ij", dA, tavg[a], jump[b])
                           + gam * np.einsum("q,qi,qj->ij", dA, jump[a], jump[b]))
                if a == b:
                    B[a][b] += th * np.einsum("q,qi,qj->ij", dA * ju0, tkap[a], phis[b])
        return B

    def jac_boundary_block(self, e, d, s, u0):
        x, dA, ph, dn, ut, dnu = self._side(e, d, s, u0)
        if s == 0:
            dn, dnu = -dn, -dnu
        gam = self.gamma(dA.sum(), (self.cell_volume(e),))
        th = self.prob.theta
        k, kp = kappa(ut), dkappa(ut)
        flux = k[:, None] * dn + (kp * dnu)[:, None] * ph
        return (-np.einsum("q,qi,qj->ij", dA, ph, flux)
                + th * np.einsum("q,qi,qj->ij", dA, k[:, None] * dn, ph)
                + th * np.einsum("q,qi,qj->ij", dA * ut * kp, dn, ph)
                + gam * np.einsum("q,qi,qj->ij", dA, ph, ph))

    def jacobian_rows(self, u0: np.ndarray, z: np.ndarray, elems) -> np.ndarray:
        """Rows of J(u0) z for the given cells; returns (len(elems), N)."""
        mesh = self.prob.mesh
        Z = np.asarray(z).reshape(-1, self.N)
        out = np.zeros((len(elems), self.N))
        for r, e in enumerate(elems):
            e = int(e)
            out[r] += self.jac_volume_block(e, u0) @ Z[e]
            for d in range(3):
                for s in range(2):
                    nb = mesh.neighbor(e, d, s)
                    if nb >= 0 and s == 1:
                        B = self.jac_interior_face_blocks(e, nb, d, u0)
                        out[r] += B[0][0] @ Z[e] + B[0][1] @ Z[nb]
                    elif nb >= 0:
                        B = self.jac_interior_face_blocks(nb, e, d, u0)
                        out[r] += B[1][1] @ Z[e] + B[1][0] @ Z[nb]
                    elif (self.prob.mask >> (2 * d + s)) & 1:
                        out[r] += self.jac_boundary_block(e, d, s, u0) @ Z[e]
        return out

    def jacobian(self, u0: np.ndarray) -> BlockMatrix:
        mesh = self.prob.mesh
        nbr = self._neighbors()
        E, N = nbr.shape[0], self.N
        blocks = np.zeros((E, NSLOT, N, N))
        for e in range(E):
            blocks[e, 0] = self.jac_volume_block(e, u0)
        for e in range(E):
            for d in range(3):
                for s in range(2):
                    nb = mesh.neighbor(e, d, s)
                    if nb >= 0 and s == 1:
                        B = self.jac_interior_face_blocks(e, nb, d, u0)
                        blocks[e, 0] += B[0][0]
                        blocks[e, slot(d, 1)] = B[0][1]
                        blocks[nb, 0] += B[1][1]
                        blocks[nb, slot(d, 0)] = B[1][0]
                    elif nb < 0 and (self.prob.mask >> (2 * d + s)) & 1:
                        blocks[e, 0] += self.jac_boundary_block(e, d, s, u0)
        return BlockMatrix(nbr, N, blocks=blocks)
