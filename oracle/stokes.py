"""DG Stokes operator by full quadrature (test infrastructure; oracle only).

The operator is the linear part of the residual of Section 5.3
(eq. stokes_weak) with mu = 1, velocity in (Q_k)^3 and pressure in Q_{k-1}:

  a((u,p),(v,q)) = sum_T (grad u, grad v)_T - (p, div v)_T - (div u, q)_T
      + sum_{F interior or Dirichlet} [ -({grad u} n, [v])_F
            + theta ([u], {grad v} n)_F + gamma_F ([u], [v])_F
            + ({p}, [v].n)_F + ([u].n, {q})_F ]

The second face term is printed garbled in the paper; it is read as
theta ([u], {grad v} n), the vector form of the scalar SIPG term of
Section 5.2 and of the boundary term grad v n of the same equation.
Neumann sides contribute nothing. Jumps, averages, normals and gamma_F are
those of the scalar operator with k the velocity degree.

Cell block layout: [u_0 (p^3) | u_1 (p^3) | u_2 (p^3) | p (k^3)], p = k+1.
"""
from __future__ import annotations

import numpy as np

from .gauss import gauss_legendre
from .problem import Problem, basis_tables, physical_gradients
from .scalar import ScalarDG


class StokesDG(ScalarDG):
    def __init__(self, prob: Problem):
        if prob.kappa is not None or prob.kappa_tensor is not None:
            raise ValueError("the Stokes operator has mu = 1 and no kappa")
        super().__init__(prob)
        self.kp = prob.k                      # pressure nodes per direction (degree k-1)
        self.pnodes, _ = gauss_legendre(self.kp)
        self.Nv = self.p ** 3
        self.Nq = self.kp ** 3
        self.N = 3 * self.Nv + self.Nq
        self.psi_c, _ = basis_tables(self.pnodes, prob.cell_xi)
        self.pface_tab = {(d, s): basis_tables(self.pnodes, prob.face_points(d, s))[0]
                          for d in range(3) for s in range(2)}

    def _sl(self, c: int) -> slice:
        """Slice of field c (0,1,2 velocity components, 3 pressure) in a cell block."""
        if c < 3:
            return slice(c * self.Nv, (c + 1) * self.Nv)
        return slice(3 * self.Nv, self.N)

    def volume_block(self, e: int) -> np.ndarray:
        pr = self.prob
        J = pr.mesh.jacobian(e, pr.cell_xi)
        wd = pr.cell_w * np.abs(np.linalg.det(J))
        g = physical_gradients(self.grad_c, J)
        A = np.zeros((self.N, self.N))
        Avv = np.einsum("p,pia,pja->ij", wd, g, g)
        for c in range(3):
            A[self._sl(c), self._sl(c)] = Avv
            Bc = -np.einsum("p,pi,pj->ij", wd, g[:, :, c], self.psi_c)  # -(p, div v)
            A[self._sl(c), self._sl(3)] = Bc
            A[self._sl(3), self._sl(c)] = Bc.T                           # -(div u, q)
        return A

    def _vside(self, e: int, d: int, s: int):
        pr = self.prob
        xi, x, dA, n = pr.face_geometry(e, d, s)
        phi, gref = self.face_tab[(d, s)]
        g = physical_gradients(gref, pr.mesh.jacobian(e, xi))
        dn = np.einsum("pja,pa->pj", g, n)
        psi = self.pface_tab[(d, s)]
        return x, dA, n, phi, dn, psi

    def _face_block(self, dA, n, gam, phi_a, dn_a, psi_a, sa, phi_b, dn_b, psi_b, sb, half):
        """Block for test functions of side a and trial functions of side b.

        sa, sb: jump signs (+1 on T^-, -1 on T^+); half: 1/2 on interior faces
        (averages), 1 on boundary faces."""
        th = self.prob.theta
        A = np.zeros((self.N, self.N))
        vv = (-half * sa * np.einsum("q,qi,qj->ij", dA, phi_a, dn_b)
              + th * half * sb * np.einsum("q,qi,qj->ij", dA, dn_a, phi_b)
              + gam * sa * sb * np.einsum("q,qi,qj->ij", dA, phi_a, phi_b))
        for c in range(3):
            A[self._sl(c), self._sl(c)] = vv
            # ({p}, [v].n): test velocity c on side a, trial pressure on side b
            A[self._sl(c), self._sl(3)] = half * sa * np.einsum("q,qi,qj->ij", dA * n[:, c], phi_a, psi_b)
            # ([u].n, {q}): test pressure on side a, trial velocity c on side b
            A[self._sl(3), self._sl(c)] = half * sb * np.einsum("q,qi,qj->ij", dA * n[:, c], psi_a, phi_b)
        return A

    def interior_face_blocks(self, em: int, ep: int, d: int):
        xm, dA, n, phim, dnm, psim = self._vside(em, d, 1)
        xp, _, _, phip, dnp, psip = self._vside(ep, d, 0)
        if not np.allclose(xm, xp, rtol=0, atol=1e-13):
            raise AssertionError("face quadrature points of the two cells do not coincide")
        gam = self.gamma(dA.sum(), (self.cell_volume(em), self.cell_volume(ep)))
        side = [(phim, dnm, psim, 1.0), (phip, dnp, psip, -1.0)]
        B = [[None, None], [None, None]]
        for a in range(2):
            for b in range(2):
                pa, da, qa, sa = side[a]
                pb, db, qb, sb = side[b]
                B[a][b] = self._face_block(dA, n, gam, pa, da, qa, sa, pb, db, qb, sb, 0.5)
        return B

    def boundary_block(self, e: int, d: int, s: int) -> np.ndarray:
        x, dA, n, phi, dn, psi = self._vside(e, d, s)
        if s == 0:
            n, dn = -n, -dn
        gam = self.gamma(dA.sum(), (self.cell_volume(e),))
        return self._face_block(dA, n, gam, phi, dn, psi, 1.0, phi, dn, psi, 1.0, 1.0)

    def kappa_gradient(self, *a, **k):
        raise NotImplementedError("the Stokes operator has no kappa")

    def dirichlet_load(self, gD) -> np.ndarray:
        """u-independent Dirichlet terms of eq. stokes_weak moved to the right-hand side:
        theta (g, grad v n) + gamma_F (g, v) + (g.n, q) on every Dirichlet face (f = 0)."""
        pr = self.prob
        mesh = pr.mesh
        b = np.zeros((mesh.nelem, self.N))
        th = pr.theta
        for e in range(mesh.nelem):
            for d in range(3):
                for s in range(2):
                    if mesh.neighbor(e, d, s) >= 0 or not (pr.mask >> (2 * d + s)) & 1:
                        continue
                    x, dA, n, phi, dn, psi = self._vside(e, d, s)
                    if s == 0:
                        n, dn = -n, -dn
                    gam = self.gamma(dA.sum(), (self.cell_volume(e),))
                    gv = gD(x)  # (P, 3)
                    for c in range(3):
                        b[e, self._sl(c)] += th * dn.T @ (dA * gv[:, c]) + gam * phi.T @ (dA * gv[:, c])
                    b[e, self._sl(3)] += psi.T @ (dA * np.sum(gv * n, axis=1))
        return b.reshape(-1)

    def interpolate_fields(self, ufn, pfn) -> np.ndarray:
        """Nodal interpolant of a velocity field ufn (P,3) and a pressure pfn (P,)."""
        mesh = self.prob.mesh
        p, kp = self.p, self.kp
        q = np.arange(p ** 3)
        xi_v = np.stack([self.nodes[q % p], self.nodes[(q // p) % p], self.nodes[q // (p * p)]], axis=1)
        r = np.arange(kp ** 3)
        xi_p = np.stack([self.pnodes[r % kp], self.pnodes[(r // kp) % kp], self.pnodes[r // (kp * kp)]], axis=1)
        out = np.zeros((mesh.nelem, self.N))
        for e in range(mesh.nelem):
            uv = ufn(mesh.map(e, xi_v))
            for c in range(3):
                out[e, self._sl(c)] = uv[:, c]
            out[e, self._sl(3)] = pfn(mesh.map(e, xi_p))
        return out.reshape(-1)
