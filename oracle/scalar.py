"""SIPG diffusion-reaction operator by full quadrature (test infrastructure; oracle only).

The operator is the Jacobian action of the residual of Section 5.2
(eq. diffreac_weak) for -div(K grad u) + c u = f with Dirichlet data on the
sides flagged in the mask:

  a(u, v) = sum_T (K grad u, grad v)_T + (c u, v)_T
          + sum_F [ -({K grad u}.n_F, [v])_F + theta ([u], {K grad v}.n_F)_F
                    + gamma_F ([u], [v])_F ]

over interior and Dirichlet boundary faces, with [w] = w^- - w^+ and
{w} = (w^- + w^+)/2 on interior faces and [w] = {w} = w on the boundary
(Section 5.2), n_F pointing from T^- to T^+ (Section 2.1), and
gamma_F = alpha k(k+1)|F| / min(|T^+|, |T^-|) (penalty_form 0) or the paper's
alpha k(k+d-1)|F| / min(...) (penalty_form 1). K is kappa * I with kappa given
per volume quadrature point (faces use the cell's interpolant of those values)
or a full tensor function of x.

Every integral is a plain tensor Gauss-Legendre sum over all quadrature points
with every basis function evaluated as a product of 1D Lagrange factors; the
sums are never factorized. The mathematical result is the one sum
factorization reaches (Section 2.2), which only reorders these sums.
"""
from __future__ import annotations

import numpy as np

from .blocks import BlockMatrix, NSLOT, slot
from .gauss import gauss_legendre
from .lagrange import lagrange_eval
from .problem import Problem, basis_tables, physical_gradients


class ScalarDG:
    def __init__(self, prob: Problem):
        self.prob = prob
        self.p = prob.k + 1
        self.N = self.p ** 3
        self.nodes, _ = gauss_legendre(self.p)  # nodal basis at the k+1 Gauss-Legendre points
        self.phi_c, self.grad_c = basis_tables(self.nodes, prob.cell_xi)
        self.face_tab = {(d, s): basis_tables(self.nodes, prob.face_points(d, s))
                         for d in range(3) for s in range(2)}
        self.coef = prob.penalty_coef(prob.k)
        self._vol_cache = {}

    # ---- coefficients ---------------------------------------------------
    def _K_cell(self, e: int, x: np.ndarray) -> np.ndarray:
        P = x.shape[0]
        if self.prob.kappa_tensor is not None:
            return self.prob.kappa_tensor(x)
        if self.prob.kappa is None:
            kap = np.ones(P)
        else:
            M = self.prob.m ** 3
            kap = self.prob.kappa[e * M:(e + 1) * M]
        return kap[:, None, None] * np.eye(3)[None]

    def _K_face(self, e: int, xi: np.ndarray, x: np.ndarray) -> np.ndarray:
        if self.prob.kappa_tensor is not None:
            return self.prob.kappa_tensor(x)
        if self.prob.kappa_face_one:
            kap = np.ones(x.shape[0])
        else:
            kap = self.prob.kappa_at(e, xi)
        return kap[:, None, None] * np.eye(3)[None]

    def cell_volume(self, e: int) -> float:
        if e not in self._vol_cache:
            self._vol_cache[e] = self.prob.cell_volume(e)
        return self._vol_cache[e]

    # ---- local matrices (test index i first, trial index j second) -------
    def volume_block(self, e: int) -> np.ndarray:
        pr = self.prob
        J = pr.mesh.jacobian(e, pr.cell_xi)
        wd = pr.cell_w * np.abs(np.linalg.det(J))
        g = physical_gradients(self.grad_c, J)
        K = self._K_cell(e, pr.mesh.map(e, pr.cell_xi))
        Kg = np.einsum("pab,pjb->pja", K, g)
        A = np.einsum("p,pia,pja->ij", wd, g, Kg)
        A += pr.c * np.einsum("p,pi,pj->ij", wd, self.phi_c, self.phi_c)
        return A

    def _side(self, e: int, d: int, s: int):
        """Face rule data of cell e on its face (d, s): points, dA, n (toward +xi_d),
        basis values and K grad(phi).n."""
        pr = self.prob
        xi, x, dA, n = pr.face_geometry(e, d, s)
        phi, gref = self.face_tab[(d, s)]
        J = pr.mesh.jacobian(e, xi)
        g = physical_gradients(gref, J)
        K = self._K_face(e, xi, x)
        Kn = np.einsum("pab,pb->pa", K, n)   # K symmetric: (K grad phi).n = grad phi . (K n)
        flux = np.einsum("pja,pa->pj", g, Kn)
        return x, dA, n, phi, flux

    def gamma(self, area: float, vols) -> float:
        return self.coef * area / min(vols)

    def interior_face_blocks(self, em: int, ep: int, d: int):
        """Blocks B[a][b] (test side a, trial side b; 0 = T^-, 1 = T^+) of one interior face."""
        xm, dA, n, phim, fluxm = self._side(em, d, 1)
        xp, dA_p, _, phip, fluxp = self._side(ep, d, 0)
        if not np.allclose(xm, xp, rtol=0, atol=1e-13):
            raise AssertionError("face quadrature points of the two cells do not coincide")
        gam = self.gamma(dA.sum(), (self.cell_volume(em), self.cell_volume(ep)))
        jump = (phim, -phip)
        avg = (0.5 * fluxm, 0.5 * fluxp)
        th = self.prob.theta
        B = [[None, None], [None, None]]
        for a in range(2):
            for b in range(2):
                B[a][b] = (-np.einsum("q,qi,qj->ij", dA, jump[a], avg[b])
                           + th * np.einsum("q,qi,qj->ij", dA, avg[a], jump[b])
                           + gam * np.einsum("q,qi,qj->ij", dA, jump[a], jump[b]))
        return B

    def boundary_block(self, e: int, d: int, s: int) -> np.ndarray:
        x, dA, n, phi, flux = self._side(e, d, s)
        if s == 0:
            flux = -flux  # outward normal
        gam = self.gamma(dA.sum(), (self.cell_volume(e),))
        th = self.prob.theta
        return (-np.einsum("q,qi,qj->ij", dA, phi, flux)
                + th * np.einsum("q,qi,qj->ij", dA, flux, phi)
                + gam * np.einsum("q,qi,qj->ij", dA, phi, phi))

    def block_row(self, e: int):
        """Blocks of block row e: {slot: (column cell, block)}."""
        mesh = self.prob.mesh
        diag = self.volume_block(e)
        row = {}
        for d in range(3):
            for s in range(2):
                nb = mesh.neighbor(e, d, s)
                if nb >= 0:
                    if s == 1:
                        B = self.interior_face_blocks(e, nb, d)
                        diag = diag + B[0][0]
                        row[slot(d, s)] = (nb, B[0][1])
                    else:
                        B = self.interior_face_blocks(nb, e, d)
                        diag = diag + B[1][1]
                        row[slot(d, s)] = (nb, B[1][0])
                elif (self.prob.mask >> (2 * d + s)) & 1:
                    diag = diag + self.boundary_block(e, d, s)
        row[0] = (e, diag)
        return row

    # ---- global matrix ----------------------------------------------------
    def _neighbors(self) -> np.ndarray:
        mesh = self.prob.mesh
        nx, ny, nz = mesh.n
        e = np.arange(mesh.nelem)
        c = [e % nx, (e // nx) % ny, e // (nx * ny)]
        stride = [1, nx, nx * ny]
        nbr = np.full((mesh.nelem, NSLOT), -1, dtype=np.int64)
        nbr[:, 0] = e
        for d in range(3):
            nbr[c[d] > 0, slot(d, 0)] = e[c[d] > 0] - stride[d]
            nbr[c[d] < mesh.n[d] - 1, slot(d, 1)] = e[c[d] < mesh.n[d] - 1] + stride[d]
        return nbr

    def translation_invariant(self) -> bool:
        pr = self.prob
        return pr.vertices is None and pr.kappa is None and pr.kappa_tensor is None

    def assemble(self, mode: str = "auto") -> BlockMatrix:
        """Global block matrix. 'explicit' stores every block; 'dedup' stores one
        block row per boundary pattern (only valid on the regular grid with
        constant coefficients, where block rows depend on nothing else)."""
        if mode == "auto":
            mode = "dedup" if self.translation_invariant() else "explicit"
        nbr = self._neighbors()
        E, N = nbr.shape[0], self.N
        if mode == "explicit":
            blocks = np.zeros((E, NSLOT, N, N))
            for e in range(E):
                for s, (col, B) in self.block_row(e).items():
                    assert nbr[e, s] == col
                    blocks[e, s] = B
            return BlockMatrix(nbr, N, blocks=blocks)
        if not self.translation_invariant():
            raise ValueError("dedup assembly needs the regular grid and constant coefficients")
        mesh = self.prob.mesh
        e = np.arange(E)
        c = [e % mesh.n[0], (e // mesh.n[0]) % mesh.n[1], e // (mesh.n[0] * mesh.n[1])]
        key = np.zeros(E, dtype=np.int64)
        for d in range(3):
            code = (c[d] == 0).astype(np.int64) + 2 * (c[d] == mesh.n[d] - 1)
            key += code * 4 ** d
        keys, first, inverse = np.unique(key, return_index=True, return_inverse=True)
        classes = np.zeros((len(keys) * NSLOT, N, N))
        for ki, rep in enumerate(first):
            for s, (_, B) in self.block_row(int(rep)).items():
                classes[ki * NSLOT + s] = B
        cls = inverse[:, None] * NSLOT + np.arange(NSLOT)[None, :]
        return BlockMatrix(nbr, N, classes=classes, cls=cls)

    # ---- sampled block rows (full-size checks without a full matrix) ------
    def apply_rows(self, x: np.ndarray, elems) -> np.ndarray:
        """Rows of A x for the given cells; returns (len(elems), N)."""
        X = np.asarray(x).reshape(-1, self.N)
        out = np.zeros((len(elems), self.N))
        for r, e in enumerate(elems):
            for s, (col, B) in self.block_row(int(e)).items():
                out[r] += B @ X[col]
        return out

    def apply_T_rows(self, g: np.ndarray, elems) -> np.ndarray:
        """Rows of A^T g for the given cells; returns (len(elems), N)."""
        G = np.asarray(g).reshape(-1, self.N)
        mesh = self.prob.mesh
        out = np.zeros((len(elems), self.N))
        for r, e in enumerate(elems):
            e = int(e)
            out[r] += self.block_row(e)[0][1].T @ G[e]
            for d in range(3):
                for s in range(2):
                    nb = mesh.neighbor(e, d, s)
                    if nb >= 0:
                        # block (row nb, column e) of A: the face shared by e and nb,
                        # test functions on nb's side, trial functions on e's side
                        if s == 1:  # e = T^-, nb = T^+
                            B = self.interior_face_blocks(e, nb, d)[1][0]
                        else:  # nb = T^-, e = T^+
                            B = self.interior_face_blocks(nb, e, d)[0][1]
                        out[r] += B.T @ G[nb]
        return out

    # ---- derivative with respect to kappa ----------------------------------
    def kappa_gradient(self, u: np.ndarray, g: np.ndarray, elems=None) -> np.ndarray:
        """dL/dkappa for L = g^T A(kappa) u, kappa given per volume quadrature point.

        L = a(u_h, g_h) is affine in kappa. Volume point q of cell T contributes
        w_q |det J| grad u_h . grad g_h. On a face, kappa_T is the cell's
        interpolant of its point values, so every face point x contributes
        dA(x) dI/dkappa_T(x) L_q(x), with I the face integrand and L_q the
        interpolation weight of point q at x.
        """
        pr = self.prob
        if pr.kappa_tensor is not None:
            raise ValueError("kappa_gradient needs a scalar kappa")
        mesh = pr.mesh
        M = pr.m ** 3
        U = np.asarray(u).reshape(-1, self.N)
        Gv = np.asarray(g).reshape(-1, self.N)
        elems = range(mesh.nelem) if elems is None else elems
        elems = [int(e) for e in elems]
        out = np.zeros((len(elems), M))
        th = pr.theta
        for r, e in enumerate(elems):
            J = mesh.jacobian(e, pr.cell_xi)
            wd = pr.cell_w * np.abs(np.linalg.det(J))
            gr = physical_gradients(self.grad_c, J)
            gu = np.einsum("pia,i->pa", gr, U[e])
            gg = np.einsum("pia,i->pa", gr, Gv[e])
            out[r] += wd * np.sum(gu * gg, axis=1)
            if pr.kappa_face_one:
                continue
            for d in range(3):
                for s in range(2):
                    nb = mesh.neighbor(e, d, s)
                    dirichlet = (pr.mask >> (2 * d + s)) & 1
                    if nb < 0 and not dirichlet:
                        continue
                    xi, x, dA, n = pr.face_geometry(e, d, s)
                    phi, gref = self.face_tab[(d, s)]
                    gp = physical_gradients(gref, mesh.jacobian(e, xi))
                    dn = np.einsum("pja,pa->pj", gp, n)
                    uT, gT = phi @ U[e], phi @ Gv[e]
                    duT, dgT = dn @ U[e], dn @ Gv[e]
                    if nb >= 0:
                        xin = pr.face_points(d, 1 - s)
                        phin, _ = self.face_tab[(d, 1 - s)]
                        uN, gN = phin @ U[nb], phin @ Gv[nb]
                        sgn = 1.0 if s == 1 else -1.0  # T is T^- when s == 1
                        ju, jg = sgn * (uT - uN), sgn * (gT - gN)
                        dI = -0.5 * duT * jg + th * 0.5 * ju * dgT
                    else:
                        sgn = 1.0 if s == 1 else -1.0  # outward normal = sgn * n
                        dI = -(sgn * duT) * gT + th * uT * (sgn * dgT)
                    Lq = self._interp_weights(xi)
                    out[r] += np.einsum("p,p,pq->q", dA, dI, Lq)
        return out

    def _interp_weights(self, xi: np.ndarray) -> np.ndarray:
        """L[p, q]: weight of volume point q in the cell interpolant at reference point p."""
        xq = self.prob.xq
        m = len(xq)
        L = [lagrange_eval(xq, xi[:, a]) for a in range(3)]
        q = np.arange(m ** 3)
        return L[0][:, q % m] * L[1][:, (q // m) % m] * L[2][:, q // (m * m)]

    # ---- right-hand side and errors ---------------------------------------
    def load_vector(self, f, gD=None) -> np.ndarray:
        """b_i = (f, phi_i) + sum over Dirichlet faces of theta (g, K grad phi_i . n)
        + gamma_F (g, phi_i): the u-independent terms of eq. diffreac_weak moved to
        the right-hand side."""
        return self.load_rows(f, gD, range(self.prob.mesh.nelem)).reshape(-1)

    def load_rows(self, f, gD, elems) -> np.ndarray:
        """The rows of the load vector of the given cells, (len(elems), N)."""
        pr = self.prob
        mesh = pr.mesh
        elems = [int(e) for e in elems]
        b = np.zeros((len(elems), self.N))
        for r, e in enumerate(elems):
            J = mesh.jacobian(e, pr.cell_xi)
            wd = pr.cell_w * np.abs(np.linalg.det(J))
            x = mesh.map(e, pr.cell_xi)
            b[r] += self.phi_c.T @ (wd * f(x))
            if gD is None:
                continue
            for d in range(3):
                for s in range(2):
                    if mesh.neighbor(e, d, s) >= 0 or not (pr.mask >> (2 * d + s)) & 1:
                        continue
                    xf, dA, n, phi, flux = self._side(e, d, s)
                    if s == 0:
                        flux = -flux
                    gam = self.gamma(dA.sum(), (self.cell_volume(e),))
                    gv = gD(xf)
                    b[r] += pr.theta * flux.T @ (dA * gv) + gam * phi.T @ (dA * gv)
        return b

    def interpolate(self, fn) -> np.ndarray:
        """Nodal interpolant of fn (values at the mapped basis nodes)."""
        mesh = self.prob.mesh
        p = self.p
        q = np.arange(p ** 3)
        xi = np.stack([self.nodes[q % p], self.nodes[(q // p) % p], self.nodes[q // (p * p)]], axis=1)
        return np.concatenate([fn(mesh.map(e, xi)) for e in range(mesh.nelem)])

    def l2_error(self, u: np.ndarray, exact, extra: int = 3) -> float:
        pr = self.prob
        mesh = pr.mesh
        mq = pr.m + extra
        xg, wg = gauss_legendre(mq)
        q = np.arange(mq ** 3)
        lex = np.stack([q % mq, (q // mq) % mq, q // (mq * mq)], axis=1)
        xi, w = xg[lex], np.prod(wg[lex], axis=1)
        phi, _ = basis_tables(self.nodes, xi)
        U = np.asarray(u).reshape(-1, self.N)
        err = 0.0
        for e in range(mesh.nelem):
            J = mesh.jacobian(e, xi)
            wd = w * np.abs(np.linalg.det(J))
            diff = phi @ U[e] - exact(mesh.map(e, xi))
            err += float(np.sum(wd * diff * diff))
        return float(np.sqrt(err))
