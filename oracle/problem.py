"""Problem description shared by the oracle's scalar and Stokes assemblers.

Test infrastructure only. The fields mirror the library's mesh descriptor but
this module shares no code with the library.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np

from .gauss import gauss_legendre
from .lagrange import lagrange_eval, lagrange_deriv
from .mesh import HexMesh


@dataclasses.dataclass
class Problem:
    nx: int
    ny: int
    nz: int
    k: int                      # polynomial degree (velocity degree for Stokes)
    m: int = 0                  # quadrature points per direction; 0 -> k + 1
    c: float = 1.0              # reaction coefficient (scalar problem)
    alpha: float = 3.0          # penalty parameter
    theta: float = -1.0         # -1: SIPG
    penalty_form: int = 0       # 0: alpha k(k+1)|F|/min|T|, 1: alpha k(k+d-1)|F|/min|T|
    mask: int = 0x3F            # Dirichlet sides, bit 2d+s for side s of direction d
    vertices: Optional[np.ndarray] = None
    kappa: Optional[np.ndarray] = None          # per volume quadrature point, (nelem*m^3,)
    kappa_face_one: bool = False                # faces use kappa = 1 instead of the trace
    kappa_tensor: Optional[Callable] = None     # x (P,3) -> K (P,3,3), replaces kappa

    def __post_init__(self):
        if self.m == 0:
            self.m = self.k + 1
        self.mesh = HexMesh(self.nx, self.ny, self.nz, self.vertices)
        self.xq, self.wq = gauss_legendre(self.m)
        m = self.m
        # tensor cell rule, q = q0 + m (q1 + m q2)
        q = np.arange(m ** 3)
        lex = np.stack([q % m, (q // m) % m, q // (m * m)], axis=1)
        self.cell_xi = self.xq[lex]
        self.cell_w = np.prod(self.wq[lex], axis=1)
        # face rule on the two tangential directions, first tangential index fastest
        ta, tb = np.meshgrid(np.arange(m), np.arange(m), indexing="xy")
        ta, tb = ta.ravel(), tb.ravel()
        self.face_t = np.stack([self.xq[ta], self.xq[tb]], axis=1)
        self.face_w = self.wq[ta] * self.wq[tb]

    @property
    def nelem(self) -> int:
        return self.mesh.nelem

    def penalty_coef(self, k: int) -> float:
        if self.penalty_form == 0:
            return self.alpha * k * (k + 1)
        return self.alpha * k * (k + 3 - 1)

    def face_points(self, d: int, side: int) -> np.ndarray:
        """Reference points of the face rule on face (d, side) of the unit cube."""
        tang = [a for a in range(3) if a != d]
        xi = np.empty((self.face_w.size, 3))
        xi[:, d] = float(side)
        xi[:, tang[0]] = self.face_t[:, 0]
        xi[:, tang[1]] = self.face_t[:, 1]
        return xi

    def face_geometry(self, e: int, d: int, side: int):
        """Physical points, area elements and unit normals on face (d, side) of cell e.

        The normal points toward increasing xi_d (from T^- to T^+ on interior
        faces); the area element is the norm of the cross product of the two
        tangential columns of J, times the tangential weights.
        """
        xi = self.face_points(d, side)
        J = self.mesh.jacobian(e, xi)
        tang = [a for a in range(3) if a != d]
        cross = np.cross(J[:, :, tang[0]], J[:, :, tang[1]])
        dA = np.linalg.norm(cross, axis=1) * self.face_w
        Jinv = np.linalg.inv(J)
        nvec = Jinv[:, d, :]
        nvec = nvec / np.linalg.norm(nvec, axis=1)[:, None]
        return xi, self.mesh.map(e, xi), dA, nvec

    def cell_volume(self, e: int) -> float:
        return self.mesh.volume(e, self.cell_w, self.cell_xi)

    def kappa_at(self, e: int, xi: np.ndarray) -> np.ndarray:
        """Scalar kappa of cell e at reference points xi: the cell's Q_{m-1} interpolant
        of its values at the volume quadrature points (1 when kappa is not given)."""
        if self.kappa is None:
            return np.ones(xi.shape[0])
        m = self.m
        kv = self.kappa[e * m ** 3:(e + 1) * m ** 3].reshape(m, m, m)  # [q2, q1, q0]
        L = [lagrange_eval(self.xq, xi[:, a]) for a in range(3)]
        return np.einsum("zyx,px,py,pz->p", kv, L[0], L[1], L[2])


def basis_tables(nodes: np.ndarray, xi: np.ndarray):
    """Values (P,N) and reference gradients (P,N,3) of the tensor Lagrange basis.

    Basis function i = i0 + n (i1 + n i2) is l_{i0}(xi_0) l_{i1}(xi_1) l_{i2}(xi_2),
    evaluated as that product at every point (no factorization).
    """
    n = len(nodes)
    L = [lagrange_eval(nodes, xi[:, a]) for a in range(3)]
    dL = [lagrange_deriv(nodes, xi[:, a]) for a in range(3)]
    P = xi.shape[0]
    phi = np.empty((P, n ** 3))
    grad = np.empty((P, n ** 3, 3))
    for i2 in range(n):
        for i1 in range(n):
            for i0 in range(n):
                i = i0 + n * (i1 + n * i2)
                phi[:, i] = L[0][:, i0] * L[1][:, i1] * L[2][:, i2]
                grad[:, i, 0] = dL[0][:, i0] * L[1][:, i1] * L[2][:, i2]
                grad[:, i, 1] = L[0][:, i0] * dL[1][:, i1] * L[2][:, i2]
                grad[:, i, 2] = L[0][:, i0] * L[1][:, i1] * dL[2][:, i2]
    return phi, grad


def physical_gradients(grad_ref: np.ndarray, J: np.ndarray) -> np.ndarray:
    """grad = J^{-T} grad_ref at every point; grad_ref (P,N,3), J (P,3,3)."""
    Jinv = np.linalg.inv(J)
    return np.einsum("pba,pnb->pna", Jinv, grad_ref)


def problem_from_workload(w, n=None, theta=None, kappa=None) -> Problem:
    """Oracle problem of a workloads.Workload (optionally on an n^3 copy of its mesh)."""
    import workloads
    if n is not None:
        w = w.scaled(n)
    return Problem(w.n, w.n, w.n, k=w.k, m=w.m, c=w.c, alpha=w.alpha,
                   theta=w.theta if theta is None else theta, penalty_form=w.penalty_form,
                   mask=w.mask, vertices=workloads.vertices(w), kappa=kappa)
