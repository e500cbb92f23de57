"""Structured hexahedral meshes of the unit cube (test infrastructure; oracle only).

Each cell T is the image of the reference cube [0,1]^3 under a map mu_T
(Section 2.1); here mu_T is the trilinear interpolation of the cell's eight
vertices. Faces carry a unit normal that points from T^- (the cell with the
lower index along the face normal direction) to T^+.
"""
from __future__ import annotations

import numpy as np


class HexMesh:
    """nx*ny*nz hexahedra; cell e = ex + nx*(ey + ny*ez).

    ``vertices`` has shape (nz+1, ny+1, nx+1, 3) with the x index fastest; None
    means the regular grid with vertex (i, j, l) at (i/nx, j/ny, l/nz).
    """

    def __init__(self, nx: int, ny: int, nz: int, vertices: np.ndarray | None = None):
        self.n = (int(nx), int(ny), int(nz))
        if vertices is None:
            xs = [np.arange(nd + 1, dtype=np.float64) / nd for nd in self.n]
            Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
            vertices = np.stack([X, Y, Z], axis=-1)
        self.vertices = np.asarray(vertices, dtype=np.float64)
        assert self.vertices.shape == (nz + 1, ny + 1, nx + 1, 3)
        self.nelem = nx * ny * nz

    # ---- topology -------------------------------------------------------
    def coords(self, e: int):
        nx, ny, _ = self.n
        return e % nx, (e // nx) % ny, e // (nx * ny)

    def index(self, ex: int, ey: int, ez: int) -> int:
        nx, ny, _ = self.n
        return ex + nx * (ey + ny * ez)

    def neighbor(self, e: int, d: int, side: int) -> int:
        """Cell across face (d, side) of cell e, or -1 on the boundary."""
        c = list(self.coords(e))
        c[d] += 1 if side == 1 else -1
        if c[d] < 0 or c[d] >= self.n[d]:
            return -1
        return self.index(*c)

    def corners(self, e: int) -> np.ndarray:
        """The 8 vertices of cell e, corner (c0, c1, c2) at row c0 + 2 c1 + 4 c2."""
        ex, ey, ez = self.coords(e)
        out = np.empty((8, 3))
        for c in range(8):
            c0, c1, c2 = c & 1, (c >> 1) & 1, (c >> 2) & 1
            out[c] = self.vertices[ez + c2, ey + c1, ex + c0]
        return out

    # ---- geometry of the trilinear map ----------------------------------
    @staticmethod
    def _shape(xi: np.ndarray):
        """Trilinear shape functions and their reference gradients at points xi (P,3)."""
        P = xi.shape[0]
        N = np.empty((P, 8))
        dN = np.empty((P, 8, 3))
        for c in range(8):
            bits = (c & 1, (c >> 1) & 1, (c >> 2) & 1)
            f = [xi[:, d] if bits[d] else 1.0 - xi[:, d] for d in range(3)]
            df = [1.0 if bits[d] else -1.0 for d in range(3)]
            N[:, c] = f[0] * f[1] * f[2]
            dN[:, c, 0] = df[0] * f[1] * f[2]
            dN[:, c, 1] = f[0] * df[1] * f[2]
            dN[:, c, 2] = f[0] * f[1] * df[2]
        return N, dN

    def map(self, e: int, xi: np.ndarray) -> np.ndarray:
        """Physical coordinates mu_T(xi) of reference points xi (P,3)."""
        N, _ = self._shape(np.atleast_2d(xi))
        return N @ self.corners(e)

    def jacobian(self, e: int, xi: np.ndarray) -> np.ndarray:
        """J[p, a, b] = d x_a / d xi_b at reference points xi (P,3)."""
        _, dN = self._shape(np.atleast_2d(xi))
        X = self.corners(e)
        return np.einsum("pcb,ca->pab", dN, X)

    def volume(self, e: int, w3: np.ndarray, xi3: np.ndarray) -> float:
        """|T| by the given cell quadrature rule."""
        J = self.jacobian(e, xi3)
        return float(np.sum(w3 * np.abs(np.linalg.det(J))))
