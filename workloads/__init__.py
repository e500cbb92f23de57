"""Seeded synthetic inputs for the sum-factorized DG operator workloads.

This module is shared by the CPU oracle and the HIP path. It holds only the
workload parameters (mesh size, polynomial degree, coefficients) and seeded
random draws. It holds none of the discretization's arithmetic: no quadrature,
no basis, no geometry beyond placing mesh vertices.

Seeds: ``100 * workload + role`` with roles x=0, kappa=1, g=2, u=3, mesh=4.
Random vectors come from ``torch.Generator('cpu')`` so that every machine
produces the same bits.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

ROLES = {"x": 0, "kappa": 1, "g": 2, "u": 3, "mesh": 4}

PROBLEM_SCALAR = 0
PROBLEM_STOKES = 1

# Boundary sides in the order (-x, +x, -y, +y, -z, +z); bit f of a mask marks
# side f as Dirichlet (Nitsche terms); the other sides carry natural
# (Neumann) conditions and contribute nothing to the operator.
MASK_ALL = 0x3F
MASK_STOKES = 0x3D  # every side but x = 1 (the outflow side of the channel)


@dataclasses.dataclass(frozen=True)
class Workload:
    """Parameters of one operator workload (a structured mesh of the unit cube)."""

    wid: int
    name: str
    problem: int
    k: int                 # polynomial degree (velocity degree for Stokes)
    m: int                 # Gauss-Legendre points per direction
    n: int                 # elements per direction (n^3 hexahedra)
    c: float = 1.0         # reaction coefficient
    alpha: float = 3.0     # penalty parameter
    theta: float = -1.0    # -1: symmetric interior penalty
    penalty_form: int = 0  # 0: alpha k(k+1)|F|/min|T|, 1: alpha k(k+d-1)|F|/min|T|
    mask: int = MASK_ALL
    perturb: float = 0.0   # max interior vertex displacement per coordinate, in units of h
    kappa_mode: int = 0    # 0: kappa = 1, 1: kappa given per volume quadrature point

    @property
    def p(self) -> int:
        return self.k + 1

    @property
    def nelem(self) -> int:
        return self.n ** 3

    @property
    def dofs_per_elem(self) -> int:
        if self.problem == PROBLEM_STOKES:
            return 3 * self.p ** 3 + self.k ** 3
        return self.p ** 3

    @property
    def ndofs(self) -> int:
        return self.nelem * self.dofs_per_elem

    def scaled(self, n: int) -> "Workload":
        """Same operator on an n^3 mesh (smaller copies for full-vector checks)."""
        return dataclasses.replace(self, n=n)

    def seed(self, role: str) -> int:
        return 100 * self.wid + ROLES[role]


WORKLOADS = {
    1: Workload(1, "diffreac_q2_4cube", PROBLEM_SCALAR, k=2, m=3, n=4),
    2: Workload(2, "diffreac_q3_64cube", PROBLEM_SCALAR, k=3, m=4, n=64),
    3: Workload(3, "stokes_q3q2_32cube_perturbed", PROBLEM_STOKES, k=3, m=4, n=32,
                mask=MASK_STOKES, perturb=0.1),
    4: Workload(4, "diffreac_q4_48cube_kappa", PROBLEM_SCALAR, k=4, m=5, n=48, kappa_mode=1),
    5: Workload(5, "diffreac_q5_40cube_solve", PROBLEM_SCALAR, k=5, m=6, n=40),
}


def _gen(seed: int) -> torch.Generator:
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed))
    return g


def uniform(n: int, seed: int) -> np.ndarray:
    """n float64 values uniform on [-1, 1)."""
    return (torch.rand(int(n), dtype=torch.float64, generator=_gen(seed)) * 2.0 - 1.0).numpy()


def lognormal(n: int, seed: int, sigma: float = 0.5) -> np.ndarray:
    """n float64 values exp(sigma * N(0, 1))."""
    z = torch.randn(int(n), dtype=torch.float64, generator=_gen(seed))
    return torch.exp(z * sigma).numpy()


def grid_vertices(nx: int, ny: int, nz: int, perturb: float = 0.0, seed: int = 0) -> np.ndarray:
    """Vertex coordinates of a structured nx*ny*nz hexahedral mesh of [0,1]^3.

    Returns an array of shape (nz+1, ny+1, nx+1, 3), i.e. vertex (i, j, l) with
    x-index i fastest lives at flat index i + (nx+1)*(j + (ny+1)*l). Interior
    vertices are displaced by independent uniform draws in
    [-perturb*h_d, perturb*h_d] per coordinate d; boundary vertices stay put so
    the domain remains the unit cube.
    """
    xs = [np.arange(nd + 1, dtype=np.float64) / nd for nd in (nx, ny, nz)]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    V = np.stack([X, Y, Z], axis=-1)
    if perturb > 0.0:
        d = uniform(V.size, seed).reshape(V.shape)
        h = np.array([1.0 / nx, 1.0 / ny, 1.0 / nz])
        interior = np.zeros(V.shape[:3], dtype=bool)
        interior[1:-1, 1:-1, 1:-1] = True
        V = V + np.where(interior[..., None], d * perturb * h, 0.0)
    return np.ascontiguousarray(V)


def inputs(w: Workload, role: str, n: int | None = None) -> np.ndarray:
    """The seeded input vector of a workload for a role ('x', 'g', 'u', 'kappa')."""
    if role == "kappa":
        count = w.nelem * w.m ** 3 if n is None else n
        return lognormal(count, w.seed("kappa"))
    count = w.ndofs if n is None else n
    return uniform(count, w.seed(role))


def vertices(w: Workload) -> np.ndarray | None:
    """Perturbed vertex coordinates of a workload, or None for the regular grid."""
    if w.perturb == 0.0:
        return None
    return grid_vertices(w.n, w.n, w.n, w.perturb, w.seed("mesh"))


def sin_solution(xyz: np.ndarray) -> np.ndarray:
    """Manufactured solution u = sin(pi x) sin(pi y) sin(pi z) of the solve workload."""
    return np.sin(math.pi * xyz[..., 0]) * np.sin(math.pi * xyz[..., 1]) * np.sin(math.pi * xyz[..., 2])


def sin_forcing(xyz: np.ndarray, c: float = 1.0) -> np.ndarray:
    """f = -Laplace(u) + c u for u = sin(pi x) sin(pi y) sin(pi z)."""
    return (3.0 * math.pi ** 2 + c) * sin_solution(xyz)
