"""Pins of the oracle's DG Stokes operator (Section 5.3, eq. stokes_weak)."""
import numpy as np
import pytest

from oracle import Problem, ScalarDG, StokesDG
import workloads


def poiseuille(x):
    """Section 5.3's manufactured flow: u = (4 y (1 - y), 0, 0)."""
    return np.stack([4 * x[:, 1] * (1 - x[:, 1]), 0 * x[:, 0], 0 * x[:, 0]], axis=1)


def pressure(x):
    """... with pressure p = 8 (1 - x)."""
    return 8.0 * (1.0 - x[:, 0])


@pytest.mark.parametrize("perturb", [0.0, 0.1])
def test_poiseuille_reproduced_exactly(perturb):
    """u_I, p_I of the manufactured solution make the discrete residual vanish:
    both lie in the discrete spaces even on trilinear cells, and with m = 4 every
    integrand (cofactor of J times polynomial traces) is a polynomial of degree
    <= 7. Dirichlet on every side but x = 1 (outflow), where the Neumann condition
    grad u n - p n = 0 holds."""
    n = 3
    V = workloads.grid_vertices(n, n, n, perturb, 404) if perturb else None
    op = StokesDG(Problem(n, n, n, k=3, m=4, mask=workloads.MASK_STOKES, vertices=V))
    A = op.assemble("explicit")
    z = op.interpolate_fields(poiseuille, pressure)
    b = op.dirichlet_load(poiseuille)
    r = A.matvec(z) - b
    assert np.max(np.abs(r)) < 1e-12 * np.max(np.abs(b))


def test_stokes_symmetric_on_perturbed_mesh():
    V = workloads.grid_vertices(2, 2, 2, 0.1, 17)
    A = StokesDG(Problem(2, 2, 2, k=3, m=4, mask=0x3D, vertices=V)).assemble("explicit").to_dense()
    assert np.max(np.abs(A - A.T)) <= 1e-14 * np.max(np.abs(A))


def test_stokes_linear_divergence_free_patch():
    """A linear, divergence-free velocity with zero pressure gives zero residual on
    rows of cells away from the Dirichlet boundary (integration by parts is exact)."""
    n = (4, 3, 3)
    V = workloads.grid_vertices(*n, 0.1, 5)
    op = StokesDG(Problem(*n, k=3, m=4, mask=0x3F, vertices=V))
    z = op.interpolate_fields(lambda x: np.stack([x[:, 1], x[:, 2], x[:, 0]], axis=1), lambda x: 0 * x[:, 0])
    inner = [op.prob.mesh.index(ex, 1, 1) for ex in (1, 2)]
    r = op.apply_rows(z, inner)
    assert np.max(np.abs(r)) < 1e-13


def test_stokes_velocity_block_is_vector_sipg():
    """On the regular grid each velocity diagonal block equals the scalar SIPG block
    with c = 0 and kappa = 1."""
    pr = dict(nx=2, ny=2, nz=2, k=3, m=4, mask=0x3D)
    st = StokesDG(Problem(**pr))
    sc = ScalarDG(Problem(**pr, c=0.0))
    for e in (0, 7):
        rs, rc = st.block_row(e), sc.block_row(e)
        Nv = st.Nv
        for s_, (col, B) in rs.items():
            for c in range(3):
                blk = B[c * Nv:(c + 1) * Nv, c * Nv:(c + 1) * Nv]
                assert np.max(np.abs(blk - rc[s_][1])) < 1e-13


def test_perturbed_mesh_cells_valid_and_fill_cube():
    V = workloads.grid_vertices(4, 4, 4, 0.1, 304)
    pr = Problem(4, 4, 4, k=3, m=4, vertices=V)
    vols = [pr.cell_volume(e) for e in range(pr.nelem)]
    assert min(vols) > 0
    assert abs(sum(vols) - 1.0) < 1e-13
