"""GPU parity of the DG Stokes apply (trilinear cells) against the oracle."""
import numpy as np
import pytest
import torch

import workloads
from oracle import Problem, StokesDG, problem_from_workload

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_apply(dg, desc, x):
    mesh = dg.Mesh(desc)
    y = mesh.apply(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    return mesh, y.cpu().numpy()


@pytest.mark.parametrize("k,shape,perturb,mask,theta", [
    (3, (3, 3, 3), 0.1, 0x3D, -1.0),
    (3, (2, 3, 2), 0.0, 0x3F, -1.0),
    (2, (3, 2, 2), 0.1, 0x3D, 1.0),
    (3, (1, 1, 2), 0.1, 0x15, -1.0),
])
def test_stokes_matches_oracle(gpu_lib, k, shape, perturb, mask, theta):
    dg = gpu_lib
    print(f"case: stokes k={k} shape={shape} perturb={perturb} mask={mask:#x}", flush=True)
    V = workloads.grid_vertices(*shape, perturb, 900 + k) if perturb else None
    NB = 3 * (k + 1) ** 3 + k ** 3
    E = shape[0] * shape[1] * shape[2]
    x = workloads.uniform(E * NB, 77)
    desc = dg.make_desc(*shape, k=k, problem=dg.DG_PROBLEM_STOKES, theta=theta, dirichlet_mask=mask, vertices=V)
    _, y = gpu_apply(dg, desc, x)
    op = StokesDG(Problem(*shape, k=k, theta=theta, mask=mask, vertices=V))
    ref = op.assemble("explicit").matvec(x)
    assert relerr(y, ref) < TOL64


def test_stokes_poiseuille_residual(gpu_lib):
    """A applied to the interpolated manufactured flow equals the Dirichlet data
    vector (Section 5.3's solution is reproduced exactly)."""
    dg = gpu_lib
    n = 4
    V = workloads.grid_vertices(n, n, n, 0.1, 31)
    op = StokesDG(Problem(n, n, n, k=3, mask=0x3D, vertices=V))
    uex = lambda x: np.stack([4 * x[:, 1] * (1 - x[:, 1]), 0 * x[:, 0], 0 * x[:, 0]], axis=1)
    z = op.interpolate_fields(uex, lambda x: 8.0 * (1.0 - x[:, 0]))
    b = op.dirichlet_load(uex)
    desc = dg.make_desc(n, k=3, problem=dg.DG_PROBLEM_STOKES, dirichlet_mask=0x3D, vertices=V)
    _, y = gpu_apply(dg, desc, z)
    assert np.max(np.abs(y - b)) < 1e-11 * np.max(np.abs(b))


def test_stokes_full_size_sampled_rows(gpu_lib):
    """The 32^3 perturbed Q3/Q2 workload at full size, 512 sampled cells
    (corners, edges, faces, the Neumann side and random interior cells; oracle
    rows in worker processes), relative L2 and elementwise."""
    from oracle_pool import rows
    dg = gpu_lib
    w = workloads.WORKLOADS[3]
    print("case: stokes 32^3 sampled rows", flush=True)
    x = workloads.inputs(w, "x")
    mesh, y = gpu_apply(dg, dg.desc_from_workload(w), x)
    n, E = w.n, w.nelem
    rng = np.random.default_rng(3)
    fixed = [0, n - 1, n * n - 1, E - 1, E - n, n * (n - 1), 31, 32 * 32 * 16, (n // 2) * (1 + n + n * n)]
    cells = np.unique(np.concatenate([fixed, rng.choice(E, 520, replace=False)]))[:512]
    (ref,) = rows("stokes", 3, cells)
    N = w.dofs_per_elem
    got = y.reshape(-1, N)[cells]
    assert relerr(got, ref) < TOL64
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_stokes_deterministic(gpu_lib):
    dg = gpu_lib
    w = workloads.WORKLOADS[3].scaled(6)
    mesh = dg.Mesh(dg.desc_from_workload(w))
    x = torch.from_numpy(workloads.inputs(w, "x")).cuda()
    assert torch.equal(mesh.apply(x), mesh.apply(x))


def test_stokes_fp32_unsupported(gpu_lib):
    dg = gpu_lib
    w = workloads.WORKLOADS[3].scaled(2)
    mesh = dg.Mesh(dg.desc_from_workload(w))
    x = torch.zeros(mesh.ndofs, dtype=torch.float32, device="cuda")
    with pytest.raises(dg.DGError):
        mesh.apply(x)


def test_stokes_flop_model_uses_the_sum_factorization_cost(gpu_lib):
    """The library's flop model of the Stokes apply counts the pressure
    interpolation forward and back with the paper's sum-factorization cost
    (eq. sumfactcost: 888 flops for 4 x 3 per direction)."""
    from oracle.cost import sumfact_cost
    dg = gpu_lib
    w = workloads.WORKLOADS[3].scaled(2)
    mesh = dg.Mesh(dg.desc_from_workload(w))
    p, kp, E = w.p, w.k, w.nelem
    csf = sumfact_cost((p, p, p), (kp, kp, kp))
    assert csf == 888
    face = 3 * (10 * p ** 3) + 60 * p * p
    assert mesh.info.flops_apply == E * (18 * p ** 4 + 2 * csf + 220 * p ** 3 + 6 * face)
