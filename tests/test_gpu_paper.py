"""GPU parity of Section 5.2's benchmark operator (K(x) = x x^T + I at every
quadrature point, c = 10, f = -6, g = |x|^2; eq. diffreac_weak) against the
oracle's full-quadrature assembly with the same tensor, through the C ABI:
the Jacobian action (dg_apply), its transpose (dg_apply_adjoint) and the full
residual with the source and Dirichlet data terms (dg_residual)."""
import numpy as np
import pytest
import torch

import workloads
from oracle import Problem, ScalarDG

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def K_paper(x):
    return np.einsum("pa,pb->pab", x, x) + np.eye(3)[None]


def f_paper(x):
    return -6.0 * np.ones(len(x))


def g_paper(x):
    return (x * x).sum(1)


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _oracle(nx, ny, nz, k, theta=-1.0, mask=0x3F, c=10.0):
    return ScalarDG(Problem(nx, ny, nz, k=k, c=c, theta=theta, mask=mask, kappa_tensor=K_paper))


def _mesh(dg, nx, ny, nz, k, theta=-1.0, mask=0x3F, c=10.0):
    return dg.Mesh(dg.make_desc(nx, ny, nz, k=k, c=c, theta=theta, dirichlet_mask=mask,
                                problem=dg.DG_PROBLEM_DIFFREAC_PAPER))


CASES = [  # (nx, ny, nz, k, theta, mask): several chunks with ragged tails along x
    (4, 4, 4, 2, -1.0, 0x3F),
    (11, 3, 2, 3, -1.0, 0x3F),
    (9, 2, 3, 3, 1.0, 0x2B),
    (6, 2, 2, 4, -1.0, 0x3F),
    (3, 2, 2, 5, 1.0, 0x17),
    (3, 1, 2, 6, -1.0, 0x3F),
    (5, 2, 1, 1, -1.0, 0x3F),
]


@pytest.mark.parametrize("nx,ny,nz,k,theta,mask", CASES)
def test_paper_operator_apply_and_transpose(gpu_lib, nx, ny, nz, k, theta, mask):
    dg = gpu_lib
    print(f"case: paper operator {nx}x{ny}x{nz} k={k} theta={theta} mask={mask:#x}", flush=True)
    op = _oracle(nx, ny, nz, k, theta, mask)
    A = op.assemble("explicit")
    mesh = _mesh(dg, nx, ny, nz, k, theta, mask)
    x = workloads.uniform(mesh.ndofs, 501 + k)
    g = workloads.uniform(mesh.ndofs, 502 + k)
    xt, gt = torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda()
    y = mesh.apply(xt)
    ATg, _ = mesh.apply_adjoint(gt, want_dkappa=False)
    torch.cuda.synchronize()
    assert relerr(y.cpu().numpy(), A.matvec(x)) < TOL64
    assert relerr(ATg.cpu().numpy(), A.rmatvec(g)) < TOL64
    # FP32: the same operator with FP32 vectors and arithmetic
    y32 = mesh.apply(xt.float())
    torch.cuda.synchronize()
    assert relerr(y32.double().cpu().numpy(), A.matvec(x)) < 1e-4


@pytest.mark.parametrize("nx,ny,nz,k", [(4, 4, 4, 2), (5, 3, 2, 3), (2, 3, 2, 5)])
def test_paper_residual(gpu_lib, nx, ny, nz, k):
    """dg_residual = A u - b with b the source f = -6 and the Dirichlet data
    g = |x|^2 of eq. diffreac_weak (the oracle's load vector)."""
    dg = gpu_lib
    print(f"case: paper residual {nx}x{ny}x{nz} k={k}", flush=True)
    op = _oracle(nx, ny, nz, k)
    A = op.assemble("explicit")
    b = op.load_vector(f_paper, g_paper)
    mesh = _mesh(dg, nx, ny, nz, k)
    u = workloads.uniform(mesh.ndofs, 601)
    r = torch.empty(mesh.ndofs, dtype=torch.float64, device="cuda")
    dg.dg_residual(mesh.handle, dg.DG_F64, torch.from_numpy(u).cuda(), r)
    torch.cuda.synchronize()
    ref = A.matvec(u) - b
    assert relerr(r.cpu().numpy(), ref) < TOL64
    # the manufactured solution |x|^2 (in Q_k, every integrand exact at m = k + 1
    # for k >= 2) makes the residual of its interpolant vanish
    uI = op.interpolate(g_paper)
    dg.dg_residual(mesh.handle, dg.DG_F64, torch.from_numpy(uI).cuda(), r)
    torch.cuda.synchronize()
    assert float(r.abs().max()) < 1e-11 * float(np.abs(b).max())


def test_paper_q3_64cube_sampled_rows(gpu_lib):
    """The benchmark size: Q3 on 64^3 cells, 16.8M DOFs; rows of 64 cells
    (corners, faces, interior, random) against the oracle's block rows."""
    dg = gpu_lib
    n, k = 64, 3
    print("case: paper operator Q3 64^3 sampled rows", flush=True)
    mesh = _mesh(dg, n, n, n, k)
    x = workloads.uniform(mesh.ndofs, 701)
    xt = torch.from_numpy(x).cuda()
    y = mesh.apply(xt)
    r = torch.empty_like(xt)
    dg.dg_residual(mesh.handle, dg.DG_F64, xt, r)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    last = n ** 3 - 1
    elems = [0, n - 1, n * n - 1, last, n ** 3 // 2 + n // 2, n * n * 5 + n * 7] + list(rng.choice(n ** 3, 58,
                                                                                                    replace=False))
    op = _oracle(n, n, n, k)
    N = (k + 1) ** 3
    Y = y.cpu().numpy().reshape(-1, N)[elems]
    ref = op.apply_rows(x, elems)
    assert relerr(Y, ref) < TOL64
    assert np.max(np.abs(Y - ref)) < 1e-12 * np.max(np.abs(ref))
    # residual rows: A x - b on the same cells
    R = r.cpu().numpy().reshape(-1, N)[elems]
    assert relerr(R, ref - op.load_rows(f_paper, g_paper, elems)) < TOL64


def test_paper_deterministic(gpu_lib):
    dg = gpu_lib
    mesh = _mesh(dg, 12, 5, 4, 3)
    x = torch.from_numpy(workloads.uniform(mesh.ndofs, 9)).cuda()
    assert torch.equal(mesh.apply(x), mesh.apply(x))
