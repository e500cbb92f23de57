"""GPU parity of the nonlinear diffusion operator (kappa(u) = 1 + u^2):
the Jacobian action J(u0) z at a linearization point (dg_apply_jacobian)
and the residual R(u) (dg_residual) against the oracle's full-quadrature
assembly, through the C ABI; at sizes the oracle cannot assemble, sampled
cells and the properties that hold at any size (J is the derivative of R;
R's small-u limit is the linear SIPG operator)."""
import numpy as np
import pytest
import torch

import workloads
from oracle import Problem
from oracle.nonlinear import NonlinearDG

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _mesh(dg, nx, ny, nz, k, theta=-1.0, mask=0x3F, c=1.0, problem=None):
    return dg.Mesh(dg.make_desc(nx, ny, nz, k=k, c=c, theta=theta, dirichlet_mask=mask,
                                problem=dg.DG_PROBLEM_NONLINEAR if problem is None else problem))


def _inputs(n, seed):
    # u0 and z uniform on [-1, 1): kappa(u0) in [1, 2]
    return workloads.uniform(n, seed), workloads.uniform(n, seed + 1)


CASES = [  # (nx, ny, nz, k, theta, mask, c): chunks with ragged tails along x, every side type
    (5, 3, 2, 1, -1.0, 0x3F, 1.0),
    (4, 4, 4, 2, -1.0, 0x3F, 1.0),
    (11, 3, 2, 3, 1.0, 0x2B, 0.5),
    (6, 2, 3, 4, -1.0, 0x17, 1.0),
    (3, 2, 2, 5, 1.0, 0x3F, 2.0),
    (3, 1, 2, 6, -1.0, 0x00, 1.0),
    (2, 2, 1, 7, -1.0, 0x3F, 1.0),
]


@pytest.mark.parametrize("nx,ny,nz,k,theta,mask,c", CASES)
def test_jacobian_and_residual_match_oracle(gpu_lib, nx, ny, nz, k, theta, mask, c):
    dg = gpu_lib
    print(f"case: nonlinear {nx}x{ny}x{nz} k={k} theta={theta} mask={mask:#x} c={c}", flush=True)
    op = NonlinearDG(Problem(nx, ny, nz, k=k, theta=theta, mask=mask, c=c))
    mesh = _mesh(dg, nx, ny, nz, k, theta, mask, c)
    u0, z = _inputs(mesh.ndofs, 700 + k)
    U0, Z = torch.from_numpy(u0).cuda(), torch.from_numpy(z).cuda()
    y = torch.empty_like(U0)
    dg.dg_apply_jacobian(mesh.handle, dg.DG_F64, U0, Z, y)
    r = torch.empty_like(U0)
    dg.dg_residual(mesh.handle, dg.DG_F64, U0, r)
    torch.cuda.synchronize()
    e_j = relerr(y.cpu().numpy(), op.jacobian(u0).matvec(z))
    e_r = relerr(r.cpu().numpy(), op.residual(u0))
    print(f"J z rel {e_j:.2e}, R rel {e_r:.2e}")
    assert e_j <= TOL64 and e_r <= TOL64
    # u0 and z may be the same vector
    dg.dg_apply_jacobian(mesh.handle, dg.DG_F64, U0, U0, y)
    torch.cuda.synchronize()
    assert relerr(y.cpu().numpy(), op.jacobian(u0).matvec(u0)) <= TOL64


def test_fp32_error(gpu_lib):
    dg = gpu_lib
    op = NonlinearDG(Problem(6, 5, 4, k=3))
    mesh = _mesh(dg, 6, 5, 4, 3)
    u0, z = _inputs(mesh.ndofs, 711)
    y = torch.empty(mesh.ndofs, dtype=torch.float32, device="cuda")
    dg.dg_apply_jacobian(mesh.handle, dg.DG_F32, torch.from_numpy(u0).float().cuda(),
                         torch.from_numpy(z).float().cuda(), y)
    r = torch.empty_like(y)
    dg.dg_residual(mesh.handle, dg.DG_F32, torch.from_numpy(u0).float().cuda(), r)
    torch.cuda.synchronize()
    e_j = relerr(y.double().cpu().numpy(), op.jacobian(u0).matvec(z))
    e_r = relerr(r.double().cpu().numpy(), op.residual(u0))
    print(f"FP32: J z rel {e_j:.2e}, R rel {e_r:.2e}")
    assert e_j <= 2e-6 and e_r <= 2e-6


def test_sampled_cells_at_32cube(gpu_lib):
    """Q3 on 32^3 (2,097,152 DOFs): 512 sampled cells (corners, edges, faces and
    random interior cells) of J(u0) z and R(u0) against the oracle's rows,
    elementwise."""
    dg = gpu_lib
    n, k = 32, 3
    mesh = _mesh(dg, n, n, n, k)
    u0, z = _inputs(mesh.ndofs, 720)
    U0, Z = torch.from_numpy(u0).cuda(), torch.from_numpy(z).cuda()
    y = torch.empty_like(U0)
    r = torch.empty_like(U0)
    dg.dg_apply_jacobian(mesh.handle, dg.DG_F64, U0, Z, y)
    dg.dg_residual(mesh.handle, dg.DG_F64, U0, r)
    torch.cuda.synchronize()
    N = (k + 1) ** 3
    Y, Rg = y.cpu().numpy().reshape(-1, N), r.cpu().numpy().reshape(-1, N)
    rng = np.random.default_rng(5)
    fixed = [0, n - 1, n * n - 1, n ** 3 - 1, n ** 3 - n, n * (n - 1), (n // 2) * (1 + n + n * n)]
    cells = np.unique(np.concatenate([fixed, rng.choice(n ** 3, 505, replace=False)]))[:512]
    op = NonlinearDG(Problem(n, n, n, k=k))
    Jr = op.jacobian_rows(u0, z, cells)
    Rr = op.residual(u0, elems=cells)
    for got, ref in ((Y[cells], Jr), (Rg[cells], Rr)):
        assert relerr(got, ref) <= TOL64
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_jacobian_is_the_derivative_of_the_gpu_residual(gpu_lib):
    """At a size the oracle cannot assemble (Q4 on 24^3, 1,728,000 DOFs): the
    central difference D(t) of the GPU residual along z is J z + t^2 C
    exactly (R is cubic along a line), so (4 D(t) - D(2t)) / 3 = J(u0) z."""
    dg = gpu_lib
    mesh = _mesh(dg, 24, 24, 24, 4, theta=1.0, mask=0x2F)
    u0, z = _inputs(mesh.ndofs, 730)
    U0, Z = torch.from_numpy(u0).cuda(), torch.from_numpy(z).cuda()

    def R(v):
        out = torch.empty_like(v)
        dg.dg_residual(mesh.handle, dg.DG_F64, v, out)
        return out

    def D(t):
        return (R(U0 + t * Z) - R(U0 - t * Z)) / (2 * t)

    t = 1e-2
    fd = (4 * D(t) - D(2 * t)) / 3
    y = torch.empty_like(U0)
    dg.dg_apply_jacobian(mesh.handle, dg.DG_F64, U0, Z, y)
    torch.cuda.synchronize()
    err = float(torch.linalg.norm(fd - y) / torch.linalg.norm(y))
    print(f"Richardson FD vs J z: {err:.2e}")
    assert err <= 1e-10


def test_small_u_limit_is_the_linear_operator_on_gpu(gpu_lib):
    """R is odd in u: (8 R(eps u) - R(2 eps u)) / (6 eps) is the kappa = 1 SIPG
    apply of the linear library path (dg_apply on a DG_PROBLEM_DIFFREAC mesh)."""
    dg = gpu_lib
    n, k = 20, 5
    mesh = _mesh(dg, n, n, n, k)
    lin = _mesh(dg, n, n, n, k, problem=dg.DG_PROBLEM_DIFFREAC)
    u = torch.from_numpy(workloads.uniform(mesh.ndofs, 740)).cuda()
    eps = 0.05
    r1, r2, Au = torch.empty_like(u), torch.empty_like(u), torch.empty_like(u)
    dg.dg_residual(mesh.handle, dg.DG_F64, eps * u, r1)
    dg.dg_residual(mesh.handle, dg.DG_F64, 2 * eps * u, r2)
    dg.dg_apply(lin.handle, dg.DG_F64, u, Au)
    torch.cuda.synchronize()
    lim = (8 * r1 - r2) / (6 * eps)
    err = float(torch.linalg.norm(lim - Au) / torch.linalg.norm(Au))
    print(f"small-u limit vs linear apply: {err:.2e}")
    assert err <= 1e-11


def test_rejections(gpu_lib):
    dg = gpu_lib
    mesh = _mesh(dg, 2, 2, 2, 2)
    x = torch.zeros(mesh.ndofs, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for call in (lambda: dg.dg_apply(mesh.handle, dg.DG_F64, x, y),
                 lambda: dg.dg_precond_apply(mesh.handle, dg.DG_F64, x, y),
                 lambda: dg.dg_apply_adjoint(mesh.handle, dg.DG_F64, x, None, None, y)):
        with pytest.raises(dg.DGError) as ei:
            call()
        assert ei.value.status == dg.DG_ERR_UNSUPPORTED
    with pytest.raises(dg.DGError) as ei:
        dg.dg_solve(mesh.handle, dg.DG_SOLVE_CG_F64, x, y)
    assert ei.value.status == dg.DG_ERR_UNSUPPORTED
    with pytest.raises(dg.DGError) as ei:
        dg.dg_apply_jacobian(mesh.handle, dg.DG_F64, x, x, x)
    assert ei.value.status == dg.DG_ERR_ARG
    lin = _mesh(dg, 2, 2, 2, 2, problem=dg.DG_PROBLEM_DIFFREAC)
    with pytest.raises(dg.DGError) as ei:
        dg.dg_apply_jacobian(lin.handle, dg.DG_F64, x, x, y)
    assert ei.value.status == dg.DG_ERR_UNSUPPORTED
