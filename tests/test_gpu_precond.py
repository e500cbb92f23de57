"""GPU parity of the block-Jacobi preconditioner (the diagonal cell blocks
inverted by fast diagonalization) against the oracle's dense block solves,
and the preconditioned solvers, through the C ABI."""
import numpy as np
import pytest
import torch

import workloads
from oracle import Problem, ScalarDG, block_jacobi, pcg, problem_from_workload

pytestmark = pytest.mark.gpu

TOL64 = 1e-12      # relative L2, FP64 (the parity bar)
TOL32 = 2e-6       # relative L2, FP32: about ten times the measured 1.2-1.7e-7


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_precond(dg, desc, r, dtype=torch.float64):
    mesh = dg.Mesh(desc)
    rt = torch.from_numpy(r).to("cuda", dtype)
    zt = torch.empty_like(rt)
    dg.dg_precond_apply(mesh.handle, dg.DG_F64 if dtype == torch.float64 else dg.DG_F32, rt, zt)
    torch.cuda.synchronize()
    return zt.double().cpu().numpy()


CASES = [(k, (3, 2, 5), 0x3F, 1.0) for k in range(1, 8)] + \
        [(k, (2, 3, 1), 0x1B, 0.3) for k in range(1, 8)] + \
        [(k, (1, 1, 1), 0x3F, 2.0) for k in (1, 3, 6)] + \
        [(2, (30, 1, 2), 0x3F, 1.0),   # p = 3: 28 cells per block, a row in two blocks
         (3, (17, 2, 2), 0x2D, 0.5),   # p = 4: 16 cells per block
         (5, (9, 3, 2), 0x3F, 0.0),    # p = 6: 7 cells per block, no reaction term
         (6, (6, 2, 2), 0x17, 1.0),    # p = 7: 5 cells per block
         (7, (5, 2, 2), 0x3F, 1.0)]    # p = 8: 4 cells per block


@pytest.mark.parametrize("k,shape,mask,c", CASES)
def test_block_jacobi_matches_oracle(gpu_lib, k, shape, mask, c):
    """Every degree; rows that span several blocks of the sweep (first, middle
    and last cells of a row in different blocks); Dirichlet and natural sides."""
    dg = gpu_lib
    print(f"case: block-Jacobi k={k} shape={shape} mask={mask:#x} c={c}", flush=True)
    nx, ny, nz = shape
    N = (k + 1) ** 3
    r = workloads.uniform(nx * ny * nz * N, 2000 + k)
    z = gpu_precond(dg, dg.make_desc(nx, ny, nz, k=k, c=c, dirichlet_mask=mask), r)
    A = ScalarDG(Problem(nx, ny, nz, k=k, c=c, mask=mask)).assemble()
    ref = block_jacobi(A, r)
    assert relerr(z, ref) < TOL64


@pytest.mark.parametrize("k", [2, 3, 5])
def test_block_jacobi_fp32_error(gpu_lib, k):
    dg = gpu_lib
    shape = (5, 3, 2)
    print(f"case: block-Jacobi FP32 k={k}", flush=True)
    r = workloads.uniform(int(np.prod(shape)) * (k + 1) ** 3, 3000 + k)
    z = gpu_precond(dg, dg.make_desc(*shape, k=k), r, torch.float32)
    ref = block_jacobi(ScalarDG(Problem(*shape, k=k)).assemble(), r)
    err = relerr(z, ref)
    print(f"k={k}: FP32 block-Jacobi relative error {err:.2e}")
    assert err < TOL32


def test_block_jacobi_full_size_sampled_cells(gpu_lib):
    """Q5 on the 40^3 solve mesh at full size: the cells of a random sample of
    blocks (interior, faces, edges, corners) against the oracle's solves with
    the same cells' diagonal blocks, assembled one block row at a time."""
    dg = gpu_lib
    w = workloads.WORKLOADS[5]
    print("case: block-Jacobi Q5 40^3 sampled cells", flush=True)
    mesh = dg.Mesh(dg.desc_from_workload(w))
    N = 216
    r = torch.from_numpy(workloads.uniform(mesh.ndofs, 4001)).cuda()
    z = torch.empty_like(r)
    dg.dg_precond_apply(mesh.handle, dg.DG_F64, r, z)
    torch.cuda.synchronize()
    sdg = ScalarDG(problem_from_workload(w))
    n = w.n
    cells = [0, n - 1, n * n - 1, n ** 3 - 1, n * n * (n // 2) + n * 3 + 7]
    cells += list(np.random.default_rng(5).integers(0, n ** 3, 8))
    rh, zh = r.cpu().numpy(), z.cpu().numpy()
    for e in cells:
        e = int(e)
        B = sdg.block_row(e)[0][1]  # slot 0: (cell, diagonal block)
        ref = np.linalg.solve(B, rh[e * N:(e + 1) * N])
        assert relerr(zh[e * N:(e + 1) * N], ref) < TOL64, e


def test_unsupported_configurations(gpu_lib):
    dg = gpu_lib
    print("case: block-Jacobi unsupported", flush=True)
    r = torch.zeros(27 * 8, dtype=torch.float64, device="cuda")
    z = torch.empty_like(r)
    for desc in (dg.make_desc(2, 2, 2, k=2, theta=1.0), dg.make_desc(2, 2, 2, k=2, kappa_mode=dg.DG_KAPPA_QP)):
        mesh = dg.Mesh(desc)
        with pytest.raises(dg.DGError) as ei:
            dg.dg_precond_apply(mesh.handle, dg.DG_F64, r, z)
        assert ei.value.status == dg.DG_ERR_UNSUPPORTED
        if desc.theta == -1.0:
            b = torch.ones(mesh.ndofs, dtype=torch.float64, device="cuda")
            x = torch.zeros_like(b)
            kap = torch.ones(mesh.info.nqp, dtype=torch.float64, device="cuda")
            with pytest.raises(dg.DGError) as ei:
                dg.dg_solve(mesh.handle, 0, b, x, kappa=kap, precond=dg.DG_PRECOND_BLOCK_JACOBI)
            assert ei.value.status == dg.DG_ERR_UNSUPPORTED


def _setup(dg, w, n):
    mesh = dg.Mesh(dg.desc_from_workload(w, n=n))
    xyz = dg.dg_mesh_qpoints(mesh.handle)
    fq = torch.from_numpy(workloads.sin_forcing(xyz, w.c)).cuda()
    b = torch.empty(mesh.ndofs, dtype=torch.float64, device="cuda")
    dg.dg_load_vector(mesh.handle, dg.DG_F64, fq, b)
    return mesh, b


def test_pcg_iterations_match_oracle_pcg(gpu_lib):
    """Preconditioned FP64 CG is the oracle's PCG iteration: counts agree."""
    dg = gpu_lib
    w = workloads.WORKLOADS[5]
    n = 3
    print(f"case: PCG Q5 {n}^3 vs oracle", flush=True)
    mesh, b = _setup(dg, w, n)
    x = torch.zeros_like(b)
    st, info = dg.dg_solve(mesh.handle, 0, b, x, rtol=1e-8, check_every=1, precond=dg.DG_PRECOND_BLOCK_JACOBI)
    assert st == dg.DG_OK
    A = ScalarDG(problem_from_workload(w, n=n)).assemble()
    _, its, _ = pcg(A.matvec, lambda v: block_jacobi(A, v), b.cpu().numpy(), rtol=1e-8)
    assert abs(info.iterations - its) <= max(2, its // 50), (info.iterations, its)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_preconditioned_solves(gpu_lib, mode):
    """Every mode with the preconditioner reaches 1e-10 on the true residual,
    agrees with the unpreconditioned FP64 CG solution and needs fewer
    iterations than its unpreconditioned run."""
    dg = gpu_lib
    w = workloads.WORKLOADS[5]
    n = 8
    print(f"case: preconditioned solve mode {mode} Q5 {n}^3", flush=True)
    mesh, b = _setup(dg, w, n)
    inner = 0.1 if mode == 2 else 1e-5
    runs = {}
    for pc in (dg.DG_PRECOND_NONE, dg.DG_PRECOND_BLOCK_JACOBI):
        x = torch.zeros_like(b)
        st, info = dg.dg_solve(mesh.handle, mode, b, x, rtol=1e-10, inner_rtol=inner, maxit=50000, precond=pc)
        assert st == dg.DG_OK, dg.lib.dg_last_error()
        assert info.rel_residual <= 1e-10
        runs[pc] = (x.cpu().numpy(), info.iterations)
        print(f"mode {mode} precond {pc}: its={info.iterations} outer={info.outer} res={info.rel_residual:.2e}")
    x0, it0 = runs[dg.DG_PRECOND_NONE]
    x1, it1 = runs[dg.DG_PRECOND_BLOCK_JACOBI]
    assert relerr(x1, x0) < 1e-7
    assert it1 < it0
