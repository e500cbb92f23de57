"""dg_solve_noalloc (fixed device workspace, no allocation) against dg_solve:
the same kernels in the same order, so the solution and the solve record
must match bitwise; two calls in a row, the second on a smaller mesh."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


def _rhs(dg, mesh, c):
    xyz = dg.dg_mesh_qpoints(mesh.handle)
    fq = torch.from_numpy(workloads.sin_forcing(xyz, c)).cuda()
    b = torch.empty(mesh.ndofs, dtype=torch.float64, device="cuda")
    dg.dg_load_vector(mesh.handle, dg.DG_F64, fq, b)
    return b


def _compare(dg, mesh, b, mode, precond, kappa=None, inner=1e-5):
    x_ref = torch.zeros_like(b)
    x_na = torch.zeros_like(b)  # the same initial guess for both
    kw = dict(rtol=1e-10, inner_rtol=inner, maxit=20000, check_every=10, precond=precond, kappa=kappa)
    st1, i1 = dg.dg_solve(mesh.handle, mode, b, x_ref, **kw)
    st2, i2 = dg.dg_solve(mesh.handle, mode, b, x_na, noalloc=True, **kw)
    torch.cuda.synchronize()
    assert st1 == st2 == dg.DG_OK, (st1, st2)
    assert (i1.iterations, i1.outer) == (i2.iterations, i2.outer)
    assert i1.rel_residual == i2.rel_residual and i2.rel_residual <= 1e-10
    assert torch.equal(x_ref, x_na)
    return i2


def test_noalloc_matches_dg_solve_two_calls(gpu_lib):
    dg = gpu_lib
    # first call: Q3 8^3 (32,768 DOFs), every mode, plain and block-Jacobi
    w = workloads.WORKLOADS[2].scaled(8)
    mesh = dg.Mesh(dg.desc_from_workload(w))
    b = _rhs(dg, mesh, w.c)
    for mode, inner in ((dg.DG_SOLVE_CG_F64, 1e-5), (dg.DG_SOLVE_IR_F32, 1e-5), (dg.DG_SOLVE_RU_F32, 0.1)):
        for pc in (dg.DG_PRECOND_NONE, dg.DG_PRECOND_BLOCK_JACOBI):
            print(f"case: noalloc vs dg_solve, {w.name} n=8, mode {mode}, precond {pc}", flush=True)
            info = _compare(dg, mesh, b, mode, pc, inner=inner)
            assert info.iterations > 0
    del mesh
    # second call, smaller: Q2 4^3 (1,728 DOFs) with kappa per point (the FP32
    # modes round it into the workspace)
    w1 = workloads.WORKLOADS[1]
    desc = dg.desc_from_workload(w1)
    desc.kappa_mode = dg.DG_KAPPA_QP
    desc.kappa_face = dg.DG_KAPPA_FACE_ONE
    mesh = dg.Mesh(desc)
    kap = torch.from_numpy(workloads.lognormal(mesh.info.nqp, 5)).cuda()
    b = _rhs(dg, mesh, w1.c)
    for mode in (dg.DG_SOLVE_CG_F64, dg.DG_SOLVE_IR_F32, dg.DG_SOLVE_CG_F64):
        print(f"case: noalloc vs dg_solve, {w1.name} with kappa, mode {mode}", flush=True)
        _compare(dg, mesh, b, mode, dg.DG_PRECOND_NONE, kappa=kap)


def test_noalloc_rejects_meshes_beyond_its_workspace(gpu_lib):
    dg = gpu_lib
    # Q5 24^3: 2,985,984 DOFs, 24 bytes per DOF for FP64 CG > 64 MiB
    print("case: noalloc size limit (Q5 24^3)", flush=True)
    mesh = dg.Mesh(dg.make_desc(24, k=5))
    b = torch.ones(mesh.ndofs, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(dg.DGError) as ei:
        dg.dg_solve(mesh.handle, dg.DG_SOLVE_CG_F64, b, x, noalloc=True)
    assert ei.value.status == dg.DG_ERR_ARG
    assert "bytes of workspace" in str(ei.value)
    torch.cuda.synchronize()
    assert float(x.abs().max()) == 0.0  # no effect
