"""Variant selection of the apply (dg_mesh_set_variant, dg_mesh_tune): every
candidate computes the same operator. The matrix-core variants (rows per
wavefront) agree bitwise among themselves, as do the two sweep orders of the
line kernels; both families match the oracle; tuning keeps the fastest."""
import numpy as np
import pytest
import torch

import workloads
from oracle import ScalarDG, problem_from_workload

pytestmark = pytest.mark.gpu


def _x(w, n, dt):
    return torch.from_numpy(workloads.inputs(w.scaled(n), "x")).to("cuda", dt)


@pytest.mark.parametrize("prec", [0, 1])
def test_q3_variants_agree(gpu_lib, prec):
    dg = gpu_lib
    w = workloads.WORKLOADS[2]
    n = 9  # ragged chunks of 4 cells along x, rows not a multiple of the march lengths
    print(f"case: Q3 variants {n}^3 precision {prec}", flush=True)
    mesh = dg.Mesh(dg.desc_from_workload(w, n=n))
    dt = torch.float64 if prec == 0 else torch.float32
    x = _x(w, n, dt)
    outs = {}
    cands = [(0, 1), (0, 2), (0, 4), (0, 8), (1, 0), (1, 1)]
    if prec == 1:  # the FP32 line kernel with its contractions on the matrix cores
        cands += [(1, 2), (1, 3)]
    for kind, param in cands:
        dg.dg_mesh_set_variant(mesh.handle, prec, kind, param)
        y = torch.empty_like(x)
        dg.dg_apply(mesh.handle, prec, x, y)
        torch.cuda.synchronize()
        outs[(kind, param)] = y.cpu().numpy()
    for r in (2, 4, 8):
        assert np.array_equal(outs[(0, r)], outs[(0, 1)]), r
    assert np.array_equal(outs[(1, 1)], outs[(1, 0)])
    keys = [(0, 1), (1, 0)]
    if prec == 1:
        assert np.array_equal(outs[(1, 3)], outs[(1, 2)])
        assert not np.array_equal(outs[(1, 2)], outs[(1, 0)])  # FP32 matrix-core products, not VALU
        keys.append((1, 2))
    ref = ScalarDG(problem_from_workload(w, n=n)).assemble().matvec(x.double().cpu().numpy())
    tol = 1e-12 if prec == 0 else 2e-6
    for key in keys:
        err = np.linalg.norm(outs[key] - ref) / np.linalg.norm(ref)
        print(key, f"{err:.2e}")
        assert err <= tol, (key, err)


def test_tune_q3_keeps_the_fastest(gpu_lib):
    dg = gpu_lib
    w = workloads.WORKLOADS[2]
    n = 16
    print(f"case: tune Q3 {n}^3", flush=True)
    mesh = dg.Mesh(dg.desc_from_workload(w, n=n))
    x = _x(w, n, torch.float64)
    y0 = torch.empty_like(x)
    dg.dg_apply(mesh.handle, 0, x, y0)
    cands, chosen = dg.dg_mesh_tune(mesh.handle, 0, trials=3)
    print(cands, chosen)
    kinds = [(k, p) for k, p, _ in cands]
    # the cost model's default (1 row at 16^3: too few wavefronts for longer
    # marches) first, the other march lengths, then the two line sweeps
    assert kinds == [(0, 1), (0, 2), (0, 4), (0, 8), (0, 16), (1, 0), (1, 1)]
    us = [t for _, _, t in cands]
    assert all(t > 0 for t in us)
    assert chosen == int(np.argmin(us))
    y1 = torch.empty_like(x)
    dg.dg_apply(mesh.handle, 0, x, y1)
    k, p, _ = cands[chosen]
    dg.dg_mesh_set_variant(mesh.handle, 0, k, p)
    y2 = torch.empty_like(x)
    dg.dg_apply(mesh.handle, 0, x, y2)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
    rel = float(torch.linalg.norm(y1 - y0) / torch.linalg.norm(y0))
    assert rel <= 1e-13


@pytest.mark.parametrize("wid", [4, 5])
def test_line_sweeps_bitwise_equal(gpu_lib, wid):
    """The sweep order changes which XCD runs a block, not what it computes:
    apply, adjoint (with dL/dkappa) and preconditioner agree bitwise."""
    dg = gpu_lib
    w = workloads.WORKLOADS[wid]
    n = 7
    print(f"case: line sweeps {w.name} {n}^3", flush=True)
    mesh = dg.Mesh(dg.desc_from_workload(w, n=n))
    x = _x(w, n, torch.float64)
    kap = None
    if w.kappa_mode:
        kap = torch.from_numpy(workloads.inputs(w.scaled(n), "kappa")).cuda()
    res = []
    for sweep in (0, 1, 0):
        dg.dg_mesh_set_variant(mesh.handle, 0, 1, sweep)
        y = torch.empty_like(x)
        dg.dg_apply(mesh.handle, 0, x, y, kap)
        out = [y]
        if kap is not None:
            g = torch.empty_like(x)
            dk = torch.empty_like(kap)
            dg.dg_apply_adjoint(mesh.handle, 0, x, x, kap, g, dk)
            out += [g, dk]
        else:
            z = torch.empty_like(x)
            dg.dg_precond_apply(mesh.handle, 0, x, z)
            out.append(z)
        torch.cuda.synchronize()
        res.append([t.cpu() for t in out])
    for a, b in zip(res[0], res[1]):
        assert torch.equal(a, b)
    for a, b in zip(res[0], res[2]):
        assert torch.equal(a, b)
    cands, chosen = dg.dg_mesh_tune(mesh.handle, 0, trials=2)
    assert [(k, p) for k, p, _ in cands] == [(1, 0), (1, 1)]


def test_solve_after_variant_change(gpu_lib):
    dg = gpu_lib
    w = workloads.WORKLOADS[5]
    mesh = dg.Mesh(dg.desc_from_workload(w, n=4))
    xyz = dg.dg_mesh_qpoints(mesh.handle)
    fq = torch.from_numpy(workloads.sin_forcing(xyz, w.c)).cuda()
    b = torch.empty(mesh.ndofs, dtype=torch.float64, device="cuda")
    dg.dg_load_vector(mesh.handle, dg.DG_F64, fq, b)
    xs = []
    for sweep in (0, 1):
        dg.dg_mesh_set_variant(mesh.handle, 0, 1, sweep)
        dg.dg_mesh_set_variant(mesh.handle, 1, 1, sweep)
        x = torch.zeros_like(b)
        st, info = dg.dg_solve(mesh.handle, dg.DG_SOLVE_CHEB_F32, b, x, precond=dg.DG_PRECOND_BLOCK_JACOBI)
        assert st == dg.DG_OK and info.rel_residual <= 1e-10
        xs.append(x)
    assert torch.equal(xs[0], xs[1])


def test_set_variant_rejects(gpu_lib):
    dg = gpu_lib
    mesh = dg.Mesh(dg.desc_from_workload(workloads.WORKLOADS[2], n=4))
    for kind, param in ((0, 3), (0, 32), (0, 0), (2, 0), (1, 2)):
        with pytest.raises(dg.DGError) as ei:
            dg.dg_mesh_set_variant(mesh.handle, 0, kind, param)
        assert ei.value.status == dg.DG_ERR_ARG
    m5 = dg.Mesh(dg.desc_from_workload(workloads.WORKLOADS[5], n=2))
    with pytest.raises(dg.DGError):
        dg.dg_mesh_set_variant(m5.handle, 0, 0, 1)  # no matrix-core kernel at k = 5
    ms = dg.Mesh(dg.desc_from_workload(workloads.WORKLOADS[3], n=2))
    with pytest.raises(dg.DGError) as ei:
        dg.dg_mesh_tune(ms.handle, 0)
    assert ei.value.status == dg.DG_ERR_UNSUPPORTED


def test_tune_q3_fp32_candidates(gpu_lib):
    """FP32 at k = 3: the matrix-core kernel (FP64 products on FP32 vectors),
    and the line kernel with FP32 VALU or FP32 matrix-core contractions."""
    dg = gpu_lib
    w = workloads.WORKLOADS[2]
    mesh = dg.Mesh(dg.desc_from_workload(w, n=16))
    cands, chosen = dg.dg_mesh_tune(mesh.handle, 1, trials=3)
    print(cands, chosen)
    assert [(k, p) for k, p, _ in cands] == [(0, 1), (0, 2), (0, 4), (0, 8), (0, 16), (1, 0), (1, 1), (1, 2), (1, 3)]
    assert chosen == int(np.argmin([t for _, _, t in cands]))


def test_fp32_kappa_lines_on_matrix_cores(gpu_lib):
    """kappa per point at k = 3 in FP32 runs the line kernel; with its
    contractions on the matrix cores it stays within FP32 accuracy of the
    oracle (kappa traces on the faces)."""
    dg = gpu_lib
    w = workloads.WORKLOADS[4]
    n = 5
    desc = dg.desc_from_workload(w, n=n)
    desc.k = 3
    desc.m = 0
    mesh = dg.Mesh(desc)
    nq = mesh.info.nqp
    kap = workloads.lognormal(nq, 17)
    x = workloads.uniform(mesh.ndofs, 18)
    from oracle import Problem, ScalarDG as SDG
    ref = SDG(Problem(n, n, n, k=3, kappa=kap)).assemble("explicit").matvec(x)
    res = {}
    for param in (0, 2):
        dg.dg_mesh_set_variant(mesh.handle, 1, 1, param)
        y = torch.empty(mesh.ndofs, dtype=torch.float32, device="cuda")
        dg.dg_apply(mesh.handle, 1, torch.from_numpy(x).float().cuda(), y, torch.from_numpy(kap).float().cuda())
        torch.cuda.synchronize()
        res[param] = np.linalg.norm(y.double().cpu().numpy() - ref) / np.linalg.norm(ref)
        print(param, res[param])
    assert res[0] <= 2e-6 and res[2] <= 2e-6
