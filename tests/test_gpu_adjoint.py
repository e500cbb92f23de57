"""GPU parity of the adjoint (A^T g and dL/dkappa for L = g^T A(kappa) u)."""
import numpy as np
import pytest
import torch

import workloads
from oracle import Problem, ScalarDG, problem_from_workload

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def cuda(a, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)


@pytest.mark.parametrize("theta", [-1.0, 1.0])
@pytest.mark.parametrize("face_one", [False, True])
@pytest.mark.parametrize("k,shape,mask", [(4, (3, 3, 3), 0x3F), (2, (4, 2, 3), 0x2D), (3, (1, 2, 1), 0x3F)])
def test_adjoint_matches_oracle(gpu_lib, theta, face_one, k, shape, mask):
    dg = gpu_lib
    print(f"case: adjoint k={k} shape={shape} theta={theta} face_one={face_one}", flush=True)
    N, M = (k + 1) ** 3, (k + 1) ** 3
    E = shape[0] * shape[1] * shape[2]
    kap = workloads.lognormal(E * M, 401)
    u = workloads.uniform(E * N, 403)
    g = workloads.uniform(E * N, 402)
    desc = dg.make_desc(*shape, k=k, theta=theta, dirichlet_mask=mask, kappa_mode=dg.DG_KAPPA_QP,
                        kappa_face=dg.DG_KAPPA_FACE_ONE if face_one else dg.DG_KAPPA_FACE_TRACE)
    mesh = dg.Mesh(desc)
    ATg, dk = mesh.apply_adjoint(cuda(g), cuda(u), cuda(kap))
    torch.cuda.synchronize()
    op = ScalarDG(Problem(*shape, k=k, theta=theta, mask=mask, kappa=kap, kappa_face_one=face_one))
    A = op.assemble("explicit")
    assert relerr(ATg.cpu().numpy(), A.rmatvec(g)) < TOL64
    assert relerr(dk.cpu().numpy(), op.kappa_gradient(u, g).reshape(-1)) < TOL64


def test_adjoint_without_kappa(gpu_lib):
    """kappa = 1 mode: dkappa is still the derivative at kappa = 1."""
    dg = gpu_lib
    k, n = 3, 3
    u = workloads.uniform(n ** 3 * 64, 1)
    g = workloads.uniform(n ** 3 * 64, 2)
    mesh = dg.Mesh(dg.make_desc(n, k=k, theta=1.0))
    ATg, dk = mesh.apply_adjoint(cuda(g), cuda(u))
    torch.cuda.synchronize()
    op = ScalarDG(Problem(n, n, n, k=k, theta=1.0, kappa=np.ones(n ** 3 * 64)))
    assert relerr(ATg.cpu().numpy(), op.assemble("explicit").rmatvec(g)) < TOL64
    assert relerr(dk.cpu().numpy(), op.kappa_gradient(u, g).reshape(-1)) < TOL64


def test_fp32_adjoint_error(gpu_lib):
    dg = gpu_lib
    k, n = 4, 3
    E = n ** 3
    kap = workloads.lognormal(E * 125, 7)
    u = workloads.uniform(E * 125, 8)
    g = workloads.uniform(E * 125, 9)
    mesh = dg.Mesh(dg.make_desc(n, k=k, kappa_mode=dg.DG_KAPPA_QP))
    ATg, dk = mesh.apply_adjoint(cuda(g, torch.float32), cuda(u, torch.float32), cuda(kap, torch.float32))
    torch.cuda.synchronize()
    op = ScalarDG(Problem(n, n, n, k=k, kappa=kap))
    e1 = relerr(ATg.double().cpu().numpy(), op.assemble("explicit").rmatvec(g))
    e2 = relerr(dk.double().cpu().numpy(), op.kappa_gradient(u, g).reshape(-1))
    print(f"FP32 adjoint: ATg error {e1:.2e}, dkappa error {e2:.2e}")
    assert e1 < 2e-5 and e2 < 2e-5


@pytest.fixture(scope="module")
def q4_full(gpu_lib):
    """The Q4 48^3 kappa workload at full size."""
    dg = gpu_lib
    w = workloads.WORKLOADS[4]
    mesh = dg.Mesh(dg.desc_from_workload(w))
    kap = workloads.inputs(w, "kappa")
    u = workloads.inputs(w, "u")
    g = workloads.inputs(w, "g")
    return w, mesh, kap, u, g


def test_q4_full_sampled_rows(gpu_lib, q4_full):
    """Full-size forward, A^T g and dkappa on 512 sampled cells (corners, edges,
    faces and random interior cells; the oracle assembles only their block rows,
    in worker processes), relative L2 and elementwise."""
    from oracle_pool import rows
    w, mesh, kap, u, g = q4_full
    print("case: Q4 48^3 sampled rows", flush=True)
    kt, ut, gt = cuda(kap), cuda(u), cuda(g)
    y = mesh.apply(ut, kt)
    ATg, dk = mesh.apply_adjoint(gt, ut, kt)
    torch.cuda.synchronize()
    n = w.n
    E = w.nelem
    rng = np.random.default_rng(4)
    fixed = [0, n - 1, n * n - 1, E - 1, E - n, n * (n - 1), 47, E // 2, (n // 2) * (1 + n + n * n)]
    cells = np.unique(np.concatenate([fixed, rng.choice(E, 520, replace=False)]))[:512]
    ya, ta, da = rows("scalar", 4, cells)
    N = 125
    for got, ref in ((y.cpu().numpy().reshape(E, N)[cells], ya), (ATg.cpu().numpy().reshape(E, N)[cells], ta),
                     (dk.cpu().numpy().reshape(E, N)[cells], da)):
        assert relerr(got, ref) < TOL64
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_q4_full_dot_product_identity(gpu_lib):
    """<A x, g> = <x, A^T g> for the non-symmetric variant at full size."""
    dg = gpu_lib
    w = workloads.WORKLOADS[4]
    mesh = dg.Mesh(dg.desc_from_workload(w, theta=1.0))
    kt = cuda(workloads.inputs(w, "kappa"))
    x = cuda(workloads.inputs(w, "u"))
    g = cuda(workloads.inputs(w, "g"))
    Ax = mesh.apply(x, kt)
    ATg, _ = mesh.apply_adjoint(g, None, kt, want_dkappa=False)
    lhs = float(torch.dot(Ax, g))
    rhs = float(torch.dot(x, ATg))
    scale = float(torch.dot(Ax.abs(), g.abs()))
    assert abs(lhs - rhs) < 1e-13 * scale


def test_q4_full_central_finite_differences(gpu_lib, q4_full):
    """dL/dkappa against central differences of L = g^T A(kappa) u on 100 random
    kappa entries, step 1e-6. L is affine in kappa, so the difference quotient has
    no truncation error; g^T (y+ - y-) is formed from the elementwise difference
    (rows away from the perturbed cell cancel exactly), leaving rounding of order
    eps |y| / (2 step |dL/dkappa|)."""
    dg = gpu_lib
    w, mesh, kap, u, g = q4_full
    print("case: Q4 48^3 finite differences", flush=True)
    kt, ut, gt = cuda(kap), cuda(u), cuda(g)
    _, dk = mesh.apply_adjoint(gt, ut, kt)
    dk = dk.cpu().numpy()
    rng = np.random.default_rng(12)
    idx = rng.choice(len(kap), 100, replace=False)
    step = 1e-6
    worst = 0.0
    for j in idx:
        kp, km = kt.clone(), kt.clone()
        kp[j] += step
        km[j] -= step
        diff = mesh.apply(ut, kp) - mesh.apply(ut, km)
        fd = float(torch.dot(gt, diff)) / (2 * step)
        worst = max(worst, abs(fd - dk[j]) / max(abs(dk[j]), 1e-300))
    print(f"central FD step 1e-6: worst relative deviation {worst:.2e}")
    assert worst < 1e-5
    # a large step is exact for an affine L
    for j in idx[:10]:
        kp, km = kt.clone(), kt.clone()
        kp[j] += 0.5
        km[j] -= 0.5
        fd = float(torch.dot(gt, mesh.apply(ut, kp) - mesh.apply(ut, km)))
        assert abs(fd - dk[j]) < 1e-11 * abs(dk[j]) + 1e-20


def test_autograd_function(gpu_lib):
    dg = gpu_lib
    n, k = 2, 3
    E = n ** 3
    kap = workloads.lognormal(E * 64, 3)
    u = workloads.uniform(E * 64, 4)
    g = workloads.uniform(E * 64, 5)
    mesh = dg.Mesh(dg.make_desc(n, k=k, kappa_mode=dg.DG_KAPPA_QP))
    ut = cuda(u).requires_grad_(True)
    kt = cuda(kap).requires_grad_(True)
    y = dg.DGApply.apply(mesh, ut, kt)
    (y * cuda(g)).sum().backward()
    op = ScalarDG(Problem(n, n, n, k=k, kappa=kap))
    assert relerr(ut.grad.cpu().numpy(), op.assemble("explicit").rmatvec(g)) < TOL64
    assert relerr(kt.grad.cpu().numpy(), op.kappa_gradient(u, g).reshape(-1)) < TOL64
