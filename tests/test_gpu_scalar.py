"""GPU parity of the sum-factorized diffusion-reaction apply against the CPU
oracle's assembled block-sparse matrix, through the C ABI."""
import numpy as np
import pytest
import torch

import workloads
from oracle import Problem, ScalarDG, problem_from_workload

pytestmark = pytest.mark.gpu

TOL64 = 1e-12      # relative L2, FP64 (the parity bar)
TOL32 = 2e-5       # relative L2, FP32 apply: ~ 1e2 x unit roundoff of float


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_apply(dg, desc, x, kappa=None, dtype=torch.float64):
    mesh = dg.Mesh(desc)
    xt = torch.from_numpy(x).to("cuda", dtype)
    kt = None if kappa is None else torch.from_numpy(kappa).to("cuda", dtype)
    y = mesh.apply(xt, kt)
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


def test_q2_4cube_matches_oracle(gpu_lib):
    dg = gpu_lib
    w = workloads.WORKLOADS[1]
    print("case: Q2 4^3 FP64", flush=True)
    x = workloads.inputs(w, "x")
    y = gpu_apply(dg, dg.desc_from_workload(w), x)
    ref = ScalarDG(problem_from_workload(w)).assemble().matvec(x)
    assert relerr(y, ref) < TOL64


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("shape,theta,mask,c", [((3, 2, 5), -1.0, 0x3F, 1.0), ((2, 3, 1), 1.0, 0x1B, 0.3),
                                                 ((1, 1, 1), -1.0, 0x00, 2.0)])
def test_degrees_shapes_masks(gpu_lib, k, shape, theta, mask, c):
    """Every built degree on ragged meshes (cells not a multiple of the block
    batch), the non-symmetric variant, Neumann sides and a single cell."""
    dg = gpu_lib
    print(f"case: k={k} shape={shape} theta={theta} mask={mask:#x}", flush=True)
    nx, ny, nz = shape
    N = (k + 1) ** 3
    x = workloads.uniform(nx * ny * nz * N, 1000 + k)
    desc = dg.make_desc(nx, ny, nz, k=k, c=c, theta=theta, dirichlet_mask=mask)
    y = gpu_apply(dg, desc, x)
    ref = ScalarDG(Problem(nx, ny, nz, k=k, c=c, theta=theta, mask=mask)).assemble().matvec(x)
    assert relerr(y, ref) < TOL64


@pytest.mark.parametrize("shape,theta,mask,c", [((6, 5, 4), 1.0, 0x2D, 0.7), ((9, 2, 3), -1.0, 0x3F, 1.0),
                                                 ((5, 1, 2), -1.0, 0x12, 0.0), ((4, 4, 4), 1.0, 0x00, 1.5)])
def test_q3_rows_and_sides(gpu_lib, shape, theta, mask, c):
    """k = 3 (the matrix-core apply) with x-rows that end in a partial group
    of cells, every mix of interior / Dirichlet / natural sides per direction,
    both theta, with and without the mass term; forward and transposed."""
    dg = gpu_lib
    print(f"case: k=3 shape={shape} theta={theta} mask={mask:#x} c={c}", flush=True)
    nx, ny, nz = shape
    x = workloads.uniform(nx * ny * nz * 64, 4242 + nx)
    desc = dg.make_desc(nx, ny, nz, k=3, c=c, theta=theta, dirichlet_mask=mask)
    A = ScalarDG(Problem(nx, ny, nz, k=3, c=c, theta=theta, mask=mask)).assemble()
    assert relerr(gpu_apply(dg, desc, x), A.matvec(x)) < TOL64
    mesh = dg.Mesh(desc)
    ATg, _ = mesh.apply_adjoint(torch.from_numpy(x).cuda(), want_dkappa=False)
    torch.cuda.synchronize()
    assert relerr(ATg.cpu().numpy(), A.rmatvec(x)) < TOL64


@pytest.mark.parametrize("penalty_form", [0, 1])
def test_penalty_forms(gpu_lib, penalty_form):
    dg = gpu_lib
    x = workloads.uniform(3 * 3 * 3 * 64, 77)
    desc = dg.make_desc(3, k=3, penalty_form=penalty_form, alpha=2.5)
    y = gpu_apply(dg, desc, x)
    ref = ScalarDG(Problem(3, 3, 3, k=3, penalty_form=penalty_form, alpha=2.5)).assemble().matvec(x)
    assert relerr(y, ref) < TOL64


@pytest.mark.parametrize("k", [2, 3, 5])
def test_fp32_apply_error(gpu_lib, k):
    dg = gpu_lib
    n = 3
    x = workloads.uniform(n ** 3 * (k + 1) ** 3, 31)
    y = gpu_apply(dg, dg.make_desc(n, k=k), x, dtype=torch.float32)
    ref = ScalarDG(Problem(n, n, n, k=k)).assemble().matvec(x)
    err = relerr(y, ref)
    print(f"FP32 apply k={k}: relative L2 error {err:.2e}")
    assert err < TOL32


@pytest.mark.parametrize("shape,mask,theta", [((9, 7, 5), 0x3F, -1.0), ((13, 10, 6), 0x2D, 1.0),
                                              ((13, 71, 45), 0x2D, -1.0), ((10, 37, 512), 0x17, -1.0)])
def test_q3_fp32_is_rounded_fp64(gpu_lib, shape, mask, theta):
    """The Q3 FP32 apply computes in FP64 on the matrix cores with the FP64
    kernel's tables and order of operations: its output is, bit for bit, the
    FP64 apply of the FP32 input rounded once to FP32 (ragged chunks, marches
    of 1, 2 and 16 rows, natural sides, the non-symmetric variant)."""
    dg = gpu_lib
    print(f"case: Q3 FP32 vs rounded FP64 {shape} mask={mask:#x} theta={theta}", flush=True)
    nx, ny, nz = shape
    mesh = dg.Mesh(dg.make_desc(nx, ny, nz, k=3, dirichlet_mask=mask, theta=theta))
    x32 = torch.from_numpy(workloads.uniform(mesh.ndofs, 6200 + nx)).to("cuda", torch.float32)
    y32 = mesh.apply(x32)
    y64 = mesh.apply(x32.double())
    a32, _ = mesh.apply_adjoint(x32, want_dkappa=False)  # the transposed operator
    a64, _ = mesh.apply_adjoint(x32.double(), want_dkappa=False)
    torch.cuda.synchronize()
    assert torch.equal(y32, y64.float())
    assert torch.equal(a32, a64.float())


@pytest.mark.parametrize("face_one", [False, True])
@pytest.mark.parametrize("theta", [-1.0, 1.0])
def test_kappa_per_point(gpu_lib, face_one, theta):
    dg = gpu_lib
    n, k = 3, 4
    w = workloads.WORKLOADS[4]
    kap = workloads.lognormal(n ** 3 * 125, w.seed("kappa"))
    x = workloads.uniform(n ** 3 * 125, w.seed("x"))
    desc = dg.make_desc(n, k=k, theta=theta, kappa_mode=dg.DG_KAPPA_QP,
                        kappa_face=dg.DG_KAPPA_FACE_ONE if face_one else dg.DG_KAPPA_FACE_TRACE)
    y = gpu_apply(dg, desc, x, kappa=kap)
    ref = ScalarDG(Problem(n, n, n, k=k, theta=theta, kappa=kap, kappa_face_one=face_one)) \
        .assemble("explicit").matvec(x)
    assert relerr(y, ref) < TOL64


def test_bitwise_deterministic(gpu_lib):
    dg = gpu_lib
    w = workloads.WORKLOADS[2].scaled(12)
    mesh = dg.Mesh(dg.desc_from_workload(w))
    x = torch.from_numpy(workloads.inputs(w, "x")).cuda()
    y1 = mesh.apply(x)
    y2 = mesh.apply(x)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)


def test_q3_64cube_full_vector(gpu_lib):
    """The benchmark workload at full size (16.8M DOFs), in the launch
    configuration the benchmark times, against the oracle's deduplicated BSR."""
    dg = gpu_lib
    w = workloads.WORKLOADS[2]
    print("case: Q3 64^3 full size", flush=True)
    x = workloads.inputs(w, "x")
    y = gpu_apply(dg, dg.desc_from_workload(w), x)
    ref = ScalarDG(problem_from_workload(w)).assemble("dedup").matvec(x)
    assert relerr(y, ref) < TOL64


@pytest.mark.parametrize("shape,mask", [((13, 71, 45), 0x2D), ((6, 130, 96), 0x17), ((10, 37, 512), 0x3F)])
def test_q3_row_march_ragged(gpu_lib, shape, mask):
    """Q3 meshes large enough that each wavefront of the matrix-core apply
    marches along y over several rows (2, 4 and 16 rows per wavefront for
    these shapes), with a shorter last march in every column, a ragged last
    x chunk and natural sides, against the oracle's deduplicated BSR."""
    dg = gpu_lib
    print(f"case: Q3 row march {shape} mask={mask:#x}", flush=True)
    nx, ny, nz = shape
    x = workloads.uniform(nx * ny * nz * 64, 6100 + ny)
    y = gpu_apply(dg, dg.make_desc(nx, ny, nz, k=3, dirichlet_mask=mask), x)
    ref = ScalarDG(Problem(nx, ny, nz, k=3, mask=mask)).assemble("dedup").matvec(x)
    assert relerr(y, ref) < TOL64


def test_q3_wide_planes_run_the_line_kernels(gpu_lib):
    """A Q3 mesh of 1500 x 1500 x 1 cells (144M DOFs): a wavefront of the
    matrix-core kernel reads within two x-y planes through 32-bit byte
    offsets, and planes this wide exceed that window, so the mesh offers no
    matrix-core variant and its apply runs the line kernels; their result
    matches the oracle's block rows on sampled cells (corners, edges,
    natural and Dirichlet sides, random cells), relative L2 and elementwise."""
    dg = gpu_lib
    nx, ny, nz, mask = 1500, 1500, 1, 0x2D
    E = nx * ny * nz
    print(f"case: Q3 wide planes {nx}x{ny}x{nz} mask={mask:#x}", flush=True)
    mesh = dg.Mesh(dg.make_desc(nx, ny, nz, k=3, dirichlet_mask=mask))
    with pytest.raises(dg.DGError) as ei:
        dg.dg_mesh_set_variant(mesh.handle, 0, dg.DG_VARIANT_MATRIX_CORE, 16)
    assert ei.value.status == dg.DG_ERR_ARG
    x = workloads.uniform(E * 64, 6200)
    y = mesh.apply(torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    rng = np.random.default_rng(6201)
    fixed = [0, nx - 1, nx * (ny - 1), E - 1, nx * (ny // 2), nx * (ny // 2) + nx - 1, E // 2 + 7]
    cells = np.unique(np.concatenate([fixed, rng.choice(E, 57, replace=False)]))
    got = y.cpu().numpy().reshape(E, 64)[cells]
    ref = ScalarDG(Problem(nx, ny, nz, k=3, mask=mask)).apply_rows(x, cells)
    assert relerr(got, ref) < TOL64
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_q5_40cube_full_vector(gpu_lib):
    """The Q5 40^3 solve workload (13.8M DOFs) at full size, FP64 (line-operator
    kernel) and FP32 (sum-factorized kernel), against the oracle's deduplicated BSR."""
    dg = gpu_lib
    w = workloads.WORKLOADS[5]
    print("case: Q5 40^3 full size", flush=True)
    x = workloads.inputs(w, "x")
    ref = ScalarDG(problem_from_workload(w)).assemble("dedup").matvec(x)
    desc = dg.desc_from_workload(w)
    assert relerr(gpu_apply(dg, desc, x), ref) < TOL64
    assert relerr(gpu_apply(dg, desc, x, dtype=torch.float32), ref) < TOL32


def test_transposed_apply(gpu_lib):
    """A^T g with the non-symmetric variant (theta = +1), no dkappa."""
    dg = gpu_lib
    n, k = 3, 3
    g = workloads.uniform(n ** 3 * 64, 5)
    mesh = dg.Mesh(dg.make_desc(n, k=k, theta=1.0))
    gt = torch.from_numpy(g).cuda()
    ATg, _ = mesh.apply_adjoint(gt, want_dkappa=False)
    torch.cuda.synchronize()
    ref = ScalarDG(Problem(n, n, n, k=k, theta=1.0)).assemble().rmatvec(g)
    assert relerr(ATg.cpu().numpy(), ref) < TOL64


def test_load_vector(gpu_lib):
    dg = gpu_lib
    w = workloads.WORKLOADS[5].scaled(3)
    mesh = dg.Mesh(dg.desc_from_workload(w))
    xyz = dg.dg_mesh_qpoints(mesh.handle)
    fq = torch.from_numpy(workloads.sin_forcing(xyz, w.c)).cuda()
    b = torch.empty(mesh.ndofs, dtype=torch.float64, device="cuda")
    dg.dg_load_vector(mesh.handle, dg.DG_F64, fq, b)
    torch.cuda.synchronize()
    op = ScalarDG(problem_from_workload(w))
    ref = op.load_vector(lambda x: workloads.sin_forcing(x, w.c))
    assert relerr(b.cpu().numpy(), ref) < 1e-13


def test_binding_rejects_bad_device_tensors(gpu_lib):
    """dtype, contiguity, length and alignment of device tensors are checked by
    the binding before any pointer reaches the library."""
    dg = gpu_lib
    print("case: binding tensor checks", flush=True)
    mesh = dg.Mesh(dg.make_desc(2, 2, 2, k=2))
    n = mesh.ndofs
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    bad = [
        (torch.zeros(n, dtype=torch.float16, device="cuda"), "float64"),
        (torch.zeros(2 * n, dtype=torch.float64, device="cuda")[::2], "contiguous"),
        (torch.zeros(n + 1, dtype=torch.float64, device="cuda"), "hold"),
        (torch.zeros(n + 1, dtype=torch.float64, device="cuda")[1:], "aligned"),
        (torch.zeros(n, dtype=torch.float32, device="cuda"), "float64"),
    ]
    for t, msg in bad:
        with pytest.raises(ValueError, match=msg):
            dg.dg_apply(mesh.handle, dg.DG_F64, t, y)
    with pytest.raises(ValueError, match="float64 or float32"):
        mesh.apply(torch.zeros(n, dtype=torch.int32, device="cuda"))
    dg.dg_apply(mesh.handle, dg.DG_F64, x, y)
    torch.cuda.synchronize()
