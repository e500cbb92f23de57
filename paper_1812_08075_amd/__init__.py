"""Python binding of libdg: matrix-free sum-factorized interior-penalty DG
operators on MI355X.

Argument marshalling only: every step of the operator runs in the HIP
kernels of libdg.so. The functions mirror include/dg.h one to one
(dg_mesh_create, dg_apply, dg_apply_adjoint, dg_solve, ...). Vectors are
torch tensors on the GPU; the current torch stream is passed to the library.
Every tensor is checked (device, dtype, contiguity, 16-byte alignment,
length) before its pointer is handed over, since the library only sees
pointers. There is no CPU fallback: the library is loaded on first use
(`lib`), and that fails loudly when libdg.so is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdg.so")

DG_OK, DG_ERR_ARG, DG_ERR_UNSUPPORTED, DG_ERR_DEVICE, DG_ERR_ALLOC = 0, -1, -2, -3, -4
DG_NOT_CONVERGED, DG_BREAKDOWN = 1, 2
DG_PROBLEM_DIFFREAC, DG_PROBLEM_STOKES, DG_PROBLEM_DIFFREAC_PAPER, DG_PROBLEM_NONLINEAR = 0, 1, 2, 3
DG_F64, DG_F32 = 0, 1
DG_KAPPA_ONE, DG_KAPPA_QP = 0, 1
DG_KAPPA_FACE_TRACE, DG_KAPPA_FACE_ONE = 0, 1
DG_SOLVE_CG_F64, DG_SOLVE_IR_F32, DG_SOLVE_RU_F32, DG_SOLVE_CHEB_F64, DG_SOLVE_CHEB_F32 = 0, 1, 2, 3, 4
DG_PRECOND_NONE, DG_PRECOND_BLOCK_JACOBI = 0, 1

_DTYPE = {DG_F64: torch.float64, DG_F32: torch.float32}


class dg_mesh_desc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("k", ctypes.c_int32), ("m", ctypes.c_int32), ("problem", ctypes.c_int32),
        ("c", ctypes.c_double), ("alpha", ctypes.c_double), ("theta", ctypes.c_double),
        ("penalty_form", ctypes.c_int32), ("dirichlet_mask", ctypes.c_uint32),
        ("vertices", ctypes.POINTER(ctypes.c_double)),
        ("kappa_mode", ctypes.c_int32), ("kappa_face", ctypes.c_int32),
    ]


class dg_mesh_info_t(ctypes.Structure):
    _fields_ = [
        ("nelem", ctypes.c_int64), ("ndofs", ctypes.c_int64), ("dofs_per_elem", ctypes.c_int64),
        ("nqp", ctypes.c_int64), ("p", ctypes.c_int32), ("m", ctypes.c_int32),
        ("axis_aligned", ctypes.c_int32), ("flops_apply", ctypes.c_double),
        ("flops_adjoint", ctypes.c_double), ("bytes_apply", ctypes.c_double * 2),
        ("bytes_adjoint", ctypes.c_double),
    ]


class dg_solve_params(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("inner_rtol", ctypes.c_double), ("maxit", ctypes.c_int32),
                ("max_outer", ctypes.c_int32), ("check_every", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("cheb_degree", ctypes.c_int32), ("cheb_lanczos", ctypes.c_int32),
                ("cheb_ratio", ctypes.c_double), ("cheb_margin", ctypes.c_double)]


class dg_solve_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("outer", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("inner_applies", ctypes.c_int32), ("lanczos_iterations", ctypes.c_int32),
                ("lambda_max", ctypes.c_double)]


DG_VARIANT_MATRIX_CORE, DG_VARIANT_LINES = 0, 1
DG_TUNE_MAX = 16


class dg_tune_result(ctypes.Structure):
    _fields_ = [("ncand", ctypes.c_int32), ("chosen", ctypes.c_int32),
                ("kind", ctypes.c_int32 * DG_TUNE_MAX), ("param", ctypes.c_int32 * DG_TUNE_MAX),
                ("us", ctypes.c_double * DG_TUNE_MAX)]


# every symbol include/dg.h declares
EXPORTS = ("dg_mesh_desc_validate", "dg_mesh_create", "dg_mesh_destroy", "dg_mesh_info", "dg_apply",
           "dg_apply_adjoint", "dg_precond_apply", "dg_solve", "dg_solve_noalloc", "dg_residual", "dg_mesh_qpoints",
           "dg_load_vector", "dg_apply_jacobian", "dg_mesh_set_variant", "dg_mesh_tune", "dg_last_error")


def _load():
    """Opens libdg.so and declares the argument types of every entry point."""
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(python -m paper_1812_08075_amd.build); there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    P, V = ctypes.POINTER, ctypes.c_void_p
    sig = {
        "dg_mesh_desc_validate": [P(dg_mesh_desc)],
        "dg_mesh_create": [P(dg_mesh_desc), V, P(V)],
        "dg_mesh_destroy": [V],
        "dg_mesh_info": [V, P(dg_mesh_info_t)],
        "dg_apply": [V, ctypes.c_int, V, V, V, V],
        "dg_apply_adjoint": [V, ctypes.c_int, V, V, V, V, V, V],
        "dg_precond_apply": [V, ctypes.c_int, V, V, V],
        "dg_solve": [V, ctypes.c_int, V, V, V, P(dg_solve_params), P(dg_solve_info), V],
        "dg_solve_noalloc": [V, ctypes.c_int, V, V, V, P(dg_solve_params), P(dg_solve_info), V],
        "dg_residual": [V, ctypes.c_int, V, V, V],
        "dg_mesh_qpoints": [V, P(ctypes.c_double)],
        "dg_load_vector": [V, ctypes.c_int, V, V, V],
        "dg_apply_jacobian": [V, ctypes.c_int, V, V, V, V],
        "dg_mesh_set_variant": [V, ctypes.c_int, ctypes.c_int, ctypes.c_int],
        "dg_mesh_tune": [V, ctypes.c_int, ctypes.c_int, V, P(dg_tune_result)],
        "dg_last_error": [],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_char_p if name == "dg_last_error" else ctypes.c_int
    return lib


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        _LIB = _load()
    return _LIB


def __getattr__(name):
    # `lib` is resolved on first access, so that importing the package (for
    # instance to build the library) never loads a missing or stale libdg.so
    if name == "lib":
        return _lib()
    raise AttributeError(name)


class DGError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libdg status {status}: {msg}")
        self.status = status


def _check(status: int, allow=()) -> int:
    if status != DG_OK and status not in allow:
        raise DGError(status, _lib().dg_last_error().decode())
    return status


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# sizes of every mesh handle this binding created (for the tensor checks)
_SIZES = {}


def _sizes(mesh):
    key = mesh.value if isinstance(mesh, ctypes.c_void_p) else int(mesh)
    sz = _SIZES.get(key)
    if sz is None:
        info = dg_mesh_info(mesh)
        sz = _SIZES[key] = (int(info.ndofs), int(info.nqp))
    return sz


def _vec(t, n, prec, name, optional=False):
    """Pointer of a device tensor after checking what the library cannot: a
    GPU tensor of the precision's dtype, contiguous, 16-byte aligned, n values."""
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    want = _DTYPE.get(prec)
    if want is None:
        raise ValueError(f"precision must be DG_F64 or DG_F32, got {prec}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU (got {t.device})")
    if t.dtype != want:
        raise ValueError(f"{name} must be {want} for this precision (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name} must hold {n} values (got {t.numel()})")
    if t.data_ptr() % 16:
        raise ValueError(f"{name} must be 16-byte aligned")
    return ctypes.c_void_p(t.data_ptr())


def _prec_of(t):
    if t.dtype == torch.float64:
        return DG_F64
    if t.dtype == torch.float32:
        return DG_F32
    raise ValueError(f"vectors must be float64 or float32 (got {t.dtype})")


def make_desc(nx, ny=None, nz=None, k=3, m=0, problem=DG_PROBLEM_DIFFREAC, c=1.0, alpha=3.0, theta=-1.0,
              penalty_form=0, dirichlet_mask=0x3F, vertices=None, kappa_mode=DG_KAPPA_ONE,
              kappa_face=DG_KAPPA_FACE_TRACE):
    """A dg_mesh_desc; `vertices` is an optional float64 numpy array (kept alive on the desc)."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    d = dg_mesh_desc(nx, ny, nz, k, m, problem, c, alpha, theta, penalty_form, dirichlet_mask, None,
                     kappa_mode, kappa_face)
    if vertices is not None:
        v = np.ascontiguousarray(vertices, dtype=np.float64)
        d._vertices_keepalive = v
        d.vertices = v.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return d


def desc_from_workload(w, n=None, theta=None):
    """Descriptor of a workloads.Workload (optionally on an n^3 copy of its mesh)."""
    import workloads
    w = w if n is None else w.scaled(n)
    verts = workloads.vertices(w)
    return make_desc(w.n, w.n, w.n, k=w.k, m=w.m, problem=w.problem, c=w.c, alpha=w.alpha,
                     theta=w.theta if theta is None else theta, penalty_form=w.penalty_form,
                     dirichlet_mask=w.mask, vertices=verts, kappa_mode=w.kappa_mode)


def dg_mesh_desc_validate(desc) -> int:
    return _lib().dg_mesh_desc_validate(ctypes.byref(desc))


def dg_mesh_create(desc, stream=None):
    h = ctypes.c_void_p()
    _check(_lib().dg_mesh_create(ctypes.byref(desc), _stream(stream), ctypes.byref(h)))
    _SIZES.pop(h.value, None)
    return h


def dg_mesh_destroy(mesh):
    key = mesh.value if isinstance(mesh, ctypes.c_void_p) else mesh
    _SIZES.pop(key, None)
    _check(_lib().dg_mesh_destroy(mesh))


def dg_mesh_info(mesh) -> dg_mesh_info_t:
    out = dg_mesh_info_t()
    _check(_lib().dg_mesh_info(mesh, ctypes.byref(out)))
    return out


def dg_apply(mesh, precision, x, y, kappa=None, stream=None):
    n, nq = _sizes(mesh)
    _check(_lib().dg_apply(mesh, precision, _vec(x, n, precision, "x"), _vec(y, n, precision, "y"),
                           _vec(kappa, nq, precision, "kappa", optional=True), _stream(stream)))


def dg_apply_adjoint(mesh, precision, g, u, kappa, ATg, dkappa=None, stream=None):
    n, nq = _sizes(mesh)
    _check(_lib().dg_apply_adjoint(mesh, precision, _vec(g, n, precision, "g"),
                                   _vec(u, n, precision, "u", optional=True),
                                   _vec(kappa, nq, precision, "kappa", optional=True),
                                   _vec(ATg, n, precision, "ATg"),
                                   _vec(dkappa, nq, precision, "dkappa", optional=True), _stream(stream)))


def dg_precond_apply(mesh, precision, r, z, stream=None):
    n, _ = _sizes(mesh)
    _check(_lib().dg_precond_apply(mesh, precision, _vec(r, n, precision, "r"), _vec(z, n, precision, "z"),
                                   _stream(stream)))


def dg_solve(mesh, mode, b, x, kappa=None, rtol=1e-10, inner_rtol=1e-5, maxit=100000, max_outer=50,
             check_every=10, precond=DG_PRECOND_NONE, stream=None, noalloc=False, cheb_degree=0,
             cheb_lanczos=0, cheb_ratio=0.0, cheb_margin=0.0):
    """dg_solve, or with noalloc=True dg_solve_noalloc (fixed device workspace)."""
    n, nq = _sizes(mesh)
    params = dg_solve_params(rtol, inner_rtol, maxit, max_outer, check_every, precond, cheb_degree, cheb_lanczos,
                             cheb_ratio, cheb_margin)
    info = dg_solve_info()
    fn = _lib().dg_solve_noalloc if noalloc else _lib().dg_solve
    st = _check(fn(mesh, mode, _vec(b, n, DG_F64, "b"), _vec(x, n, DG_F64, "x"),
                                _vec(kappa, nq, DG_F64, "kappa", optional=True), ctypes.byref(params),
                                ctypes.byref(info), _stream(stream)), allow=(DG_NOT_CONVERGED, DG_BREAKDOWN))
    return st, info


def dg_residual(mesh, precision, u, r, stream=None):
    n, _ = _sizes(mesh)
    _check(_lib().dg_residual(mesh, precision, _vec(u, n, precision, "u"), _vec(r, n, precision, "r"),
                              _stream(stream)))


def dg_apply_jacobian(mesh, precision, u0, z, y, stream=None):
    n, _ = _sizes(mesh)
    _check(_lib().dg_apply_jacobian(mesh, precision, _vec(u0, n, precision, "u0"), _vec(z, n, precision, "z"),
                                    _vec(y, n, precision, "y"), _stream(stream)))


def dg_mesh_set_variant(mesh, precision, kind, param):
    _check(_lib().dg_mesh_set_variant(mesh, precision, kind, param))


def dg_mesh_tune(mesh, precision, trials=5, stream=None):
    """Times the apply variants of this mesh and keeps the fastest; returns
    [(kind, param, microseconds), ...] and the index chosen."""
    out = dg_tune_result()
    _check(_lib().dg_mesh_tune(mesh, precision, trials, _stream(stream), ctypes.byref(out)))
    cands = [(out.kind[i], out.param[i], out.us[i]) for i in range(out.ncand)]
    return cands, out.chosen


def dg_mesh_qpoints(mesh) -> np.ndarray:
    info = dg_mesh_info(mesh)
    out = np.empty((info.nqp, 3), dtype=np.float64)
    _check(_lib().dg_mesh_qpoints(mesh, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def dg_load_vector(mesh, precision, fq, b, stream=None):
    n, nq = _sizes(mesh)
    _check(_lib().dg_load_vector(mesh, precision, _vec(fq, nq, precision, "fq"), _vec(b, n, precision, "b"),
                                 _stream(stream)))


class Mesh:
    """Owning wrapper of a dg_mesh handle with tensor-allocating helpers."""

    def __init__(self, desc, stream=None):
        self.desc = desc
        self.handle = dg_mesh_create(desc, stream)
        self.info = dg_mesh_info(self.handle)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _LIB is not None:
            _SIZES.pop(h.value, None)
            _LIB.dg_mesh_destroy(h)
            self.handle = None

    @property
    def ndofs(self) -> int:
        return int(self.info.ndofs)

    def apply(self, x, kappa=None, out=None):
        prec = _prec_of(x)
        y = torch.empty_like(x) if out is None else out
        dg_apply(self.handle, prec, x, y, kappa)
        return y

    def apply_adjoint(self, g, u=None, kappa=None, want_dkappa=True):
        prec = _prec_of(g)
        ATg = torch.empty_like(g)
        dk = torch.empty(int(self.info.nqp), dtype=g.dtype, device=g.device) if want_dkappa else None
        dg_apply_adjoint(self.handle, prec, g, u, kappa, ATg, dk)
        return ATg, dk


class DGApply(torch.autograd.Function):
    """y = A(kappa) u; backward returns A^T g and dL/dkappa from dg_apply_adjoint."""

    @staticmethod
    def forward(ctx, mesh: Mesh, u, kappa):
        ctx.mesh = mesh
        ctx.save_for_backward(u, kappa)
        return mesh.apply(u, kappa)

    @staticmethod
    def backward(ctx, g):
        u, kappa = ctx.saved_tensors
        need_k = ctx.needs_input_grad[2]
        ATg, dk = ctx.mesh.apply_adjoint(g.contiguous(), u if need_k else None, kappa, want_dkappa=need_k)
        return None, ATg, dk
