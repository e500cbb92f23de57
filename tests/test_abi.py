"""The C ABI without a GPU: the library loads, exports every symbol the header
declares, and rejects bad descriptors and arguments before any HIP call."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dg():
    import paper_1812_08075_amd as dg
    return dg


def declared_functions():
    text = open(os.path.join(ROOT, "include", "dg.h")).read()
    return sorted(set(re.findall(r"^(?:dg_status|const char\*)\s+(dg_\w+)\s*\(", text, re.M)))


def test_header_declarations_are_exported(dg):
    decl = declared_functions()
    assert len(decl) >= 10
    for name in decl:
        assert hasattr(dg.lib, name), name
    assert sorted(dg.EXPORTS) == decl


def test_validate_accepts_workload_descriptors(dg):
    import workloads
    for w in workloads.WORKLOADS.values():
        assert dg.dg_mesh_desc_validate(dg.desc_from_workload(w, n=2)) == dg.DG_OK, w.name


@pytest.mark.parametrize("kw,status", [
    (dict(nx=0), -1), (dict(k=0), -1), (dict(k=8), -2), (dict(m=7, k=3), -2), (dict(m=-1), -1),
    (dict(problem=5), -1), (dict(penalty_form=2), -1), (dict(dirichlet_mask=0x40), -1),
    (dict(kappa_mode=3), -1), (dict(alpha=-1.0), -1), (dict(theta=float("nan")), -1),
    (dict(problem=1, k=1), -2), (dict(problem=1, kappa_mode=1), -1), (dict(nx=65536, ny=1, nz=1), -1),
])
def test_validate_rejects(dg, kw, status):
    base = dict(nx=2, k=3)
    base.update(kw)
    d = dg.make_desc(**base)
    assert dg.dg_mesh_desc_validate(d) == status
    assert len(dg.lib.dg_last_error()) > 0


def test_scalar_with_vertices_unsupported(dg):
    import workloads
    v = workloads.grid_vertices(2, 2, 2, 0.1, 1)
    assert dg.dg_mesh_desc_validate(dg.make_desc(2, k=2, vertices=v)) == dg.DG_ERR_UNSUPPORTED


def test_null_arguments_rejected_without_gpu(dg):
    assert dg.lib.dg_mesh_desc_validate(None) == dg.DG_ERR_ARG
    assert dg.lib.dg_apply(None, 0, None, None, None, None) == dg.DG_ERR_ARG
    assert dg.lib.dg_apply_adjoint(None, 0, None, None, None, None, None, None) == dg.DG_ERR_ARG
    assert dg.lib.dg_mesh_info(None, None) == dg.DG_ERR_ARG
    assert dg.lib.dg_mesh_destroy(None) == dg.DG_OK
    out = ctypes.c_void_p()
    assert dg.lib.dg_mesh_create(None, None, ctypes.byref(out)) == dg.DG_ERR_ARG
    assert dg.lib.dg_solve(None, 0, None, None, None, None, None, None) < 0
    assert dg.lib.dg_precond_apply(None, 0, None, None, None) == dg.DG_ERR_ARG
    assert b"NULL" in dg.lib.dg_last_error()


def test_solve_params_layout_matches_header(dg):
    """The ctypes mirror of dg_solve_params has the header's fields in order."""
    text = open(os.path.join(ROOT, "include", "dg.h")).read()
    body = re.search(r"typedef struct \{([^}]*)\} dg_solve_params;", text).group(1)
    fields = re.findall(r"^\s*(?:double|int32_t)\s+(\w+);", body, re.M)
    assert fields == [f for f, _ in dg.dg_solve_params._fields_]


def test_misaligned_vectors_rejected_without_gpu(dg):
    """Vectors must be 16-byte aligned (the kernels move 16-byte groups): a
    pointer 8 bytes off is DG_ERR_ARG before the library looks at anything else."""
    buf = (ctypes.c_double * 8)()
    base = ctypes.addressof(buf)
    base += (-base) % 16
    ok, off = ctypes.c_void_p(base), ctypes.c_void_p(base + 8)
    cases = [
        lambda: dg.lib.dg_apply(None, 0, off, ok, None, None),
        lambda: dg.lib.dg_apply(None, 0, ok, off, None, None),
        lambda: dg.lib.dg_apply(None, 0, ok, ok, off, None),
        lambda: dg.lib.dg_apply_adjoint(None, 0, ok, ok, None, ok, off, None),
        lambda: dg.lib.dg_apply_adjoint(None, 0, off, ok, None, ok, None, None),
        lambda: dg.lib.dg_precond_apply(None, 0, ok, off, None),
        lambda: dg.lib.dg_load_vector(None, 0, off, ok, None),
        lambda: dg.lib.dg_solve(None, 0, ok, off, None, None, None, None),
    ]
    for i, call in enumerate(cases):
        assert call() == dg.DG_ERR_ARG, i
        assert b"16-byte" in dg.lib.dg_last_error(), i


def test_build_module_imports_without_library(tmp_path):
    """The build step must work in a fresh checkout: importing the package (and
    its build module) must not load libdg.so, which does not exist yet there."""
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / "paper_1812_08075_amd"
    pkg.mkdir()
    for f in ("__init__.py", "build.py"):
        shutil.copy(os.path.join(ROOT, "paper_1812_08075_amd", f), pkg / f)
    code = ("import paper_1812_08075_amd as p, paper_1812_08075_amd.build as b; "
            "assert callable(b.build); assert p._LIB is None; "
            "import os; assert not os.path.exists(p.LIB_PATH)\n"
            "try:\n    p.lib\nexcept ImportError:\n    pass\nelse:\n    raise SystemExit('lib loaded')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=tmp_path, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_binding_rejects_bad_tensors(dg):
    """The binding checks what the C side cannot see behind a pointer."""
    import torch
    t = torch.zeros(16, dtype=torch.float64)
    with pytest.raises(ValueError, match="GPU"):
        dg._vec(t, 16, dg.DG_F64, "x")
    with pytest.raises(ValueError, match="precision"):
        dg._vec(t, 16, 7, "x")
    with pytest.raises(ValueError, match="required"):
        dg._vec(None, 16, dg.DG_F64, "x")
    assert dg._vec(None, 16, dg.DG_F64, "kappa", optional=True) is None
    with pytest.raises(ValueError, match="float64 or float32"):
        dg._prec_of(torch.zeros(4, dtype=torch.float16))
    with pytest.raises(TypeError):
        dg._vec(np.zeros(16), 16, dg.DG_F64, "x")


def test_solve_info_layout_matches_header(dg):
    """The ctypes mirror of dg_solve_info has the header's fields in order."""
    text = open(os.path.join(ROOT, "include", "dg.h")).read()
    body = re.search(r"typedef struct \{([^}]*)\} dg_solve_info;", text).group(1)
    fields = re.findall(r"^\s*(?:double|int32_t)\s+(\w+);", body, re.M)
    assert fields == [f for f, _ in dg.dg_solve_info._fields_]
    assert ctypes.sizeof(dg.dg_solve_info) == 40 and ctypes.sizeof(dg.dg_solve_params) == 56
