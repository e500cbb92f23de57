"""The C ABI without a GPU: the library loads, exports every symbol the header
declares, and rejects bad descriptors and arguments before any HIP call."""
import ctypes
import os
import re

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
