"""Oracle block rows at full size, computed in parallel worker processes.

Test infrastructure: the workers are fresh interpreters (spawn; they never
touch the GPU) that rebuild the seeded workload inputs and the oracle, and
return its rows for their share of the sampled cells."""
from __future__ import annotations

import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _path():
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)


def _scalar_rows(args):
    wid, cells = args
    _path()
    import workloads
    from oracle import ScalarDG, problem_from_workload
    w = workloads.WORKLOADS[wid]
    kap = workloads.inputs(w, "kappa")
    u, g = workloads.inputs(w, "u"), workloads.inputs(w, "g")
    op = ScalarDG(problem_from_workload(w, kappa=kap))
    return op.apply_rows(u, cells), op.apply_T_rows(g, cells), op.kappa_gradient(u, g, cells)


def _stokes_rows(args):
    wid, cells = args
    _path()
    import workloads
    from oracle import StokesDG, problem_from_workload
    w = workloads.WORKLOADS[wid]
    return (StokesDG(problem_from_workload(w)).apply_rows(workloads.inputs(w, "x"), cells),)


def rows(kind: str, wid: int, cells, workers: int | None = None):
    """Oracle rows of the sampled cells: ('scalar': A u, A^T g, dL/dkappa of the
    kappa workload; 'stokes': A x), each stacked in the order of `cells`."""
    cells = [int(c) for c in cells]
    workers = workers or max(1, min(8, (os.cpu_count() or 2) // 2))
    chunks = [c for c in np.array_split(np.array(cells), workers) if len(c)]
    fn = _scalar_rows if kind == "scalar" else _stokes_rows
    with mp.get_context("spawn").Pool(len(chunks)) as pool:
        parts = pool.map(fn, [(wid, [int(v) for v in c]) for c in chunks])
    return [np.concatenate([p[i] for p in parts]) for i in range(len(parts[0]))]
