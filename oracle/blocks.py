"""Block-sparse global matrix of a DG operator (test infrastructure; oracle only).

DG spaces are blocked per cell and the global vector is accessed block-wise
(Section 1 and Section 3.1): the matrix has one block row per cell with at
most seven nonzero blocks, the cell itself (slot 0) and its face neighbours
(slot 1 + 2 d + s for side s of direction d).

Blocks are stored either explicitly per (cell, slot) or, for meshes on which
many block rows coincide, once per class with a class index per (cell, slot).
"""
from __future__ import annotations

import numpy as np

NSLOT = 7


def slot(d: int, side: int) -> int:
    return 1 + 2 * d + side


class BlockMatrix:
    """y = A x with A given by block rows.

    nbr[e, s]: column block of slot s in row e (-1: absent; slot 0 is e itself).
    Either ``blocks`` (E, 7, N, N) or ``classes`` (C, N, N) with ``cls`` (E, 7).
    """

    def __init__(self, nbr: np.ndarray, bsize: int, blocks: np.ndarray | None = None,
                 classes: np.ndarray | None = None, cls: np.ndarray | None = None):
        self.nbr = np.asarray(nbr, dtype=np.int64)
        self.nelem = self.nbr.shape[0]
        self.bsize = int(bsize)
        self.blocks = blocks
        self.classes = classes
        self.cls = cls
        assert (blocks is None) != (classes is None)

    @property
    def shape(self):
        n = self.nelem * self.bsize
        return (n, n)

    def _slot_terms(self, s: int):
        """Yield (rows, cols, block or per-row blocks) for slot s."""
        valid = np.nonzero(self.nbr[:, s] >= 0)[0]
        if self.blocks is not None:
            yield valid, self.nbr[valid, s], self.blocks[valid, s]
        else:
            cl = self.cls[valid, s]
            for c in np.unique(cl):
                rows = valid[cl == c]
                yield rows, self.nbr[rows, s], self.classes[c]

    def matvec(self, x: np.ndarray) -> np.ndarray:
        N = self.bsize
        X = np.asarray(x, dtype=np.float64).reshape(self.nelem, N)
        Y = np.zeros_like(X)
        for s in range(NSLOT):
            for rows, cols, B in self._slot_terms(s):
                if B.ndim == 2:
                    Y[rows] += X[cols] @ B.T
                else:
                    Y[rows] += np.einsum("eij,ej->ei", B, X[cols])
        return Y.reshape(-1)

    def rmatvec(self, g: np.ndarray) -> np.ndarray:
        """A^T g: block (e, s) contributes B^T g_e to block row nbr[e, s]."""
        N = self.bsize
        G = np.asarray(g, dtype=np.float64).reshape(self.nelem, N)
        Z = np.zeros_like(G)
        for s in range(NSLOT):
            for rows, cols, B in self._slot_terms(s):
                # within one slot every column block appears at most once
                if B.ndim == 2:
                    Z[cols] += G[rows] @ B
                else:
                    Z[cols] += np.einsum("eji,ej->ei", B, G[rows])
        return Z.reshape(-1)

    def row_block(self, e: int, s: int) -> np.ndarray:
        if self.blocks is not None:
            return self.blocks[e, s]
        return self.classes[self.cls[e, s]]

    def to_dense(self) -> np.ndarray:
        N = self.bsize
        A = np.zeros(self.shape)
        for e in range(self.nelem):
            for s in range(NSLOT):
                c = self.nbr[e, s]
                if c >= 0:
                    A[e * N:(e + 1) * N, c * N:(c + 1) * N] += self.row_block(e, s)
        return A

    def to_scipy(self):
        import scipy.sparse as sp
        N = self.bsize
        rows, cols, vals = [], [], []
        ii, jj = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
        for e in range(self.nelem):
            for s in range(NSLOT):
                c = self.nbr[e, s]
                if c >= 0:
                    rows.append((e * N + ii).ravel())
                    cols.append((c * N + jj).ravel())
                    vals.append(self.row_block(e, s).ravel())
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=self.shape)


def _c_lib():
    """The oracle's C block SpMV (oracle/spmv.c), built by oracle/build_c.py."""
    import ctypes
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liboracle_spmv.so")
    if not os.path.exists(path):  # a fresh checkout: one gcc call
        from .build_c import build
        build()
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.oracle_bsr_matvec.argtypes = [ctypes.c_int64, ctypes.c_int32, P, P, P, P, P, ctypes.c_int32]
    lib.oracle_bsr_matvec.restype = None
    return lib


class CBlockMatvec:
    """y = A x of a BlockMatrix by the C routine of oracle/spmv.c: the plain
    block-row definition, block rows split over `threads` OpenMP threads."""

    def __init__(self, A: BlockMatrix):
        self.lib = _c_lib()
        self.nelem, self.n = A.nelem, A.bsize
        self.nbr = np.ascontiguousarray(A.nbr, dtype=np.int64)
        if A.classes is not None:
            self.blocks = np.ascontiguousarray(A.classes, dtype=np.float64)
            self.cls = np.ascontiguousarray(A.cls, dtype=np.int64)
        else:
            self.blocks = np.ascontiguousarray(A.blocks.reshape(-1, self.n, self.n), dtype=np.float64)
            self.cls = np.arange(self.nelem * NSLOT, dtype=np.int64).reshape(self.nelem, NSLOT)

    def __call__(self, x: np.ndarray, threads: int = 1, out: np.ndarray | None = None) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        assert x.size == self.nelem * self.n
        y = np.empty_like(x) if out is None else out
        self.lib.oracle_bsr_matvec(self.nelem, self.n, self.nbr.ctypes.data, self.cls.ctypes.data,
                                   self.blocks.ctypes.data, x.ctypes.data, y.ctypes.data, int(threads))
        return y
