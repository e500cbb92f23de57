"""Pins of the oracle's block-Jacobi preconditioner and preconditioned CG
(the element block-Jacobi preconditioner named among the matrix-free
preconditioners of Section 1) against things other than themselves."""
import numpy as np
import pytest

from oracle import Problem, ScalarDG, block_jacobi, cg, pcg


def _rand(n, seed):
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("mask", [0x3F, 0x15])
def test_single_cell_block_jacobi_is_the_inverse(k, mask):
    # one cell: the diagonal block is the whole matrix, so A z = r through the
    # full block-row product
    A = ScalarDG(Problem(1, 1, 1, k=k, mask=mask)).assemble("explicit")
    r = _rand(A.shape[0], 3)
    z = block_jacobi(A, r)
    assert np.linalg.norm(A.matvec(z) - r) <= 1e-12 * np.linalg.norm(r)


@pytest.mark.parametrize("k", [1, 2])
def test_block_jacobi_solves_each_dense_diagonal_block(k):
    # the cell blocks cut out of the dense matrix, solved one by one, on a
    # mesh with interior, boundary and corner cells
    prob = Problem(3, 2, 2, k=k, mask=0x2D)
    dg = ScalarDG(prob)
    Ad = dg.assemble("explicit")
    D = Ad.to_dense()
    N = Ad.bsize
    r = _rand(Ad.shape[0], 5)
    z = block_jacobi(Ad, r)
    for e in range(Ad.nelem):
        s = slice(e * N, (e + 1) * N)
        assert np.allclose(D[s, s] @ z[s], r[s], rtol=0, atol=1e-12 * np.abs(r).max())
    # the class-deduplicated storage gives the same result
    zd = block_jacobi(dg.assemble("dedup"), r)
    assert np.linalg.norm(zd - z) <= 1e-13 * np.linalg.norm(z)


@pytest.mark.parametrize("k", [2, 3, 4])
@pytest.mark.parametrize("cell", [13, 0, 2])  # interior (1,1,1), corner (0,0,0), edge (2,0,0)
def test_diagonal_block_is_a_kronecker_sum(k, cell):
    # The premise of inverting the block by fast diagonalization: with the
    # collocated GL basis on an axis-aligned cell and kappa = 1, the diagonal
    # block is sum_d (W x W x K_d), W = diag(w) on the two other directions.
    # So (1) two nodes that differ in two or three indices do not couple, and
    # (2) for nodes differing only along d the entry divided by the two
    # tangential weights does not depend on the tangential indices.
    p = k + 1
    prob = Problem(3, 3, 3, k=k)
    dg = ScalarDG(prob)
    A = dg.assemble("explicit")
    B = A.blocks[cell, 0]
    w = np.polynomial.legendre.leggauss(p)[1] / 2.0
    idx = [(i0, i1, i2) for i2 in range(p) for i1 in range(p) for i0 in range(p)]
    scale = np.abs(B).max()
    for a, ia in enumerate(idx):
        for b, ib in enumerate(idx):
            if sum(x != y for x, y in zip(ia, ib)) >= 2:
                assert abs(B[a, b]) <= 1e-13 * scale
    for d in range(3):
        t = [e for e in range(3) if e != d]
        ref = {}
        for a, ia in enumerate(idx):
            for b, ib in enumerate(idx):
                if ia[d] != ib[d] and all(ia[e] == ib[e] for e in t):
                    v = B[a, b] / (w[ia[t[0]]] * w[ia[t[1]]])
                    key = (ia[d], ib[d])
                    if key in ref:
                        assert abs(v - ref[key]) <= 1e-11 * scale / w.min() ** 2
                    else:
                        ref[key] = v


def test_pcg_with_exact_inverse_takes_one_iteration():
    A = ScalarDG(Problem(1, 1, 1, k=3)).assemble("explicit")
    b = _rand(A.shape[0], 7)
    x, its, res = pcg(A.matvec, lambda r: block_jacobi(A, r), b, rtol=1e-12)
    assert its == 1 and res <= 1e-12


@pytest.mark.parametrize("k", [2, 4])
def test_pcg_matches_cg_with_fewer_iterations(k):
    A = ScalarDG(Problem(3, 3, 3, k=k)).assemble("dedup")
    b = _rand(A.shape[0], 11)
    x0, it0, res0 = cg(A.matvec, b, rtol=1e-11)
    x1, it1, res1 = pcg(A.matvec, lambda r: block_jacobi(A, r), b, rtol=1e-11)
    assert res0 <= 1e-10 and res1 <= 1e-10
    assert np.linalg.norm(x1 - x0) <= 1e-8 * np.linalg.norm(x0)
    assert it1 < it0
