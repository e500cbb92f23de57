"""Pins of the oracle's SIPG diffusion-reaction operator (Section 5.2,
eq. diffreac_weak) against things other than itself."""
import math

import mpmath
import numpy as np
import pytest

from oracle import gauss_legendre, Problem, ScalarDG, cg
from oracle.blocks import slot
from oracle.problem import basis_tables
import workloads

mpmath.mp.dps = 50


# ---------------------------------------------------------------------------
# closed-form element and face matrices on an axis-aligned cube
# ---------------------------------------------------------------------------
def _mp_gl_nodes(p):
    """GL nodes on [0,1] at 50 digits by polishing numpy's nodes with findroot."""
    t, _ = np.polynomial.legendre.leggauss(p)
    return [mpmath.findroot(lambda s: mpmath.legendre(p, 2 * s - 1), (float(ti) + 1) / 2) for ti in t]


def _mp_lagrange(nodes, j, s):
    v = mpmath.mpf(1)
    for i, xi in enumerate(nodes):
        if i != j:
            v *= (s - xi) / (nodes[j] - xi)
    return v


def _mp_dlagrange(nodes, j, s):
    return mpmath.diff(lambda t: _mp_lagrange(nodes, j, t), s)


def _closed_form_1d(p):
    nodes = _mp_gl_nodes(p)
    M = np.zeros((p, p))
    K = np.zeros((p, p))
    for i in range(p):
        for j in range(p):
            M[i, j] = float(mpmath.quad(lambda s: _mp_lagrange(nodes, i, s) * _mp_lagrange(nodes, j, s), [0, 1]))
            K[i, j] = float(mpmath.quad(lambda s: _mp_dlagrange(nodes, i, s) * _mp_dlagrange(nodes, j, s), [0, 1]))
    e = [np.array([float(_mp_lagrange(nodes, j, mpmath.mpf(s))) for j in range(p)]) for s in (0, 1)]
    de = [np.array([float(_mp_dlagrange(nodes, j, mpmath.mpf(s))) for j in range(p)]) for s in (0, 1)]
    return M, K, e, de


@pytest.mark.parametrize("k", [1, 2, 3])
def test_closed_form_kronecker_blocks(k):
    """Volume block = c h^3 M(x)M(x)M + h (K(x)M(x)M + M(x)K(x)M + M(x)M(x)K) and
    face blocks = h^2 (M(x)M) (x) (1D normal factor), all 1D factors from 50-digit
    quadrature; lexicographic index i0 fastest, so the x factor is last in kron."""
    p = k + 1
    n = 2
    h = 1.0 / n
    c = 1.7
    M, K, e, de = _closed_form_1d(p)
    kr = lambda a, b, cc: np.kron(cc, np.kron(b, a))  # a acts on x (fastest)
    pr = Problem(n, n, n, k=k, c=c)
    op = ScalarDG(pr)
    vol = c * h ** 3 * kr(M, M, M) + h * (kr(K, M, M) + kr(M, K, M) + kr(M, M, K))
    assert np.max(np.abs(op.volume_block(0) - vol)) < 1e-13 * np.max(np.abs(vol))
    gam = 3.0 * k * (k + 1) / h  # alpha k(k+1) |F| / |T| with alpha = 3 on a cube of side h
    th = pr.theta
    # boundary face x = 0 of cell 0: outward normal -e_x, d/dn = -(1/h) d/dxi
    N1 = (-np.outer(e[0], -de[0] / h) + th * np.outer(-de[0] / h, e[0]) + gam * np.outer(e[0], e[0]))
    ref = h * h * kr(N1, M, M)
    got = op.boundary_block(0, 0, 0)
    assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref))
    # interior face between cells 0 (T-) and 1 (T+) along x, n = +e_x
    B = op.interior_face_blocks(0, 1, 0)
    sides = [(e[1], de[1] / h, 1.0), (e[0], de[0] / h, -1.0)]  # trace, normal derivative, jump sign
    for a in range(2):
        for b in range(2):
            ea, da, sa = sides[a]
            eb, db, sb = sides[b]
            N1 = (-sa * 0.5 * np.outer(ea, db) + th * sb * 0.5 * np.outer(da, eb) + gam * sa * sb * np.outer(ea, eb))
            ref = h * h * kr(N1, M, M)
            assert np.max(np.abs(B[a][b] - ref)) < 1e-13 * np.max(np.abs(ref)), (a, b)


# ---------------------------------------------------------------------------
# structure: symmetry, definiteness, explicit vs deduplicated storage
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("k,n", [(1, 3), (2, 2), (3, 2)])
def test_sipg_symmetric(k, n):
    pr = Problem(n, n, n, k=k, kappa=workloads.lognormal(n ** 3 * (k + 1) ** 3, 7))
    A = ScalarDG(pr).assemble("explicit").to_dense()
    assert np.max(np.abs(A - A.T)) <= 1e-14 * np.max(np.abs(A))


def test_nonsymmetric_variant_is_not_symmetric():
    pr = Problem(2, 2, 2, k=2, theta=1.0)
    A = ScalarDG(pr).assemble("explicit").to_dense()
    assert np.max(np.abs(A - A.T)) > 1e-3 * np.max(np.abs(A))


@pytest.mark.parametrize("k", [2, 3, 4, 5])
@pytest.mark.parametrize("n", [1, 2])
def test_sipg_positive_definite(k, n):
    """The k(k+1)/h penalty is coercive: Cholesky succeeds."""
    if k == 5 and n == 2:
        pytest.skip("covered by smaller cases; dense 1728^2 factorisation is slow")
    A = ScalarDG(Problem(n, n, n, k=k)).assemble().to_dense()
    np.linalg.cholesky(A)


def test_dedup_matches_explicit():
    op = ScalarDG(Problem(3, 2, 4, k=2))
    A1 = op.assemble("explicit").to_dense()
    A2 = op.assemble("dedup").to_dense()
    assert np.max(np.abs(A1 - A2)) <= 1e-14 * np.max(np.abs(A1))


def test_matvec_rmatvec_rows_agree_with_dense():
    pr = Problem(3, 2, 2, k=2, theta=1.0, kappa=workloads.lognormal(12 * 27, 3))
    op = ScalarDG(pr)
    A = op.assemble("explicit")
    D = A.to_dense()
    x = workloads.uniform(D.shape[0], 1)
    g = workloads.uniform(D.shape[0], 2)
    assert np.max(np.abs(A.matvec(x) - D @ x)) < 1e-12
    assert np.max(np.abs(A.rmatvec(g) - D.T @ g)) < 1e-12
    rows = [0, 5, 11]
    assert np.max(np.abs(op.apply_rows(x, rows) - (D @ x).reshape(-1, 27)[rows])) < 1e-12
    assert np.max(np.abs(op.apply_T_rows(g, rows) - (D.T @ g).reshape(-1, 27)[rows])) < 1e-12


def test_kronecker_identity_of_tensor_basis():
    """(A(x)A(x)A) X evaluated factor by factor (Section 2.2) equals the oracle's
    product-of-1D-factors basis table, pinning its lexicographic ordering."""
    p, m = 4, 6
    nodes, _ = gauss_legendre(p)
    xq, _ = gauss_legendre(m)
    from oracle import lagrange_eval
    A1 = lagrange_eval(nodes, xq)  # (m, p)
    q = np.arange(m ** 3)
    xi = np.stack([xq[q % m], xq[(q // m) % m], xq[q // (m * m)]], axis=1)
    phi, _ = basis_tables(nodes, xi)
    X = workloads.uniform(p ** 3, 9)
    T = X.reshape(p, p, p)  # [i2, i1, i0]
    T = np.einsum("ai,zyi->zya", A1, T)
    T = np.einsum("bj,zjx->zbx", A1, T)
    T = np.einsum("ck,kyx->cyx", A1, T)
    assert np.max(np.abs(T.reshape(-1) - phi @ X)) < 1e-13


# ---------------------------------------------------------------------------
# consistency and exactness on polynomial and manufactured solutions
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("k", [2, 3])
def test_polynomial_consistency(k):
    """For u in Q_k with Dirichlet data u, A u_I equals (f, v) plus the Dirichlet
    terms exactly (SIPG is consistent and every integrand is a polynomial the
    rule integrates exactly)."""
    c = 2.5
    cases = [
        (lambda x: np.ones(len(x)), lambda x: c * np.ones(len(x))),
        (lambda x: x[:, 0] - 2 * x[:, 2], lambda x: c * (x[:, 0] - 2 * x[:, 2])),
        (lambda x: (x * x).sum(1), lambda x: -6.0 + c * (x * x).sum(1)),
        (lambda x: x[:, 0] * x[:, 1] ** 2 + x[:, 2], lambda x: -2 * x[:, 0] + c * (x[:, 0] * x[:, 1] ** 2 + x[:, 2])),
    ]
    op = ScalarDG(Problem(3, 2, 2, k=k, c=c))
    A = op.assemble()
    for u, f in cases:
        uI = op.interpolate(u)
        b = op.load_vector(f, u)
        r = A.matvec(uI) - b
        assert np.max(np.abs(r)) < 1e-11 * max(1.0, np.max(np.abs(b))), np.max(np.abs(r))


@pytest.mark.parametrize("k", [2, 3])
def test_paper_manufactured_solution_tensor_coefficient(k):
    """Section 5.2's data K = x x^T + I, c = 10, f = -6, g = |x|^2: u = |x|^2 solves
    the PDE, lies in Q_k and every integrand has degree <= 2m-1, so the discrete
    residual of its interpolant vanishes."""
    Kfn = lambda x: np.einsum("pa,pb->pab", x, x) + np.eye(3)[None]
    pr = Problem(2, 3, 2, k=k, c=10.0, kappa_tensor=Kfn)
    op = ScalarDG(pr)
    A = op.assemble("explicit")
    g = lambda x: (x * x).sum(1)
    uI = op.interpolate(g)
    b = op.load_vector(lambda x: -6.0 * np.ones(len(x)), g)
    r = A.matvec(uI) - b
    assert np.max(np.abs(r)) < 1e-12 * np.max(np.abs(b))
    # and the solve reproduces it
    import scipy.sparse.linalg as spla
    u = spla.spsolve(A.to_scipy().tocsc(), b)
    assert np.max(np.abs(u - uI)) < 1e-10


@pytest.mark.slow
@pytest.mark.parametrize("k", [1, 2, 3])
def test_manufactured_sin_convergence_rate(k):
    """SIPG L2 error for u = sin(pi x) sin(pi y) sin(pi z) decays like h^(k+1)."""
    import scipy.sparse.linalg as spla
    errs = []
    ns = [2, 4, 8] if k < 3 else [2, 4]
    for n in ns:
        op = ScalarDG(Problem(n, n, n, k=k))
        A = op.assemble()
        b = op.load_vector(lambda x: workloads.sin_forcing(x, 1.0))
        u = spla.spsolve(A.to_scipy().tocsc(), b)
        errs.append(op.l2_error(u, workloads.sin_solution))
    rate = math.log2(errs[-2] / errs[-1])
    assert rate > k + 1 - 0.35, (errs, rate)


def test_oracle_cg_solves():
    op = ScalarDG(Problem(3, 3, 3, k=2))
    A = op.assemble()
    b = op.load_vector(lambda x: workloads.sin_forcing(x, 1.0))
    x, its, res = cg(A.matvec, b, rtol=1e-10)
    assert res < 2e-10 and its > 10
    import scipy.sparse.linalg as spla
    xd = spla.spsolve(A.to_scipy().tocsc(), b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-8


# ---------------------------------------------------------------------------
# derivative with respect to kappa: L = g^T A(kappa) u is affine in kappa
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("theta", [-1.0, 1.0])
def test_kappa_gradient_matches_finite_differences(theta):
    n, k = 2, 2
    M = (k + 1) ** 3
    kap = workloads.lognormal(n ** 3 * M, 11)
    u = workloads.uniform(n ** 3 * 27, 12)
    g = workloads.uniform(n ** 3 * 27, 13)
    op = ScalarDG(Problem(n, n, n, k=k, theta=theta, kappa=kap, mask=0x2B))
    grad = op.kappa_gradient(u, g).reshape(-1)
    rng = np.random.default_rng(0)
    for j in rng.choice(len(kap), 12, replace=False):
        vals = []
        for step in (+1.0, -1.0):
            kk = kap.copy()
            kk[j] += step
            A = ScalarDG(Problem(n, n, n, k=k, theta=theta, kappa=kk, mask=0x2B)).assemble("explicit")
            vals.append(g @ A.matvec(u))
        fd = (vals[0] - vals[1]) / 2.0  # exact: L is affine in kappa
        assert abs(fd - grad[j]) < 1e-11 * max(1.0, abs(fd)), (j, fd, grad[j])


def test_kappa_gradient_volume_closed_form_when_faces_use_one():
    """With kappa = 1 on faces only the volume term w |J| grad u . grad g remains;
    for u = x and g = y it vanishes, for u = g = x it is w |J|."""
    n, k = 2, 2
    kap = workloads.lognormal(n ** 3 * 27, 5)
    op = ScalarDG(Problem(n, n, n, k=k, kappa=kap, kappa_face_one=True))
    ux = op.interpolate(lambda x: x[:, 0])
    uy = op.interpolate(lambda x: x[:, 1])
    assert np.max(np.abs(op.kappa_gradient(ux, uy))) < 1e-13
    h3 = (1.0 / n) ** 3
    ref = np.tile(op.prob.cell_w * h3, (n ** 3, 1))
    assert np.max(np.abs(op.kappa_gradient(ux, ux) - ref)) < 1e-13


# ---------------------------------------------------------------------------
# kappa per volume quadrature point: layout and face traces; the paper's penalty
# ---------------------------------------------------------------------------
def _layout_points(nx, ny, nz, m):
    """Physical volume points in the library's kappa layout, written out from its
    definition (cell e = ex + nx (ey + ny ez), point q0 + m (q1 + m q2), nodes of
    numpy's Gauss-Legendre rule mapped to [0, 1])."""
    t, _ = np.polynomial.legendre.leggauss(m)
    xi = (t + 1.0) / 2.0
    pts = []
    for ez in range(nz):
        for ey in range(ny):
            for ex in range(nx):
                for q2 in range(m):
                    for q1 in range(m):
                        for q0 in range(m):
                            pts.append(((ex + xi[q0]) / nx, (ey + xi[q1]) / ny, (ez + xi[q2]) / nz))
    return np.array(pts)


def _kappa_linear(X):
    return 1.0 + X[:, 0] + 2.0 * X[:, 1] + 3.0 * X[:, 2]


@pytest.mark.parametrize("theta", [-1.0, 1.0])
def test_kappa_per_point_layout_and_face_trace(theta):
    """kappa(x) = 1 + x + 2y + 3z sampled in the layout above and passed per point
    gives the same matrix as the full-tensor path with K = kappa(x) I evaluated
    directly at every volume and face point (eq. diffreac_weak): the function is
    not symmetric in x, y, z, so a permuted point layout or cell order fails, and
    it has degree 1 per direction, so the face-trace interpolant of the point
    values is exact. Mixed Dirichlet / natural sides, a non-cubic mesh."""
    nx, ny, nz, k, mask = 3, 2, 2, 2, 0x2B
    kap = _kappa_linear(_layout_points(nx, ny, nz, k + 1))
    K = lambda X: _kappa_linear(X)[:, None, None] * np.eye(3)[None]
    A1 = ScalarDG(Problem(nx, ny, nz, k=k, theta=theta, mask=mask, kappa=kap)).assemble("explicit").to_dense()
    A2 = ScalarDG(Problem(nx, ny, nz, k=k, theta=theta, mask=mask, kappa_tensor=K)).assemble("explicit").to_dense()
    assert np.max(np.abs(A1 - A2)) <= 1e-13 * np.max(np.abs(A2))
    # the check has teeth: the same values with the point axes q0 and q2 swapped differ
    m = k + 1
    swapped = kap.reshape(-1, m, m, m).transpose(0, 3, 2, 1).reshape(-1)
    A3 = ScalarDG(Problem(nx, ny, nz, k=k, theta=theta, mask=mask, kappa=swapped)).assemble("explicit").to_dense()
    assert np.max(np.abs(A3 - A2)) > 1e-3 * np.max(np.abs(A2))


def _lagrange_at(nodes, s):
    return np.array([np.prod([(s - xi) / (xj - xi) for i, xi in enumerate(nodes) if i != j])
                     for j, xj in enumerate(nodes)])


@pytest.mark.parametrize("k", [1, 2, 3])
def test_paper_penalty_form(k):
    """penalty_form = 1 is the paper's gamma_F = alpha k(k+d-1)|F|/min|T| (Section 5.2),
    3k(k+2)/h on cubes of side h, against 3k(k+1)/h for penalty_form = 0: the two
    matrices differ by 3k/h times sum_F ([u], [v])_F over interior and Dirichlet
    faces, written out here with Kronecker products of 1D factors (numpy nodes and
    weights, Lagrange values at 0 and 1 by the product formula)."""
    n, p = 2, k + 1
    h = 1.0 / n
    t, wt = np.polynomial.legendre.leggauss(p)
    nodes, w = (t + 1.0) / 2.0, wt / 2.0
    e = [_lagrange_at(nodes, 0.0), _lagrange_at(nodes, 1.0)]
    Mt = h * np.diag(w)  # tangential 1D mass of the collocated basis
    kr = lambda a, b, c: np.kron(c, np.kron(b, a))  # a acts on x (fastest)

    def face(d, N1):
        f = [Mt, Mt, Mt]
        f[d] = N1
        return kr(*f)

    N = p ** 3
    S = np.zeros((n ** 3 * N, n ** 3 * N))
    cell = lambda c: c[0] + n * (c[1] + n * c[2])
    for ez in range(n):
        for ey in range(n):
            for ex in range(n):
                c = (ex, ey, ez)
                a = cell(c)
                for d in range(3):
                    for s in range(2):
                        nb = list(c)
                        nb[d] += 1 if s else -1
                        if 0 <= nb[d] < n:
                            b = cell(nb)
                            # ([u],[v]) seen from cell a: own trace at side s, neighbour's at side 1-s
                            S[a * N:(a + 1) * N, a * N:(a + 1) * N] += face(d, np.outer(e[s], e[s]))
                            S[a * N:(a + 1) * N, b * N:(b + 1) * N] -= face(d, np.outer(e[s], e[1 - s]))
                        else:
                            S[a * N:(a + 1) * N, a * N:(a + 1) * N] += face(d, np.outer(e[s], e[s]))
    A0 = ScalarDG(Problem(n, n, n, k=k, penalty_form=0)).assemble("explicit").to_dense()
    A1 = ScalarDG(Problem(n, n, n, k=k, penalty_form=1)).assemble("explicit").to_dense()
    ref = (3.0 * k * (k + 2) / h - 3.0 * k * (k + 1) / h) * S
    assert np.max(np.abs((A1 - A0) - ref)) <= 1e-13 * np.max(np.abs(A1))


@pytest.mark.parametrize("mode", ["explicit", "dedup"])
def test_c_block_spmv_matches_numpy(mode):
    """The oracle's C block SpMV (used for the CPU baseline timing) against the
    NumPy block products and the dense matrix, 1 and 4 threads."""
    from oracle.blocks import CBlockMatvec
    op = ScalarDG(Problem(3, 2, 4, k=2, theta=1.0))
    A = op.assemble(mode)
    x = workloads.uniform(A.shape[0], 17)
    ref = A.to_dense() @ x
    mv = CBlockMatvec(A)
    for t in (1, 4):
        y = mv(x, threads=t)
        assert np.max(np.abs(y - ref)) <= 1e-13 * np.max(np.abs(ref))
        assert np.max(np.abs(y - A.matvec(x))) <= 1e-13 * np.max(np.abs(ref))
