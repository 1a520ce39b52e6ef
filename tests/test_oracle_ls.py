"""Pins for the oracle's least-squares map (Section 2, eq. approx_map and the
column split) against independent methods: the full-height dense problem
solved by LAPACK's SVD least squares, exact rational normal equations, closed
forms and the fixed points the definition implies.  CPU only."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import pde_inputs as P


def to_scipy(A):
    return sp.csc_matrix((A.val, A.rowind, A.colptr), shape=(A.n, A.n))


def pat_scipy(S, val):
    return sp.csc_matrix((val, S.rowind, S.colptr), shape=(S.n, S.n))


def colmax_rel(M, Mref, S):
    """max over columns of ||m - m*||_inf / ||m*||_inf"""
    worst = 0.0
    for j in range(S.n):
        a, b = S.colptr[j], S.colptr[j + 1]
        den = np.abs(Mref[a:b]).max()
        if den > 0:
            worst = max(worst, np.abs(M[a:b] - Mref[a:b]).max() / den)
    return worst


def lstsq_map(Ak, A0, S, cols=None):
    """Each column solved on the FULL n-row dense problem with numpy's SVD
    least squares: independent of the row-set restriction and of QR."""
    Ad, A0d = Ak.to_dense(), A0.to_dense()
    M = np.full(S.nnz, np.nan)
    rho = np.full(S.n, np.nan)
    for j in (range(S.n) if cols is None else cols):
        J = S.rowind[S.colptr[j]:S.colptr[j + 1]]
        m, *_ = np.linalg.lstsq(Ad[:, J], A0d[:, j], rcond=None)
        M[S.colptr[j]:S.colptr[j + 1]] = m
        rho[j] = np.sum((Ad[:, J] @ m - A0d[:, j]) ** 2)
    return M, rho


@pytest.mark.parametrize("power", [1, 2, 3])
def test_config1_vs_lstsq(power):
    A0, (A1,) = P.config1()
    S = O.pattern(A1, power)
    M, rho, st, _ = O.sam_build(A1, A0, S)
    cols = np.arange(0, A1.n, 7)
    Ml, rl = lstsq_map(A1, A0, S, cols)
    sel = np.concatenate([np.arange(S.colptr[j], S.colptr[j + 1]) for j in cols])
    assert np.max(np.abs(M[sel] - Ml[sel]) / np.abs(Ml[sel]).max()) < 1e-12
    assert np.allclose(rho[cols], rl[cols], rtol=1e-9, atol=1e-14)


def test_nonsymmetric_vs_lstsq():
    A0, As = P.config3(m=6)
    Ak = As[-1]
    S = O.pattern(Ak, 2)
    M, rho, st, _ = O.sam_build(Ak, A0, S)
    Ml, rl = lstsq_map(Ak, A0, S)
    assert colmax_rel(M, Ml, S) < 1e-12
    assert np.allclose(rho, rl, rtol=1e-9, atol=1e-14)


def test_exact_rational_normal_equations():
    """Small integer blocks: the unique minimiser solves A^T A m = A^T b
    exactly; compare with the rational solution."""
    rng = np.random.default_rng(11)
    n = 9
    Bd = rng.random((n, n)) < 0.35
    Ad = np.where(Bd, rng.integers(-3, 4, (n, n)), 0).astype(float) + 6 * np.eye(n)
    A0d = np.where(rng.random((n, n)) < 0.3, rng.integers(-2, 3, (n, n)), 0).astype(float) + np.eye(n)
    Ak, A0 = P.dense_to_csc(Ad), P.dense_to_csc(A0d)
    S = O.pattern(Ak, 1)
    M, rho, _, _ = O.sam_build(Ak, A0, S)
    for j in range(n):
        J = list(S.rowind[S.colptr[j]:S.colptr[j + 1]])
        A = [[Fraction(int(Ad[i, l])) for l in J] for i in range(n)]
        b = [Fraction(int(A0d[i, j])) for i in range(n)]
        k = len(J)
        G = [[sum(A[i][a] * A[i][c] for i in range(n)) for c in range(k)] for a in range(k)]
        g = [sum(A[i][a] * b[i] for i in range(n)) for a in range(k)]
        # Gauss-Jordan in exact arithmetic
        for c in range(k):
            piv = next(r for r in range(c, k) if G[r][c] != 0)
            G[c], G[piv] = G[piv], G[c]
            g[c], g[piv] = g[piv], g[c]
            for r in range(k):
                if r != c and G[r][c] != 0:
                    f = G[r][c] / G[c][c]
                    G[r] = [x - f * y for x, y in zip(G[r], G[c])]
                    g[r] -= f * g[c]
        m_exact = np.array([float(g[c] / G[c][c]) for c in range(k)])
        m = M[S.colptr[j]:S.colptr[j + 1]]
        assert np.max(np.abs(m - m_exact)) <= 1e-13 * max(1.0, np.abs(m_exact).max())


def test_single_entry_closed_form():
    """|J_j| = 1 (diagonal pattern): m = a^T b / a^T a with a = A_k(:,j)."""
    A0, (A1,) = P.config1()
    n = A1.n
    S = O.Pattern(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32))
    M, rho, _, _ = O.sam_build(A1, A0, S)
    Ad, A0d = A1.to_dense(), A0.to_dense()
    want = np.einsum("ij,ij->j", Ad, A0d) / np.einsum("ij,ij->j", Ad, Ad)
    assert np.allclose(M, want, rtol=1e-13, atol=0)
    r = Ad * want - A0d
    assert np.allclose(rho, (r ** 2).sum(axis=0), rtol=1e-10)


def test_full_pattern_gives_exact_map():
    """S full: M = A_k^{-1} A_0 (eq. exact_map) and R = 0."""
    A0, As = P.config3(m=3)
    Ak = As[2]
    n = Ak.n
    S = O.Pattern(n, (np.arange(n + 1) * n).astype(np.int32), np.tile(np.arange(n), n).astype(np.int32))
    M, rho, _, _ = O.sam_build(Ak, A0, S)
    N = np.linalg.solve(Ak.to_dense(), A0.to_dense())
    assert np.abs(M.reshape(n, n).T - N).max() < 1e-11 * np.abs(N).max()
    assert rho.max() < 1e-20 * (A0.val ** 2).sum()


def test_identity_when_source_equals_target():
    A0, _ = P.config1()
    S = O.pattern(A0, 2)
    M, rho, _, _ = O.sam_build(A0, A0, S)
    cols = np.repeat(np.arange(S.n), np.diff(S.colptr))
    assert np.abs(M - (S.rowind == cols)).max() < 1e-13
    assert rho.max() < 1e-24 * (A0.val ** 2).sum()


def test_column_scaling_fixed_point():
    """A_k = A_0 D  =>  M = D^{-1} and R = 0."""
    A0, _ = P.config1()
    rng = np.random.default_rng(5)
    d = rng.uniform(0.5, 2.0, A0.n)
    cols = np.repeat(np.arange(A0.n), np.diff(A0.colptr))
    Ak = A0.with_values(A0.val * d[cols])
    S = O.pattern(Ak, 1)
    M, rho, _, _ = O.sam_build(Ak, A0, S)
    scol = np.repeat(np.arange(S.n), np.diff(S.colptr))
    want = np.where(S.rowind == scol, 1.0 / d[scol], 0.0)
    assert np.abs(M - want).max() < 1e-13
    assert rho.max() < 1e-24 * (A0.val ** 2).sum()


def test_invariances():
    """Common scalar and a common row permutation leave M unchanged; column
    scaling of A_k by D maps M to D^{-1} M (fixed pattern S)."""
    A0, As = P.config3(m=4)
    Ak = As[3]
    S = O.pattern(Ak, 2)
    M, rho, _, _ = O.sam_build(Ak, A0, S)
    M2, rho2, _, _ = O.sam_build(Ak.with_values(3.5 * Ak.val), A0.with_values(3.5 * A0.val), S)
    assert colmax_rel(M2, M, S) < 1e-13
    assert np.allclose(rho2, 3.5 ** 2 * rho, rtol=1e-10, atol=1e-20)
    rng = np.random.default_rng(9)
    perm = rng.permutation(Ak.n)
    Akp = P.dense_to_csc(Ak.to_dense()[perm])
    A0p = P.dense_to_csc(A0.to_dense()[perm])
    M3, rho3, _, _ = O.sam_build(Akp, A0p, S)
    assert colmax_rel(M3, M, S) < 1e-12
    d = rng.uniform(0.5, 2.0, Ak.n)
    cols = np.repeat(np.arange(Ak.n), np.diff(Ak.colptr))
    M4, _, _, _ = O.sam_build(Ak.with_values(Ak.val * d[cols]), A0, S)
    assert colmax_rel(M4 * d[S.rowind], M, S) < 1e-12


def test_zero_residual_when_pattern_contains_exact_map():
    """Block-diagonal A_k: the exact map lives inside the closure pattern,
    so the SAM on that pattern has zero residual."""
    rng = np.random.default_rng(21)
    blocks = [rng.uniform(-1, 1, (3, 3)) + 3 * np.eye(3) for _ in range(5)]
    Ad = np.zeros((15, 15))
    A0d = np.zeros((15, 15))
    for b, B in enumerate(blocks):
        s = slice(3 * b, 3 * b + 3)
        Ad[s, s] = B
        A0d[s, s] = np.triu(rng.uniform(-1, 1, (3, 3))) + np.eye(3)
    Ak, A0 = P.dense_to_csc(Ad), P.dense_to_csc(A0d)
    S = O.pattern(Ak, 15)
    M, rho, _, _ = O.sam_build(Ak, A0, S)
    assert rho.max() < 1e-26 * (A0d ** 2).sum()
    r2, _ = O.residual(Ak, A0, S, M)
    assert r2 < 1e-26 * (A0d ** 2).sum()


def test_residual_matches_scipy_and_column_sum():
    A0, As = P.config3(m=5)
    Ak = As[-1]
    S = O.pattern(Ak, 2)
    M, rho, _, _ = O.sam_build(Ak, A0, S)
    r2, a2 = O.residual(Ak, A0, S, M)
    R = to_scipy(Ak) @ pat_scipy(S, M) - to_scipy(A0)
    assert np.isclose(r2, sp.linalg.norm(R, "fro") ** 2, rtol=1e-12)
    assert np.isclose(a2, sp.linalg.norm(to_scipy(A0), "fro") ** 2, rtol=1e-14)
    assert np.isclose(r2, rho.sum(), rtol=1e-9)


def test_out_of_rowset_term():
    """A_0 entries outside I_j only add out_j to the residual: build a target
    with an entry no column of J_j can reach."""
    n = 6
    Ad = np.eye(n) * 2.0
    Ad[1, 0] = 1.0
    A0d = np.eye(n)
    A0d[5, 0] = 3.0  # row 5 is not in I_0 = {0, 1}
    Ak, A0 = P.dense_to_csc(Ad), P.dense_to_csc(A0d)
    S = O.pattern(Ak, 1)
    M, rho, _, _ = O.sam_build(Ak, A0, S)
    Ml, rl = lstsq_map(Ak, A0, S)
    assert np.allclose(M, Ml, atol=1e-14)
    assert np.isclose(rho[0], rl[0]) and rho[0] >= 9.0


def test_apply_matches_scipy():
    A0, (A1,) = P.config1()
    S = O.pattern(A1, 2)
    M, _, _, _ = O.sam_build(A1, A0, S)
    x = np.random.default_rng(1).standard_normal(A1.n)
    assert np.allclose(O.apply(S, M, x), pat_scipy(S, M) @ x, rtol=1e-13, atol=1e-13)


def test_rank_deficient_block_reported():
    """Two identical columns in J_j make the block rank deficient."""
    n = 5
    Ad = np.eye(n) * 2.0
    Ad[:, 3] = Ad[:, 2]          # columns 2 and 3 identical -> singular A_k
    Ad[4, 2] = Ad[4, 3] = 1.0
    Ak = P.dense_to_csc(Ad)
    S = O.Pattern(n, np.array([0, 1, 2, 4, 5, 6], dtype=np.int32),
                  np.array([0, 1, 2, 3, 3, 4], dtype=np.int32))
    _, _, st, bad = O.sam_build(Ak, Ak, S, raise_on_error=False)
    assert st == 5 and bad == 2
    with pytest.raises(O.OracleError):
        O.sam_build(Ak, Ak, S)


def test_column_subset_matches_full():
    A0, As = P.config2(m=24, nmat=3)
    S = O.pattern(As[1], 2)
    M, rho, _, _ = O.sam_build(As[1], A0, S)
    cols = np.array([0, 5, 77, 300, 575])
    Mc, rc, _, _ = O.sam_build(As[1], A0, S, cols=cols)
    for j in cols:
        a, b = S.colptr[j], S.colptr[j + 1]
        assert np.array_equal(Mc[a:b], M[a:b])
    assert np.array_equal(rc[cols], rho[cols])
    assert np.isnan(rc[1])


def test_near_diagonal_blocks_stable():
    """Off-diagonal couplings 1e-9 of the diagonal: the Householder vector
    must be formed without cancellation (beta of opposite sign to alpha), or
    the map loses all accuracy against the SVD solution."""
    rng = np.random.default_rng(4)
    n = 40
    Bd = rng.random((n, n)) < 0.1
    Ad = np.where(Bd, 1e-9 * rng.uniform(-1, 1, (n, n)), 0.0) + np.diag(rng.uniform(1, 2, n))
    A0d = np.where(Bd, rng.uniform(-1, 1, (n, n)), 0.0) + np.eye(n)
    Ak, A0 = P.dense_to_csc(Ad), P.dense_to_csc(A0d)
    S = O.pattern(Ak, 2)
    M, rho, _, _ = O.sam_build(Ak, A0, S)
    Ml, rl = lstsq_map(Ak, A0, S)
    assert colmax_rel(M, Ml, S) < 1e-10


def test_frobenius_sum_is_exactly_rounded():
    """The oracle's ||R||_F^2 (sum of column residuals) equals the exact
    rational sum of the same doubles, rounded once, also where plain
    left-to-right summation loses the small terms."""
    rng = np.random.default_rng(7)
    rho = np.concatenate([[1e16], rng.uniform(0, 1, 5000), [-1e16]])
    exact = float(sum(Fraction(float(x)) for x in rho))
    assert O.frobenius_sq(rho) == exact
    naive = 0.0
    for x in rho:
        naive += x
    assert naive != exact          # the case does separate the two sums
    r = rng.uniform(0, 1, 1000)
    assert O.frobenius_sq(r) == float(sum(Fraction(float(x)) for x in r))
