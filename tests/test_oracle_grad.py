"""Pins for the oracle's soft-weighted map and its gradient: central finite
differences of the oracle's own forward loss, the w -> 0 and w = 1 limits.
CPU only."""
import numpy as np
import pytest

import oracle as O
import pde_inputs as P


def small_problem(seed=0, m=4):
    rng = np.random.default_rng(seed)
    k0 = rng.lognormal(0.0, 0.5, (m, m, m))
    k1 = k0 * np.exp(0.1 * rng.standard_normal((m, m, m)))
    A0, A1 = P.diffusion_3d(k0), P.diffusion_3d(k1)
    S = O.pattern(A1, 2)
    w = P.candidate_weights(A1.n, S.colptr, S.rowind, A1, seed=seed)
    mu = P.penalty_scale(A1)
    return A0, A1, S, w, mu


def loss(Ak, A0, S, w, mu):
    M, rho, _, _ = O.sam_build(Ak, A0, S, weights=w, mu=mu)
    return rho.sum()


def central(f, x, idx, h):
    xp = x.copy(); xp[idx] += h
    xm = x.copy(); xm[idx] -= h
    return (f(xp) - f(xm)) / (2 * h)


@pytest.mark.parametrize("seed", [0, 3])
def test_weighted_map_solves_penalised_normal_equations(seed):
    """Direct pin of the soft-weighted map: for every column, m solves
    (A^T A + P) m = A^T b with A = A_k(:, J_j) taken whole (all n rows, so no
    row set is involved), b = A_0(:, j) and P = diag(mu (1/w - 1)), by
    numpy's dense solver; the column residual is ||A m - b||^2 without the
    penalty."""
    import scipy.sparse as sp
    A0, A1, S, w, mu = small_problem(seed)
    M, rho, _, _ = O.sam_build(A1, A0, S, weights=w, mu=mu)
    Ak = sp.csc_matrix((A1.val, A1.rowind, A1.colptr), shape=(A1.n, A1.n)).toarray()
    A0d = sp.csc_matrix((A0.val, A0.rowind, A0.colptr), shape=(A0.n, A0.n)).toarray()
    worst = 0.0
    for j in range(A1.n):
        a, b = S.colptr[j], S.colptr[j + 1]
        J = S.rowind[a:b]
        A = Ak[:, J]
        p = mu * (1.0 / w[a:b] - 1.0)
        m = np.linalg.solve(A.T @ A + np.diag(p), A.T @ A0d[:, j])
        worst = max(worst, np.abs(M[a:b] - m).max() / np.abs(m).max())
        r = A @ m - A0d[:, j]
        assert np.isclose(rho[j], r @ r, rtol=1e-9, atol=1e-15)
    assert worst <= 1e-10, worst
    assert (w < 1.0).any() and (w > 0.0).all()    # the penalty is active on the candidates


def test_loss_equals_build_residual():
    A0, A1, S, w, mu = small_problem(1)
    gAk, gA0, gw, L = O.backward(A1, A0, S, w, mu)
    assert np.isclose(L, loss(A1, A0, S, w, mu), rtol=1e-13)


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_vs_central_fd(seed):
    A0, A1, S, w, mu = small_problem(seed)
    gAk, gA0, gw, L = O.backward(A1, A0, S, w, mu)
    rng = np.random.default_rng(seed + 50)
    scale = np.abs(gAk).max()
    for e in rng.choice(A1.nnz, 12, replace=False):
        h = 1e-6 * max(1.0, abs(A1.val[e]))
        fd = central(lambda v: loss(A1.with_values(v), A0, S, w, mu), A1.val, e, h)
        assert abs(fd - gAk[e]) <= 1e-6 * scale, (e, fd, gAk[e])
    scale = np.abs(gA0).max()
    for e in rng.choice(A0.nnz, 12, replace=False):
        h = 1e-6 * max(1.0, abs(A0.val[e]))
        fd = central(lambda v: loss(A1, A0.with_values(v), S, w, mu), A0.val, e, h)
        assert abs(fd - gA0[e]) <= 1e-6 * scale, (e, fd, gA0[e])
    cand = np.nonzero(w < 1.0)[0]
    scale = np.abs(gw).max()
    for e in rng.choice(cand, 12, replace=False):
        h = 1e-6
        fd = central(lambda ww: loss(A1, A0, S, ww, mu), w, e, h)
        assert abs(fd - gw[e]) <= 1e-6 * scale, (e, fd, gw[e])


def test_directional_derivative():
    A0, A1, S, w, mu = small_problem(3)
    gAk, gA0, gw, L = O.backward(A1, A0, S, w, mu)
    rng = np.random.default_rng(8)
    dA = rng.standard_normal(A1.nnz)
    d0 = rng.standard_normal(A0.nnz)
    h = 1e-6
    f = lambda t: loss(A1.with_values(A1.val + t * dA), A0.with_values(A0.val + t * d0), S, w, mu)
    fd = (f(h) - f(-h)) / (2 * h)
    an = gAk @ dA + gA0 @ d0
    assert abs(fd - an) <= 1e-6 * abs(an)


def test_unit_weights_envelope():
    """w = 1 everywhere: no penalty, lambda = 0 at the least-squares optimum
    (A^T r = 0), so dL/dA_k(i,l) reduces to the envelope term
    sum_j 2 r_j(i) m_j(l), evaluated here with scipy's sparse products."""
    import scipy.sparse as sp
    A0, A1, S, w, mu = small_problem(2)
    ones = np.ones(S.nnz)
    gAk, gA0, gw, L = O.backward(A1, A0, S, ones, mu)
    M, _, _, _ = O.sam_build(A1, A0, S)
    Ms = sp.csc_matrix((M, S.rowind, S.colptr), shape=(S.n, S.n))
    As = sp.csc_matrix((A1.val, A1.rowind, A1.colptr), shape=(A1.n, A1.n))
    A0s = sp.csc_matrix((A0.val, A0.rowind, A0.colptr), shape=(A0.n, A0.n))
    R = (As @ Ms - A0s).toarray()
    G = 2 * R @ Ms.toarray().T
    cols = np.repeat(np.arange(A1.n), np.diff(A1.colptr))
    assert np.allclose(gAk, G[A1.rowind, cols], rtol=1e-8, atol=1e-10 * np.abs(G).max())
    assert np.allclose(gA0, -2 * R[A0.rowind, np.repeat(np.arange(A0.n), np.diff(A0.colptr))],
                       rtol=1e-8, atol=1e-10 * np.abs(R).max())


def test_small_weights_reach_level_one_map():
    """w -> 0 on the level-2 candidates drives those entries to zero: the loss
    approaches the plain map on S(A_k) (level 1)."""
    A0, A1, S, w, mu = small_problem(4)
    tiny = np.where(w < 1.0, 1e-14, 1.0)
    Lw = loss(A1, A0, S, tiny, mu)
    S1 = O.pattern(A1, 1)
    _, rho1, _, _ = O.sam_build(A1, A0, S1)
    assert np.isclose(Lw, rho1.sum(), rtol=1e-6)
    _, rho2, _, _ = O.sam_build(A1, A0, S)
    assert rho2.sum() < rho1.sum()  # level 2 improves on level 1


def test_weight_domain():
    A0, A1, S, w, mu = small_problem(0)
    bad = w.copy()
    bad[0] = 1.5
    with pytest.raises(O.OracleError):
        O.sam_build(A1, A0, S, weights=bad, mu=mu)
