"""Pins of the adaptive-pattern oracle functions (candidate weights and the
top-k selection), against brute force on small random patterns with ties and
NaN, the special cases k = 0 and k >= every candidate count, and the
monotonicity of the least-squares residual in the pattern
(B subset S' subset S => ||R(B)|| >= ||R(S')|| >= ||R(S)||)."""
import numpy as np
import pytest

import oracle as O
import pde_inputs as P


def random_pattern(n, per_col, rng, base=None):
    cp, ri = [0], []
    for j in range(n):
        rows = set(rng.choice(n, size=min(per_col, n), replace=False).tolist())
        if base is not None:
            rows |= set(base.rowind[base.colptr[j]:base.colptr[j + 1]].tolist())
        rows = sorted(rows)
        ri += rows
        cp.append(len(ri))
    return O.Pattern(n, np.array(cp, dtype=np.int32), np.array(ri, dtype=np.int32))


def brute_topk(S, w, g, k):
    cp, ri = [0], []
    for j in range(S.n):
        es = list(range(S.colptr[j], S.colptr[j + 1]))
        cands = [e for e in es if not w[e] >= 1.0]
        key = lambda e: (np.inf if np.isnan(g[e]) else g[e], int(S.rowind[e]))
        chosen = set(sorted(cands, key=key)[:k])
        kept = [int(S.rowind[e]) for e in es if w[e] >= 1.0 or e in chosen]
        ri += kept
        cp.append(len(ri))
    return np.array(cp), np.array(ri, dtype=np.int64)


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("k", [0, 1, 3, 50])
def test_topk_brute_force(seed, k):
    rng = np.random.default_rng(seed)
    B = random_pattern(30, 3, rng)
    S = random_pattern(30, 9, rng, base=B)
    w = O.candidate_weights(S, B, 1.0, 0.2)
    g = np.round(rng.standard_normal(S.nnz), 1)     # many ties
    g[rng.random(S.nnz) < 0.1] = np.nan
    out = O.select_topk(S, w, g, k)
    cp, ri = brute_topk(S, w, g, k)
    assert np.array_equal(out.colptr, cp) and np.array_equal(out.rowind, ri)


def test_candidate_weights_membership():
    """Membership by sparse-matrix algebra instead of per-column sets: the
    entries of S shared with B are where the elementwise product of the two
    0/1 patterns is nonzero."""
    import scipy.sparse as sp
    rng = np.random.default_rng(4)
    B = random_pattern(25, 4, rng)
    S = random_pattern(25, 8, rng, base=B)
    w = O.candidate_weights(S, B, 1.0, 0.3)
    Sm = sp.csc_matrix((np.arange(1, S.nnz + 1, dtype=np.float64), S.rowind, S.colptr), shape=(S.n, S.n))
    Bm = sp.csc_matrix((np.ones(B.nnz), B.rowind, B.colptr), shape=(B.n, B.n))
    shared = Sm.multiply(Bm).tocsc()
    expect = np.full(S.nnz, 0.3)
    expect[shared.data.astype(np.int64) - 1] = 1.0    # the data carry S's entry numbers
    assert np.array_equal(w, expect)
    assert (w == 1.0).sum() == B.nnz          # B is a subset of S


def test_topk_extremes_on_levels():
    A0, (A1,) = P.config1()
    B, S = O.pattern(A1, 1), O.pattern(A1, 2)
    w = O.candidate_weights(S, B)
    g = np.random.default_rng(0).standard_normal(S.nnz)
    S0 = O.select_topk(S, w, g, 0)
    assert np.array_equal(S0.colptr, B.colptr) and np.array_equal(S0.rowind, B.rowind)
    Sall = O.select_topk(S, w, g, 10 ** 6)
    assert np.array_equal(Sall.colptr, S.colptr) and np.array_equal(Sall.rowind, S.rowind)


def test_residual_monotone_in_pattern():
    """The column least-squares residual can only drop when the pattern
    grows: level 1 >= adapted >= level 2, on the oracle's own gradient."""
    A0, (A1,) = P.config1()
    B, S = O.pattern(A1, 1), O.pattern(A1, 2)
    w = O.candidate_weights(S, B, 1.0, 0.1)
    mu = P.penalty_scale(A1)
    _, _, gw, _ = O.backward(A1, A0, S, weights=w, mu=mu)
    assert np.all(np.isfinite(gw))
    res = []
    for Sp in (B, O.select_topk(S, w, gw, 2), S):
        _, rho, _, _ = O.sam_build(A1, A0, Sp)
        res.append(rho.sum())
    assert res[0] >= res[1] * (1 - 1e-12) and res[1] >= res[2] * (1 - 1e-12)
    assert res[0] > res[2]


def test_gradient_choice_beats_worst_choice():
    """Keeping the k most negative dL/dw lowers the residual at least as much
    as keeping the k least negative ones (k = 2, cfg1)."""
    A0, (A1,) = P.config1()
    B, S = O.pattern(A1, 1), O.pattern(A1, 2)
    w = O.candidate_weights(S, B, 1.0, 0.1)
    _, _, gw, _ = O.backward(A1, A0, S, weights=w, mu=P.penalty_scale(A1))
    best = O.select_topk(S, w, gw, 2)
    worst = O.select_topk(S, w, -gw, 2)
    rb = O.sam_build(A1, A0, best)[1].sum()
    rw = O.sam_build(A1, A0, worst)[1].sum()
    assert rb < rw
