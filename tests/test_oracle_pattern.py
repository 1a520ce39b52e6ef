"""Pins for the oracle's pattern construction (Sections 3 and 4 of the paper)
against values the paper prints, brute-force boolean matrix powers and
hand-built columns.  CPU only."""
import json
import os

import numpy as np
import pytest

import oracle as O
import pde_inputs as P

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load_7x7():
    mats, cur = {}, None
    for line in open(os.path.join(GOLD, "paper_7x7.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line in ("A0", "A1"):
            cur = line
            mats[cur] = []
            continue
        mats[cur].append([int(t) for t in line.split()])
    return np.array(mats["A0"], dtype=bool), np.array(mats["A1"], dtype=bool)


def pattern_to_bool(S):
    d = np.zeros((S.n, S.n), dtype=bool)
    cols = np.repeat(np.arange(S.n), np.diff(S.colptr))
    d[S.rowind, cols] = True
    return d


def brute_power(Bd, p):
    """Boolean (I + B)^p by repeated dense integer products."""
    n = Bd.shape[0]
    M = (Bd | np.eye(n, dtype=bool)).astype(np.int64)
    R = M.copy()
    for _ in range(p - 1):
        R = ((R @ M) > 0).astype(np.int64)
    return R > 0


def closure(Bd):
    """Reflexive transitive closure by Warshall's algorithm."""
    n = Bd.shape[0]
    R = Bd | np.eye(n, dtype=bool)
    for k in range(n):
        R = R | (R[:, [k]] & R[[k], :])
    return R


@pytest.mark.parametrize("row", json.load(open(os.path.join(GOLD, "cd2d_table_counts.json")))["rows"],
                         ids=lambda r: r["label"])
def test_table_counts(row):
    L = P.laplacian_2d(64)
    kw = {k: row[k] for k in ("tau", "lfil") if k in row}
    S = O.pattern(L, row["power"], row["kind"], **kw)
    assert S.nnz == row["nnz"]


def test_7x7_subset_and_closure():
    A0, A1 = load_7x7()
    assert not np.any(A0 & ~A1)  # eq. (property) for the pair
    c1 = closure(A1)
    assert c1.sum() == 49        # G*(A_1) is complete
    assert closure(A0).sum() == 24  # negative control: upper triangle
    # oracle level-n pattern equals the closure
    A1c = P.dense_to_csc(A1.astype(float))
    S = O.pattern(A1c, 7)
    assert np.array_equal(pattern_to_bool(S), c1)
    # the exact map with random values on these patterns is dense (49 nnz)
    rng = np.random.default_rng(0)
    V1 = np.where(A1, rng.uniform(0.5, 1.5, A1.shape), 0.0) + 3 * np.eye(7)
    V0 = np.where(A0, rng.uniform(0.5, 1.5, A0.shape), 0.0)
    N = np.linalg.solve(V1, V0)
    assert (np.abs(N) > 1e-12 * np.abs(N).max()).sum() == 49


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("p", [1, 2, 3])
def test_power_matches_boolean_matmul(seed, p):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 40))
    Bd = rng.random((n, n)) < 0.12
    A = P.dense_to_csc(np.where(Bd, 1.0, 0.0) + np.eye(n) * 0)  # no forced diagonal
    if A.nnz == 0:
        pytest.skip("empty")
    S = O.pattern(A, p)
    assert np.array_equal(pattern_to_bool(S), brute_power(Bd, p))
    # rows sorted ascending inside each column
    for j in range(n):
        seg = S.rowind[S.colptr[j]:S.colptr[j + 1]]
        assert np.all(np.diff(seg) > 0)


@pytest.mark.parametrize("seed", range(4))
def test_exact_map_inside_closure(seed):
    """Section 3 claim, as an inclusion: with S(A_0) inside S(A_k) the exact
    map's pattern lies inside the reflexive closure of G(A_k)."""
    rng = np.random.default_rng(100 + seed)
    n = 24
    Bk = rng.random((n, n)) < 0.08
    B0 = Bk & (rng.random((n, n)) < 0.7)
    Ak = np.where(Bk, rng.uniform(-1, 1, (n, n)), 0.0) + 4 * np.eye(n)
    A0 = np.where(B0, rng.uniform(-1, 1, (n, n)), 0.0) + 2 * np.eye(n)
    N = np.linalg.solve(Ak, A0)
    Sn = np.abs(N) > 1e-12 * np.abs(N).max()
    S = O.pattern(P.dense_to_csc(Ak), n)
    assert not np.any(Sn & ~pattern_to_bool(S))


def _col(vals_rows, n):
    """Single-column helper: matrix with the given (row, value) entries in
    column 0 and 1 on the rest of the diagonal."""
    d = np.eye(n)
    d[0, 0] = 0.0
    for r, v in vals_rows:
        d[r, 0] = v
    return P.dense_to_csc(d)


def col0(S):
    return list(S.rowind[S.colptr[0]:S.colptr[1]])


def test_column_tau_rule():
    A = _col([(0, 4.0), (1, -1.0), (2, 2.0), (3, 3.0), (4, -3.9)], 6)
    # threshold (1 - tau) * max|a| with max = 4, strict '>'
    assert col0(O.sparsify(A, "column", tau=0.0)) == [0]            # nothing exceeds the max
    assert col0(O.sparsify(A, "column", tau=1.0)) == [0, 1, 2, 3, 4]  # every nonzero
    assert col0(O.sparsify(A, "column", tau=0.25)) == [0, 4]        # > 3.0
    assert col0(O.sparsify(A, "column", tau=0.5)) == [0, 3, 4]      # > 2.0
    with pytest.raises(O.OracleError):
        O.sparsify(A, "column", tau=1.5)


def test_lfil_rule_ties_and_overflow():
    A = _col([(0, 5.0), (1, 2.0), (2, -2.0), (3, 1.0), (5, 2.0)], 6)
    # diagonal + (lfil - 1) largest off-diagonals, ties to the smaller row
    assert col0(O.sparsify(A, "lfil", lfil=1)) == [0]
    assert col0(O.sparsify(A, "lfil", lfil=2)) == [0, 1]
    assert col0(O.sparsify(A, "lfil", lfil=3)) == [0, 1, 2]
    assert col0(O.sparsify(A, "lfil", lfil=4)) == [0, 1, 2, 5]
    # lfil above the column count keeps the column as is
    assert col0(O.sparsify(A, "lfil", lfil=50)) == [0, 1, 2, 3, 5]


def test_global_rule_scaling_and_zero_diagonal():
    # column 0 has a zero diagonal: D_00 = 1 (Section 4 definition of D)
    d = np.diag([0.0, 4.0, 16.0, 1.0])
    d[1, 0] = 1.0    # |a| / sqrt(D_11 D_00) = 1/2
    d[2, 0] = 1.0    # 1/4
    d[3, 0] = 0.3    # 0.3
    A = P.dense_to_csc(d)
    assert col0(O.sparsify(A, "global", thresh=0.29)) == [0, 1, 3]
    assert col0(O.sparsify(A, "global", thresh=0.26)) == [0, 1, 3]
    assert col0(O.sparsify(A, "global", thresh=0.2)) == [0, 1, 2, 3]
    # the printed D^{1/2} A D^{1/2} form (flag +1): |a| * sqrt(D_ii D_jj)
    assert col0(O.sparsify(A, "global", thresh=1.9, global_scale=1)) == [0, 1, 2]
    assert col0(O.sparsify(A, "global", thresh=4.0, global_scale=1)) == [0]
    # the diagonal is part of the pattern even when it is not stored
    assert 0 in col0(O.sparsify(A, "none"))


def test_global_rule_scale_invariant():
    rng = np.random.default_rng(3)
    A0, _ = P.config1()
    A = A0.with_values(A0.val * 1e3)
    s1 = O.pattern(A0, 2, "global", thresh=0.2)
    s2 = O.pattern(A, 2, "global", thresh=0.2)
    assert np.array_equal(s1.rowind, s2.rowind) and np.array_equal(s1.colptr, s2.colptr)
    del rng


def test_row_sets_brute_force():
    rng = np.random.default_rng(7)
    n = 30
    Bd = rng.random((n, n)) < 0.1
    A = P.dense_to_csc(np.where(Bd, 1.0, 0.0) + np.eye(n))
    S = O.pattern(A, 2)
    I = O.row_sets(S, A)
    Ad = A.to_dense() != 0
    for j in range(n):
        J = S.rowind[S.colptr[j]:S.colptr[j + 1]]
        want = np.nonzero(Ad[:, J].any(axis=1))[0]
        assert list(I.rowind[I.colptr[j]:I.colptr[j + 1]]) == list(want)
