"""Shared helpers of the GPU parity tests: device upload, comparisons."""
import numpy as np


def colmax_rel(M, Mref, colptr, cols=None):
    """Largest per-column ||m - m*||_inf / ||m*||_inf and the largest
    entrywise |m - m*| / |m*| (over entries with |m*| > 0), over the columns
    `cols` (all columns when None)."""
    M = np.asarray(M, dtype=np.float64)
    Mref = np.asarray(Mref, dtype=np.float64)
    colptr = np.asarray(colptr, dtype=np.int64)
    if cols is None:
        return _colmax_all(M, Mref, colptr)
    worst_col, worst_ent = 0.0, 0.0
    for j in cols:
        a, b = int(colptr[j]), int(colptr[j + 1])
        if b == a:
            continue
        ref = Mref[a:b]
        den = np.abs(ref).max()
        d = np.abs(M[a:b] - ref)
        if den > 0:
            worst_col = max(worst_col, d.max() / den)
        nz = np.abs(ref) > 0
        if nz.any():
            worst_ent = max(worst_ent, (d[nz] / np.abs(ref[nz])).max())
    return worst_col, worst_ent


def _colmax_all(M, Mref, colptr):
    """colmax_rel over every column, vectorised with segment maxima."""
    nnz = int(colptr[-1])
    if nnz == 0:
        return 0.0, 0.0
    d = np.abs(M[:nnz] - Mref[:nnz])
    a = np.abs(Mref[:nnz])
    starts = colptr[:-1][np.diff(colptr) > 0]
    dmax = np.maximum.reduceat(d, starts)
    amax = np.maximum.reduceat(a, starts)
    ok = amax > 0
    worst_col = float((dmax[ok] / amax[ok]).max()) if ok.any() else 0.0
    nz = a > 0
    worst_ent = float((d[nz] / a[nz]).max()) if nz.any() else 0.0
    return worst_col, worst_ent


def entrywise_rel(M, Mref, colptr, floor):
    """Largest |m_i - m*_i| / |m*_i| over the entries with |m*_i| at least
    `floor` times the largest |m*| of their column.  Entries far below their
    column's scale are resolved by no FP64 least-squares solver to a relative
    1e-6 (the FP64 oracle's own error there is ~1e-16 of the column maximum),
    so the entrywise bar applies above the floor; the column bar covers the
    rest."""
    M = np.asarray(M, dtype=np.float64)
    Mref = np.asarray(Mref, dtype=np.float64)
    colptr = np.asarray(colptr, dtype=np.int64)
    nnz = int(colptr[-1])
    if nnz == 0:
        return 0.0
    a = np.abs(Mref[:nnz])
    lens = np.diff(colptr)
    starts = colptr[:-1][lens > 0]
    amax = np.repeat(np.maximum.reduceat(a, starts), lens[lens > 0])
    sel = (a > 0) & (a >= floor * amax)
    if not sel.any():
        return 0.0
    return float((np.abs(M[:nnz] - Mref[:nnz])[sel] / a[sel]).max())


def sample_columns(n, colptr_S, k=2000, seed=0):
    """A seeded sample of columns plus the first/last ones and one column of
    every distinct pattern size (boundary and rare shapes)."""
    rng = np.random.default_rng(seed)
    cols = set(rng.choice(n, size=min(k, n), replace=False).tolist())
    cols.update([0, 1, n - 2, n - 1])
    sizes = np.diff(np.asarray(colptr_S))
    for s in np.unique(sizes):
        cols.add(int(np.nonzero(sizes == s)[0][0]))
        cols.add(int(np.nonzero(sizes == s)[0][-1]))
    return np.array(sorted(c for c in cols if 0 <= c < n), dtype=np.int32)


# Map entries: per column ||m - m*||_inf <= TOL ||m*||_inf, and in FP32 +
# refinement also entrywise |m_i - m*_i| <= TOL |m*_i| on every entry of at
# least ENTRY_FLOOR times its column's largest (M is stored in FP32, whose
# rounding alone is 6e-8 relative; the refined FP64 solution is within about
# 1e-12 of the column maximum, so the bar holds with a margin of ten above
# the floor).
TOL = {"f64": 1e-10, "f32": 1e-6}
ENTRY_FLOOR = 1e-5
