"""Shared helpers of the GPU parity tests: device upload, comparisons."""
import numpy as np


def colmax_rel(M, Mref, colptr, cols=None):
    """Largest per-column ||m - m*||_inf / ||m*||_inf and the largest
    entrywise |m - m*| / |m*| (over entries with |m*| > 0)."""
    M = np.asarray(M, dtype=np.float64)
    Mref = np.asarray(Mref, dtype=np.float64)
    worst_col, worst_ent = 0.0, 0.0
    js = range(len(colptr) - 1) if cols is None else cols
    for j in js:
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


TOL = {"f64": 1e-10, "f32": 1e-6}
