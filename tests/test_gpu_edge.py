"""Degenerate inputs through the C ABI, against the FP64 oracle: a 1 x 1
system, diagonal sources (every block 1 x 1, whatever the power), a target
whose columns reach outside the row sets (only out_j), columns with a single
pattern entry next to full ones, and a replanned sequence over a 3 x 3 grid
(fewer columns than one wave holds)."""
import numpy as np
import pytest
import torch

import oracle as O
import pde_inputs as P
from parity_util import TOL, colmax_rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2406_17656_amd import Context
    c = Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(A):
    from paper_2406_17656_amd import DeviceCSC
    return DeviceCSC.from_host(A)


def host(t):
    return t.detach().cpu().numpy()


def check(ctx, A0, Ak, power, prec, **kw):
    Sp = O.pattern(Ak, power, **kw)
    dAk, dA0 = dev(Ak), dev(A0)
    Scp, Sri = ctx.pattern(dAk, power, **kw)
    assert np.array_equal(host(Scp), Sp.colptr) and np.array_equal(host(Sri), Sp.rowind)
    M, col, res2 = ctx.build(dAk, dA0, Scp, Sri, prec)
    ctx.sync_status()
    Mo, rho, _, _ = O.sam_build(Ak, A0, Sp)
    wc, _ = colmax_rel(host(M).astype(np.float64), Mo, Sp.colptr)
    assert wc <= TOL[prec], wc
    assert np.allclose(host(col), rho, rtol=1e-9, atol=1e-13 * max(rho.max(), 1e-300))
    assert np.isclose(float(host(res2)[0]), rho.sum(), rtol=1e-9, atol=1e-300)
    return Mo, rho


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_one_by_one(ctx, prec):
    Ak = P.dense_to_csc(np.array([[4.0]]))
    A0 = P.dense_to_csc(np.array([[3.0]]))
    Mo, rho = check(ctx, A0, Ak, 1, prec)
    assert np.isclose(Mo[0], 0.75) and rho[0] < 1e-30


@pytest.mark.parametrize("power", [1, 3])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_diagonal_source_target_outside_row_sets(ctx, power, prec):
    """A diagonal A_k keeps every block 1 x 1 at any power; a tridiagonal A_0
    has entries outside every row set, which enter the residual as out_j."""
    rng = np.random.default_rng(11)
    n = 300
    Ak = P.dense_to_csc(np.diag(rng.uniform(1.0, 2.0, n)))
    d0 = np.diag(rng.uniform(1.0, 2.0, n)) + np.diag(rng.uniform(-1, 1, n - 1), 1) + \
        np.diag(rng.uniform(-1, 1, n - 1), -1)
    A0 = P.dense_to_csc(d0)
    Mo, rho = check(ctx, A0, Ak, power, prec)
    offd = (d0 - np.diag(np.diag(d0))) ** 2
    assert np.allclose(rho, offd.sum(axis=0), rtol=1e-12)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_mixed_single_and_full_columns(ctx, prec):
    """Columns of A_k with only the diagonal next to 5-point columns: blocks
    from 1 x 1 to 13 x 5 in one build, several size classes."""
    A0, As = P.config2(m=16, nmat=2)
    Ak = As[0]
    rng = np.random.default_rng(12)
    dense = np.zeros((Ak.n, Ak.n))
    cols = np.repeat(np.arange(Ak.n), np.diff(Ak.colptr))
    dense[Ak.rowind, cols] = Ak.val
    iso = rng.choice(Ak.n, 40, replace=False)
    for j in iso:  # keep only the diagonal of these columns
        dj = dense[j, j]
        dense[:, j] = 0.0
        dense[j, j] = dj
    check(ctx, A0, P.dense_to_csc(dense), 1, prec)
    check(ctx, A0, P.dense_to_csc(dense), 2, prec)


def test_small_replanned_sequence(ctx):
    """A 3 x 3 grid (9 columns): fewer columns than one wave's problems."""
    A0, As = P.config2(m=3, nmat=3)
    dA0 = dev(A0)
    dAs = [dev(A) for A in As]
    seq = ctx.sequence(dA0, dAs[0], len(As), prec="f32", power=2, replan_each_run=True)
    Ms = seq.alloc_maps()
    res2 = torch.zeros(len(As), dtype=torch.float64, device="cuda")
    for _ in range(2):
        seq.run([d.val for d in dAs], Ms, res2)
        ctx.sync_status()
    for k, Ak in enumerate(As):
        Sp = O.pattern(Ak, 2)
        cp, ri = seq.pattern(k)
        assert np.array_equal(host(cp), Sp.colptr) and np.array_equal(host(ri), Sp.rowind)
        Mo, rho, _, _ = O.sam_build(Ak, A0, Sp)
        wc, _ = colmax_rel(host(Ms[k][:Sp.nnz]).astype(np.float64), Mo, Sp.colptr)
        assert wc <= TOL["f32"], (k, wc)
        assert np.isclose(float(host(res2)[k]), rho.sum(), rtol=1e-9, atol=1e-300)
    seq.close()


@pytest.mark.parametrize("nsrc", [1, 2, 5])
def test_replanned_source_counts(ctx, nsrc):
    """Replanned sequences of one, two and five sources: the sources rotate
    over three graph branches, so these cover two empty branches, one empty
    branch, and branches of unequal length.  Every map against the oracle, and
    a second replay bit for bit equal to the first."""
    A0, As = P.config2(m=20, nmat=nsrc + 1)   # the target and nsrc sources
    assert len(As) == nsrc
    dA0 = dev(A0)
    dAs = [dev(A) for A in As]
    seq = ctx.sequence(dA0, dAs[0], nsrc, prec="f32", power=2, replan_each_run=True)
    Ms = seq.alloc_maps()
    res2 = torch.zeros(nsrc, dtype=torch.float64, device="cuda")
    seq.run([d.val for d in dAs], Ms, res2)
    ctx.sync_status()
    first = [host(M).copy() for M in Ms]
    r_first = host(res2).copy()
    seq.run([d.val for d in dAs], Ms, res2)
    ctx.sync_status()
    for k, Ak in enumerate(As):
        assert np.array_equal(host(Ms[k]), first[k]), k
        Sp = O.pattern(Ak, 2)
        Mo, rho, _, _ = O.sam_build(Ak, A0, Sp)
        wc, _ = colmax_rel(host(Ms[k][:Sp.nnz]).astype(np.float64), Mo, Sp.colptr)
        assert wc <= TOL["f32"], (k, wc)
        assert np.isclose(float(host(res2)[k]), rho.sum(), rtol=1e-9, atol=1e-300)
    assert np.array_equal(host(res2), r_first)
    seq.close()
