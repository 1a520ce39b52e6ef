"""Full-size GPU parity on the larger workloads: the 3D upwind
convection-diffusion sequence on a 64^3 grid (n = 262144) with the level-2
pattern and the column-threshold variant, and the 1024 x 1024 ragged
9-point sequence (n = 1048576) with the global threshold then level 2, run
through the graph-captured sequence.  Integer patterns are compared in full
(bit-exact); map entries on a seeded sample of columns plus every distinct
column size, against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle as O
import pde_inputs as P
from parity_util import TOL, colmax_rel, sample_columns

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


@pytest.fixture(scope="module")
def cfg3():
    return P.config3()


@pytest.fixture(scope="module")
def cfg4():
    return P.config4(nmat=3)


def check_one(ctx, A0, Ak, prec, power, kind="none", seed=0, **kw):
    Sp = O.pattern(Ak, power, kind, **kw)
    dAk, dA0 = dev(Ak), dev(A0)
    Scp, Sri = ctx.pattern(dAk, power, kind, **kw)
    assert np.array_equal(Scp.cpu().numpy(), Sp.colptr)
    assert np.array_equal(Sri.cpu().numpy(), Sp.rowind)
    M, col, res2 = ctx.build(dAk, dA0, Scp, Sri, prec)
    ctx.sync_status()
    cols = sample_columns(Ak.n, Sp.colptr, k=2000, seed=seed)
    Mo, rho, _, _ = O.sam_build(Ak, A0, Sp, cols=cols)
    wc, we = colmax_rel(M.cpu().numpy().astype(np.float64), Mo, Sp.colptr, cols)
    assert wc <= TOL[prec], (wc, we)
    colg = col.cpu().numpy()
    assert np.allclose(colg[cols], rho[cols], rtol=1e-9, atol=1e-13 * rho[cols].max())
    assert np.isclose(float(res2.cpu()[0]), colg.sum(), rtol=1e-12)
    return wc, we


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_config3_level2(ctx, cfg3, prec):
    A0, As = cfg3
    wc, we = check_one(ctx, A0, As[-1], prec, 2, seed=3)   # Pe = 100, D perturbed
    print(f"cfg3 64^3 level 2 {prec}: colmax {wc:.2e} entrywise {we:.2e}")


def test_config3_column_threshold(ctx, cfg3):
    A0, As = cfg3
    check_one(ctx, A0, As[-1], "f32", 2, kind="column", tau=0.85, seed=4)


def test_config4_sequence_thresholded(ctx, cfg4):
    """Global threshold 0.1 then level 2, replanned per source on the device
    inside one HIP graph; every source's pattern bit-exact, sampled maps."""
    A0, As = cfg4
    dA0 = dev(A0)
    dAs = [dev(A) for A in As]
    seq = ctx.sequence(dA0, dAs[0], len(As), prec="f32", power=2, kind="global", thresh=0.1)
    Ms = seq.alloc_maps()
    res2 = torch.zeros(len(As), dtype=torch.float64, device="cuda")
    seq.run([d.val for d in dAs], Ms, res2)
    ctx.sync_status()
    for k, Ak in enumerate(As):
        Sp = O.pattern(Ak, 2, "global", thresh=0.1)
        cp, ri = seq.pattern(k)
        assert np.array_equal(cp.cpu().numpy(), Sp.colptr)
        assert np.array_equal(ri.cpu().numpy(), Sp.rowind)
        cols = sample_columns(Ak.n, Sp.colptr, k=1500, seed=10 + k)
        Mo, rho, _, _ = O.sam_build(Ak, A0, Sp, cols=cols)
        wc, we = colmax_rel(Ms[k][:Sp.nnz].cpu().numpy().astype(np.float64), Mo, Sp.colptr, cols)
        assert wc <= TOL["f32"], (k, wc, we)
    seq.close()


def test_config4_level2_f64(ctx, cfg4):
    A0, As = cfg4
    check_one(ctx, A0, As[0], "f64", 2, kind="global", thresh=0.1, seed=5)
