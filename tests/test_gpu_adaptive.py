"""GPU parity of the adaptive-pattern calls: candidate weights bit-exact
against the oracle, the top-k selection bit-exact against the oracle run on
the GPU's own gradient (the decision is taken on the same numbers), the
penalty scale, and the map on the adapted pattern against the FP64 oracle,
with the residual ordering level 1 >= adapted >= level 2."""
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


def pat(cp, ri):
    return O.Pattern(cp.numel() - 1, cp.cpu().numpy(), ri.cpu().numpy())


def cases():
    A0, As = P.config2(m=40, nmat=2)
    yield "cfg2-40", A0, As[0]
    A0, As = P.config4(m=24, nmat=2)
    yield "cfg4-24", A0, As[0]


CASES = list(cases())


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_candidate_weights_and_penalty(ctx, case):
    _, A0, Ak = case
    dAk = dev(Ak)
    Bcp, Bri = ctx.pattern(dAk, 1)
    Scp, Sri = ctx.pattern(dAk, 2)
    w = ctx.candidate_weights(Scp, Sri, Bcp, Bri, 1.0, 0.25)
    want = O.candidate_weights(pat(Scp, Sri), pat(Bcp, Bri), 1.0, 0.25)
    assert np.array_equal(w.cpu().numpy(), want)
    assert np.isclose(ctx.penalty_scale(dAk), P.penalty_scale(Ak), rtol=1e-12)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("k", [0, 1, 3, 100])
def test_topk_bitexact(ctx, case, k):
    _, A0, Ak = case
    from paper_2406_17656_amd.adaptive import adaptive_pattern
    dAk, dA0 = dev(Ak), dev(A0)
    cp, ri, info = adaptive_pattern(ctx, dAk, dA0, k, w_cand=0.1)
    ctx.sync_status()
    S = pat(*info["S"])
    want = O.select_topk(S, info["w"].cpu().numpy(), info["gw"].cpu().numpy(), k)
    assert np.array_equal(cp.cpu().numpy(), want.colptr)
    assert np.array_equal(ri.cpu().numpy(), want.rowind)
    if k == 0:
        B = pat(*info["B"])
        assert np.array_equal(want.colptr, B.colptr) and np.array_equal(want.rowind, B.rowind)


def test_gradient_matches_oracle(ctx):
    _, A0, Ak = CASES[0]
    from paper_2406_17656_amd.adaptive import adaptive_pattern
    cp, ri, info = adaptive_pattern(ctx, dev(Ak), dev(A0), 2, w_cand=0.1)
    ctx.sync_status()
    S = pat(*info["S"])
    _, _, gw, _ = O.backward(Ak, A0, S, weights=info["w"].cpu().numpy(), mu=info["mu"])
    g = info["gw"].cpu().numpy()
    assert np.abs(g - gw).max() <= 1e-6 * np.abs(gw).max()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_adaptive_map_parity_and_ordering(ctx, case):
    _, A0, Ak = case
    from paper_2406_17656_amd.adaptive import adaptive_map
    dAk, dA0 = dev(Ak), dev(A0)
    cp, ri, M, res2, info = adaptive_map(ctx, dAk, dA0, 2, w_cand=0.1, prec="f32")
    ctx.sync_status()
    Sp = pat(cp, ri)
    Mo, rho, _, _ = O.sam_build(Ak, A0, Sp)
    wc, we = colmax_rel(M.cpu().numpy().astype(np.float64), Mo, Sp.colptr)
    assert wc <= TOL["f32"], (wc, we)
    r_adapt = float(res2.cpu()[0])
    assert np.isclose(r_adapt, rho.sum(), rtol=1e-9)
    r1 = O.sam_build(Ak, A0, pat(*info["B"]))[1].sum()
    r2 = O.sam_build(Ak, A0, pat(*info["S"]))[1].sum()
    assert r1 * (1 + 1e-9) >= r_adapt >= r2 * (1 - 1e-9)
