"""Every numeric kernel variant of the menu, put first in the bucket order,
gives oracle-parity maps (the autotuner may pick any of them), and the
autotuner's choice keeps parity."""
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


def cases():
    A0, As = P.config2(m=40, nmat=2)
    yield "cfg2-40-p1", A0, As[0], 1, {}
    yield "cfg2-40-p2", A0, As[0], 2, {}
    A0, As = P.config3(m=10)
    yield "cfg3-10-p2", A0, As[-1], 2, {}
    # ragged blocks of every width from a few to ~20 columns
    A0, As = P.config4(m=24, nmat=2)
    yield "cfg4-24-glob-p2", A0, As[0], 2, {"kind": "global", "thresh": 0.1}


CASES = list(cases())


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_each_variant_first(ctx, case, prec):
    from paper_2406_17656_amd import SamError, autotune
    _, A0, Ak, p, kw = case
    Sp = O.pattern(Ak, p, **kw)
    Mo, rho, _, _ = O.sam_build(Ak, A0, Sp)
    dA0, dAk = dev(A0), dev(Ak)
    Scp, Sri = torch.as_tensor(Sp.colptr).cuda(), torch.as_tensor(Sp.rowind).cuda()
    plan = ctx.plan(dAk, dA0, Scp, Sri)
    served = 0
    for order in autotune.candidate_orders(len(autotune.menu(prec))):
        try:
            plan.select(order, prec)
        except SamError:
            continue
        M, _, r = plan.build(dAk.val, dA0.val, prec)
        ctx.sync_status()
        wc, we = colmax_rel(M.cpu().numpy().astype(np.float64), Mo, Sp.colptr)
        assert wc <= TOL[prec], (order[:2], wc)
        assert np.isclose(float(r.cpu()[0]), rho.sum(), rtol=1e-9)
        served += 1
    assert served >= 2
    plan.close()


def test_autotune_keeps_parity(ctx, tmp_path, monkeypatch):
    from paper_2406_17656_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tune.json"))
    _, A0, Ak, p, kw = CASES[1]
    Sp = O.pattern(Ak, p, **kw)
    dA0, dAk = dev(A0), dev(Ak)
    plan = ctx.plan(dAk, dA0, torch.as_tensor(Sp.colptr).cuda(), torch.as_tensor(Sp.rowind).cuda())
    res = autotune.tune(plan, dAk.val, dA0.val, "f32", reps=3)
    assert not res["cached"] and len(res["timings"]) >= 2
    M, _, _ = plan.build(dAk.val, dA0.val, "f32")
    Mo, _, _, _ = O.sam_build(Ak, A0, Sp)
    assert colmax_rel(M.cpu().numpy().astype(np.float64), Mo, Sp.colptr)[0] <= TOL["f32"]
    again = autotune.tune(plan, dAk.val, dA0.val, "f32", reps=3)
    assert again["cached"] and again["order"] == res["order"]
    plan.close()
