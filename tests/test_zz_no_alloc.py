"""The allocation-free entry point sam_build_noalloc (the plan in the
library's fixed device array) against sam_build with a torch workspace,
through the C ABI: two calls in a row, the second on a smaller problem (the
array keeps the first call's contents), give the same map and residual bit
for bit; a problem whose plan exceeds the array is refused before any kernel
runs.  Collected last: runs alone in a fresh process or after the others."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
import pde_inputs as P
from paper_2406_17656_amd import _capi as C
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


def ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def both(ctx, dAk, dA0, Scp, Sri, prec):
    """(M, res2, cols) of sam_build with a torch workspace and of
    sam_build_noalloc, each into fresh outputs filled with a sentinel."""
    lib = ctx.lib
    a, b = dAk.struct(), dA0.struct()
    nnz = int(Sri.numel())
    n = dAk.n
    p = C.SAM_PREC_F32_REFINE if prec == "f32" else C.SAM_PREC_F64
    dt = torch.float32 if prec == "f32" else torch.float64
    outs = []
    for noalloc in (False, True):
        M = torch.full((nnz,), -7.0, dtype=dt, device="cuda")
        r = torch.full((1,), -7.0, dtype=torch.float64, device="cuda")
        c = torch.full((n,), -7.0, dtype=torch.float64, device="cuda")
        if noalloc:
            st = lib.sam_build_noalloc(ctx.h, ctypes.byref(a), ctypes.byref(b), ptr(Scp), ptr(Sri), nnz, p, ptr(M),
                                       ptr(c), ptr(r), stream())
        else:
            nb = ctypes.c_size_t()
            assert lib.sam_workspace_size(ctx.h, ctypes.byref(a), ctypes.byref(b), ptr(Scp), ptr(Sri), nnz, p,
                                          ctypes.byref(nb), stream()) == C.SAM_OK
            ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
            st = lib.sam_build(ctx.h, ctypes.byref(a), ctypes.byref(b), ptr(Scp), ptr(Sri), nnz, p, ptr(M), ptr(c),
                               ptr(r), ptr(ws), nb.value, stream())
        assert st == C.SAM_OK, lib.sam_last_error(ctx.h)
        torch.cuda.synchronize()
        outs.append((M, r, c))
    ctx.sync_status()
    return outs


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_noalloc_matches_workspace_build(ctx, prec):
    from paper_2406_17656_amd import SamError  # noqa: F401
    cases = [P.config2(m=512, nmat=2), P.config2(m=96, nmat=2)]   # the second call is smaller
    for A0, As in cases:
        Ak = As[0]
        dAk, dA0 = dev(Ak), dev(A0)
        Scp, Sri = ctx.pattern(dAk, 2)
        (M1, r1, c1), (M2, r2, c2) = both(ctx, dAk, dA0, Scp, Sri, prec)
        iv = torch.int32 if prec == "f32" else torch.int64
        assert torch.equal(M1.view(iv), M2.view(iv))
        assert torch.equal(r1, r2) and torch.equal(c1, c2)
        if Ak.n <= 96 * 96:    # and the map is the oracle's
            S = O.pattern(Ak, 2)
            Mo, rho, _, _ = O.sam_build(Ak, A0, S)
            wc, we = colmax_rel(M2.cpu().numpy().astype(np.float64), Mo, S.colptr)
            assert wc <= TOL[prec], (wc, we)
            assert abs(float(r2.cpu()[0]) - O.frobenius_sq(rho)) <= 1e-9 * O.frobenius_sq(rho)


def test_noalloc_refuses_plans_beyond_the_array(ctx):
    """The 1024 x 1024 level-2 plan (68 M gathered entries) needs more than
    the fixed 48 MiB: refused with SAM_ERR_UNSUPPORTED and a message, outputs
    untouched."""
    A0, As = P.config2(m=1024, nmat=2)
    dAk, dA0 = dev(As[0]), dev(A0)
    Scp, Sri = ctx.pattern(dAk, 2)
    a, b = dAk.struct(), dA0.struct()
    nnz = int(Sri.numel())
    M = torch.full((nnz,), -7.0, dtype=torch.float32, device="cuda")
    st = ctx.lib.sam_build_noalloc(ctx.h, ctypes.byref(a), ctypes.byref(b), ptr(Scp), ptr(Sri), nnz,
                                   C.SAM_PREC_F32_REFINE, ptr(M), None, None, stream())
    assert st == C.SAM_ERR_UNSUPPORTED
    assert b"fixed scratch" in ctx.lib.sam_last_error(ctx.h)
    torch.cuda.synchronize()
    ctx.sync_status()
    assert bool((M == -7.0).all())
