"""GPU tests of the C ABI's memory and validation contract, called through
ctypes with torch-allocated device memory: the sizes the library reports are
enough and are checked, the one-shot build in a caller workspace matches the
oracle, two streams with their own workspaces run on one context at once,
and malformed CSC structures are rejected (SAM_ERR_UNSORTED, first bad
column) before any other kernel reads their indices."""
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


def raw_build(ctx, dAk, dA0, Scp, Sri, prec, ws=None, extra=0):
    """sam_workspace_size + sam_build through the C ABI; returns (status, M, res2, bytes)."""
    lib = ctx.lib
    a, b = dAk.struct(), dA0.struct()
    nnz = int(Sri.numel())
    p = C.SAM_PREC_F32_REFINE if prec == "f32" else C.SAM_PREC_F64
    nb = ctypes.c_size_t()
    assert lib.sam_workspace_size(ctx.h, ctypes.byref(a), ctypes.byref(b), ptr(Scp), ptr(Sri), nnz, p,
                                  ctypes.byref(nb), stream()) == C.SAM_OK
    size = nb.value + extra
    if ws is None:
        ws = torch.empty(max(size, 256), dtype=torch.uint8, device="cuda")
    M = torch.full((max(nnz, 1),), -7.0, dtype=torch.float32 if prec == "f32" else torch.float64, device="cuda")
    res2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = lib.sam_build(ctx.h, ctypes.byref(a), ctypes.byref(b), ptr(Scp), ptr(Sri), nnz, p, ptr(M), None,
                       ptr(res2), ptr(ws), size, stream())
    return st, M, res2, nb.value


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_build_in_caller_workspace(ctx, prec):
    A0, As = P.config2(m=48, nmat=2)
    Ak = As[0]
    dAk, dA0 = dev(Ak), dev(A0)
    Scp, Sri = ctx.pattern(dAk, 2)
    st, M, res2, nbytes = raw_build(ctx, dAk, dA0, Scp, Sri, prec)
    assert st == C.SAM_OK, ctx.lib.sam_last_error(ctx.h)
    ctx.sync_status()
    S = O.pattern(Ak, 2)
    Mo, rho, _, _ = O.sam_build(Ak, A0, S)
    wc, we = colmax_rel(M.cpu().numpy().astype(np.float64), Mo, S.colptr)
    assert wc <= TOL[prec], (wc, we)
    assert abs(float(res2.cpu()[0]) - O.frobenius_sq(rho)) <= 1e-9 * O.frobenius_sq(rho)
    # the workspace is what the library said it needs: one byte less is refused
    st, M2, _, _ = raw_build(ctx, dAk, dA0, Scp, Sri, prec, extra=-1)
    assert st == C.SAM_ERR_ARG and b"plan memory" in ctx.lib.sam_last_error(ctx.h)
    torch.cuda.synchronize()
    assert bool((M2 == -7.0).all())          # nothing was written


def test_two_streams_own_workspaces(ctx):
    """Two one-shot builds of different sources on one context, each on its
    own stream with its own workspace and outputs, at the same time: both
    equal the serial builds bit for bit."""
    A0, As = P.config2(m=64, nmat=3)
    dA0 = dev(A0)
    dAs = [dev(A) for A in As[:2]]
    pats = [ctx.pattern(d, 2) for d in dAs]
    serial = []
    for d, (cp, ri) in zip(dAs, pats):
        st, M, r, _ = raw_build(ctx, d, dA0, cp, ri, "f32")
        assert st == C.SAM_OK
        serial.append((M.clone(), r.clone()))
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for s, d, (cp, ri) in zip((s1, s2), dAs, pats):
        with torch.cuda.stream(s):
            st, M, r, _ = raw_build(ctx, d, dA0, cp, ri, "f32")
            assert st == C.SAM_OK
            outs.append((M, r))
    torch.cuda.synchronize()
    ctx.sync_status()
    for (M, r), (Ms, rs) in zip(outs, serial):
        assert torch.equal(M.view(torch.int32), Ms.view(torch.int32))
        assert torch.equal(r, rs)


def bad_structures(n=6):
    """(name, colptr, rowind, first bad column) of malformed n x n CSC arrays."""
    good_cp = np.arange(0, 2 * n + 1, 2, dtype=np.int32)
    good_ri = np.array([v for j in range(n) for v in sorted((j, (j + 1) % n))], dtype=np.int32)
    out = []
    ri = good_ri.copy()
    ri[6], ri[7] = ri[7], ri[6]                     # column 3 unsorted
    out.append(("unsorted", good_cp, ri, 3))
    ri = good_ri.copy()
    ri[5] = ri[4]                                   # column 2 repeats a row
    out.append(("duplicate", good_cp, ri, 2))
    ri = good_ri.copy()
    ri[9] = n + 3                                   # column 4 row out of range
    out.append(("row_too_large", good_cp, ri, 4))
    ri = good_ri.copy()
    ri[2] = -1                                      # column 1 negative row
    out.append(("negative_row", good_cp, ri, 1))
    cp = good_cp.copy()
    cp[3], cp[4] = cp[4], cp[3]                     # colptr decreases after column 2
    out.append(("colptr_decreasing", cp, good_ri, 2))
    return good_cp, good_ri, out


def to_dev(cp, ri, n, val=True):
    from paper_2406_17656_amd import DeviceCSC
    v = torch.ones(len(ri), dtype=torch.float64, device="cuda") if val else None
    return DeviceCSC(n, torch.as_tensor(cp).cuda(), torch.as_tensor(ri).cuda(), v)


@pytest.mark.parametrize("case", range(5))
def test_check_csc_rejects_malformed(ctx, case):
    from paper_2406_17656_amd import SamError
    n = 6
    good_cp, good_ri, bad = bad_structures(n)
    name, cp, ri, col = bad[case]
    ctx.check_csc(to_dev(good_cp, good_ri, n))          # the good one passes
    with pytest.raises(SamError) as e:
        ctx.check_csc(to_dev(cp, ri, n))
    assert e.value.status == C.SAM_ERR_UNSORTED
    msg = str(e.value)
    if name != "colptr_decreasing":
        assert f"column {col}" in msg, (name, msg)


@pytest.mark.parametrize("case", range(5))
def test_entry_points_validate_before_reading(ctx, case):
    """A malformed A_k, A_0 or S is refused by every call that first receives
    it, and no kernel of the call ran: the status word stays clear and the
    outputs keep their sentinel."""
    from paper_2406_17656_amd import SamError
    n = 6
    good_cp, good_ri, bad = bad_structures(n)
    name, cp, ri, col = bad[case]
    good, broken = to_dev(good_cp, good_ri, n), to_dev(cp, ri, n)
    gS = (good.colptr, good.rowind)
    calls = {
        "pattern(A_k)": lambda: ctx.pattern(broken, 2),
        "plan(A_k)": lambda: ctx.plan(broken, good, *gS),
        "plan(A_0)": lambda: ctx.plan(good, broken, *gS),
        "plan(S)": lambda: ctx.plan(good, good, broken.colptr, broken.rowind),
        "build(S)": lambda: ctx.build(good, good, broken.colptr, broken.rowind, "f32"),
        "sequence(A_k)": lambda: ctx.sequence(good, broken, 2, power=2),
        "sequence(A_0)": lambda: ctx.sequence(broken, good, 2, power=2),
        "apply_prepare(M)": lambda: ctx.apply_prepare(n, broken.colptr, broken.rowind),
    }
    for what, call in calls.items():
        with pytest.raises(SamError) as e:
            call()
        assert e.value.status == C.SAM_ERR_UNSORTED, (what, name, str(e.value))
    ctx.sync_status()     # no kernel reported anything
