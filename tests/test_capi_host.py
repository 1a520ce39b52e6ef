"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/sam.h declares, and validates arguments before it
touches a device."""
import ctypes

import pytest

from paper_2406_17656_amd import _capi as C


def test_exports_every_declared_symbol():
    lib = C.load()
    names = C.header_symbols()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(C.SIGNATURES), set(names) ^ set(C.SIGNATURES)


def test_status_strings_and_version():
    lib = C.load()
    for code, name in C.STATUS_NAMES.items():
        assert lib.sam_status_string(code).decode() == name
    assert lib.sam_version().decode().count(".") == 2


@pytest.fixture
def hctx():
    lib = C.load()
    h = ctypes.c_void_p()
    assert lib.sam_create(ctypes.byref(h), C.SAM_NO_DEVICE) == C.SAM_OK
    yield lib, h
    lib.sam_destroy(h)


def csc(n=4, nnz=4, ptr=1):
    return C.sam_csc(n, nnz, ptr, ptr, ptr)


def spec(**kw):
    d = dict(kind=0, power=1, thresh=0.0, global_scale=-1, tau=0.0, lfil=1)
    d.update(kw)
    return C.sam_pattern_spec(d["kind"], d["power"], d["thresh"], d["global_scale"], d["tau"], d["lfil"])


def test_null_context_rejected():
    lib = C.load()
    nnz = ctypes.c_int64()
    a = csc()
    sp = spec()
    assert lib.sam_pattern_count(None, ctypes.byref(a), ctypes.byref(sp), ctypes.byref(nnz), None) == 1
    assert lib.sam_create(None, 0) == 1


@pytest.mark.parametrize("bad,code", [
    (dict(power=0), 1), (dict(kind=7), 1), (dict(kind=2, tau=1.5), 1), (dict(kind=2, tau=-0.1), 1),
    (dict(kind=3, lfil=0), 1), (dict(kind=1, global_scale=0), 1),
])
def test_pattern_spec_validation(hctx, bad, code):
    lib, h = hctx
    nnz = ctypes.c_int64()
    a = csc()
    sp = spec(**bad)
    assert lib.sam_pattern_count(h, ctypes.byref(a), ctypes.byref(sp), ctypes.byref(nnz), None) == code
    assert lib.sam_last_error(h).decode()


def test_valid_arguments_reach_the_device_check(hctx):
    lib, h = hctx
    nnz = ctypes.c_int64()
    a = csc()
    sp = spec(power=2)
    assert lib.sam_pattern_count(h, ctypes.byref(a), ctypes.byref(sp), ctypes.byref(nnz), None) == 8
    assert "no device" in lib.sam_last_error(h).decode()


def test_plan_shape_and_overflow_checks(hctx):
    lib, h = hctx
    pl = ctypes.c_void_p()
    a, b = csc(n=4), csc(n=5)
    assert lib.sam_plan_create(h, ctypes.byref(a), ctypes.byref(b), 1, 1, 4, ctypes.byref(pl), None) == 2
    b = csc(n=4)
    assert lib.sam_plan_create(h, ctypes.byref(a), ctypes.byref(b), 1, 1, 2 ** 31, ctypes.byref(pl), None) == 4
    assert lib.sam_plan_create(h, ctypes.byref(a), ctypes.byref(b), 1, 1, -1, ctypes.byref(pl), None) == 1
    neg = csc(n=-1)
    assert lib.sam_plan_create(h, ctypes.byref(neg), ctypes.byref(b), 1, 1, 4, ctypes.byref(pl), None) == 1
    nullrows = C.sam_csc(4, 4, 1, None, 1)
    assert lib.sam_plan_create(h, ctypes.byref(nullrows), ctypes.byref(b), 1, 1, 4, ctypes.byref(pl), None) == 1


def test_build_and_residual_argument_checks(hctx):
    lib, h = hctx
    a, b = csc(n=4), csc(n=4)
    # unknown precision
    assert lib.sam_build(h, ctypes.byref(a), ctypes.byref(b), 1, 1, 4, 7, 1, None, None, None) == 1
    # missing M
    assert lib.sam_build(h, ctypes.byref(a), ctypes.byref(b), 1, 1, 4, 0, None, None, None, None) == 1
    # residual: order mismatch, nnz overflow, null res2
    c = csc(n=3)
    assert lib.sam_residual(h, ctypes.byref(a), ctypes.byref(c), 1, 1, 4, 1, 0, 1, None, None) == 2
    assert lib.sam_residual(h, ctypes.byref(a), ctypes.byref(b), 1, 1, 2 ** 31, 1, 0, 1, None, None) == 4
    assert lib.sam_residual(h, ctypes.byref(a), ctypes.byref(b), 1, 1, 4, 1, 0, None, None, None) == 1
    # apply
    assert lib.sam_apply_prepare(h, 4, 1, 1, 2 ** 31, 1, 1, 1, None) == 4
    assert lib.sam_apply(h, 4, 1, 1, 1, 1, 9, 1, 1, None) == 1


def test_empty_matrices_rejected(hctx):
    lib, h = hctx
    pl = ctypes.c_void_p()
    a, b = csc(n=4, nnz=0), csc(n=4)
    assert lib.sam_plan_create(h, ctypes.byref(a), ctypes.byref(b), 1, 1, 4, ctypes.byref(pl), None) == 1
    assert "stored entries" in lib.sam_last_error(h).decode()


def test_empty_sequence_rejected(hctx):
    lib, h = hctx
    sq = ctypes.c_void_p()
    a = csc(n=0, nnz=0)
    spec = C.sam_pattern_spec(0, 2, 0.0, -1, 0.0, 1)
    assert lib.sam_sequence_create(h, ctypes.byref(a), ctypes.byref(a), ctypes.byref(spec), 2, 1, 1,
                                   ctypes.byref(sq), None) == 1
    assert "empty" in lib.sam_last_error(h).decode()


def test_menu_without_device():
    from paper_2406_17656_amd import autotune
    for prec in ("f32", "f64"):
        m = autotune.menu(prec)
        assert len(m) >= 6 and all(v["max_rows"] >= 13 and v["NC"] >= 5 for v in m)
        assert autotune.menu(prec, weighted=1)
    orders = autotune.candidate_orders(5)
    assert orders[0] == [0, 1, 2, 3, 4] and [3, 0, 1, 2, 4] in orders
    lib = C.load()
    cnt = ctypes.c_int32()
    assert lib.sam_menu(7, 0, 0, ctypes.byref(cnt), None, None, None, None) == 1


def test_plan_select_validation(hctx):
    lib, h = hctx
    # no plan: argument error before anything else
    arr = (ctypes.c_int32 * 1)(0)
    assert lib.sam_plan_select(None, 1, arr, 1, None) == 1


def test_adaptive_calls_validate_arguments(hctx):
    """Argument checks of the adaptive-pattern calls come before any device
    work: NULLs, negative sizes and k < 0 are SAM_ERR_ARG, oversized patterns
    SAM_ERR_OVERFLOW; valid arguments on a context without a device reach
    SAM_ERR_UNSUPPORTED."""
    lib, h = hctx
    out = ctypes.c_int64()
    w = ctypes.c_double()
    # sam_candidate_weights(ctx, n, S_cp, S_ri, nnz_S, B_cp, B_ri, nnz_B, w_base, w_cand, w, stream)
    assert lib.sam_candidate_weights(h, -1, 1, 1, 4, 1, 1, 4, 1.0, 0.1, 1, None) == C.SAM_ERR_ARG
    assert lib.sam_candidate_weights(h, 4, None, 1, 4, 1, 1, 4, 1.0, 0.1, 1, None) == C.SAM_ERR_ARG
    assert lib.sam_candidate_weights(h, 4, 1, 1, 4, 1, 1, 4, 1.0, 0.1, None, None) == C.SAM_ERR_ARG
    assert lib.sam_candidate_weights(h, 4, 1, 1, 2 ** 31, 1, 1, 4, 1.0, 0.1, 1, None) == C.SAM_ERR_OVERFLOW
    assert lib.sam_candidate_weights(h, 4, 1, 1, 4, 1, 1, 4, 1.0, 0.1, 1, None) == C.SAM_ERR_UNSUPPORTED
    # sam_pattern_topk(ctx, n, S_cp, S_ri, nnz_S, w, grad, k, out_cp, out_ri, nnz_out, stream)
    assert lib.sam_pattern_topk(h, 4, 1, 1, 4, 1, 1, -1, 1, 1, ctypes.byref(out), None) == C.SAM_ERR_ARG
    assert lib.sam_pattern_topk(h, 4, 1, 1, 4, None, 1, 2, 1, 1, ctypes.byref(out), None) == C.SAM_ERR_ARG
    assert lib.sam_pattern_topk(h, 4, 1, 1, 4, 1, 1, 2, 1, 1, None, None) == C.SAM_ERR_ARG
    assert lib.sam_pattern_topk(h, 4, 1, 1, 4, 1, 1, 2, 1, 1, ctypes.byref(out), None) == C.SAM_ERR_UNSUPPORTED
    # sam_penalty_scale(ctx, Ak, mu, stream)
    a = csc()
    assert lib.sam_penalty_scale(h, ctypes.byref(a), None, None) == C.SAM_ERR_ARG
    e = csc(n=0, nnz=0)
    assert lib.sam_penalty_scale(h, ctypes.byref(e), ctypes.byref(w), None) == C.SAM_ERR_ARG
    nv = C.sam_csc(4, 4, 1, 1, None)
    assert lib.sam_penalty_scale(h, ctypes.byref(nv), ctypes.byref(w), None) == C.SAM_ERR_ARG
    assert lib.sam_penalty_scale(h, ctypes.byref(a), ctypes.byref(w), None) == C.SAM_ERR_UNSUPPORTED
