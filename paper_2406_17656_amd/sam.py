"""Python binding of the SAM C ABI over torch tensors (device memory and
streams only; every step runs in the HIP library).

Names follow include/sam.h: ``Context.pattern`` wraps sam_pattern_count +
sam_pattern_fill, ``Context.plan`` sam_plan_create, ``Plan.build``
sam_build_planned, ``Context.build`` sam_build, ``Context.residual``
sam_residual, ``Context.apply_prepare`` / ``Context.apply`` the y = M x calls,
``Context.sequence`` the sequence calls, ``Plan.build_weighted`` /
``Plan.backward`` the soft-weighted map and its adjoint.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _capi as C

PREC = {"f64": C.SAM_PREC_F64, "f32": C.SAM_PREC_F32_REFINE, "f32_refine": C.SAM_PREC_F32_REFINE}


class SamError(RuntimeError):
    def __init__(self, status: int, message: str, column: int = -1):
        name = C.STATUS_NAMES.get(status, str(status))
        super().__init__(f"{name}: {message}" if message else name)
        self.status = status
        self.name = name
        self.column = column


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _buf(nbytes: int, device) -> torch.Tensor:
    """Device memory for the library (torch allocations are 512-byte aligned;
    freed tensors return to torch's pool in stream order, after the kernels
    already enqueued on the same stream)."""
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _size(fn, *args) -> int:
    nb = ctypes.c_size_t()
    st = fn(*args, ctypes.byref(nb))
    if st != C.SAM_OK:
        raise SamError(st, fn.__name__)
    return nb.value


def _prec(p) -> int:
    if isinstance(p, str):
        return PREC[p]
    return int(p)


def _mdtype(prec: int):
    return torch.float32 if prec == C.SAM_PREC_F32_REFINE else torch.float64


@dataclass
class DeviceCSC:
    """Square CSC matrix held in device tensors."""
    n: int
    colptr: torch.Tensor   # int32 n+1
    rowind: torch.Tensor   # int32 nnz
    val: torch.Tensor | None = None  # float64 nnz

    @property
    def nnz(self) -> int:
        return int(self.rowind.numel())

    @staticmethod
    def from_host(A, device="cuda") -> "DeviceCSC":
        """From any object with n, colptr, rowind, val numpy arrays."""
        return DeviceCSC(int(A.n),
                         torch.as_tensor(np.ascontiguousarray(A.colptr, dtype=np.int32)).to(device),
                         torch.as_tensor(np.ascontiguousarray(A.rowind, dtype=np.int32)).to(device),
                         None if getattr(A, "val", None) is None else
                         torch.as_tensor(np.ascontiguousarray(A.val, dtype=np.float64)).to(device))

    def struct(self) -> C.sam_csc:
        return C.sam_csc(self.n, self.nnz, self.colptr.data_ptr(), self.rowind.data_ptr(),
                         None if self.val is None else self.val.data_ptr())


def _spec(kind="none", power=1, thresh=0.0, global_scale=-1, tau=0.0, lfil=1) -> C.sam_pattern_spec:
    return C.sam_pattern_spec(C.SPARSIFY[kind] if isinstance(kind, str) else int(kind), int(power),
                              float(thresh), int(global_scale), float(tau), int(lfil))


class Context:
    """A sam_ctx bound to one HIP device."""

    def __init__(self, device: int = 0):
        self.lib = C.load()
        self.device = device
        h = ctypes.c_void_p()
        st = self.lib.sam_create(ctypes.byref(h), device)
        if st != C.SAM_OK:
            raise SamError(st, f"sam_create(device={device}) failed")
        self.h = h

    # -- plumbing
    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.sam_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stream(self):
        if self.device == C.SAM_NO_DEVICE:
            return None
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def check(self, st: int):
        if st != C.SAM_OK:
            msg = self.lib.sam_last_error(self.h)
            raise SamError(st, msg.decode() if msg else "")

    def sync_status(self):
        col = ctypes.c_int32(-1)
        st = self.lib.sam_sync_status(self.h, self.stream(), ctypes.byref(col))
        if st != C.SAM_OK:
            msg = self.lib.sam_last_error(self.h)
            raise SamError(st, msg.decode() if msg else "", col.value)

    def check_csc(self, A: DeviceCSC):
        s = A.struct()
        self.check(self.lib.sam_check_csc(self.h, ctypes.byref(s), self.stream()))

    # -- pattern (Sections 3-4)
    def pattern(self, Ak: DeviceCSC, power=1, kind="none", **kw):
        s = Ak.struct()
        sp = _spec(kind, power, **kw)
        dev = Ak.colptr.device
        nb = ctypes.c_size_t()
        self.check(self.lib.sam_pattern_workspace_size(self.h, ctypes.byref(s), ctypes.byref(sp), ctypes.byref(nb),
                                                       self.stream()))
        ws = _buf(nb.value, dev)
        nnz = ctypes.c_int64()
        self.check(self.lib.sam_pattern_count(self.h, ctypes.byref(s), ctypes.byref(sp), _ptr(ws), nb.value,
                                              ctypes.byref(nnz), self.stream()))
        cp = torch.empty(Ak.n + 1, dtype=torch.int32, device=dev)
        ri = torch.empty(max(nnz.value, 1), dtype=torch.int32, device=dev)
        self.check(self.lib.sam_pattern_fill(self.h, ctypes.byref(s), ctypes.byref(sp), _ptr(ws), nb.value,
                                             _ptr(cp), _ptr(ri), self.stream()))
        return cp, ri[:nnz.value]

    # -- build (Section 2)
    def plan(self, Ak: DeviceCSC, A0: DeviceCSC, S_colptr, S_rowind) -> "Plan":
        return Plan(self, Ak, A0, S_colptr, S_rowind)

    def build(self, Ak: DeviceCSC, A0: DeviceCSC, S_colptr, S_rowind, prec="f64", want_cols=True):
        p = _prec(prec)
        nnz = int(S_rowind.numel())
        dev = Ak.colptr.device
        M = torch.empty(max(nnz, 1), dtype=_mdtype(p), device=dev)
        cols = torch.empty(max(Ak.n, 1), dtype=torch.float64, device=dev) if want_cols else None
        res2 = torch.empty(1, dtype=torch.float64, device=dev)
        a, b = Ak.struct(), A0.struct()
        nb = ctypes.c_size_t()
        self.check(self.lib.sam_workspace_size(self.h, ctypes.byref(a), ctypes.byref(b), _ptr(S_colptr),
                                               _ptr(S_rowind), nnz, p, ctypes.byref(nb), self.stream()))
        ws = _buf(nb.value, dev)
        self.check(self.lib.sam_build(self.h, ctypes.byref(a), ctypes.byref(b), _ptr(S_colptr),
                                      _ptr(S_rowind), nnz, p, _ptr(M), _ptr(cols), _ptr(res2),
                                      _ptr(ws), nb.value, self.stream()))
        return M[:nnz], (cols[:Ak.n] if cols is not None else None), res2

    # -- residual (Section 2 eq. res)
    def residual(self, Ak: DeviceCSC, A0: DeviceCSC, M_colptr, M_rowind, M_val, prec="f64"):
        p = _prec(prec)
        dev = Ak.colptr.device
        res2 = torch.empty(1, dtype=torch.float64, device=dev)
        a02 = torch.empty(1, dtype=torch.float64, device=dev)
        a, b = Ak.struct(), A0.struct()
        nb = _size(self.lib.sam_residual_workspace_size, Ak.n, A0.nnz)
        ws = _buf(nb, dev)
        self.check(self.lib.sam_residual(self.h, ctypes.byref(a), ctypes.byref(b), _ptr(M_colptr),
                                         _ptr(M_rowind), int(M_rowind.numel()), _ptr(M_val), p,
                                         _ptr(res2), _ptr(a02), _ptr(ws), nb, self.stream()))
        return res2, a02

    # -- y = M x
    def apply_prepare(self, n, M_colptr, M_rowind):
        nnz = int(M_rowind.numel())
        dev = M_colptr.device
        rp = torch.empty(n + 1, dtype=torch.int32, device=dev)
        ci = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
        pm = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
        nb = _size(self.lib.sam_apply_workspace_size, n)
        ws = _buf(nb, dev)
        self.check(self.lib.sam_apply_prepare(self.h, n, _ptr(M_colptr), _ptr(M_rowind), nnz, _ptr(rp),
                                              _ptr(ci), _ptr(pm), _ptr(ws), nb, self.stream()))
        return rp, ci, pm

    def apply_permute(self, T, M_val, prec="f64"):
        """M's values in the row view's order (sam_apply_permute), for
        apply(..., permuted=True)."""
        pm = T[2]
        nnz = int(M_val.numel())
        out = torch.empty_like(M_val)
        self.check(self.lib.sam_apply_permute(self.h, nnz, _ptr(pm), _ptr(M_val), _prec(prec), _ptr(out),
                                              self.stream()))
        return out

    def apply(self, T, M_val, x, prec="f64", y=None, permuted=False):
        """y = M x; permuted: M_val comes from apply_permute (row order)."""
        rp, ci, pm = T
        n = rp.numel() - 1
        if y is None:
            y = torch.empty(n, dtype=torch.float64, device=x.device)
        self.check(self.lib.sam_apply(self.h, n, _ptr(rp), _ptr(ci), None if permuted else _ptr(pm), _ptr(M_val),
                                      _prec(prec), _ptr(x), _ptr(y), self.stream()))
        return y

    # -- adaptive patterns (future work of the paper, end of Section 2)
    def candidate_weights(self, S_colptr, S_rowind, B_colptr, B_rowind, w_base=1.0, w_cand=0.1):
        """sam_candidate_weights: w over S's entries, w_base on B's entries."""
        n = S_colptr.numel() - 1
        w = torch.empty(max(int(S_rowind.numel()), 1), dtype=torch.float64, device=S_colptr.device)
        self.check(self.lib.sam_candidate_weights(self.h, n, _ptr(S_colptr), _ptr(S_rowind), int(S_rowind.numel()),
                                                  _ptr(B_colptr), _ptr(B_rowind), int(B_rowind.numel()),
                                                  float(w_base), float(w_cand), _ptr(w), self.stream()))
        return w[:S_rowind.numel()]

    def pattern_topk(self, S_colptr, S_rowind, w, grad, k):
        """sam_pattern_topk: base entries (w >= 1) plus the k smallest-grad candidates per column."""
        n = S_colptr.numel() - 1
        nnz = int(S_rowind.numel())
        dev = S_colptr.device
        cp = torch.empty(n + 1, dtype=torch.int32, device=dev)
        ri = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
        out = ctypes.c_int64()
        nb = _size(self.lib.sam_topk_workspace_size, n)
        ws = _buf(nb, dev)
        self.check(self.lib.sam_pattern_topk(self.h, n, _ptr(S_colptr), _ptr(S_rowind), nnz, _ptr(w), _ptr(grad),
                                             int(k), _ptr(cp), _ptr(ri), ctypes.byref(out), _ptr(ws), nb,
                                             self.stream()))
        return cp, ri[:out.value]

    def penalty_scale(self, Ak: DeviceCSC) -> float:
        """sam_penalty_scale: ||A_k||_F^2 / n."""
        a = Ak.struct()
        mu = ctypes.c_double()
        nb = _size(self.lib.sam_penalty_workspace_size, Ak.nnz)
        ws = _buf(nb, Ak.colptr.device)
        self.check(self.lib.sam_penalty_scale(self.h, ctypes.byref(a), ctypes.byref(mu), _ptr(ws), nb,
                                              self.stream()))
        return mu.value

    # -- sequence
    def sequence(self, A0: DeviceCSC, Ak_struct: DeviceCSC, n_src: int, prec="f32", power=1,
                 kind="none", replan_each_run=False, **kw) -> "Sequence":
        return Sequence(self, A0, Ak_struct, n_src, _prec(prec), _spec(kind, power, **kw),
                        replan_each_run)


class Plan:
    """sam_plan: symbolic analysis of the column problems."""

    def __init__(self, ctx: Context, Ak: DeviceCSC, A0: DeviceCSC, S_colptr, S_rowind):
        self.ctx = ctx
        self.Ak, self.A0 = Ak, A0          # keep the structure arrays alive
        self.S_colptr, self.S_rowind = S_colptr, S_rowind
        self.n = Ak.n
        self.nnz_S = int(S_rowind.numel())
        self._bwd = None                   # backward workspace, prepared on first use
        h = ctypes.c_void_p()
        a, b = Ak.struct(), A0.struct()
        nb = ctypes.c_size_t()
        ctx.check(ctx.lib.sam_plan_size(ctx.h, ctypes.byref(a), ctypes.byref(b), _ptr(S_colptr), _ptr(S_rowind),
                                        self.nnz_S, ctypes.byref(nb), ctx.stream()))
        self.mem = _buf(nb.value, Ak.colptr.device)   # owned by the plan until close()
        ctx.check(ctx.lib.sam_plan_create(ctx.h, ctypes.byref(a), ctypes.byref(b), _ptr(S_colptr),
                                          _ptr(S_rowind), self.nnz_S, _ptr(self.mem), nb.value, ctypes.byref(h),
                                          ctx.stream()))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            torch.cuda.synchronize(self.ctx.device)
            self.ctx.lib.sam_plan_destroy(self.h)
            self.h = None
            self.mem = None
            self._bwd = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        n = ctypes.c_int32(); mr = ctypes.c_int32(); mc = ctypes.c_int32()
        ga = ctypes.c_int64(); nb = ctypes.c_int32(); bc = (ctypes.c_int32 * 16)()
        self.ctx.check(self.ctx.lib.sam_plan_info(self.h, ctypes.byref(n), ctypes.byref(mr),
                                                  ctypes.byref(mc), ctypes.byref(ga), ctypes.byref(nb), bc))
        return {"n": n.value, "max_rows": mr.value, "max_cols": mc.value, "gathered": ga.value,
                "bucket_cols": list(bc[:nb.value])}

    def select(self, order, prec="f32"):
        """sam_plan_select: serve columns with the first listed menu variant that fits."""
        arr = (ctypes.c_int32 * len(order))(*order)
        self.ctx.check(self.ctx.lib.sam_plan_select(self.h, _prec(prec), arr, len(order), self.ctx.stream()))

    def cost(self, prec="f32") -> dict:
        f32 = ctypes.c_double(); f64 = ctypes.c_double(); by = ctypes.c_double()
        self.ctx.check(self.ctx.lib.sam_plan_cost(self.h, _prec(prec), ctypes.byref(f32), ctypes.byref(f64),
                                                  ctypes.byref(by)))
        return {"flops32": f32.value, "flops64": f64.value, "bytes": by.value}

    def cost_weighted(self, prec="f32", backward=False) -> dict:
        """sam_plan_cost_weighted: algorithmic flops of one weighted build or
        one adjoint on this plan."""
        f32 = ctypes.c_double(); f64 = ctypes.c_double()
        self.ctx.check(self.ctx.lib.sam_plan_cost_weighted(self.h, _prec(prec), 1 if backward else 0,
                                                           ctypes.byref(f32), ctypes.byref(f64)))
        return {"flops32": f32.value, "flops64": f64.value}

    def _outs(self, prec, M, cols, res2, fro=True):
        dev = self.S_colptr.device
        if M is None:
            M = torch.empty(max(self.nnz_S, 1), dtype=_mdtype(prec), device=dev)
        if res2 is None and fro:
            res2 = torch.empty(1, dtype=torch.float64, device=dev)
        return M, cols, res2

    def build(self, Ak_val, A0_val, prec="f64", M=None, col_res2=None, res2=None, fro=True):
        """sam_build_planned.  fro=False (and no res2) leaves out the
        Frobenius sum: the launches are then the numeric kernels alone."""
        p = _prec(prec)
        M, col_res2, res2 = self._outs(p, M, col_res2, res2, fro)
        self.ctx.check(self.ctx.lib.sam_build_planned(self.h, _ptr(Ak_val), _ptr(A0_val), p, _ptr(M),
                                                      _ptr(col_res2), _ptr(res2), self.ctx.stream()))
        return M[:self.nnz_S], col_res2, res2

    def build_weighted(self, Ak_val, A0_val, w, mu, prec="f32", M=None, col_res2=None, res2=None):
        p = _prec(prec)
        M, col_res2, res2 = self._outs(p, M, col_res2, res2)
        self.ctx.check(self.ctx.lib.sam_build_weighted(self.h, _ptr(Ak_val), _ptr(A0_val), _ptr(w),
                                                       float(mu), p, _ptr(M), _ptr(col_res2), _ptr(res2),
                                                       self.ctx.stream()))
        return M[:self.nnz_S], col_res2, res2

    def backward(self, Ak_val, A0_val, w, mu, dL=1.0, prec="f32", want_gw=True):
        p = _prec(prec)
        dev = Ak_val.device
        gAk = torch.empty_like(Ak_val)
        gA0 = torch.empty_like(A0_val)
        gw = torch.empty(max(self.nnz_S, 1), dtype=torch.float64, device=dev) if want_gw else None
        loss = torch.empty(1, dtype=torch.float64, device=dev)
        if self._bwd is None:
            nb = ctypes.c_size_t()
            self.ctx.check(self.ctx.lib.sam_backward_workspace_size(self.h, ctypes.byref(nb)))
            ws = _buf(nb.value, dev)
            self.ctx.check(self.ctx.lib.sam_backward_prepare(self.h, _ptr(ws), nb.value, self.ctx.stream()))
            self._bwd = (ws, nb.value)
        ws, nb = self._bwd
        self.ctx.check(self.ctx.lib.sam_backward(self.h, _ptr(Ak_val), _ptr(A0_val), _ptr(w), float(mu),
                                                 float(dL), p, _ptr(gAk), _ptr(gA0), _ptr(gw), _ptr(loss),
                                                 _ptr(ws), nb, self.ctx.stream()))
        return gAk, gA0, (gw[:self.nnz_S] if gw is not None else None), loss


class Sequence:
    """sam_seq: maps A_1..A_N to A_0 with one graph launch per run."""

    def __init__(self, ctx: Context, A0: DeviceCSC, Ak_struct: DeviceCSC, n_src: int, prec: int,
                 spec: C.sam_pattern_spec, replan_each_run: bool):
        self.ctx = ctx
        self.A0, self.Ak_struct = A0, Ak_struct
        self.n_src = n_src
        self.prec = prec
        self.spec = spec
        h = ctypes.c_void_p()
        a, b = A0.struct(), Ak_struct.struct()
        dev = A0.colptr.device
        replan = 1 if replan_each_run else 0
        nb = ctypes.c_size_t()
        ctx.check(ctx.lib.sam_pattern_workspace_size(ctx.h, ctypes.byref(b), ctypes.byref(spec), ctypes.byref(nb),
                                                     ctx.stream()))
        ws = _buf(nb.value, dev)
        total = ctypes.c_size_t()
        ctx.check(ctx.lib.sam_sequence_size(ctx.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(spec), n_src,
                                            prec, replan, _ptr(ws), nb.value, ctypes.byref(total), ctx.stream()))
        del ws
        self.mem = _buf(total.value, dev)   # owned by the sequence until close()
        ctx.check(ctx.lib.sam_sequence_create(ctx.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(spec),
                                              n_src, prec, replan, _ptr(self.mem), total.value, ctypes.byref(h),
                                              ctx.stream()))
        self.h = h
        nb = ctypes.c_int64()
        ctx.check(ctx.lib.sam_sequence_info(self.h, ctypes.byref(nb)))
        self.nnz_bound = nb.value

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            torch.cuda.synchronize(self.ctx.device)
            self.ctx.lib.sam_sequence_destroy(self.h)
            self.h = None
            self.mem = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def alloc_maps(self):
        dev = self.A0.colptr.device
        return [torch.empty(max(self.nnz_bound, 1), dtype=_mdtype(self.prec), device=dev)
                for _ in range(self.n_src)]

    def select(self, order):
        arr = (ctypes.c_int32 * len(order))(*order)
        self.ctx.check(self.ctx.lib.sam_sequence_select(self.h, arr, len(order), self.ctx.stream()))

    def run(self, Ak_vals, M_vals, res2):
        arr_a = (ctypes.c_void_p * self.n_src)(*[t.data_ptr() for t in Ak_vals])
        arr_m = (ctypes.c_void_p * self.n_src)(*[t.data_ptr() for t in M_vals])
        self.ctx.check(self.ctx.lib.sam_sequence_run(self.h, arr_a, arr_m, _ptr(res2), self.ctx.stream()))

    def pattern(self, k: int):
        """Pattern of source k from the last run (colptr, rowind tensors)."""
        dev = self.A0.colptr.device
        cp = torch.empty(self.A0.n + 1, dtype=torch.int32, device=dev)
        ri = torch.empty(max(self.nnz_bound, 1), dtype=torch.int32, device=dev)
        nnz = ctypes.c_int64()
        self.ctx.check(self.ctx.lib.sam_sequence_pattern(self.h, k, _ptr(cp), _ptr(ri), ctypes.byref(nnz),
                                                         self.ctx.stream()))
        return cp, ri[:nnz.value]
