"""Batched Newton-Raphson AC power flow on AMD MI355X (gfx950).

Thin Python binding over the C ABI in ``include/pf.h``: argument marshalling only.
Device memory and streams come from PyTorch; every step of the solve runs in the HIP
library ``libpf_hip.so`` built from ``csrc/``.  Nothing here falls back to the CPU:
if the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpf_hip.so")

PF_BUS_PQ, PF_BUS_PV, PF_BUS_REF = 1, 2, 3
PF_ORDER_NATURAL, PF_ORDER_MIN_DEGREE, PF_ORDER_USER = 0, 1, 2
PF_FP64, PF_FP32_LU = 0, 1
PF_LAUNCH_AUTO, PF_LAUNCH_FUSED, PF_LAUNCH_PHASES = 0, 1, 2
PF_REORDER_AUTO, PF_REORDER_OFF = 0, 1
PF_ST_CONVERGED, PF_ST_MAXITER, PF_ST_NONFINITE, PF_ST_PIVOT, PF_ST_INTERNAL = 0, 1, 2, 3, -1

EXPORTED = ["pf_analyze", "pf_plan_info", "pf_plan_order", "pf_plan_lu_pattern",
            "pf_workspace_bytes", "pf_solve_batch", "pf_eval_mismatch", "pf_eval_factor",
            "pf_eval_step", "pf_plan_destroy", "pf_last_error", "pf_mlp_gemm",
            "pf_mlp_act_backward", "pf_mlp_mse", "pf_mlp_adam", "pf_mlp_to_bf16",
            "pf_mlp_features", "pf_mlp_warm_v0", "pf_queue_create", "pf_queue_add",
            "pf_queue_run", "pf_queue_info", "pf_queue_destroy", "pf_tune", "pf_tune_cache_save",
            "pf_tune_cache_load", "pf_tune_cache_clear", "pf_tune_cache_size", "pf_solve_batch_warm",
            "pf_resolve_opts", "pf_branch_flows", "pf_plan_schedule", "pf_solve_host",
            "pf_plan_levels", "pf_cpu_solve_batch", "pf_cpu_solve_pivoting", "pf_solve_fallback",
            "pf_solve_batch_noalloc", "pf_plan_ring"]


class PfError(RuntimeError):
    pass


class _PlanInfo(ctypes.Structure):
    _fields_ = [("n_bus", ctypes.c_int32), ("n_pv", ctypes.c_int32), ("n_pq", ctypes.c_int32),
                ("n_unknowns", ctypes.c_int32), ("nnz_y", ctypes.c_int32), ("nnz_j", ctypes.c_int32),
                ("nnz_lu", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("n_bs_levels", ctypes.c_int32), ("n_panels", ctypes.c_int32),
                ("slot_rows", ctypes.c_int32), ("max_col", ctypes.c_int32),
                ("n_updates", ctypes.c_int64), ("flops_refactor", ctypes.c_int64),
                ("bytes_iter_fp64", ctypes.c_int64), ("bytes_iter_fp32", ctypes.c_int64),
                ("pattern_hash", ctypes.c_uint64)]


class _Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("tile", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("long_slots", ctypes.c_int32), ("launch", ctypes.c_int32),
                ("reorder", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _QueueInfo(ctypes.Structure):
    _fields_ = [("n_items", ctypes.c_int32), ("n_groups", ctypes.c_int32), ("built", ctypes.c_int32),
                ("grid", ctypes.c_int32 * 18), ("n_tiles", ctypes.c_int64),
                ("n_instances", ctypes.c_int64), ("workspace_bytes", ctypes.c_size_t),
                ("wall_clock_hz", ctypes.c_double)]


_lib = None
_vp = ctypes.c_void_p
_i32p = ctypes.POINTER(ctypes.c_int32)
_i8p = ctypes.POINTER(ctypes.c_int8)


def lib():
    """Load libpf_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PfError(f"HIP library not built: {LIB_PATH} is missing "
                          "(run paper_2101_02270_amd.build.build())")
        L = ctypes.CDLL(LIB_PATH)
        L.pf_analyze.argtypes = [ctypes.c_int32, ctypes.c_int32, _i32p, _i32p, _i8p, ctypes.c_int32,
                                 _i32p, ctypes.POINTER(_vp)]
        L.pf_plan_info.argtypes = [_vp, ctypes.POINTER(_PlanInfo)]
        L.pf_plan_order.argtypes = [_vp, _i32p]
        L.pf_plan_levels.argtypes = [_vp, _i32p, ctypes.POINTER(ctypes.c_int64)]
        L.pf_cpu_solve_batch.argtypes = [_vp, ctypes.c_int32, _vp, _vp, _vp, ctypes.c_double, ctypes.c_int32,
                                         ctypes.c_int32, _vp, _vp, _vp, _vp]
        L.pf_cpu_solve_pivoting.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp, _vp, ctypes.c_double,
                                            ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp]
        L.pf_solve_fallback.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp, _vp, ctypes.c_double,
                                        ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp, _i32p, _vp]
        L.pf_solve_batch_noalloc.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp, _vp, ctypes.c_double,
                                             ctypes.c_int32, ctypes.POINTER(_Opts), _vp, _vp, _vp, _vp, _vp]
        L.pf_plan_lu_pattern.argtypes = [_vp, _i32p, _i32p, _i32p]
        L.pf_plan_ring.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _i32p, _i32p, _i32p, _i32p]
        L.pf_workspace_bytes.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(_Opts)]
        L.pf_workspace_bytes.restype = ctypes.c_size_t
        L.pf_solve_batch.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp, _vp,
                                     ctypes.c_double, ctypes.c_int32, ctypes.POINTER(_Opts), _vp,
                                     ctypes.c_size_t, _vp, _vp, _vp, _vp, _vp]
        for f in ("pf_eval_mismatch",):
            getattr(L, f).argtypes = [_vp, ctypes.c_int32, _vp, _vp, _vp, ctypes.POINTER(_Opts), _vp,
                                      ctypes.c_size_t, _vp, _vp, _vp]
        for f in ("pf_eval_factor", "pf_eval_step"):
            getattr(L, f).argtypes = [_vp, ctypes.c_int32, _vp, _vp, _vp, ctypes.POINTER(_Opts), _vp,
                                      ctypes.c_size_t, _vp, _vp]
        L.pf_plan_destroy.argtypes = [_vp]
        i32, i64, f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float
        L.pf_mlp_gemm.argtypes = [i32, i32, i32, i32, i32, _vp, _vp, _vp, i32, _vp, _vp, _vp, _vp]
        L.pf_mlp_act_backward.argtypes = [i32, i32, _vp, _vp, i32, _vp, _vp, _vp]
        L.pf_mlp_mse.argtypes = [i64, _vp, _vp, _vp, _vp, i32, _vp]
        L.pf_mlp_adam.argtypes = [i64, _vp, _vp, _vp, _vp, _vp, f32, f32, f32, f32, i32, _vp]
        L.pf_mlp_to_bf16.argtypes = [i64, _vp, _vp, _vp]
        L.pf_mlp_features.argtypes = [i32, i32, _vp, _vp, _vp, _vp, i32, _vp, _vp, _vp, _vp]
        L.pf_mlp_warm_v0.argtypes = [i32, i32, _vp, _vp, i32, _vp, _vp, _vp, _vp, _vp, _vp]
        L.pf_solve_batch_warm.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp, _vp, _vp,
                                          ctypes.c_double, ctypes.c_int32, ctypes.POINTER(_Opts), _vp,
                                          ctypes.c_size_t, _vp, _vp, _vp, _vp, _vp]
        L.pf_branch_flows.argtypes = [i32, i32, _vp, _vp, _vp, _vp, _vp, i32, _vp, _vp, _vp, _vp, _vp]
        L.pf_solve_host.argtypes = [_vp, i32, _vp, _vp, _vp, ctypes.c_double, i32, ctypes.POINTER(_Opts), i32,
                                    _vp, _vp, _vp, _vp, _vp]
        L.pf_plan_schedule.argtypes = [_vp, i32, _i32p, _i32p, _i32p, _i32p]
        L.pf_resolve_opts.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(_Opts), ctypes.POINTER(_Opts)]
        L.pf_queue_create.argtypes = [ctypes.POINTER(_vp)]
        L.pf_queue_add.argtypes = [_vp, _vp, i32, _vp, _vp, _vp, ctypes.c_double, i32,
                                   ctypes.POINTER(_Opts), _vp, _vp, _vp, _vp, _vp]
        L.pf_queue_run.argtypes = [_vp, _vp]
        L.pf_queue_info.argtypes = [_vp, ctypes.POINTER(_QueueInfo)]
        L.pf_queue_destroy.argtypes = [_vp]
        L.pf_queue_destroy.restype = None
        L.pf_tune_cache_save.argtypes = [ctypes.c_char_p]
        L.pf_tune_cache_load.argtypes = [ctypes.c_char_p]
        L.pf_tune_cache_clear.argtypes = []
        L.pf_tune_cache_size.argtypes = []
        L.pf_tune_cache_size.restype = ctypes.c_int32
        L.pf_tune.argtypes = [_vp, i32, _vp, _vp, _vp, ctypes.c_double, i32, i32, i32, i32, i32,
                              ctypes.POINTER(_Opts), ctypes.POINTER(ctypes.c_double), _vp]
        L.pf_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        msg = lib().pf_last_error().decode()
        raise PfError(f"{what} failed ({rc}): {msg}")


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class Plan:
    """Analysed Ybus pattern (pf_analyze).  Device data live on the current device."""

    def __init__(self, row_ptr, col_idx, bus_type, ordering: int = PF_ORDER_MIN_DEGREE,
                 user_perm=None):
        rp = _np(row_ptr, np.int32)
        ci = _np(col_idx, np.int32)
        bt = _np(bus_type, np.int8)
        up = None if user_perm is None else _np(user_perm, np.int32)
        h = _vp()
        rc = lib().pf_analyze(int(rp.shape[0] - 1), int(ci.shape[0]),
                              rp.ctypes.data_as(_i32p), ci.ctypes.data_as(_i32p),
                              bt.ctypes.data_as(_i8p), int(ordering),
                              up.ctypes.data_as(_i32p) if up is not None else None,
                              ctypes.byref(h))
        _check(rc, "pf_analyze")
        self._h = h
        info = _PlanInfo()
        _check(lib().pf_plan_info(self._h, ctypes.byref(info)), "pf_plan_info")
        self.info = {f: getattr(info, f) for f, _ in _PlanInfo._fields_}
        self.n = self.info["n_bus"]
        self.N = self.info["n_unknowns"]
        self.nnz_y = self.info["nnz_y"]
        self.nnz_lu = self.info["nnz_lu"]

    @classmethod
    def from_ybus(cls, yb, bus_type, **kw):
        return cls(yb.row_ptr, yb.col_idx, bus_type, **kw)

    def close(self):
        if getattr(self, "_h", None):
            lib().pf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def order(self) -> np.ndarray:
        p = np.zeros(self.N, np.int32)
        _check(lib().pf_plan_order(self._h, p.ctypes.data_as(_i32p)), "pf_plan_order")
        return p

    def levels(self):
        """(columns per level, multiply-adds per level) of the refactorization's column DAG."""
        nl = self.info["n_levels"]
        cols = np.zeros(nl, np.int32)
        madds = np.zeros(nl, np.int64)
        _check(lib().pf_plan_levels(self._h, cols.ctypes.data_as(_i32p),
                                    madds.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))), "pf_plan_levels")
        return cols, madds

    def lu_pattern(self):
        cp = np.zeros(self.N + 1, np.int32)
        ri = np.zeros(self.nnz_lu, np.int32)
        lv = np.zeros(self.N, np.int32)
        _check(lib().pf_plan_lu_pattern(self._h, cp.ctypes.data_as(_i32p), ri.ctypes.data_as(_i32p),
                                        lv.ctypes.data_as(_i32p)), "pf_plan_lu_pattern")
        return cp, ri, lv

    def schedule(self, order: int = 0):
        """(first column, width, rank among the long panels or -1, first column of the long
        panel one rank earlier or -1) of every panel in processing order."""
        np_ = self.info["n_panels"]
        out = [np.zeros(np_, np.int32) for _ in range(4)]
        _check(lib().pf_plan_schedule(self._h, int(order), *[a.ctypes.data_as(_i32p) for a in out]),
               "pf_plan_schedule")
        return tuple(out)

    def ring(self, order: int, n_long: int):
        """(offset, rows, wait_lo, wait_hi) of every long panel's place in the LDS ring for an
        LDS budget of n_long pairs of max_col rows (pf_plan_ring)."""
        nl = int((self.schedule(order)[2] >= 0).sum())
        out = [np.zeros(max(nl, 1), np.int32) for _ in range(4)]
        _check(lib().pf_plan_ring(self._h, int(order), int(n_long), *[a.ctypes.data_as(_i32p) for a in out]),
               "pf_plan_ring")
        return tuple(a[:nl] for a in out)

    def resolve(self, batch: int, precision=PF_FP64, tile=0, waves=0, schedule=0, long_slots=0, launch=0,
                reorder=0) -> dict:
        """The configuration a solve of batch instances would use (pf_resolve_opts)."""
        o = _Opts()
        _check(lib().pf_resolve_opts(self._h, int(batch),
                                     ctypes.byref(_Opts(precision, tile, waves, schedule, long_slots, launch, reorder)),
                                     ctypes.byref(o)), "pf_resolve_opts")
        return {"precision": o.precision, "tile": o.tile, "waves": o.waves, "schedule": o.schedule,
                "long_slots": o.long_slots, "launch": o.launch, "reorder": o.reorder}

    def workspace_bytes(self, batch: int, precision=PF_FP64, tile=0, waves=0) -> int:
        o = _Opts(precision, tile, waves)
        return int(lib().pf_workspace_bytes(self._h, int(batch), ctypes.byref(o)))


@dataclass
class Result:
    v: "object"          # torch float64 [B][n][2]
    iters: "object"      # torch int32 [B]
    converged: "object"  # torch uint8 [B]
    status: "object"     # torch int8 [B]


def _torch():
    import torch
    return torch


def _dev_ptr(t, dtype, shape=None, name="tensor"):
    torch = _torch()
    if not t.is_cuda:
        raise PfError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise PfError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise PfError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise PfError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return _vp(t.data_ptr())


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return _vp(s.cuda_stream)


def _workspace(plan: Plan, batch, opts, workspace):
    torch = _torch()
    need = int(lib().pf_workspace_bytes(plan._h, int(batch), ctypes.byref(opts)))
    if need == 0:
        raise PfError("pf_workspace_bytes failed: " + lib().pf_last_error().decode())
    if workspace is None or workspace.numel() * workspace.element_size() < need:
        workspace = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    ptr = workspace.data_ptr()
    aligned = (ptr + 255) & ~255
    avail = workspace.numel() * workspace.element_size() - (aligned - ptr)
    return workspace, _vp(aligned), avail


def _ybus_view(plan: Plan, ybus, batch=None):
    """Shared Ybus values [nnz_y] (complex128) or [nnz_y][2], or with batch per-instance
    values [batch][nnz_y] / [batch][nnz_y][2].  Returns (pointer, tensor, batched flag)."""
    torch = _torch()
    if ybus.dtype == torch.complex128:
        ybus = torch.view_as_real(ybus)
    if ybus.dim() == 3:
        return _dev_ptr(ybus, torch.float64, (batch, plan.nnz_y, 2), "ybus"), ybus, 1
    return _dev_ptr(ybus, torch.float64, (plan.nnz_y, 2), "ybus"), ybus, 0


def _as_pairs(x, name):
    torch = _torch()
    if x.dtype == torch.complex128:
        x = torch.view_as_real(x)
    return x


def solve_batch(plan: Plan, ybus, sbus, v0, tol: float = 1e-8, max_iter: int = 10,
                precision: int = PF_FP64, tile: int = 0, waves: int = 0, workspace=None,
                stream=None, out: Optional[Result] = None, schedule: int = 0,
                v_fallback=None, long_slots: int = 0, pivot_fallback: bool = False, launch: int = 0,
                reorder: int = 0) -> Result:
    """Run pf_solve_batch on device tensors: ybus complex128 [nnz_y] (or [B][nnz_y]: one set of
    values per instance), sbus complex128 [B][n],
    v0 float64 [B][n][2].  With v_fallback (same shape as v0) pf_solve_batch_warm runs
    instead: instances that fail from v0 restart once from v_fallback inside the kernel.
    With pivot_fallback, pf_solve_fallback then re-solves every instance that reported
    PF_ST_PIVOT or PF_ST_NONFINITE with a threshold-pivoting factorization (synchronises the
    stream; out.n_resolved counts them).
    Returns device tensors (valid once the stream synchronises)."""
    torch = _torch()
    B = int(v0.shape[0])
    yp, _, yb_batched = _ybus_view(plan, ybus, B)
    s2 = _as_pairs(sbus, "sbus")
    sp = _dev_ptr(s2, torch.float64, (B, plan.n, 2), "sbus")
    vp = _dev_ptr(v0, torch.float64, (B, plan.n, 2), "v0")
    if out is None:
        out = Result(v=torch.empty((B, plan.n, 2), dtype=torch.float64, device=v0.device),
                     iters=torch.empty(B, dtype=torch.int32, device=v0.device),
                     converged=torch.empty(B, dtype=torch.uint8, device=v0.device),
                     status=torch.empty(B, dtype=torch.int8, device=v0.device))
    opts = _Opts(precision, tile, waves, schedule, long_slots, launch, reorder)
    workspace, wp, avail = _workspace(plan, B, opts, workspace)
    outs = (_vp(out.v.data_ptr()), _vp(out.iters.data_ptr()), _vp(out.converged.data_ptr()),
            _vp(out.status.data_ptr()), _stream_ptr(stream))
    if v_fallback is None:
        rc = lib().pf_solve_batch(plan._h, B, yp, yb_batched, sp, vp, float(tol), int(max_iter),
                                  ctypes.byref(opts), wp, avail, *outs)
        _check(rc, "pf_solve_batch")
    else:
        fp = _dev_ptr(v_fallback, torch.float64, (B, plan.n, 2), "v_fallback")
        rc = lib().pf_solve_batch_warm(plan._h, B, yp, yb_batched, sp, vp, fp, float(tol), int(max_iter),
                                       ctypes.byref(opts), wp, avail, *outs)
        _check(rc, "pf_solve_batch_warm")
    out._workspace = workspace
    if pivot_fallback:
        nr = ctypes.c_int32(0)
        rc = lib().pf_solve_fallback(plan._h, B, yp, yb_batched, sp, vp, float(tol), int(max_iter), 0,
                                     _vp(out.v.data_ptr()), _vp(out.iters.data_ptr()),
                                     _vp(out.converged.data_ptr()), _vp(out.status.data_ptr()),
                                     ctypes.byref(nr), _stream_ptr(stream))
        _check(rc, "pf_solve_fallback")
        out.n_resolved = int(nr.value)
    return out


def solve_batch_noalloc(plan: Plan, ybus, sbus, v0, out: Result, tol: float = 1e-8, max_iter: int = 10,
                        precision: int = PF_FP64, tile: int = 0, waves: int = 0, schedule: int = 0,
                        long_slots: int = 0, stream=None) -> Result:
    """pf_solve_batch_noalloc: pf_solve_batch into the caller's `out` tensors, with the
    library's fixed device scratch as workspace (no allocation by the library or here)."""
    torch = _torch()
    B = int(v0.shape[0])
    yp, _, yb_batched = _ybus_view(plan, ybus, B)
    s2 = _as_pairs(sbus, "sbus")
    sp = _dev_ptr(s2, torch.float64, (B, plan.n, 2), "sbus")
    vp = _dev_ptr(v0, torch.float64, (B, plan.n, 2), "v0")
    outs = (_dev_ptr(out.v, torch.float64, (B, plan.n, 2), "v_out"), _dev_ptr(out.iters, torch.int32, (B,), "iters"),
            _dev_ptr(out.converged, torch.uint8, (B,), "converged"), _dev_ptr(out.status, torch.int8, (B,), "status"))
    opts = _Opts(precision, tile, waves, schedule, long_slots)
    rc = lib().pf_solve_batch_noalloc(plan._h, B, yp, yb_batched, sp, vp, float(tol), int(max_iter),
                                      ctypes.byref(opts), *outs, _stream_ptr(stream))
    _check(rc, "pf_solve_batch_noalloc")
    return out


def _eval(fn, plan: Plan, ybus, sbus, v, out_shape, precision, tile, waves, extra_out=None,
          workspace=None, stream=None):
    torch = _torch()
    B = int(v.shape[0])
    yp, _, _ = _ybus_view(plan, ybus)
    s2 = _as_pairs(sbus, "sbus")
    sp = _dev_ptr(s2, torch.float64, (B, plan.n, 2), "sbus")
    vp = _dev_ptr(v, torch.float64, (B, plan.n, 2), "v")
    opts = _Opts(precision, tile, waves)
    workspace, wp, avail = _workspace(plan, B, opts, workspace)
    out = torch.empty(out_shape, dtype=torch.float64, device=v.device)
    args = [plan._h, B, yp, sp, vp, ctypes.byref(opts), wp, avail, _vp(out.data_ptr())]
    if extra_out is not None:
        args.append(_vp(extra_out.data_ptr()))
    args.append(_stream_ptr(stream))
    _check(fn(*args), fn.__name__)
    return out


def eval_mismatch(plan: Plan, ybus, sbus, v, precision=PF_FP64, tile=0, waves=0, **kw):
    """(F [B][N] in unknown order, max|F| [B]) at V."""
    torch = _torch()
    B = int(v.shape[0])
    normf = torch.empty(B, dtype=torch.float64, device=v.device)
    F = _eval(lib().pf_eval_mismatch, plan, ybus, sbus, v, (B, plan.N), precision, tile, waves,
              extra_out=normf, **kw)
    return F, normf


def eval_factor(plan: Plan, ybus, sbus, v, precision=PF_FP64, tile=0, waves=0, **kw):
    """Values of L+U-I [B][nnz_lu] of A = P J(V) P^T in lu_pattern() order."""
    B = int(v.shape[0])
    return _eval(lib().pf_eval_factor, plan, ybus, sbus, v, (B, plan.nnz_lu), precision, tile,
                 waves, **kw)


def eval_step(plan: Plan, ybus, sbus, v, precision=PF_FP64, tile=0, waves=0, **kw):
    """Newton step dx [B][N] (unknown order) solving J(V) dx = F(V)."""
    B = int(v.shape[0])
    return _eval(lib().pf_eval_step, plan, ybus, sbus, v, (B, plan.N), precision, tile, waves, **kw)


def tune(plan: Plan, ybus, sbus, v0, tol: float = 1e-8, max_iter: int = 10,
         precision: int = PF_FP64, waves: int = 0, reps: int = 2, force: bool = False,
         stream=None):
    """pf_tune on device tensors shaped as for solve_batch.  Returns
    ({"precision", "tile", "waves", "schedule", "long_slots"}, mean ms per solve)."""
    torch = _torch()
    B = int(v0.shape[0])
    yp, _, _ = _ybus_view(plan, ybus)
    sp = _dev_ptr(_as_pairs(sbus, "sbus"), torch.float64, (B, plan.n, 2), "sbus")
    vp = _dev_ptr(v0, torch.float64, (B, plan.n, 2), "v0")
    best = _Opts()
    ms = ctypes.c_double(0.0)
    rc = lib().pf_tune(plan._h, B, yp, sp, vp, float(tol), int(max_iter), int(precision), int(waves),
                       int(reps), 1 if force else 0, ctypes.byref(best), ctypes.byref(ms),
                       _stream_ptr(stream))
    _check(rc, "pf_tune")
    return ({"precision": best.precision, "tile": best.tile, "waves": best.waves,
             "schedule": best.schedule, "long_slots": best.long_slots}, ms.value)


def tune_cache_save(path: str) -> None:
    """pf_tune_cache_save: write the tuner's cache to a text file."""
    _check(lib().pf_tune_cache_save(os.fsencode(path)), "pf_tune_cache_save")


def tune_cache_load(path: str) -> None:
    """pf_tune_cache_load: add a saved cache's entries to the tuner's cache."""
    _check(lib().pf_tune_cache_load(os.fsencode(path)), "pf_tune_cache_load")


def tune_cache_clear() -> None:
    _check(lib().pf_tune_cache_clear(), "pf_tune_cache_clear")


def tune_cache_size() -> int:
    return int(lib().pf_tune_cache_size())


class Queue:
    """pf_queue_*: several plans' batches solved by one replayable graph of persistent
    kernels.  Every tensor handed to add() is kept referenced here, because the graph
    holds its address."""

    def __init__(self):
        h = _vp()
        _check(lib().pf_queue_create(ctypes.byref(h)), "pf_queue_create")
        self._h = h
        self._keep = []
        self.results = []

    def add(self, plan: Plan, ybus, sbus, v0, tol: float = 1e-8, max_iter: int = 10,
            precision: int = PF_FP64, tile: int = 0, waves: int = 0, schedule: int = 0,
            ticks: bool = True, long_slots: int = 0) -> Result:
        torch = _torch()
        B = int(v0.shape[0])
        yp, yv, _ = _ybus_view(plan, ybus)
        s2 = _as_pairs(sbus, "sbus")
        sp = _dev_ptr(s2, torch.float64, (B, plan.n, 2), "sbus")
        vp = _dev_ptr(v0, torch.float64, (B, plan.n, 2), "v0")
        dev = v0.device
        out = Result(v=torch.empty((B, plan.n, 2), dtype=torch.float64, device=dev),
                     iters=torch.empty(B, dtype=torch.int32, device=dev),
                     converged=torch.empty(B, dtype=torch.uint8, device=dev),
                     status=torch.empty(B, dtype=torch.int8, device=dev))
        out.ticks = torch.zeros(B, dtype=torch.int64, device=dev) if ticks else None
        opts = _Opts(precision, tile, waves, schedule, long_slots)
        rc = lib().pf_queue_add(self._h, plan._h, B, yp, sp, vp, float(tol), int(max_iter),
                                ctypes.byref(opts), _vp(out.v.data_ptr()), _vp(out.iters.data_ptr()),
                                _vp(out.converged.data_ptr()), _vp(out.status.data_ptr()),
                                _vp(out.ticks.data_ptr()) if ticks else None)
        _check(rc, "pf_queue_add")
        self._keep.append((plan, yv, s2, v0, out))
        self.results.append(out)
        return out

    def run(self, stream=None):
        _check(lib().pf_queue_run(self._h, _stream_ptr(stream)), "pf_queue_run")

    def info(self) -> dict:
        q = _QueueInfo()
        _check(lib().pf_queue_info(self._h, ctypes.byref(q)), "pf_queue_info")
        d = {f: getattr(q, f) for f, _ in _QueueInfo._fields_}
        d["grid"] = list(q.grid)[: q.n_groups]
        return d

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.pf_queue_destroy(self._h)
        self._h = None
        self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def branch_flows(from_bus, to_bus, r, x, b_total, n_bus: int, v, losses: bool = True, stream=None):
    """pf_branch_flows on device tensors: from_bus/to_bus int32 [m], r/x/b_total float64 [m],
    v float64 [B][n_bus][2].  Returns (s_from, s_to, loss) complex128 tensors ([B][m],
    [B][m], [B] or None)."""
    torch = _torch()
    m = int(from_bus.shape[0])
    B = int(v.shape[0])
    dev = v.device
    sf = torch.empty((B, m, 2), dtype=torch.float64, device=dev)
    st = torch.empty((B, m, 2), dtype=torch.float64, device=dev)
    loss = torch.empty((B, 2), dtype=torch.float64, device=dev) if losses else None
    rc = lib().pf_branch_flows(int(n_bus), m, _dev_ptr(from_bus, torch.int32, (m,), "from_bus"),
                               _dev_ptr(to_bus, torch.int32, (m,), "to_bus"), _dev_ptr(r, torch.float64, (m,), "r"),
                               _dev_ptr(x, torch.float64, (m,), "x"), _dev_ptr(b_total, torch.float64, (m,), "b_total"),
                               B, _dev_ptr(v, torch.float64, (B, n_bus, 2), "v"), _vp(sf.data_ptr()),
                               _vp(st.data_ptr()), _vp(loss.data_ptr()) if losses else None, _stream_ptr(stream))
    _check(rc, "pf_branch_flows")
    return (torch.view_as_complex(sf), torch.view_as_complex(st),
            torch.view_as_complex(loss) if losses else None)


def solve_host(plan: Plan, ybus, sbus, v0, tol: float = 1e-8, max_iter: int = 10, precision: int = PF_FP64,
               tile: int = 0, waves: int = 0, chunk: int = 2048, stream=None):
    """pf_solve_host: ybus a device tensor as in solve_batch; sbus complex128 [B][n] and v0
    float64 [B][n][2] host tensors (pinned for overlap).  Returns a Result of pinned host
    tensors."""
    torch = _torch()
    B = int(v0.shape[0])
    yp, _, _ = _ybus_view(plan, ybus)
    s2 = _as_pairs(sbus, "sbus")
    for t_, nm in ((s2, "sbus"), (v0, "v0")):
        if t_.is_cuda or t_.dtype != torch.float64 or not t_.is_contiguous() or tuple(t_.shape) != (B, plan.n, 2):
            raise PfError(f"{nm} must be a contiguous float64 host tensor of shape {(B, plan.n, 2)}")
    out = Result(v=torch.empty((B, plan.n, 2), dtype=torch.float64, pin_memory=True),
                 iters=torch.empty(B, dtype=torch.int32, pin_memory=True),
                 converged=torch.empty(B, dtype=torch.uint8, pin_memory=True),
                 status=torch.empty(B, dtype=torch.int8, pin_memory=True))
    rc = lib().pf_solve_host(plan._h, B, yp, _vp(s2.data_ptr()), _vp(v0.data_ptr()), float(tol), int(max_iter),
                             ctypes.byref(_Opts(precision, tile, waves, 0)), int(chunk), _vp(out.v.data_ptr()),
                             _vp(out.iters.data_ptr()), _vp(out.converged.data_ptr()), _vp(out.status.data_ptr()),
                             _stream_ptr(stream))
    _check(rc, "pf_solve_host")
    return out


@dataclass
class HostResult:
    v: np.ndarray          # float64 [B][n][2]
    iters: np.ndarray      # int32 [B]
    converged: np.ndarray  # bool [B]
    status: np.ndarray     # int8 [B]


def cpu_solve_pivoting(plan: Plan, ybus, sbus, v0, tol: float = 1e-8, max_iter: int = 10,
                       threads: int = 0) -> HostResult:
    """pf_cpu_solve_pivoting on host arrays: ybus complex128 [nnz_y] or [B][nnz_y], sbus
    complex128 [B][n], v0 float64 [B][n][2].  Newton-Raphson with a fresh threshold-pivoting
    sparse LU every iteration (the factorization pf_solve_fallback gives flagged instances)."""
    y = np.ascontiguousarray(np.asarray(ybus, dtype=np.complex128)).view(np.float64)
    s = np.ascontiguousarray(np.asarray(sbus, dtype=np.complex128)).view(np.float64)
    v = np.ascontiguousarray(v0, dtype=np.float64)
    B = int(v.shape[0])
    batched = 1 if y.ndim == 2 else 0
    if y.shape[-1] != 2 * plan.nnz_y or (batched and y.shape[0] != B) or s.shape != (B, 2 * plan.n) \
            or v.shape != (B, plan.n, 2):
        raise PfError("ybus, sbus or v0 has the wrong shape for this plan")
    out = HostResult(v=np.empty((B, plan.n, 2)), iters=np.empty(B, np.int32),
                     converged=np.empty(B, np.uint8), status=np.empty(B, np.int8))
    rc = lib().pf_cpu_solve_pivoting(plan._h, B, _vp(y.ctypes.data), batched, _vp(s.ctypes.data),
                                     _vp(v.ctypes.data), float(tol), int(max_iter), int(threads),
                                     _vp(out.v.ctypes.data), _vp(out.iters.ctypes.data),
                                     _vp(out.converged.ctypes.data), _vp(out.status.ctypes.data))
    _check(rc, "pf_cpu_solve_pivoting")
    out.converged = out.converged.astype(bool)
    return out


def cpu_solve_batch(plan: Plan, ybus, sbus, v0, tol: float = 1e-8, max_iter: int = 10,
                    threads: int = 0) -> HostResult:
    """pf_cpu_solve_batch on host arrays: ybus complex128 [nnz_y], sbus complex128 [B][n],
    v0 float64 [B][n][2].  The batched CPU engine (mini-batches of 8 in SIMD lanes, worker
    threads over mini-batches; threads = 0 uses every online core).  It is a separate
    engine, not a fallback of the GPU entry points."""
    y = np.ascontiguousarray(np.asarray(ybus, dtype=np.complex128)).view(np.float64)
    s = np.ascontiguousarray(np.asarray(sbus, dtype=np.complex128)).view(np.float64)
    v = np.ascontiguousarray(v0, dtype=np.float64)
    B = int(v.shape[0])
    if y.shape[0] != 2 * plan.nnz_y or s.shape != (B, 2 * plan.n) or v.shape != (B, plan.n, 2):
        raise PfError("ybus, sbus or v0 has the wrong shape for this plan")
    out = HostResult(v=np.empty((B, plan.n, 2)), iters=np.empty(B, np.int32),
                     converged=np.empty(B, np.uint8), status=np.empty(B, np.int8))
    rc = lib().pf_cpu_solve_batch(plan._h, B, _vp(y.ctypes.data), _vp(s.ctypes.data), _vp(v.ctypes.data),
                                  float(tol), int(max_iter), int(threads), _vp(out.v.ctypes.data),
                                  _vp(out.iters.ctypes.data), _vp(out.converged.ctypes.data),
                                  _vp(out.status.ctypes.data))
    _check(rc, "pf_cpu_solve_batch")
    out.converged = out.converged.astype(bool)
    return out
