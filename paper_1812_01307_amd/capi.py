"""ctypes binding of libbsgd.so (the C ABI declared in include/bsgd.h).

Argument marshalling only: torch tensors are passed as device pointers, the
current torch stream as the HIP stream.  Every function here has the name
of the C entry point it calls.  The library must have been built
(``python paper_1812_01307_amd/build.py`` or ``__graft_entry__.build()``);
importing this module without it raises ImportError.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbsgd.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is not built; run __graft_entry__.build() first")
_lib = ctypes.CDLL(_LIB_PATH)

BSGD_OK = 0
BSGD_ERR_INVALID = -1
BSGD_ERR_WORKSPACE = -2
BSGD_ERR_HIP = -3
BSGD_ERR_UNSUPPORTED = -4
BSGD_ERR_DIVERGED = -5
BSGD_VAL_F32 = 0
BSGD_VAL_F16 = 1
BSGD_PLAN_F16 = 1
BSGD_PLAN_AUTOTUNE = 2
BSGD_PLAN_STAGED_FWD = 4
BSGD_PLAN_STAGED_BWD = 8
BSGD_PLAN_STAGED = 12
BSGD_PLAN_FWD_ONLY = 16
BSGD_PLAN_SINGLE_PASS_ONLY = 32
BSGD_LAUNCH_NT = 128
BSGD_STATE_VOLUME = 1
BSGD_STATE_BLOCK_SELECT = 2
BSGD_METHOD_BSGD = 0
BSGD_METHOD_ISTA = 1
BSGD_FUSED_WIDE = 1

_STATUS = {0: "OK", -1: "INVALID", -2: "WORKSPACE", -3: "HIP", -4: "UNSUPPORTED", -5: "DIVERGED"}


class BsgdError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn}: {_STATUS.get(status, status)}: {msg}")
        self.status = status


class bsgd_csr(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int
_f32 = ctypes.c_float
_sz = ctypes.c_size_t
_PROTOS = {
    "bsgd_plan_workspace_size": [_i64, _i64, _i64, _i32, _i32, _i32, _i32, _i32, _i64,
                                 ctypes.c_uint, ctypes.POINTER(_sz)],
    "bsgd_plan_create": [ctypes.POINTER(bsgd_csr), ctypes.POINTER(bsgd_csr), _i32, _i32,
                         ctypes.POINTER(_i64), ctypes.POINTER(_i64), _i32, _i32, _i32, _i64,
                         ctypes.c_uint, _vp, _sz, _vp, ctypes.POINTER(_vp)],
    "bsgd_plan_lanes": [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)],
    "bsgd_plan_set_lanes": [_vp, _i32, _i32],
    "bsgd_plan_staged": [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)],
    "bsgd_plan_set_staged": [_vp, _i32, _i32],
    "bsgd_plan_staged_shape": [_vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                               ctypes.POINTER(_i64)],
    "bsgd_tile_nnz": [_vp, _i32, _i32, _vp, ctypes.POINTER(_i64)],
    "bsgd_tile_export": [_vp, _i32, _i32, _i32, _vp, _vp, _vp, _vp],
    "bsgd_forward": [_vp, _i32, _vp, _vp, _vp, _vp],
    "bsgd_backproject": [_vp, _i32, _vp, _vp, _f32, _vp, _vp],
    "bsgd_forward_block": [_vp, _i32, _i32, _i32, _vp, _vp, _vp],
    "bsgd_backproject_block": [_vp, _i32, _i32, _i32, _vp, _vp, _vp],
    "bsgd_tv_workspace_size": [_i32, _i32, _i32, ctypes.POINTER(_sz)],
    "bsgd_tv_prox": [_i32, _i32, _i32, _vp, _f32, _i32, _vp, _vp, _sz, _vp],
    "bsgd_tv_prox_noalloc": [_i32, _i32, _i32, _vp, _f32, _i32, _vp, _vp],
    "bsgd_tv_value": [_i32, _i32, _i32, _vp, _vp, _sz, _vp, ctypes.POINTER(ctypes.c_double)],
    "bsgd_power_workspace_size": [_vp, ctypes.POINTER(_sz)],
    "bsgd_power_umax": [_vp, _i32, _i32, _vp, _sz, _vp, ctypes.POINTER(_f32)],
    "bsgd_lanczos_workspace_size": [_vp, _i32, ctypes.POINTER(_sz)],
    "bsgd_lanczos_umax": [_vp, _i32, _i32, _vp, _sz, _vp, ctypes.POINTER(_f32)],
    "bsgd_lanczos_workspace_size_fused": [_vp, _i32, ctypes.POINTER(_sz)],
    "bsgd_lanczos_umax_fused": [_vp, _i32, _i32, _vp, _sz, _vp, ctypes.POINTER(_f32)],
    "bsgd_state_workspace_size": [_vp, _i32, ctypes.c_uint, ctypes.POINTER(_sz)],
    "bsgd_state_create": [_vp, _i32, _i32, ctypes.c_uint, _vp, _sz, ctypes.POINTER(_vp)],
    "bsgd_state_set_rhs": [_vp, _i32, _vp, _vp, _vp],
    "bsgd_state_set_lambda": [_vp, ctypes.POINTER(_f32), _vp],
    "bsgd_get_x_rhs": [_vp, _i32, _vp, _vp],
    "bsgd_get_stats_rhs": [_vp, _vp, ctypes.POINTER(ctypes.c_double)],
    "bsgd_get_res_change_rhs": [_vp, _vp, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double)],
    "bsgd_graph_create": [_vp, _f32, _f32, _i32, _i32, _vp, ctypes.POINTER(_vp)],
    "bsgd_graph_launch": [_vp, _vp],
    "bsgd_state_init": [_vp, _vp, _vp, _vp],
    "bsgd_state_load": [_vp, _vp, _vp, _i64, _vp],
    "bsgd_run_epochs": [_vp, _f32, _f32, _i32, _i32, _vp],
    "bsgd_get_x": [_vp, _vp, _vp],
    "bsgd_get_r": [_vp, _vp, _vp],
    "bsgd_get_stats": [_vp, _vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)],
    "bsgd_state_enable_timing": [_vp, _i32],
    "bsgd_state_enable_timing_sampled": [_vp, _i32, _i32],
    "bsgd_state_set_overlap": [_vp, _i32],
    "bsgd_state_set_prox_schedule": [_vp, _i32],
    "bsgd_state_set_launch": [_vp, _i32, _i32],
    "bsgd_state_launch": [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)],
    "bsgd_state_autotune": [_vp, _f32, _f32, _i32, _i32, _vp, ctypes.POINTER(_i32)],
    "bsgd_state_timing": [_vp] + [ctypes.POINTER(ctypes.c_double)] * 3 + [ctypes.POINTER(_i64)],
    "bsgd_fused_workspace_size": [_vp, _i32, ctypes.c_uint, _vp, ctypes.POINTER(_sz)],
    "bsgd_fused_create": [_vp, _i32, ctypes.c_uint, _vp, _sz, _vp, ctypes.POINTER(_vp)],
    "bsgd_fused_shape": [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i64),
                         ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i32)],
    "bsgd_fused_set_waves": [_vp, _i32],
    "bsgd_fused_partials_size": [_vp, ctypes.POINTER(_sz)],
    "bsgd_fused_partials_size_rhs": [_vp, _i32, ctypes.POINTER(_sz)],
    "bsgd_fused_apply": [_vp, _i32, _vp, _vp, _vp, _vp, _f32, _vp, _vp, _vp, _sz, _vp],
    "bsgd_state_attach_fused": [_vp, _vp, _vp, _sz],
    "bsgd_state_set_method": [_vp, _i32],
    "bsgd_run_selected": [_vp, _f32, _f32, _i32, _i32, ctypes.POINTER(ctypes.c_uint64),
                          ctypes.POINTER(ctypes.c_uint64), _vp],
}
for _name, _args in _PROTOS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.bsgd_plan_destroy.argtypes = [_vp]
_lib.bsgd_plan_destroy.restype = None
_lib.bsgd_state_destroy.argtypes = [_vp]
_lib.bsgd_state_destroy.restype = None
_lib.bsgd_graph_destroy.argtypes = [_vp]
_lib.bsgd_graph_destroy.restype = None
_lib.bsgd_fused_destroy.argtypes = [_vp]
_lib.bsgd_fused_destroy.restype = None
_lib.bsgd_last_error.argtypes = []
_lib.bsgd_last_error.restype = ctypes.c_char_p

EXPORTED = sorted(list(_PROTOS) + ["bsgd_plan_destroy", "bsgd_state_destroy", "bsgd_graph_destroy",
                                   "bsgd_fused_destroy", "bsgd_last_error"])


def library_path() -> str:
    return _LIB_PATH


def _check(fn: str, status: int, allow=()):
    if status != BSGD_OK and status not in allow:
        raise BsgdError(fn, status, _lib.bsgd_last_error().decode())
    return status


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ws(nbytes: int, device) -> torch.Tensor:
    # torch's caching allocator returns 512-byte aligned blocks
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _chk(t, n=None, name="tensor"):
    if t.dtype != torch.float32:
        raise ValueError(f"{name} must be float32")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return t


# --------------------------------------------------------------------------
# Plan
# --------------------------------------------------------------------------

class Plan:
    """Block store of A and A^T in a torch-owned device workspace."""

    def __init__(self, handle, workspace, M, N, row_off, col_off, H, W, D, nrows, ncols, flags):
        self.handle = handle
        self.workspace = workspace
        self.M, self.N = M, N
        self.row_off, self.col_off = list(row_off), list(col_off)
        self.H, self.W, self.D = H, W, D
        self.nrows, self.ncols = nrows, ncols
        self.flags = flags
        self.source = None  # A's device arrays, kept alive by BSGD_PLAN_SINGLE_PASS_ONLY plans

    # the destroy function is bound at class creation: at interpreter exit the
    # module's globals may already be gone when the last objects are collected
    def __del__(self, _destroy=_lib.bsgd_plan_destroy):
        h = getattr(self, "handle", None)
        if h:
            self.handle = None
            _destroy(h)


def bsgd_plan_workspace_size(nrows, ncols, nnz, M, N, H, W, D=1, view_len=0, flags=0) -> int:
    out = _sz()
    _check("bsgd_plan_workspace_size",
           _lib.bsgd_plan_workspace_size(nrows, ncols, nnz, M, N, H, W, D, view_len, flags,
                                         ctypes.byref(out)))
    return out.value


def bsgd_plan_create(A, At, M, N, row_off, col_off, H, W, D=1, view_len=0, flags=0,
                     stream=None) -> Plan:
    """A, At: (row_ptr int64, col int32, val float32) device tensor triples plus shapes.

    A = (nrows, ncols, row_ptr, col, val); At likewise for the transpose.  With
    BSGD_PLAN_FWD_ONLY the transpose's column array may be None (only its row
    pointers and values are read).  A BSGD_PLAN_SINGLE_PASS_ONLY plan reads A's
    arrays again when its tile-sliced store is built: the Plan holds them.
    """
    nrows, ncols, rp, cl, vl = A
    tn, tc, trp, tcl, tvl = At
    for t, dt in ((rp, torch.int64), (cl, torch.int32), (vl, torch.float32),
                  (trp, torch.int64), (tcl, torch.int32), (tvl, torch.float32)):
        if t is not None and t.dtype != dt:
            raise ValueError(f"CSR array has dtype {t.dtype}, expected {dt}")
    a = bsgd_csr(nrows, ncols, cl.numel(), _ptr(rp), _ptr(cl), _ptr(vl))
    at = bsgd_csr(tn, tc, tvl.numel(), _ptr(trp), _ptr(tcl) if tcl is not None else None,
                  _ptr(tvl))
    nbytes = bsgd_plan_workspace_size(nrows, ncols, cl.numel(), M, N, H, W, D, view_len, flags)
    ws = _ws(nbytes, rp.device)
    ro = (_i64 * (M + 1))(*[int(v) for v in row_off])
    co = (_i64 * (N + 1))(*[int(v) for v in col_off])
    h = _vp()
    _check("bsgd_plan_create", _lib.bsgd_plan_create(
        ctypes.byref(a), ctypes.byref(at), M, N, ro, co, H, W, D, view_len, flags, _ptr(ws),
        nbytes, _stream(stream), ctypes.byref(h)))
    plan = Plan(h, ws, M, N, row_off, col_off, H, W, D, nrows, ncols, flags)
    if flags & BSGD_PLAN_SINGLE_PASS_ONLY:
        plan.source = (rp, cl, vl)
    return plan


def bsgd_plan_lanes(plan: Plan):
    f, b = _i32(), _i32()
    _check("bsgd_plan_lanes", _lib.bsgd_plan_lanes(plan.handle, ctypes.byref(f), ctypes.byref(b)))
    return f.value, b.value


def bsgd_plan_staged(plan: Plan):
    """Lanes per row of the staged kernels (fwd, bwd): 0 = row kernels, -1 = not built."""
    f, b = _i32(), _i32()
    _check("bsgd_plan_staged", _lib.bsgd_plan_staged(plan.handle, ctypes.byref(f), ctypes.byref(b)))
    return f.value, b.value


def bsgd_plan_staged_shape(plan: Plan, transposed: int):
    """(stages, stage width, stored entries) of one direction's staged store."""
    p_, w_, e_ = _i32(), _i32(), _i64()
    _check("bsgd_plan_staged_shape", _lib.bsgd_plan_staged_shape(
        plan.handle, int(transposed), ctypes.byref(p_), ctypes.byref(w_), ctypes.byref(e_)))
    return p_.value, w_.value, e_.value


def bsgd_plan_set_staged(plan: Plan, fwd_lanes: int, bwd_lanes: int):
    _check("bsgd_plan_set_staged", _lib.bsgd_plan_set_staged(plan.handle, int(fwd_lanes),
                                                             int(bwd_lanes)))


def bsgd_plan_set_lanes(plan: Plan, fwd_lanes: int, bwd_lanes: int):
    _check("bsgd_plan_set_lanes", _lib.bsgd_plan_set_lanes(plan.handle, fwd_lanes, bwd_lanes))


def bsgd_tile_nnz(plan: Plan, i, j, stream=None) -> int:
    out = _i64()
    _check("bsgd_tile_nnz", _lib.bsgd_tile_nnz(plan.handle, i, j, _stream(stream), ctypes.byref(out)))
    return out.value


def bsgd_tile_export(plan: Plan, i, j, transposed=False, stream=None):
    """Block (i, j) (or its transpose) as block-local (ptr, col, val) device tensors."""
    nnz = bsgd_tile_nnz(plan, i, j, stream)
    dev = plan.workspace.device
    rows = (plan.row_off[i + 1] - plan.row_off[i]) if not transposed else \
        (plan.col_off[j + 1] - plan.col_off[j])
    ptr = torch.empty(rows + 1, dtype=torch.int64, device=dev)
    col = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
    val = torch.empty(max(nnz, 1), dtype=torch.float32, device=dev)
    _check("bsgd_tile_export", _lib.bsgd_tile_export(plan.handle, i, j, int(bool(transposed)),
                                                     _ptr(ptr), _ptr(col), _ptr(val), _stream(stream)))
    return ptr, col[:nnz], val[:nnz]


# --------------------------------------------------------------------------
# Products
# --------------------------------------------------------------------------

def bsgd_forward(plan: Plan, x, y=None, out=None, vt=BSGD_VAL_F32, stream=None):
    _chk(x, plan.ncols, "x")
    if y is not None:
        _chk(y, plan.nrows, "y")
    if out is None:
        out = torch.empty(plan.nrows, dtype=torch.float32, device=x.device)
    _chk(out, plan.nrows, "out")
    _check("bsgd_forward", _lib.bsgd_forward(plan.handle, vt, _ptr(x), _ptr(y), _ptr(out),
                                             _stream(stream)))
    return out


def bsgd_backproject(plan: Plan, r, x=None, mu=0.0, out=None, vt=BSGD_VAL_F32, stream=None):
    _chk(r, plan.nrows, "r")
    if x is not None:
        _chk(x, plan.ncols, "x")
    if out is None:
        out = torch.empty(plan.ncols, dtype=torch.float32, device=r.device)
    _chk(out, plan.ncols, "out")
    _check("bsgd_backproject", _lib.bsgd_backproject(plan.handle, vt, _ptr(r), _ptr(x), float(mu),
                                                     _ptr(out), _stream(stream)))
    return out


def bsgd_forward_block(plan: Plan, i, j, xj, out=None, vt=BSGD_VAL_F32, stream=None):
    _chk(xj, plan.col_off[j + 1] - plan.col_off[j], "xj")
    n = plan.row_off[i + 1] - plan.row_off[i]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=xj.device)
    _chk(out, n, "z")
    _check("bsgd_forward_block", _lib.bsgd_forward_block(plan.handle, vt, i, j, _ptr(xj), _ptr(out),
                                                         _stream(stream)))
    return out


def bsgd_backproject_block(plan: Plan, i, j, ri, out=None, vt=BSGD_VAL_F32, stream=None):
    _chk(ri, plan.row_off[i + 1] - plan.row_off[i], "ri")
    n = plan.col_off[j + 1] - plan.col_off[j]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=ri.device)
    _chk(out, n, "g")
    _check("bsgd_backproject_block", _lib.bsgd_backproject_block(
        plan.handle, vt, i, j, _ptr(ri), _ptr(out), _stream(stream)))
    return out


# --------------------------------------------------------------------------
# TV
# --------------------------------------------------------------------------

def bsgd_tv_workspace_size(H, W, D=1) -> int:
    out = _sz()
    _check("bsgd_tv_workspace_size", _lib.bsgd_tv_workspace_size(H, W, D, ctypes.byref(out)))
    return out.value


def bsgd_tv_prox(b, theta, iters, out=None, ws=None, stream=None):
    """b: (H, W) or (D, H, W) float32 device tensor."""
    shape = tuple(b.shape)
    D, H, W = (1,) + shape if len(shape) == 2 else shape
    _chk(b)
    if out is None:
        out = torch.empty_like(b)
    nbytes = bsgd_tv_workspace_size(H, W, D)
    if ws is None:
        ws = _ws(nbytes, b.device)
    _check("bsgd_tv_prox", _lib.bsgd_tv_prox(H, W, D, _ptr(b), float(theta), int(iters), _ptr(out),
                                             _ptr(ws), ws.numel(), _stream(stream)))
    return out


def bsgd_tv_prox_noalloc(b, theta, iters, out, stream=None):
    """bsgd_tv_prox on the library's own scratch array: `out` is caller-provided
    (same shape as b), nothing is allocated."""
    shape = tuple(b.shape)
    D, H, W = (1,) + shape if len(shape) == 2 else shape
    _chk(b)
    _chk(out, b.numel(), "out")
    _check("bsgd_tv_prox_noalloc", _lib.bsgd_tv_prox_noalloc(
        H, W, D, _ptr(b), float(theta), int(iters), _ptr(out), _stream(stream)))
    return out


def bsgd_tv_value(x, ws=None, stream=None) -> float:
    shape = tuple(x.shape)
    D, H, W = (1,) + shape if len(shape) == 2 else shape
    _chk(x)
    nbytes = bsgd_tv_workspace_size(H, W, D)
    if ws is None:
        ws = _ws(nbytes, x.device)
    out = ctypes.c_double()
    _check("bsgd_tv_value", _lib.bsgd_tv_value(H, W, D, _ptr(x), _ptr(ws), ws.numel(),
                                               _stream(stream), ctypes.byref(out)))
    return out.value


# --------------------------------------------------------------------------
# Step size
# --------------------------------------------------------------------------

def bsgd_power_workspace_size(plan: Plan) -> int:
    out = _sz()
    _check("bsgd_power_workspace_size", _lib.bsgd_power_workspace_size(plan.handle, ctypes.byref(out)))
    return out.value


def bsgd_power_umax(plan: Plan, iters, vt=BSGD_VAL_F32, ws=None, stream=None) -> float:
    nbytes = bsgd_power_workspace_size(plan)
    if ws is None:
        ws = _ws(nbytes, plan.workspace.device)
    out = ctypes.c_float()
    _check("bsgd_power_umax", _lib.bsgd_power_umax(plan.handle, vt, int(iters), _ptr(ws), ws.numel(),
                                                   _stream(stream), ctypes.byref(out)))
    return float(out.value)


def bsgd_lanczos_workspace_size(plan: Plan, steps: int) -> int:
    out = _sz()
    _check("bsgd_lanczos_workspace_size", _lib.bsgd_lanczos_workspace_size(plan.handle, int(steps),
                                                                           ctypes.byref(out)))
    return out.value


def bsgd_lanczos_umax(plan: Plan, steps, vt=BSGD_VAL_F32, ws=None, stream=None) -> float:
    nbytes = bsgd_lanczos_workspace_size(plan, steps)
    if ws is None:
        ws = _ws(nbytes, plan.workspace.device)
    out = ctypes.c_float()
    _check("bsgd_lanczos_umax", _lib.bsgd_lanczos_umax(plan.handle, vt, int(steps), _ptr(ws),
                                                       ws.numel(), _stream(stream),
                                                       ctypes.byref(out)))
    return float(out.value)


# --------------------------------------------------------------------------
# Epochs
# --------------------------------------------------------------------------

class State:
    def __init__(self, handle, workspace, plan, nrhs=1, flags=0):
        self.handle = handle
        self.workspace = workspace
        self.plan = plan
        self.nrhs = nrhs
        self.flags = flags

    # the destroy function is bound at class creation: at interpreter exit the
    # module's globals may already be gone when the last objects are collected
    def __del__(self, _destroy=_lib.bsgd_state_destroy):
        h = getattr(self, "handle", None)
        if h:
            self.handle = None
            _destroy(h)


def bsgd_state_workspace_size(plan: Plan, nrhs=1, flags=0) -> int:
    out = _sz()
    _check("bsgd_state_workspace_size", _lib.bsgd_state_workspace_size(plan.handle, nrhs, flags,
                                                                       ctypes.byref(out)))
    return out.value


def bsgd_state_create(plan: Plan, nrhs=1, vt=BSGD_VAL_F32, flags=0) -> State:
    nbytes = bsgd_state_workspace_size(plan, nrhs, flags)
    ws = _ws(nbytes, plan.workspace.device)
    h = _vp()
    _check("bsgd_state_create", _lib.bsgd_state_create(plan.handle, nrhs, vt, flags, _ptr(ws),
                                                       nbytes, ctypes.byref(h)))
    return State(h, ws, plan, nrhs, flags)


def bsgd_state_init(state: State, y, x0=None, stream=None):
    """y: [r] or [r, nrhs]; x0: [c] or [c, nrhs] (row-major, RHS fastest)."""
    _chk(y, state.plan.nrows * state.nrhs, "y")
    if x0 is not None:
        _chk(x0, state.plan.ncols * state.nrhs, "x0")
    _check("bsgd_state_init", _lib.bsgd_state_init(state.handle, _ptr(y), _ptr(x0), _stream(stream)))


def bsgd_state_load(state: State, x, r, epoch, stream=None):
    _chk(x, state.plan.ncols * state.nrhs, "x")
    _chk(r, state.plan.nrows * state.nrhs, "r")
    _check("bsgd_state_load", _lib.bsgd_state_load(state.handle, _ptr(x), _ptr(r), int(epoch),
                                                   _stream(stream)))


def bsgd_run_epochs(state: State, mu, lam, epochs, prox_iters, stream=None):
    _check("bsgd_run_epochs", _lib.bsgd_run_epochs(state.handle, float(mu), float(lam), int(epochs),
                                                   int(prox_iters), _stream(stream)))


def bsgd_get_x(state: State, out=None, stream=None):
    n = state.plan.ncols * state.nrhs
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=state.workspace.device)
    _chk(out, n, "x")
    _check("bsgd_get_x", _lib.bsgd_get_x(state.handle, _ptr(out), _stream(stream)))
    return out


def bsgd_get_r(state: State, out=None, stream=None):
    n = state.plan.nrows * state.nrhs
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=state.workspace.device)
    _chk(out, n, "r")
    _check("bsgd_get_r", _lib.bsgd_get_r(state.handle, _ptr(out), _stream(stream)))
    return out


def bsgd_get_stats(state: State, stream=None, allow_diverged=False):
    """(||r||^2, epochs_done); raises on divergence unless allow_diverged."""
    rn = ctypes.c_double()
    ep = _i64()
    st = _lib.bsgd_get_stats(state.handle, _stream(stream), ctypes.byref(rn), ctypes.byref(ep))
    _check("bsgd_get_stats", st, allow=(BSGD_ERR_DIVERGED,) if allow_diverged else ())
    return rn.value, ep.value, st == BSGD_ERR_DIVERGED


def bsgd_last_error() -> str:
    return _lib.bsgd_last_error().decode()


def bsgd_state_enable_timing(state: State, max_epochs: int, stride: int = 1):
    """Time up to max_epochs epochs: one in every `stride` (1: every epoch)."""
    if stride == 1:
        _check("bsgd_state_enable_timing",
               _lib.bsgd_state_enable_timing(state.handle, int(max_epochs)))
    else:
        _check("bsgd_state_enable_timing_sampled",
               _lib.bsgd_state_enable_timing_sampled(state.handle, int(max_epochs), int(stride)))


def bsgd_state_timing(state: State):
    """(forward ms, backprojection ms, prox ms, epochs timed) summed over timed epochs."""
    f, b, x = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    n = _i64()
    _check("bsgd_state_timing", _lib.bsgd_state_timing(state.handle, ctypes.byref(f), ctypes.byref(b),
                                                       ctypes.byref(x), ctypes.byref(n)))
    return f.value, b.value, x.value, n.value


def bsgd_state_set_method(state: State, method: int):
    """BSGD_METHOD_BSGD (Algorithm 1, delayed residual) or BSGD_METHOD_ISTA (no delay)."""
    _check("bsgd_state_set_method", _lib.bsgd_state_set_method(state.handle, int(method)))


def bsgd_run_selected(state: State, mu, lam, rows_sel, cols_sel, prox_iters, stream=None):
    """Iterations over drawn block subsets: rows_sel[t], cols_sel[t] are bit masks."""
    rows = np.ascontiguousarray(np.asarray(rows_sel, dtype=np.uint64))
    cols = np.ascontiguousarray(np.asarray(cols_sel, dtype=np.uint64))
    if rows.shape != cols.shape or rows.ndim != 1:
        raise ValueError("rows_sel and cols_sel must be 1-D arrays of equal length")
    u64p = ctypes.POINTER(ctypes.c_uint64)
    _check("bsgd_run_selected", _lib.bsgd_run_selected(
        state.handle, float(mu), float(lam), int(rows.size), int(prox_iters),
        rows.ctypes.data_as(u64p), cols.ctypes.data_as(u64p), _stream(stream)))


def bsgd_state_set_overlap(state: State, mode: int):
    _check("bsgd_state_set_overlap", _lib.bsgd_state_set_overlap(state.handle, int(mode)))


def bsgd_state_set_rhs(state: State, k: int, y=None, x0=None, stream=None):
    if y is not None:
        _chk(y, state.plan.nrows, "y")
    if x0 is not None:
        _chk(x0, state.plan.ncols, "x0")
    _check("bsgd_state_set_rhs", _lib.bsgd_state_set_rhs(state.handle, int(k), _ptr(y), _ptr(x0),
                                                         _stream(stream)))


def bsgd_state_set_lambda(state: State, lam, stream=None):
    arr = (ctypes.c_float * state.nrhs)(*[float(v) for v in lam])
    _check("bsgd_state_set_lambda", _lib.bsgd_state_set_lambda(state.handle, arr, _stream(stream)))


def bsgd_get_x_rhs(state: State, k: int, out=None, stream=None):
    if out is None:
        out = torch.empty(state.plan.ncols, dtype=torch.float32, device=state.workspace.device)
    _chk(out, state.plan.ncols, "x")
    _check("bsgd_get_x_rhs", _lib.bsgd_get_x_rhs(state.handle, int(k), _ptr(out), _stream(stream)))
    return out


def bsgd_get_stats_rhs(state: State, stream=None, allow_diverged=False):
    """Per-RHS ||r_k||^2 (list of floats)."""
    arr = (ctypes.c_double * state.nrhs)()
    st = _lib.bsgd_get_stats_rhs(state.handle, _stream(stream), arr)
    _check("bsgd_get_stats_rhs", st, allow=(BSGD_ERR_DIVERGED,) if allow_diverged else ())
    return list(arr)


def bsgd_get_res_change_rhs(state: State, stream=None):
    """Per-RHS squared residual norms of the last two epochs: (now, prev) lists."""
    now = (ctypes.c_double * state.nrhs)()
    prev = (ctypes.c_double * state.nrhs)()
    _check("bsgd_get_res_change_rhs",
           _lib.bsgd_get_res_change_rhs(state.handle, _stream(stream), now, prev))
    return list(now), list(prev)


class Graph:
    def __init__(self, handle, state):
        self.handle = handle
        self.state = state
        # the captured kernels read the attached store and its partial sums
        self.fused = getattr(state, "fused", None)
        self.fused_partials = getattr(state, "fused_partials", None)

    # the destroy function is bound at class creation: at interpreter exit the
    # module's globals may already be gone when the last objects are collected
    def __del__(self, _destroy=_lib.bsgd_graph_destroy):
        h = getattr(self, "handle", None)
        if h:
            self.handle = None
            _destroy(h)


def bsgd_graph_create(state: State, mu, lam, epochs, prox_iters, stream=None) -> Graph:
    s = stream if stream is not None else torch.cuda.current_stream()
    if s.cuda_stream == 0:
        raise ValueError("graph capture needs a non-default stream")
    h = _vp()
    _check("bsgd_graph_create", _lib.bsgd_graph_create(state.handle, float(mu), float(lam),
                                                       int(epochs), int(prox_iters),
                                                       ctypes.c_void_p(s.cuda_stream),
                                                       ctypes.byref(h)))
    return Graph(h, state)


def bsgd_graph_launch(graph: Graph, stream=None):
    _check("bsgd_graph_launch", _lib.bsgd_graph_launch(graph.handle, _stream(stream)))


def bsgd_state_set_launch(state: State, pass_waves: int = 0, prox_split: int = 0):
    _check("bsgd_state_set_launch", _lib.bsgd_state_set_launch(state.handle, int(pass_waves),
                                                               int(prox_split)))


def bsgd_state_launch(state: State):
    """(pass wavefronts, prox split) of the state's epochs (0: defaults)."""
    w, sp = _i32(), _i32()
    _check("bsgd_state_launch", _lib.bsgd_state_launch(state.handle, ctypes.byref(w),
                                                       ctypes.byref(sp)))
    return w.value, sp.value


def bsgd_state_autotune(state: State, mu, lam, prox_iters, reps=3, stream=None):
    """Time the launch shapes on this (not yet initialised) state; returns the choice."""
    ch = (_i32 * 2)()
    _check("bsgd_state_autotune", _lib.bsgd_state_autotune(
        state.handle, float(mu), float(lam), int(prox_iters), int(reps), _stream(stream), ch))
    return ch[0], ch[1]


def bsgd_state_set_prox_schedule(state: State, schedule: int):
    _check("bsgd_state_set_prox_schedule", _lib.bsgd_state_set_prox_schedule(state.handle,
                                                                             int(schedule)))


# --------------------------------------------------------------------------
# Single-pass epochs (tile-sliced store)
# --------------------------------------------------------------------------

class Fused:
    """Tile-sliced store of a plan's matrix in a torch-owned device workspace."""

    def __init__(self, handle, workspace, plan):
        self.handle = handle
        self.workspace = workspace
        self.plan = plan  # keeps the plan alive

    # the destroy function is bound at class creation: at interpreter exit the
    # module's globals may already be gone when the last objects are collected
    def __del__(self, _destroy=_lib.bsgd_fused_destroy):
        h = getattr(self, "handle", None)
        if h:
            self.handle = None
            _destroy(h)


def bsgd_fused_workspace_size(plan: Plan, chunks=0, flags=0, stream=None) -> int:
    out = _sz()
    _check("bsgd_fused_workspace_size", _lib.bsgd_fused_workspace_size(
        plan.handle, int(chunks), int(flags), _stream(stream), ctypes.byref(out)))
    return out.value


def bsgd_fused_create(plan: Plan, chunks=0, flags=0, stream=None) -> Fused:
    nbytes = bsgd_fused_workspace_size(plan, chunks, flags, stream)
    ws = _ws(nbytes, plan.workspace.device)
    h = _vp()
    _check("bsgd_fused_create", _lib.bsgd_fused_create(plan.handle, int(chunks), int(flags),
                                                       _ptr(ws), nbytes, _stream(stream),
                                                       ctypes.byref(h)))
    return Fused(h, ws, plan)


def bsgd_lanczos_workspace_size_fused(fused: Fused, steps: int) -> int:
    out = _sz()
    _check("bsgd_lanczos_workspace_size_fused",
           _lib.bsgd_lanczos_workspace_size_fused(fused.handle, int(steps), ctypes.byref(out)))
    return out.value


def bsgd_lanczos_umax_fused(fused: Fused, steps, vt=BSGD_VAL_F32, ws=None, stream=None) -> float:
    """u_max by Lanczos steps whose products run on the tile-sliced store."""
    nbytes = bsgd_lanczos_workspace_size_fused(fused, steps)
    if ws is None:
        ws = _ws(nbytes, fused.workspace.device)
    out = ctypes.c_float()
    _check("bsgd_lanczos_umax_fused",
           _lib.bsgd_lanczos_umax_fused(fused.handle, vt, int(steps), _ptr(ws), ws.numel(),
                                        _stream(stream), ctypes.byref(out)))
    return float(out.value)


def bsgd_fused_shape(fused: Fused):
    """(tiles, chunks, segments, slices, stored entries, bytes per stored column)."""
    t, q, cb = _i32(), _i32(), _i32()
    g, sl, e = _i64(), _i64(), _i64()
    _check("bsgd_fused_shape", _lib.bsgd_fused_shape(fused.handle, ctypes.byref(t), ctypes.byref(q),
                                                     ctypes.byref(g), ctypes.byref(sl),
                                                     ctypes.byref(e), ctypes.byref(cb)))
    return t.value, q.value, g.value, sl.value, e.value, cb.value


def bsgd_fused_set_waves(fused: Fused, waves: int):
    _check("bsgd_fused_set_waves", _lib.bsgd_fused_set_waves(fused.handle, int(waves)))


def bsgd_fused_partials_size(fused: Fused) -> int:
    out = _sz()
    _check("bsgd_fused_partials_size", _lib.bsgd_fused_partials_size(fused.handle, ctypes.byref(out)))
    return out.value


def bsgd_fused_partials_size_rhs(fused: Fused, nrhs: int) -> int:
    out = _sz()
    _check("bsgd_fused_partials_size_rhs", _lib.bsgd_fused_partials_size_rhs(
        fused.handle, int(nrhs), ctypes.byref(out)))
    return out.value


def bsgd_fused_apply(fused: Fused, x, r, y=None, xadd=None, mu=0.0, out_r=None, out_x=None,
                     vt=BSGD_VAL_F32, partials=None, stream=None):
    """One single-pass product: (y - A x or A x, xadd + mu 2 A^T r or 2 A^T r)."""
    plan = fused.plan
    _chk(x, plan.ncols, "x")
    _chk(r, plan.nrows, "r")
    if y is not None:
        _chk(y, plan.nrows, "y")
    if xadd is not None:
        _chk(xadd, plan.ncols, "xadd")
    dev = x.device
    if out_r is None:
        out_r = torch.empty(plan.nrows, dtype=torch.float32, device=dev)
    if out_x is None:
        out_x = torch.empty(plan.ncols, dtype=torch.float32, device=dev)
    _chk(out_r, plan.nrows, "out_r")
    _chk(out_x, plan.ncols, "out_x")
    if partials is None:
        partials = _ws(bsgd_fused_partials_size(fused), dev)
    _check("bsgd_fused_apply", _lib.bsgd_fused_apply(
        fused.handle, vt, _ptr(x), _ptr(y), _ptr(r), _ptr(xadd), float(mu), _ptr(out_r),
        _ptr(out_x), _ptr(partials), partials.numel(), _stream(stream)))
    return out_r, out_x


def bsgd_state_attach_fused(state: State, fused, partials=None):
    """Run the state's epochs through the single-pass form (fused=None detaches)."""
    if fused is None:
        _check("bsgd_state_attach_fused", _lib.bsgd_state_attach_fused(state.handle, None, None, 0))
        state.fused = state.fused_partials = None
        return
    if partials is None:
        partials = _ws(bsgd_fused_partials_size_rhs(fused, state.nrhs), state.workspace.device)
    _check("bsgd_state_attach_fused", _lib.bsgd_state_attach_fused(
        state.handle, fused.handle, _ptr(partials), partials.numel()))
    state.fused = fused
    state.fused_partials = partials
