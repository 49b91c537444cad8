"""Thin Python binding of the C ABI in ``include/batchsolve.h``.

Each ``bs_*`` function here marshals its arguments (torch device tensors, numpy
host arrays, the current HIP stream) into the call of the same name in
``libbatchsolve.so``; every step of the solve runs in the HIP kernels.  There
is no CPU fallback: if the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbatchsolve.so")

# enums of batchsolve.h
CSR, ELL, DENSE = 0, 1, 2
CG, BICGSTAB, GMRES, TRSV_LOWER, TRSV_UPPER = 0, 1, 2, 3, 4
PREC_NONE, PREC_JACOBI, PREC_BLOCK_JACOBI, PREC_ILU = 0, 1, 2, 3
FP64, MIXED = 0, 1
CONVERGED, MAX_ITER, BREAKDOWN, NONFINITE = 0, 1, 2, 3
OK, ERR_INVALID_ARG, ERR_PATTERN, ERR_UNSUPPORTED, ERR_HIP, ERR_NO_DEVICE = 0, -1, -2, -3, -4, -5
FLAG_X0_ZERO = 1
FLAG_PLAIN_LAYOUT = 2
FLAG_ABS_TOL = 4
MAX_ROWS, MAX_ROW_NNZ, MAX_RESTART = 2048, 64, 30


class BatchSolveError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = bs_error_string(code)
        extra = bs_last_error() if code == ERR_HIP else ""
        super().__init__(f"{where}: {msg} ({code}){' - ' + extra if extra else ''}")


class bs_options(C.Structure):
    _fields_ = [("restart", C.c_int32), ("precision", C.c_int32), ("inner_tol", C.c_double),
                ("flags", C.c_int32), ("team", C.c_int32), ("rows_per_lane", C.c_int32),
                ("outer_iters", C.c_void_p), ("x_alt", C.c_void_p), ("alt_used", C.c_void_p),
                ("block_size", C.c_int32), ("n_rhs", C.c_int32), ("varlen_policy", C.c_int32),
                ("structure_generation", C.c_int32)]


class bs_pattern_dev(C.Structure):
    _fields_ = [("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("nnz", C.c_int32),
                ("ell_width", C.c_int32)]


class bs_plan_info(C.Structure):
    _fields_ = [("team", C.c_int32), ("rows_per_lane", C.c_int32), ("slots", C.c_int32),
                ("group_size", C.c_int32), ("systems_per_group", C.c_int32),
                ("lds_bytes", C.c_int32), ("stage_values", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib() -> C.CDLL:
    """Load ``libbatchsolve.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2308_08417_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.bs_pattern_create_csr.argtypes = [i32, i32, vp, vp, C.POINTER(vp)]
    L.bs_pattern_create_ell.argtypes = [i32, i32, vp, C.POINTER(vp)]
    L.bs_pattern_create_dense.argtypes = [i32, C.POINTER(vp)]
    L.bs_pattern_destroy.argtypes = [vp]
    L.bs_pattern_query.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
    L.bs_pattern_ell_cols.argtypes = [vp, vp]
    L.bs_wave_layout.argtypes = [i32, i32, vp, vp, i32, i32, vp, vp, vp, vp]
    L.bs_pattern_layout.argtypes = [vp, C.POINTER(i32), vp]
    L.bs_values_csr_to_ell.argtypes = [vp, i64, vp, vp, vp]
    L.bs_matrix_storage.argtypes = [C.c_int, i64, i32, i32, i32, C.POINTER(i64), C.POINTER(i64)]
    L.bs_batch_solve.argtypes = [C.c_int, i64, i32, vp, vp, vp, vp, C.c_int, C.c_int, dbl, i32,
                                 vp, vp, vp, C.POINTER(bs_options), vp]
    L.bs_plan.argtypes = [C.c_int, i32, i32, i32, C.c_int, C.POINTER(bs_options),
                          C.POINTER(bs_plan_info)]
    L.bs_plan_precond.argtypes = [C.c_int, i32, i32, i32, C.c_int, C.c_int,
                                  C.POINTER(bs_options), C.POINTER(bs_plan_info)]
    sz = C.c_size_t
    L.bs_varbatch_create.argtypes = [i64, i32, vp, vp, vp, vp, vp, vp, C.POINTER(vp)]
    L.bs_varbatch_destroy.argtypes = [vp]
    L.bs_varbatch_query.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i32),
                                    C.POINTER(i32)]
    L.bs_varbatch_set_policy.argtypes = [vp, i32]
    L.bs_varbatch_create_ell.argtypes = [i64, i32, vp, vp, vp, vp, vp, C.POINTER(vp)]
    L.bs_varbatch_set_plan.argtypes = [vp, vp]
    L.bs_varbatch_get_plan.argtypes = [vp, vp, vp]
    _vsolve = [vp, vp, vp, vp, C.c_int, C.c_int, dbl, i32, vp, vp, vp, C.POINTER(bs_options)]
    L.bs_varbatch_solve.argtypes = _vsolve + [vp]
    L.bs_varbatch_tune.argtypes = _vsolve + [i32, C.c_char_p, C.c_char_p, sz, vp]
    L.bs_varbatch_capture.argtypes = _vsolve
    L.bs_varbatch_replay.argtypes = [vp, vp]
    L.bs_batch_solve_varlen.argtypes = [i64, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp,
                                        C.c_int, C.c_int, dbl, i32, vp, vp, vp,
                                        C.POINTER(bs_options), vp, sz, vp]
    L.bs_batch_solve_varlen.restype = C.c_int
    L.bs_varlen_workspace_size.argtypes = [i64]
    L.bs_varlen_workspace_size.restype = sz
    L.bs_batch_solve_dev.argtypes = [C.c_int, i64, i32, C.POINTER(bs_pattern_dev), vp, vp, vp,
                                     C.c_int, C.c_int, dbl, i32, vp, vp, vp,
                                     C.POINTER(bs_options), vp, sz, vp]
    L.bs_batch_solve_dev.restype = C.c_int
    L.bs_workspace_size.argtypes = [C.c_int, i64, i32, vp, C.c_int, C.POINTER(bs_options)]
    L.bs_workspace_size.restype = sz
    f32p = vp
    L.bs_ws_create.argtypes = [i32, i32, vp, vp, C.POINTER(vp)]
    L.bs_ws_destroy.argtypes = [vp]
    L.bs_ws_param_count.argtypes = [vp, C.POINTER(i64)]
    L.bs_ws_set_params.argtypes = [vp, vp]
    L.bs_ws_get_params.argtypes = [vp, vp]
    L.bs_ws_features.argtypes = [vp, i64, vp, vp, vp, vp, f32p, f32p, vp]
    L.bs_ws_fit_scaling.argtypes = [vp, i64, vp, vp, vp]
    L.bs_ws_get_scaling.argtypes = [vp, vp, vp, vp]
    L.bs_ws_set_scaling.argtypes = [vp, vp, vp, vp]
    L.bs_ws_forward.argtypes = [vp, i64, vp, vp, vp, vp]
    L.bs_ws_grad.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp]
    L.bs_ws_train_step.argtypes = [vp, i64, vp, vp, vp, C.c_float, vp, vp]
    L.bs_ws_infer.argtypes = [vp, i64, vp, vp, vp, vp, vp]
    L.bs_ws_train_step_noalloc.argtypes = [vp, i64, vp, vp, vp, C.c_float, vp, vp]
    L.bs_ws_train_step_noalloc.restype = C.c_int
    L.bs_ws_packed_bytes.argtypes = [i32]
    L.bs_ws_packed_bytes.restype = sz
    L.bs_ws_pack.argtypes = [vp, vp, sz, vp]
    L.bs_ws_pack.restype = C.c_int
    L.bs_ws_infer_packed.argtypes = [i64, i32, vp, vp, vp, vp, vp, vp]
    L.bs_ws_infer_packed.restype = C.c_int
    L.bs_error_string.argtypes = [C.c_int]
    L.bs_error_string.restype = C.c_char_p
    L.bs_last_error.argtypes = []
    L.bs_last_error.restype = C.c_char_p
    for name in ("bs_pattern_create_csr", "bs_pattern_create_ell", "bs_pattern_create_dense",
                 "bs_pattern_destroy",
                 "bs_pattern_query", "bs_pattern_ell_cols", "bs_wave_layout",
                 "bs_pattern_layout", "bs_values_csr_to_ell",
                 "bs_matrix_storage", "bs_batch_solve", "bs_plan", "bs_plan_precond",
                 "bs_varbatch_create", "bs_varbatch_create_ell", "bs_varbatch_set_plan",
                 "bs_varbatch_get_plan",
                 "bs_varbatch_destroy", "bs_varbatch_query", "bs_varbatch_set_policy",
                 "bs_varbatch_solve", "bs_varbatch_tune", "bs_varbatch_capture",
                 "bs_varbatch_replay", "bs_ws_create", "bs_ws_destroy", "bs_ws_param_count",
                 "bs_ws_set_params", "bs_ws_get_params", "bs_ws_features", "bs_ws_fit_scaling",
                 "bs_ws_get_scaling", "bs_ws_set_scaling", "bs_ws_forward", "bs_ws_grad",
                 "bs_ws_train_step", "bs_ws_infer"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(code: int, where: str):
    if code != OK:
        raise BatchSolveError(code, where)


def bs_error_string(code: int) -> str:
    return lib().bs_error_string(code).decode()


def bs_last_error() -> str:
    return lib().bs_last_error().decode()


def _host_i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.int32)


def _ptr(t) -> Optional[int]:
    """Device pointer of a torch tensor (None stays NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


_DTYPES = {"f64": "torch.float64", "f32": "torch.float32", "i32": "torch.int32",
           "i64": "torch.int64"}


def _expect(t, name: str, dtype: str, numel: int, optional: bool = False,
            at_least: bool = False) -> None:
    """Check a tensor argument before its raw pointer reaches the library: the
    kernels trust the element type and count, so a wrong one would make them
    read or write past the allocation.  ``dtype`` is "f64", "f32" or "i32";
    ``numel`` the element count the call will touch.  Raises ValueError."""
    if t is None:
        if optional:
            return
        raise ValueError(f"{name} is required")
    if str(t.dtype) != _DTYPES[dtype]:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {_DTYPES[dtype]}")
    if t.numel() < numel if at_least else t.numel() != numel:
        raise ValueError(f"{name}: {t.numel()} elements, expected {'at least ' if at_least else ''}"
                         f"{numel}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous tensor")


def check_solve_args(fmt: int, n_rows: int, nnz: int, ell_width: int, values, b, x, iters, resid,
                     status=None, opts: Optional["bs_options"] = None) -> tuple:
    """Element types and counts of a ``bs_batch_solve`` call for a pattern of
    ``n_rows`` rows, ``nnz`` entries and ELL width ``ell_width``; returns
    ``(n_batch, n_solves)``.  Raises ValueError on any mismatch."""
    if b is None or b.dim() != 2 or b.shape[1] != n_rows:
        raise ValueError(f"b: expected a [n_solves][{n_rows}] tensor")
    k = opts.n_rhs if opts is not None and opts.n_rhs > 1 else 1
    n_solves = int(b.shape[0])
    if n_solves % k:
        raise ValueError("b holds a whole number of right-hand sides per matrix")
    n_batch = n_solves // k
    stored = {CSR: nnz, ELL: ell_width * n_rows, DENSE: n_rows * n_rows}.get(fmt)
    if stored is None:
        raise ValueError(f"unknown format {fmt}")
    _expect(values, "values", "f64", n_batch * stored)
    _expect(b, "b", "f64", n_solves * n_rows)
    _expect(x, "x", "f64", n_solves * n_rows)
    _expect(iters, "iters", "i32", n_solves)
    _expect(resid, "resid", "f64", n_solves)
    _expect(status, "status", "i32", n_solves, optional=True)
    if opts is not None:
        keep = getattr(opts, "_keep", (None, None, None))
        if (opts.outer_iters or opts.x_alt or opts.alt_used) and keep == (None, None, None):
            raise ValueError("options with device pointers must come from make_options")
        outer, x_alt, alt_used = keep
        _expect(outer, "outer_iters", "i32", n_solves, optional=True)
        _expect(x_alt, "x_alt", "f64", n_solves * n_rows, optional=True)
        _expect(alt_used, "alt_used", "i32", n_solves, optional=True)
    return n_batch, n_solves


def _stream(stream) -> Optional[int]:
    if stream is not None:
        return int(stream)
    import torch
    return torch.cuda.current_stream().cuda_stream


# ------------------------------------------------------------------ patterns
def bs_pattern_create_csr(row_ptr, col_idx) -> int:
    rp, ci = _host_i32(row_ptr), _host_i32(col_idx)
    h = C.c_void_p()
    _check(lib().bs_pattern_create_csr(rp.size - 1, ci.size, rp.ctypes.data,
                                       ci.ctypes.data if ci.size else None, C.byref(h)),
           "bs_pattern_create_csr")
    return h.value


def bs_pattern_create_dense(n_rows: int) -> int:
    h = C.c_void_p()
    _check(lib().bs_pattern_create_dense(n_rows, C.byref(h)), "bs_pattern_create_dense")
    return h.value


def bs_pattern_create_ell(n_rows: int, ell_col) -> int:
    ec = _host_i32(ell_col)
    width = ec.size // n_rows
    h = C.c_void_p()
    _check(lib().bs_pattern_create_ell(n_rows, width, ec.ctypes.data if ec.size else None,
                                       C.byref(h)), "bs_pattern_create_ell")
    return h.value


def bs_pattern_destroy(handle: int) -> None:
    _check(lib().bs_pattern_destroy(handle), "bs_pattern_destroy")


def bs_pattern_query(handle: int) -> dict:
    v = [C.c_int32() for _ in range(4)]
    _check(lib().bs_pattern_query(handle, *[C.byref(x) for x in v]), "bs_pattern_query")
    return dict(zip(("n_rows", "nnz", "ell_width", "max_row_nnz"), (x.value for x in v)))


def bs_pattern_ell_cols(handle: int) -> np.ndarray:
    q = bs_pattern_query(handle)
    out = np.empty(max(q["ell_width"] * q["n_rows"], 1), np.int32)
    _check(lib().bs_pattern_ell_cols(handle, out.ctypes.data), "bs_pattern_ell_cols")
    return out[: q["ell_width"] * q["n_rows"]]


def bs_wave_layout(row_ptr, col_idx, slots: int, steps: int = 20000) -> dict:
    """Bank-aware one-wave layout of a CSR pattern (host only): lane_row[64],
    lane_win[64], col_pos[n] and the model costs (chosen, plain)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    n = rp.size - 1
    lane_row = np.empty(64, np.int32)
    lane_win = np.empty(64, np.int32)
    col_pos = np.empty(n, np.int32)
    cost = np.empty(2, np.int64)
    _check(lib().bs_wave_layout(n, ci.size, rp.ctypes.data, ci.ctypes.data, slots, steps,
                                lane_row.ctypes.data, lane_win.ctypes.data, col_pos.ctypes.data,
                                cost.ctypes.data), "bs_wave_layout")
    return {"lane_row": lane_row, "lane_win": lane_win, "col_pos": col_pos,
            "cost": int(cost[0]), "plain_cost": int(cost[1])}


def bs_pattern_layout(handle: int):
    """(slots, lane_row, lane_win, col_pos) of the pattern's layout, or None."""
    q = bs_pattern_query(handle)
    slots = C.c_int32()
    out = np.empty(128 + q["n_rows"], np.int32)
    _check(lib().bs_pattern_layout(handle, C.byref(slots), out.ctypes.data), "bs_pattern_layout")
    if slots.value == 0:
        return None
    return slots.value, out[:64].copy(), out[64:128].copy(), out[128:].copy()


def bs_values_csr_to_ell(handle: int, csr_values, ell_values, stream=None) -> None:
    _check(lib().bs_values_csr_to_ell(handle, csr_values.shape[0], _ptr(csr_values),
                                      _ptr(ell_values), _stream(stream)), "bs_values_csr_to_ell")


def bs_matrix_storage(fmt: int, n_batch: int, n_rows: int, nnz: int, ell_width: int):
    vc, ic = C.c_int64(), C.c_int64()
    _check(lib().bs_matrix_storage(fmt, n_batch, n_rows, nnz, ell_width, C.byref(vc), C.byref(ic)),
           "bs_matrix_storage")
    return vc.value, ic.value


def make_options(restart: int = 0, precision: int = FP64, inner_tol: float = 0.0, flags: int = 0,
                 team: int = 0, rows_per_lane: int = 0, outer_iters=None, x_alt=None,
                 alt_used=None, block_size: int = 0, n_rhs: int = 0, varlen_policy: int = 0,
                 structure_generation: int = 0) -> bs_options:
    o = bs_options(restart, precision, inner_tol, flags, team, rows_per_lane, _ptr(outer_iters),
                   _ptr(x_alt), _ptr(alt_used), block_size, n_rhs, varlen_policy,
                   structure_generation)
    # the structure holds raw device pointers: keep their tensors alive with it
    o._keep = (outer_iters, x_alt, alt_used)
    return o


def bs_plan(fmt: int, n_rows: int, nnz: int, max_row_nnz: int, solver: int,
            opts: Optional[bs_options] = None) -> dict:
    out = bs_plan_info()
    _check(lib().bs_plan(fmt, n_rows, nnz, max_row_nnz, solver,
                         C.byref(opts) if opts is not None else None, C.byref(out)), "bs_plan")
    return out.as_dict()


def bs_plan_precond(fmt: int, n_rows: int, nnz: int, max_row_nnz: int, solver: int,
                    precond: int, opts: Optional[bs_options] = None) -> dict:
    out = bs_plan_info()
    _check(lib().bs_plan_precond(fmt, n_rows, nnz, max_row_nnz, solver, precond,
                                 C.byref(opts) if opts is not None else None, C.byref(out)),
           "bs_plan_precond")
    return out.as_dict()


# ------------------------------------------------------------------ solve
def bs_batch_solve(fmt: int, pattern: int, values, b, x, solver: int, precond: int, tol: float,
                   max_iter: int, iters, resid, status=None, opts: Optional[bs_options] = None,
                   stream=None) -> None:
    """Launch the fused solve on ``stream`` (default: torch's current stream).

    ``values``/``b``/``x``: float64 device tensors ``[B, nnz]`` (CSR) or ``[B, W*n]``
    (ELL), ``[B, n]``, ``[B, n]``; ``iters``/``status`` int32 ``[B]``; ``resid``
    float64 ``[B]``.  With ``opts.n_rhs = k > 1``, B counts matrices and ``b``/``x``
    (and the per-solve outputs) hold ``B*k`` rows, matrix by matrix.
    Asynchronous: synchronise the stream before reading results.
    """
    q = bs_pattern_query(pattern)
    n_rows = q["n_rows"]
    n_batch, _ = check_solve_args(fmt, n_rows, q["nnz"], q["ell_width"], values, b, x, iters,
                                  resid, status, opts)
    _check(lib().bs_batch_solve(fmt, n_batch, n_rows, pattern, _ptr(values), _ptr(b), _ptr(x),
                                solver, precond, float(tol), int(max_iter), _ptr(iters),
                                _ptr(resid), _ptr(status),
                                C.byref(opts) if opts is not None else None, _stream(stream)),
           "bs_batch_solve")


def bs_batch_solve_dev(fmt: int, n_rows: int, row_ptr, col_idx, values, b, x, solver: int,
                       precond: int, tol: float, max_iter: int, iters, resid, status=None,
                       opts: Optional[bs_options] = None, ell_width: int = 0, workspace=None,
                       stream=None) -> None:
    """``bs_batch_solve`` with the shared pattern as int32 device tensors the
    caller owns: CSR ``row_ptr`` [n+1] and ``col_idx`` [nnz]; ELL ``col_idx``
    [ell_width*n] slot-major (``row_ptr`` None); DENSE neither."""
    if fmt == CSR:
        for t, name in ((row_ptr, "row_ptr"), (col_idx, "col_idx")):
            if t is None or str(t.dtype) != _DTYPES["i32"] or not t.is_cuda:
                raise ValueError(f"{name}: expected an int32 device tensor")
        _expect(row_ptr, "row_ptr", "i32", n_rows + 1)
        nnz = int(col_idx.numel())
    elif fmt == ELL:
        if col_idx is None or str(col_idx.dtype) != _DTYPES["i32"] or not col_idx.is_cuda:
            raise ValueError("col_idx: expected an int32 device tensor")
        _expect(col_idx, "col_idx", "i32", ell_width * n_rows)
        nnz = ell_width * n_rows
    else:
        nnz = n_rows * n_rows
    n_batch, _ = check_solve_args(fmt, n_rows, nnz, ell_width, values, b, x, iters, resid,
                                  status, opts)
    pd = bs_pattern_dev(_ptr(row_ptr) if fmt == CSR else None,
                        _ptr(col_idx) if fmt != DENSE else None,
                        nnz if fmt != DENSE else 0, ell_width if fmt == ELL else 0)
    ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _check(lib().bs_batch_solve_dev(fmt, n_batch, n_rows, C.byref(pd), _ptr(values), _ptr(b),
                                    _ptr(x), solver, precond, float(tol), int(max_iter),
                                    _ptr(iters), _ptr(resid), _ptr(status),
                                    C.byref(opts) if opts is not None else None,
                                    _ptr(workspace), ws_bytes, _stream(stream)),
           "bs_batch_solve_dev")


@dataclass
class Pattern:
    """Owns a pattern handle; releases its device copy when collected."""

    handle: int
    n_rows: int
    nnz: int
    ell_width: int
    max_row_nnz: int

    @classmethod
    def from_csr(cls, row_ptr, col_idx) -> "Pattern":
        h = bs_pattern_create_csr(row_ptr, col_idx)
        return cls(h, **bs_pattern_query(h))

    @classmethod
    def dense(cls, n_rows: int) -> "Pattern":
        """The full pattern, for BatchDense values ``[B][n][n]`` (``DENSE``)."""
        h = bs_pattern_create_dense(n_rows)
        return cls(h, **bs_pattern_query(h))

    @classmethod
    def from_ell(cls, n_rows: int, ell_col) -> "Pattern":
        h = bs_pattern_create_ell(n_rows, ell_col)
        return cls(h, **bs_pattern_query(h))

    def __del__(self):
        if self.handle and _lib is not None:
            _lib.bs_pattern_destroy(self.handle)
            self.handle = 0


def solve(pattern: Pattern, values, b, x=None, fmt: int = CSR, solver: int = BICGSTAB,
          precond: int = PREC_JACOBI, tol: float = 1e-10, max_iter: int = 500,
          opts: Optional[bs_options] = None, stream=None):
    """Allocate the outputs with torch and call :func:`bs_batch_solve`.

    Returns ``(x, iters, resid, status)`` as device tensors (not synchronised).
    If ``x`` is None the solve starts from zero (``BS_FLAG_X0_ZERO``).
    """
    import torch
    B = b.shape[0]
    dev = b.device
    if x is None:
        x = torch.empty_like(b)
        # a copy: the caller's options stay as they were
        base = opts if opts is not None else make_options()
        opts = bs_options.from_buffer_copy(base)
        opts._keep = getattr(base, "_keep", (None, None, None))
        opts.flags |= FLAG_X0_ZERO
    iters = torch.empty(B, dtype=torch.int32, device=dev)
    resid = torch.empty(B, dtype=torch.float64, device=dev)
    status = torch.empty(B, dtype=torch.int32, device=dev)
    bs_batch_solve(fmt, pattern.handle, values, b, x, solver, precond, tol, max_iter, iters, resid,
                   status, opts, stream)
    return x, iters, resid, status


# ------------------------------------------------------------------ uneven batches
def _host(a, dt) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=dt)


# systems of each uneven-batch handle made here (for the argument checks)
_VB_SYSTEMS: dict = {}


def bs_varbatch_create(pat_rows, pat_rowptr_off, rowptr_all, pat_col_off, col_all, sys_pat) -> int:
    pr, pro, rpa = _host(pat_rows, np.int32), _host(pat_rowptr_off, np.int64), _host(rowptr_all, np.int32)
    pco, ca, sp = _host(pat_col_off, np.int64), _host(col_all, np.int32), _host(sys_pat, np.int32)
    h = C.c_void_p()
    _check(lib().bs_varbatch_create(sp.size, pr.size, pr.ctypes.data, pro.ctypes.data,
                                    rpa.ctypes.data, pco.ctypes.data,
                                    ca.ctypes.data if ca.size else None,
                                    sp.ctypes.data if sp.size else None, C.byref(h)),
           "bs_varbatch_create")
    _VB_SYSTEMS[h.value] = int(sp.size)
    return h.value


def bs_varbatch_create_ell(pat_rows, pat_width, pat_col_off, col_all, sys_pat) -> int:
    """ELL patterns: slot-major columns [width][rows] per pattern, -1 padding."""
    pr, pw, pco = _host(pat_rows, np.int32), _host(pat_width, np.int32), _host(pat_col_off, np.int64)
    ca, sp = _host(col_all, np.int32), _host(sys_pat, np.int32)
    h = C.c_void_p()
    _check(lib().bs_varbatch_create_ell(sp.size, pr.size, pr.ctypes.data, pw.ctypes.data,
                                        pco.ctypes.data, ca.ctypes.data if ca.size else None,
                                        sp.ctypes.data if sp.size else None, C.byref(h)),
           "bs_varbatch_create_ell")
    _VB_SYSTEMS[h.value] = int(sp.size)
    return h.value


def bs_varbatch_set_plan(handle: int, class_codes) -> None:
    """One launch per size class; ``class_codes`` holds 5 codes
    (shape + 3 * walk + 6 * placement)."""
    cc = _host(class_codes, np.int32)
    if cc.size != 5:
        raise ValueError("class_codes: expected 5 codes")
    _check(lib().bs_varbatch_set_plan(handle, cc.ctypes.data), "bs_varbatch_set_plan")


def bs_varbatch_get_plan(handle: int) -> tuple:
    """(policy, [5 class codes]); policy -1 under a per-class plan."""
    p = C.c_int32()
    cc = np.zeros(5, np.int32)
    _check(lib().bs_varbatch_get_plan(handle, C.byref(p), cc.ctypes.data), "bs_varbatch_get_plan")
    return p.value, cc.tolist()


def bs_varbatch_destroy(handle: int) -> None:
    _VB_SYSTEMS.pop(handle, None)
    _check(lib().bs_varbatch_destroy(handle), "bs_varbatch_destroy")


def bs_varbatch_query(handle: int) -> dict:
    r, v = C.c_int64(), C.c_int64()
    t, p = C.c_int32(), C.c_int32()
    _check(lib().bs_varbatch_query(handle, C.byref(r), C.byref(v), C.byref(t), C.byref(p)),
           "bs_varbatch_query")
    return {"total_rows": r.value, "total_values": v.value, "n_tasks": t.value, "policy": p.value}


def bs_varbatch_set_policy(handle: int, policy: int) -> None:
    _check(lib().bs_varbatch_set_policy(handle, policy), "bs_varbatch_set_policy")


def check_varbatch_args(total_values: int, total_rows: int, n_batch: int, values, b, x, iters,
                        resid, status=None, opts: Optional["bs_options"] = None) -> None:
    """Element types and counts of an uneven-batch solve; raises ValueError."""
    _expect(values, "values", "f64", total_values)
    _expect(b, "b", "f64", total_rows)
    _expect(x, "x", "f64", total_rows)
    _expect(iters, "iters", "i32", n_batch)
    _expect(resid, "resid", "f64", n_batch)
    _expect(status, "status", "i32", n_batch, optional=True)
    if opts is not None:
        outer, x_alt, alt_used = getattr(opts, "_keep", (None, None, None))
        if x_alt is not None or alt_used is not None:
            raise ValueError("the uneven-batch path takes no second initial guess")
        _expect(outer, "outer_iters", "i32", n_batch, optional=True)


def _vargs(handle, values, b, x, solver, precond, tol, max_iter, iters, resid, status, opts):
    q = bs_varbatch_query(handle)
    n_batch = _VB_SYSTEMS[handle]
    check_varbatch_args(q["total_values"], q["total_rows"], n_batch, values, b, x, iters, resid,
                        status, opts)
    return (handle, _ptr(values), _ptr(b), _ptr(x), solver, precond, float(tol), int(max_iter),
            _ptr(iters), _ptr(resid), _ptr(status), C.byref(opts) if opts is not None else None)


def bs_varbatch_solve(handle: int, values, b, x, solver: int, precond: int, tol: float,
                      max_iter: int, iters, resid, status=None, opts: Optional[bs_options] = None,
                      stream=None) -> None:
    """Solve an uneven batch: ``values``/``b``/``x`` are the concatenated float64
    device vectors, ``iters``/``status`` int32 and ``resid`` float64 per system."""
    _check(lib().bs_varbatch_solve(*_vargs(handle, values, b, x, solver, precond, tol, max_iter,
                                           iters, resid, status, opts), _stream(stream)),
           "bs_varbatch_solve")


def bs_varbatch_tune(handle: int, values, b, x, solver: int, precond: int, tol: float,
                     max_iter: int, iters, resid, status=None, opts: Optional[bs_options] = None,
                     reps: int = 3, cache_path: Optional[str] = None, stream=None) -> str:
    """Time the single-launch policies and the per-class plans, keep the
    fastest; returns the report line."""
    buf = C.create_string_buffer(1024)
    _check(lib().bs_varbatch_tune(*_vargs(handle, values, b, x, solver, precond, tol, max_iter,
                                          iters, resid, status, opts), int(reps),
                                  cache_path.encode() if cache_path else None, buf, len(buf),
                                  _stream(stream)), "bs_varbatch_tune")
    return buf.value.decode()


def bs_varbatch_capture(handle: int, values, b, x, solver: int, precond: int, tol: float,
                        max_iter: int, iters, resid, status=None,
                        opts: Optional[bs_options] = None) -> None:
    _check(lib().bs_varbatch_capture(*_vargs(handle, values, b, x, solver, precond, tol, max_iter,
                                             iters, resid, status, opts)), "bs_varbatch_capture")


def bs_varbatch_replay(handle: int, stream=None) -> None:
    _check(lib().bs_varbatch_replay(handle, _stream(stream)), "bs_varbatch_replay")


def bs_varlen_workspace_size(n_batch: int) -> int:
    return int(lib().bs_varlen_workspace_size(int(n_batch)))


def bs_workspace_size(fmt: int, n_batch: int, n_rows: int, pattern: int, solver: int,
                      opts: Optional[bs_options] = None) -> int:
    return int(lib().bs_workspace_size(fmt, int(n_batch), int(n_rows), pattern, solver,
                                       C.byref(opts) if opts is not None else None))


def check_varlen_args(n_batch: int, n_patterns: int, sys_rows, row_off, val_off, pat_id,
                      pat_rowptr_off, pat_col_off, rowptr_all, col_all, ws) -> None:
    """Element types and counts of the structure arrays of
    ``bs_batch_solve_varlen`` and the size of its workspace; raises ValueError.
    (The contents are validated by the library.)"""
    _expect(sys_rows, "sys_rows", "i32", n_batch)
    _expect(pat_id, "pat_id", "i32", n_batch)
    _expect(row_off, "row_off", "i64", n_batch + 1)
    _expect(val_off, "val_off", "i64", n_batch + 1)
    _expect(pat_rowptr_off, "pat_rowptr_off", "i64", n_patterns)
    _expect(pat_col_off, "pat_col_off", "i64", n_patterns)
    for t, name in ((rowptr_all, "rowptr_all"), (col_all, "col_all")):
        if t is None or str(t.dtype) != _DTYPES["i32"]:
            raise ValueError(f"{name}: expected an int32 tensor")
    if ws is None or ws.numel() * ws.element_size() < bs_varlen_workspace_size(n_batch):
        raise ValueError("ws: smaller than bs_varlen_workspace_size(n_batch)")


def bs_batch_solve_varlen(sys_rows, row_off, val_off, pat_id, pat_rowptr_off, pat_col_off,
                          rowptr_all, col_all, values, b, x, solver: int, precond: int,
                          tol: float, max_iter: int, iters, resid, status=None,
                          opts: Optional[bs_options] = None, ws=None, stream=None) -> None:
    """Uneven batch on device tensors the caller owns (``bs_batch_solve_varlen``):
    int32 ``sys_rows``/``pat_id`` [B], int64 ``row_off``/``val_off`` [B+1] and
    ``pat_rowptr_off``/``pat_col_off`` [P], int32 ``rowptr_all``/``col_all``;
    ``ws`` a device tensor of at least ``bs_varlen_workspace_size(B)`` bytes."""
    n_batch = int(sys_rows.numel())
    n_patterns = int(pat_rowptr_off.numel())
    check_varlen_args(n_batch, n_patterns, sys_rows, row_off, val_off, pat_id, pat_rowptr_off,
                      pat_col_off, rowptr_all, col_all, ws)
    _expect(iters, "iters", "i32", n_batch)
    _expect(resid, "resid", "f64", n_batch)
    _expect(status, "status", "i32", n_batch, optional=True)
    for t, name in ((values, "values"), (b, "b"), (x, "x")):
        if t is None or str(t.dtype) != _DTYPES["f64"]:
            raise ValueError(f"{name}: expected a float64 tensor")
    _check(lib().bs_batch_solve_varlen(
        n_batch, _ptr(sys_rows), _ptr(row_off), _ptr(val_off), n_patterns, _ptr(pat_id),
        _ptr(pat_rowptr_off), _ptr(pat_col_off), _ptr(rowptr_all), _ptr(col_all), _ptr(values),
        _ptr(b), _ptr(x), solver, precond, float(tol), int(max_iter), _ptr(iters), _ptr(resid),
        _ptr(status), C.byref(opts) if opts is not None else None, _ptr(ws),
        ws.numel() * ws.element_size(), _stream(stream)), "bs_batch_solve_varlen")


class VarBatch:
    """Owns an uneven-batch handle (see ``bs_varbatch_create``; with
    ``ell=True`` the arguments are those of ``bs_varbatch_create_ell``)."""

    def __init__(self, *args, ell: bool = False):
        self.handle = bs_varbatch_create_ell(*args) if ell else bs_varbatch_create(*args)
        self.n_batch = int(np.asarray(args[-1]).size)
        q = bs_varbatch_query(self.handle)
        self.total_rows, self.total_values = q["total_rows"], q["total_values"]

    def query(self) -> dict:
        return bs_varbatch_query(self.handle)

    def __del__(self):
        if getattr(self, "handle", 0) and _lib is not None:
            _VB_SYSTEMS.pop(self.handle, None)
            _lib.bs_varbatch_destroy(self.handle)
            self.handle = 0


# ------------------------------------------------------------------ learned initial guess
def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.float32)


def _f64h(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.float64)


# (n, nnz) of each learned-start model made here (for the argument checks)
_WS_SHAPES: dict = {}


def bs_ws_create(n: int, row_ptr, col_idx) -> int:
    rp, ci = _host_i32(row_ptr), _host_i32(col_idx)
    h = C.c_void_p()
    _check(lib().bs_ws_create(n, ci.size, rp.ctypes.data, ci.ctypes.data if ci.size else None,
                              C.byref(h)), "bs_ws_create")
    _WS_SHAPES[h.value] = (int(n), int(ci.size))
    return h.value


def bs_ws_destroy(handle: int) -> None:
    _WS_SHAPES.pop(handle, None)
    _check(lib().bs_ws_destroy(handle), "bs_ws_destroy")


def check_ws_args(n: int, nnz: int, n_rows: int, *, values=None, b=None, x_prev=None,
                  x_next=None, x0=None, feat=None, delta=None, rows=None, y=None,
                  n_feat_rows: Optional[int] = None) -> None:
    """Element types and counts of a learned-start call on a model of n
    unknowns and nnz pattern entries; ``n_rows`` is the number of systems or
    samples the call processes (``n_feat_rows`` the rows of ``feat``/``delta``
    when ``rows`` selects among them).  Raises ValueError."""
    fr = n_rows if n_feat_rows is None else n_feat_rows
    for t, name, dt, cnt in ((values, "values", "f64", n_rows * nnz),
                             (b, "b", "f64", n_rows * n), (x_prev, "x_prev", "f64", n_rows * n),
                             (x_next, "x_next", "f64", n_rows * n), (x0, "x0", "f64", n_rows * n),
                             (feat, "feat", "f32", fr * 3 * n), (delta, "delta", "f32", fr * n),
                             (y, "y", "f32", n_rows * n)):
        _expect(t, name, dt, cnt, optional=True)
    _expect(rows, "rows", "i32", n_rows, optional=True, at_least=True)


def bs_ws_param_count(handle: int) -> int:
    c = C.c_int64()
    _check(lib().bs_ws_param_count(handle, C.byref(c)), "bs_ws_param_count")
    return c.value


def bs_ws_set_params(handle: int, params) -> None:
    p = _f32(params)
    if p.size != bs_ws_param_count(handle):
        raise ValueError("parameter vector has the wrong length")
    _check(lib().bs_ws_set_params(handle, p.ctypes.data), "bs_ws_set_params")


def bs_ws_get_params(handle: int) -> np.ndarray:
    p = np.empty(bs_ws_param_count(handle), np.float32)
    _check(lib().bs_ws_get_params(handle, p.ctypes.data), "bs_ws_get_params")
    return p


def bs_ws_features(handle: int, values, b, x_prev, feat, x_next=None, delta=None,
                   stream=None) -> None:
    n, nnz = _WS_SHAPES[handle]
    B = b.numel() // n
    check_ws_args(n, nnz, B, values=values, b=b, x_prev=x_prev, x_next=x_next, feat=feat,
                  delta=delta)
    if (x_next is None) != (delta is None):
        raise ValueError("x_next and delta go together")
    _check(lib().bs_ws_features(handle, b.shape[0], _ptr(values), _ptr(b), _ptr(x_prev),
                                _ptr(x_next), _ptr(feat), _ptr(delta), _stream(stream)),
           "bs_ws_features")


def bs_ws_fit_scaling(handle: int, feat, delta, stream=None) -> None:
    n, nnz = _WS_SHAPES[handle]
    check_ws_args(n, nnz, feat.shape[0], feat=feat, delta=delta)
    _check(lib().bs_ws_fit_scaling(handle, feat.shape[0], _ptr(feat), _ptr(delta),
                                   _stream(stream)), "bs_ws_fit_scaling")


def bs_ws_get_scaling(handle: int, n: int):
    mu, sd, sdd = np.empty(3 * n), np.empty(3 * n), np.empty(n)
    _check(lib().bs_ws_get_scaling(handle, mu.ctypes.data, sd.ctypes.data, sdd.ctypes.data),
           "bs_ws_get_scaling")
    return mu, sd, sdd


def bs_ws_set_scaling(handle: int, mu_f, sd_f, sd_d) -> None:
    mu, sd, sdd = _f64h(mu_f), _f64h(sd_f), _f64h(sd_d)
    _check(lib().bs_ws_set_scaling(handle, mu.ctypes.data, sd.ctypes.data, sdd.ctypes.data),
           "bs_ws_set_scaling")


def bs_ws_forward(handle: int, feat, y, rows=None, stream=None) -> None:
    n, nnz = _WS_SHAPES[handle]
    check_ws_args(n, nnz, y.shape[0], feat=feat, rows=rows, y=y,
                  n_feat_rows=feat.shape[0] if rows is not None else None)
    _check(lib().bs_ws_forward(handle, y.shape[0], _ptr(feat), _ptr(rows), _ptr(y),
                               _stream(stream)), "bs_ws_forward")


def bs_ws_grad(handle: int, feat, delta, grad, loss, rows=None, n_samples=None,
               stream=None) -> None:
    M = n_samples if n_samples is not None else (rows.shape[0] if rows is not None else feat.shape[0])
    n, nnz = _WS_SHAPES[handle]
    check_ws_args(n, nnz, M, feat=feat, delta=delta, rows=rows,
                  n_feat_rows=feat.shape[0])
    if rows is None and feat.shape[0] < M:
        raise ValueError(f"feat: {feat.shape[0]} rows, expected at least {M}")
    _expect(grad, "grad", "f32", bs_ws_param_count(handle))
    _expect(loss, "loss", "f32", 1, optional=True)
    _check(lib().bs_ws_grad(handle, M, _ptr(feat), _ptr(delta), _ptr(rows), _ptr(grad), _ptr(loss),
                            _stream(stream)), "bs_ws_grad")


def bs_ws_train_step(handle: int, feat, delta, lr: float, loss=None, rows=None, n_samples=None,
                     stream=None) -> None:
    M = n_samples if n_samples is not None else (rows.shape[0] if rows is not None else feat.shape[0])
    n, nnz = _WS_SHAPES[handle]
    check_ws_args(n, nnz, M, feat=feat, delta=delta, rows=rows,
                  n_feat_rows=feat.shape[0])
    if rows is None and feat.shape[0] < M:
        raise ValueError(f"feat: {feat.shape[0]} rows, expected at least {M}")
    _expect(loss, "loss", "f32", 1, optional=True)
    _check(lib().bs_ws_train_step(handle, M, _ptr(feat), _ptr(delta), _ptr(rows), float(lr),
                                  _ptr(loss), _stream(stream)), "bs_ws_train_step")


def bs_ws_train_step_noalloc(handle: int, feat, delta, lr: float, loss=None, rows=None,
                             n_samples=None, stream=None) -> None:
    """``bs_ws_train_step`` on the library's static workspace (no allocation;
    at most 2048 samples)."""
    M = n_samples if n_samples is not None else (rows.shape[0] if rows is not None else feat.shape[0])
    n, nnz = _WS_SHAPES[handle]
    check_ws_args(n, nnz, M, feat=feat, delta=delta, rows=rows,
                  n_feat_rows=feat.shape[0])
    if rows is None and feat.shape[0] < M:
        raise ValueError(f"feat: {feat.shape[0]} rows, expected at least {M}")
    _expect(loss, "loss", "f32", 1, optional=True)
    _check(lib().bs_ws_train_step_noalloc(handle, M, _ptr(feat), _ptr(delta), _ptr(rows),
                                          float(lr), _ptr(loss), _stream(stream)),
           "bs_ws_train_step_noalloc")


def bs_ws_infer(handle: int, values, b, x_prev, x0, stream=None) -> None:
    n, nnz = _WS_SHAPES[handle]
    check_ws_args(n, nnz, b.numel() // n, values=values, b=b, x_prev=x_prev, x0=x0)
    _check(lib().bs_ws_infer(handle, b.shape[0], _ptr(values), _ptr(b), _ptr(x_prev), _ptr(x0),
                             _stream(stream)), "bs_ws_infer")


def bs_ws_packed_bytes(n: int) -> int:
    return int(lib().bs_ws_packed_bytes(int(n)))


def bs_ws_pack(handle: int, weights, stream=None) -> None:
    """Copy the model's inference weights into the uint8 device tensor ``weights``
    (at least ``bs_ws_packed_bytes(n)`` bytes)."""
    n, _ = _WS_SHAPES[handle]
    if weights is None or weights.numel() * weights.element_size() < bs_ws_packed_bytes(n):
        raise ValueError("weights: smaller than bs_ws_packed_bytes(n)")
    _check(lib().bs_ws_pack(handle, _ptr(weights), weights.numel() * weights.element_size(),
                            _stream(stream)), "bs_ws_pack")


def bs_ws_infer_packed(weights, n: int, diag, b, x_prev, x0, stream=None) -> None:
    """x0 from packed weights and the diagonals ``diag`` [B][n] (float64)."""
    B = b.numel() // n
    if weights is None or weights.numel() * weights.element_size() < bs_ws_packed_bytes(n):
        raise ValueError("weights: smaller than bs_ws_packed_bytes(n)")
    for t, name in ((diag, "diag"), (b, "b"), (x_prev, "x_prev"), (x0, "x0")):
        _expect(t, name, "f64", B * n)
    _check(lib().bs_ws_infer_packed(B, int(n), _ptr(weights), _ptr(diag), _ptr(b), _ptr(x_prev),
                                    _ptr(x0), _stream(stream)), "bs_ws_infer_packed")


class WarmStartModel:
    """Owns a learned-initial-guess model (see ``bs_ws_create``)."""

    def __init__(self, n: int, row_ptr, col_idx):
        self.n = n
        self.handle = bs_ws_create(n, row_ptr, col_idx)
        self.param_count = bs_ws_param_count(self.handle)

    def __del__(self):
        if getattr(self, "handle", 0) and _lib is not None:
            _WS_SHAPES.pop(self.handle, None)
            _lib.bs_ws_destroy(self.handle)
            self.handle = 0
