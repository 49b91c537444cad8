"""CPU FP64 oracle for the batched Krylov solvers -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The HIP library never calls it, and it shares no code with it.

``liboracle.so`` is plain C (``oracle.c``); this module marshals numpy arrays
into it.  The MLP oracle for the learned initial guess lives in ``oracle.mlp``.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

from . import build as _build

CSR, ELL = 0, 1
CG, BICGSTAB, GMRES, TRSV_LOWER, TRSV_UPPER = 0, 1, 2, 3, 4
PREC_NONE, PREC_JACOBI, PREC_BLOCK_JACOBI, PREC_ILU = 0, 1, 2, 3
# ILU(0) with the column-oriented backward substitution (same operations,
# decreasing column order): the oracle's second order, for rounding studies
PREC_ILU_COL = 4
CONVERGED, MAX_ITER, BREAKDOWN, NONFINITE = 0, 1, 2, 3

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
        I, I64, D = C.c_int, C.c_int64, C.c_double
        L.or_batch_solve.argtypes = [I, I64, I, i32p, i32p, I, I, i32p, f64p, f64p, f64p,
                                     I, I, I, D, I, I, I, i32p, f64p, i32p, I]
        L.or_batch_solve.restype = I
        L.or_batch_solve_log.argtypes = [I, I64, I, i32p, i32p, I, I, i32p, f64p, f64p, f64p,
                                         I, I, I, D, I, I, I, i32p, f64p, i32p, I, i32p, I]
        L.or_batch_solve_log.restype = I
        L.or_batch_spmv.argtypes = [I, I64, I, i32p, i32p, I, I, i32p, f64p, f64p, f64p]
        L.or_batch_spmv.restype = None
        L.or_batch_true_residual.argtypes = [I, I64, I, i32p, i32p, I, I, i32p, f64p, f64p,
                                             f64p, f64p, I]
        L.or_batch_true_residual.restype = None
        L.or_batch_jacobi.argtypes = [I, I64, I, i32p, i32p, I, I, i32p, f64p, f64p]
        L.or_batch_jacobi.restype = None
        L.or_batch_block_jacobi.argtypes = [I, I64, I, i32p, i32p, I, I, i32p, f64p, I, f64p]
        L.or_batch_block_jacobi.restype = None
        L.or_batch_ilu0.argtypes = [I, I64, I, i32p, i32p, I, I, i32p, f64p, f64p, i32p]
        L.or_batch_ilu0.restype = None
        L.or_batch_ilu0_apply.argtypes = [I, I64, I, i32p, i32p, I, I, i32p, f64p, f64p,
                                          f64p, f64p, I]
        L.or_batch_ilu0_apply.restype = None
        L.or_dot.argtypes = [I, f64p, f64p]
        L.or_dot.restype = D
        L.or_csr_to_ell.argtypes = [I, i32p, i32p, C.c_void_p]
        L.or_csr_to_ell.restype = I
        L.or_csr_values_to_ell.argtypes = [I64, I, i32p, I, I, f64p, f64p]
        L.or_csr_values_to_ell.restype = None
        L.or_dense_solve.argtypes = [I, f64p, f64p]
        L.or_dense_solve.restype = I
        _lib = L
    return _lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


_DUMMY_I = np.zeros(1, np.int32)


class Pattern:
    """A shared pattern in CSR form, plus its ELL form built by the oracle."""

    def __init__(self, n: int, row_ptr, col_idx):
        self.n = int(n)
        self.row_ptr = _i32(row_ptr)
        self.col_idx = _i32(col_idx)
        self.nnz = int(self.col_idx.size)
        self.width, self.ell_col = csr_to_ell(self.n, self.row_ptr, self.col_idx)

    def args(self, fmt: int):
        if fmt == CSR:
            return (self.row_ptr, self.col_idx, self.nnz, 0, _DUMMY_I)
        return (_DUMMY_I if self.row_ptr is None else self.row_ptr, _DUMMY_I, 0,
                self.width, self.ell_col)


def csr_to_ell(n: int, row_ptr, col_idx):
    """BatchEll pattern from BatchCsr (Sec. 3.1): returns (width, ell_col[W*n])."""
    rp, ci = _i32(row_ptr), _i32(col_idx)
    w = lib().or_csr_to_ell(n, rp, ci, None)
    out = np.empty(max(w, 1) * n, np.int32)
    lib().or_csr_to_ell(n, rp, ci, out.ctypes.data)
    return w, out[: w * n]


def csr_values_to_ell(pat: Pattern, values) -> np.ndarray:
    v = _f64(values)
    B = v.shape[0]
    out = np.empty((B, pat.width * pat.n))
    lib().or_csr_values_to_ell(B, pat.n, pat.row_ptr, pat.nnz, pat.width, v, out)
    return out


def batch_solve(pat: Pattern, values, b, x0=None, fmt: int = CSR, solver: int = BICGSTAB,
                precond: int = PREC_JACOBI, tol: float = 1e-10, max_iter: int = 500,
                restart: int = 30, nthreads: Optional[int] = None, absolute: bool = False,
                block_size: int = 4):
    """Solve every system; ``values`` in the layout of ``fmt``.

    Stop test (Tab. 2): relative ||r|| <= tol ||b|| by default, absolute
    ||r|| <= tol with ``absolute``.  ``precond``: none, scalar Jacobi, block
    Jacobi with blocks of ``block_size`` consecutive rows, or ILU(0).
    ``solver`` TRSV_LOWER / TRSV_UPPER solve with the lower / upper triangle of
    A (diagonal included) by substitution.  Returns ``(x, iters, resid, status)``;
    ``resid`` is the true residual ||b - A x||, divided by ||b|| for the
    relative criterion.
    """
    v = _f64(values)
    b = _f64(b)
    B = b.shape[0]
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, order="C")
    iters = np.zeros(B, np.int32)
    resid = np.zeros(B)
    status = np.zeros(B, np.int32)
    nt = nthreads if nthreads is not None else (os.cpu_count() or 1)
    rp, ci, nnz, w, ec = pat.args(fmt)
    lib().or_batch_solve(fmt, B, pat.n, rp, ci, nnz, w, ec, v, b, x, solver, precond,
                         int(block_size), float(tol), int(bool(absolute)), int(max_iter),
                         int(restart), iters, resid, status, nt)
    return x, iters, resid, status


def batch_solve_log(pat: Pattern, values, b, x0=None, fmt: int = CSR, solver: int = BICGSTAB,
                    precond: int = PREC_JACOBI, tol: float = 1e-10, max_iter: int = 500,
                    log_cap: int = 16, nthreads: Optional[int] = None, absolute: bool = False,
                    block_size: int = 4):
    """``batch_solve`` (CG or BiCGSTAB) that also returns each system's restart
    log ``[B][log_cap]``: entry 0 counts the restarts from the true residual,
    entries 1.. hold the iteration count at which each one happened."""
    v = _f64(values)
    b = _f64(b)
    B = b.shape[0]
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, order="C")
    iters = np.zeros(B, np.int32)
    resid = np.zeros(B)
    status = np.zeros(B, np.int32)
    log = np.zeros((B, log_cap), np.int32)
    nt = nthreads if nthreads is not None else (os.cpu_count() or 1)
    rp, ci, nnz, w, ec = pat.args(fmt)
    lib().or_batch_solve_log(fmt, B, pat.n, rp, ci, nnz, w, ec, v, b, x, solver, precond,
                             int(block_size), float(tol), int(bool(absolute)), int(max_iter), 30,
                             iters, resid, status, nt, log, int(log_cap))
    return x, iters, resid, status, log


def batch_spmv(pat: Pattern, values, x, fmt: int = CSR) -> np.ndarray:
    v, x = _f64(values), _f64(x)
    y = np.empty_like(x)
    rp, ci, nnz, w, ec = pat.args(fmt)
    lib().or_batch_spmv(fmt, x.shape[0], pat.n, rp, ci, nnz, w, ec, v, x, y)
    return y


def true_residual(pat: Pattern, values, b, x, fmt: int = CSR,
                  nthreads: Optional[int] = None) -> np.ndarray:
    """``||b - A x|| / ||b||`` per system, computed by the oracle in FP64."""
    v, b, x = _f64(values), _f64(b), _f64(x)
    out = np.empty(b.shape[0])
    rp, ci, nnz, w, ec = pat.args(fmt)
    nt = nthreads if nthreads is not None else (os.cpu_count() or 1)
    lib().or_batch_true_residual(fmt, b.shape[0], pat.n, rp, ci, nnz, w, ec, v, b, x, out, nt)
    return out


def block_jacobi(pat: Pattern, values, bs: int, fmt: int = CSR) -> np.ndarray:
    """Block-Jacobi inverse rows ``[B][n][bs]``: row i holds entries (i, b0..b0+bs-1)
    of the inverse of its diagonal block (b0 = i - i % bs)."""
    v = _f64(values)
    B = v.shape[0]
    out = np.empty((B, pat.n, bs))
    rp, ci, nnz, w, ec = pat.args(fmt)
    lib().or_batch_block_jacobi(fmt, B, pat.n, rp, ci, nnz, w, ec, v, int(bs), out)
    return out


def ilu0(pat: Pattern, values, fmt: int = CSR):
    """ILU(0) factors ``[B][n][n]`` (dense, L strictly below the diagonal with
    unit diagonal implied, U on and above, zero off the pattern) and a flag per
    system that is False where a pivot was zero or an entry not finite."""
    v = _f64(values)
    B = v.shape[0]
    lu = np.empty((B, pat.n, pat.n))
    ok = np.empty(B, np.int32)
    rp, ci, nnz, w, ec = pat.args(fmt)
    lib().or_batch_ilu0(fmt, B, pat.n, rp, ci, nnz, w, ec, v, lu, ok)
    return lu, ok.astype(bool)


def ilu0_apply(pat: Pattern, values, lu, v_in, fmt: int = CSR, col: bool = False) -> np.ndarray:
    """z = (L U)^{-1} v per system with the factors returned by ``ilu0``
    (``col``: column-oriented backward substitution)."""
    v = _f64(values)
    x = _f64(v_in)
    z = np.empty_like(x)
    rp, ci, nnz, w, ec = pat.args(fmt)
    lib().or_batch_ilu0_apply(fmt, x.shape[0], pat.n, rp, ci, nnz, w, ec, v, _f64(lu), x, z,
                              int(bool(col)))
    return z


def jacobi(pat: Pattern, values, fmt: int = CSR) -> np.ndarray:
    v = _f64(values)
    d = np.empty((v.shape[0], pat.n))
    rp, ci, nnz, w, ec = pat.args(fmt)
    lib().or_batch_jacobi(fmt, v.shape[0], pat.n, rp, ci, nnz, w, ec, v, d)
    return d


def dot(a, b) -> float:
    a, b = _f64(a), _f64(b)
    return float(lib().or_dot(a.size, a, b))


def dense_solve(A, b) -> np.ndarray:
    """Own dense LU with partial pivoting; raises on a zero pivot."""
    A = np.array(A, dtype=np.float64, order="C")
    x = np.array(b, dtype=np.float64, order="C")
    if lib().or_dense_solve(A.shape[0], A, x) != 0:
        raise np.linalg.LinAlgError("zero pivot")
    return x


def to_dense(pat: Pattern, values_one) -> np.ndarray:
    """Dense matrix of one system from its CSR values (test helper)."""
    A = np.zeros((pat.n, pat.n))
    rows = np.repeat(np.arange(pat.n), np.diff(pat.row_ptr))
    A[rows, pat.col_idx] = values_one
    return A
