"""Seeded synthetic batches of small sparse systems that share one pattern.

This module only *draws inputs*: sparsity patterns, matrix values, right-hand
sides and drifting time-step sequences.  It contains none of the solver's
arithmetic (no products, no norms, no solves), so both the CPU oracle and the
GPU path can take their inputs from it without sharing any method code.

The shapes follow the workloads the paper evaluates (Sec. 4.1, Tab. 3): a
3-point-stencil family whose size can grow, and n = 22..144 chemistry
Jacobians from a reacting-flow code, which share one pattern across 2^17 cells.
The chemistry matrices themselves are not available, so a random pattern of the
same size and a stiff ``I - gamma*J`` value model stand in for them.

All generators use ``numpy.random.default_rng(seed)`` (PCG64) and draw in a fixed,
documented order, so a batch is reproducible bit for bit from its seed.
Large batches are drawn in chunks from the same stream, which yields the same
numbers as one big draw.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Iterator, Optional

import numpy as np

__all__ = [
    "Batch",
    "VarBatch",
    "tridiag_stencil",
    "chem_jacobian",
    "chem_pattern",
    "collision_stencil",
    "uneven_banded",
    "chem_trajectory",
    "grid9_pattern",
    "MECHANISMS",
    "mechanism_pattern",
    "mechanism_batch",
]

_CHUNK = 8192  # systems per draw chunk; the stream is consumed sequentially


@dataclass
class Batch:
    """A batch of ``n_batch`` systems of ``n`` rows sharing one CSR pattern.

    ``values`` is system-major, ``[n_batch][nnz]`` in CSR order of the shared
    pattern; ``b`` and ``x0`` are ``[n_batch][n]``.
    """

    name: str
    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col_idx: np.ndarray  # int32 [nnz]
    values: np.ndarray  # float64 [n_batch][nnz]
    b: np.ndarray  # float64 [n_batch][n]
    x0: np.ndarray  # float64 [n_batch][n]
    meta: dict = field(default_factory=dict)

    @property
    def n_batch(self) -> int:
        return int(self.values.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    def subset(self, idx) -> "Batch":
        idx = np.asarray(idx)
        return Batch(self.name, self.n, self.row_ptr, self.col_idx,
                     np.ascontiguousarray(self.values[idx]),
                     np.ascontiguousarray(self.b[idx]),
                     np.ascontiguousarray(self.x0[idx]), dict(self.meta))


def _csr_from_mask(mask: np.ndarray):
    rows, cols = np.nonzero(mask)  # row-major, columns ascending in each row
    n = mask.shape[0]
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    return row_ptr, cols.astype(np.int32)


def _uniform(rng: np.random.Generator, shape, chunk_axis0: bool = True) -> np.ndarray:
    """``rng.random(shape)`` drawn in chunks along axis 0 (identical stream)."""
    shape = tuple(int(s) for s in shape)
    if not chunk_axis0 or shape[0] <= _CHUNK:
        return rng.random(shape)
    out = np.empty(shape)
    for s in range(0, shape[0], _CHUNK):
        e = min(shape[0], s + _CHUNK)
        out[s:e] = rng.random((e - s,) + shape[1:])
    return out


# --------------------------------------------------------------------------
# 3-point stencil family (Sec. 4.2): tridiagonal, diagonally dominant.
# --------------------------------------------------------------------------
def tridiag_stencil(n_batch: int = 64, n: int = 32, seed: int = 0,
                    diag_lo: float = 4.0, off_center: float = -1.0,
                    off_spread: float = 0.1) -> Batch:
    """Tridiagonal batch: ``a_ii = 4+U(0,1)``, ``a_{i,i+-1} = -1+U(-0.1,0.1)``.

    Draw order: values ``rng.random((B, nnz))`` in CSR order, then
    ``b = 2*rng.random((B, n)) - 1``.  x0 = 0.
    """
    mask = np.zeros((n, n), dtype=bool)
    i = np.arange(n)
    mask[i, i] = True
    mask[i[1:], i[1:] - 1] = True
    mask[i[:-1], i[:-1] + 1] = True
    row_ptr, col_idx = _csr_from_mask(mask)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    is_diag = rows == col_idx
    rng = np.random.default_rng(seed)
    u = _uniform(rng, (n_batch, col_idx.size))
    values = np.where(is_diag[None, :], diag_lo + u,
                      off_center + off_spread * (2.0 * u - 1.0))
    b = 2.0 * _uniform(rng, (n_batch, n)) - 1.0
    return Batch("tridiag_stencil", n, row_ptr, col_idx, values, b,
                 np.zeros((n_batch, n)), {"seed": seed})


# --------------------------------------------------------------------------
# Chemistry-Jacobian stand-in (Sec. 4.3, Tab. 3 sizes): A = I - gamma * J.
# --------------------------------------------------------------------------
def chem_pattern(n: int = 54, fill: float = 0.35, seed: int = 0,
                 rng: Optional[np.random.Generator] = None):
    """Full diagonal plus Bernoulli(``fill``) off-diagonal entries.

    Draws ``rng.random((n, n))`` once (the first draw of the stream).
    """
    rng = np.random.default_rng(seed) if rng is None else rng
    mask = rng.random((n, n)) < fill
    np.fill_diagonal(mask, True)
    return _csr_from_mask(mask)


def _log_uniform_signed(d: np.ndarray, lo_exp: float, hi_exp: float) -> np.ndarray:
    sign = np.where(d[..., 0] < 0.5, -1.0, 1.0)
    return sign * np.power(10.0, lo_exp + (hi_exp - lo_exp) * d[..., 1])


def chem_jacobian(n_batch: int = 1 << 17, n: int = 54, fill: float = 0.35,
                  gamma: float = 1e-6, seed: int = 0) -> Batch:
    """``A = I - gamma*J``; ``J_ij = +-10^U(-3,3)`` on a shared random pattern.

    Draw order: pattern ``rng.random((n, n))``; then ``rng.random((B, nnz, 2))``
    as (sign, exponent) pairs per stored entry in CSR order; then
    ``b = 2*rng.random((B, n)) - 1``.  x0 = 0.
    """
    rng = np.random.default_rng(seed)
    row_ptr, col_idx = chem_pattern(n, fill, rng=rng)
    nnz = col_idx.size
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    is_diag = rows == col_idx
    values = np.empty((n_batch, nnz))
    for s in range(0, n_batch, _CHUNK):
        e = min(n_batch, s + _CHUNK)
        J = _log_uniform_signed(rng.random((e - s, nnz, 2)), -3.0, 3.0)
        values[s:e] = -gamma * J
        values[s:e, is_diag] += 1.0
    b = 2.0 * _uniform(rng, (n_batch, n)) - 1.0
    return Batch("chem_jacobian", n, row_ptr, col_idx, values, b,
                 np.zeros((n_batch, n)), {"seed": seed, "gamma": gamma, "fill": fill})


# --------------------------------------------------------------------------
# Stand-ins for the reacting-flow mechanisms of Tab. 3: their sizes, their
# counts of distinct matrices, replicated over the batch.
# --------------------------------------------------------------------------
# name: (distinct matrices, rows, stored entries per matrix), Tab. 3
MECHANISMS = {
    "drm19": (67, 22, 438),
    "gri12": (73, 33, 978),
    "gri30": (90, 54, 2560),
    "dodecane_lu": (78, 54, 2332),
    "isooctane": (72, 144, 6135),
}


def mechanism_pattern(n: int, nnz: int, rng: np.random.Generator):
    """Full diagonal plus ``nnz - n`` off-diagonal positions drawn uniformly
    without replacement: one ``rng.permutation`` of the n(n-1) off-diagonal
    positions (row-major order), whose first ``nnz - n`` are kept."""
    if not n <= nnz <= n * n:
        raise ValueError("need n <= nnz <= n^2")
    off = np.flatnonzero(~np.eye(n, dtype=bool))
    pick = rng.permutation(off.size)[: nnz - n]
    mask = np.eye(n, dtype=bool)
    mask.flat[off[pick]] = True
    return _csr_from_mask(mask)


def mechanism_batch(name: str, n_batch: int = 1 << 17, gamma: float = 1e-6,
                    seed: int = 0) -> Batch:
    """One Tab. 3 input: its ``unique`` distinct systems, ``A = I - gamma*J``
    (``J_ij = +-10^U(-3,3)``, the chemistry model above) on a shared pattern
    of the table's size, each with its own b ~ U(-1,1), replicated over the
    batch in turn (system s is distinct system s mod unique), as the paper
    fills its batches from the matrices of a few cells (Sec. 4.1).

    Draw order: the pattern's permutation; ``rng.random((unique, nnz, 2))``
    as (sign, exponent) pairs per stored entry in CSR order; then
    ``2*rng.random((unique, n)) - 1`` for b.  x0 = 0.
    """
    unique, n, nnz = MECHANISMS[name]
    rng = np.random.default_rng(seed)
    row_ptr, col_idx = mechanism_pattern(n, nnz, rng)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    is_diag = rows == col_idx
    vu = -gamma * _log_uniform_signed(rng.random((unique, nnz, 2)), -3.0, 3.0)
    vu[:, is_diag] += 1.0
    bu = 2.0 * rng.random((unique, n)) - 1.0
    reps = -(-n_batch // unique)
    values = np.ascontiguousarray(np.tile(vu, (reps, 1))[:n_batch])
    b = np.ascontiguousarray(np.tile(bu, (reps, 1))[:n_batch])
    return Batch(name, n, row_ptr, col_idx, values, b, np.zeros((n_batch, n)),
                 {"seed": seed, "gamma": gamma, "unique": unique})


# --------------------------------------------------------------------------
# Collision-operator stand-in: 9-point nonsymmetric stencil on a 2D grid.
# --------------------------------------------------------------------------
def grid9_pattern(nx: int = 32, ny: int = 31):
    """9-point, non-periodic stencil on an ``nx`` x ``ny`` grid (x fastest).

    Returns ``row_ptr, col_idx, dx, dy`` with the neighbour offset of every
    stored entry (0, 0 on the diagonal).  Columns ascend within each row.
    """
    n = nx * ny
    rp = [0]
    cols, dxs, dys = [], [], []
    for y in range(ny):
        for x in range(nx):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    xx, yy = x + dx, y + dy
                    if 0 <= xx < nx and 0 <= yy < ny:
                        cols.append(yy * nx + xx)
                        dxs.append(dx)
                        dys.append(dy)
            rp.append(len(cols))
    return (np.asarray(rp, np.int32), np.asarray(cols, np.int32),
            np.asarray(dxs, np.int8), np.asarray(dys, np.int8))


def collision_stencil(n_batch: int = 4096, nx: int = 32, ny: int = 31,
                      seed: int = 0, dominance: float = 1.2) -> Batch:
    """Diagonally dominant 9-point operator with a random advection-like skew.

    Per system ``(u_x, u_y) ~ U(-1,1)^2``; off-diagonal
    ``w = -(1 + 0.5 (dx u_x + dy u_y)) * c * (1 + 0.05 U(-1,1))`` with ``c = 1``
    for axis and ``0.5`` for diagonal neighbours; ``a_ii = dominance * sum|w|``.
    Draw order: ``rng.random((B, 2))`` for u, ``rng.random((B, nnz))`` per stored
    entry (the diagonal's draw is unused), then ``b = 2*rng.random((B,n)) - 1``.
    """
    rng = np.random.default_rng(seed)
    row_ptr, col_idx, dx, dy = grid9_pattern(nx, ny)
    n = nx * ny
    nnz = col_idx.size
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    is_diag = (dx == 0) & (dy == 0)
    c = np.where((dx != 0) & (dy != 0), 0.5, 1.0)
    u = 2.0 * rng.random((n_batch, 2)) - 1.0
    values = np.empty((n_batch, nnz))
    for s in range(0, n_batch, _CHUNK):
        e = min(n_batch, s + _CHUNK)
        noise = 2.0 * rng.random((e - s, nnz)) - 1.0
        skew = 1.0 + 0.5 * (dx[None, :] * u[s:e, 0:1] + dy[None, :] * u[s:e, 1:2])
        w = -skew * c[None, :] * (1.0 + 0.05 * noise)
        w[:, is_diag] = 0.0
        absw = np.zeros((e - s, n))
        np.add.at(absw.T, rows, np.abs(w).T)
        w[:, is_diag] = dominance * absw
        values[s:e] = w
    b = 2.0 * _uniform(rng, (n_batch, n)) - 1.0
    return Batch("collision_stencil", n, row_ptr, col_idx, values, b,
                 np.zeros((n_batch, n)), {"seed": seed, "nx": nx, "ny": ny})


# --------------------------------------------------------------------------
# Uneven batch: per-system size and band, patterns deduplicated.
# --------------------------------------------------------------------------
@dataclass
class VarBatch:
    """Systems of different sizes; each references one of ``n_patterns``.

    ``rowptr_all``/``col_all`` concatenate the distinct CSR patterns;
    ``pat_rowptr_off[p]``/``pat_col_off[p]`` locate pattern ``p``.  Values,
    ``b`` and ``x0`` are concatenated system after system, located by
    ``val_off`` and ``row_off`` (length ``n_batch+1``).
    """

    sys_rows: np.ndarray  # int32 [B]
    pat_id: np.ndarray  # int32 [B]
    pat_rows: np.ndarray  # int32 [P]
    pat_rowptr_off: np.ndarray  # int64 [P]
    pat_col_off: np.ndarray  # int64 [P]
    rowptr_all: np.ndarray  # int32
    col_all: np.ndarray  # int32
    row_off: np.ndarray  # int64 [B+1]
    val_off: np.ndarray  # int64 [B+1]
    values: np.ndarray  # float64 [sum nnz]
    b: np.ndarray  # float64 [sum n]
    x0: np.ndarray  # float64 [sum n]
    meta: dict = field(default_factory=dict)

    @property
    def n_batch(self) -> int:
        return int(self.sys_rows.shape[0])

    def system(self, s: int):
        """(row_ptr, col_idx, values, b, x0) of system ``s`` (views)."""
        p = int(self.pat_id[s])
        n = int(self.sys_rows[s])
        ro = int(self.pat_rowptr_off[p])
        rp = self.rowptr_all[ro:ro + n + 1]
        co = int(self.pat_col_off[p])
        ci = self.col_all[co:co + int(rp[-1])]
        v = self.values[self.val_off[s]:self.val_off[s + 1]]
        r0, r1 = self.row_off[s], self.row_off[s + 1]
        return rp, ci, v, self.b[r0:r1], self.x0[r0:r1]

    def ell(self, extra_slots: int = 0, pad_value: float = 0.0):
        """The same batch in the ELL layout: per pattern ``w = longest row +
        extra_slots`` slots, slot-major columns ``[w][n]`` with -1 padding, and
        every system's values ``[w][n]`` in the same layout (padding slots hold
        ``pad_value``).  Returns ``(pat_rows, pat_width, pat_col_off, col_all,
        pat_id, values)``; a re-layout only, entry k of row i stays slot k."""
        P = self.pat_rows.size
        widths = np.empty(P, np.int32)
        cols, offs, slot_of = [], [], []
        at = 0
        for p in range(P):
            n = int(self.pat_rows[p])
            ro, co = int(self.pat_rowptr_off[p]), int(self.pat_col_off[p])
            rp = self.rowptr_all[ro:ro + n + 1].astype(np.int64)
            ci = self.col_all[co:co + int(rp[-1])]
            lens = np.diff(rp)
            w = int(lens.max(initial=0)) + extra_slots
            widths[p] = w
            rows = np.repeat(np.arange(n), lens)
            k = np.arange(rp[-1]) - rp[rows]
            dst = k * n + rows  # slot-major position of every CSR entry
            c = np.full(w * n, -1, np.int32)
            c[dst] = ci
            cols.append(c)
            offs.append(at)
            slot_of.append(dst)
            at += w * n
        val_off = np.zeros(self.n_batch + 1, np.int64)
        sizes = np.asarray([widths[p] * self.pat_rows[p] for p in self.pat_id], np.int64)
        val_off[1:] = np.cumsum(sizes)
        vals = np.full(int(val_off[-1]), pad_value, np.float64)
        for s in range(self.n_batch):
            p = int(self.pat_id[s])
            vals[val_off[s] + slot_of[p]] = self.values[self.val_off[s]:self.val_off[s + 1]]
        return (self.pat_rows.copy(), widths, np.asarray(offs, np.int64),
                np.concatenate(cols) if cols else np.zeros(0, np.int32), self.pat_id.copy(), vals)


def _band_pattern(n: int, kl: int, ku: int):
    rp = np.zeros(n + 1, dtype=np.int32)
    cols = []
    for i in range(n):
        lo, hi = max(0, i - kl), min(n - 1, i + ku)
        cols.extend(range(lo, hi + 1))
        rp[i + 1] = len(cols)
    return rp, np.asarray(cols, dtype=np.int32)


def uneven_banded(n_batch: int = 100_000, n_min: int = 16, n_max: int = 1024,
                  w_min: int = 5, w_max: int = 9, seed: int = 0,
                  dominance: float = 1.2) -> VarBatch:
    """Banded nonsymmetric systems with ``n ~ U{n_min..n_max}``, width ``U{w_min..w_max}``.

    Per system: band with ``kl = (w-1)//2`` sub- and ``ku = w-1-kl`` super-diagonals,
    a skew ``s ~ U(-1,1)``; off-diagonal ``-(1 + 0.3 s sgn(j-i)) (1 + 0.1 U(-1,1))``;
    ``a_ii = dominance * sum|off|``.  Draw order: ``n`` (``rng.integers``), ``w``,
    ``s`` (``rng.random``), then one ``rng.random`` per stored entry of every
    system in system order, then ``b`` per system in system order.
    """
    rng = np.random.default_rng(seed)
    sys_rows = rng.integers(n_min, n_max + 1, size=n_batch).astype(np.int32)
    widths = rng.integers(w_min, w_max + 1, size=n_batch)
    skew = 2.0 * rng.random(n_batch) - 1.0
    kl = (widths - 1) // 2
    ku = widths - 1 - kl
    keys = {}
    pat_id = np.empty(n_batch, dtype=np.int32)
    pats = []
    for s in range(n_batch):
        k = (int(sys_rows[s]), int(kl[s]), int(ku[s]))
        if k not in keys:
            keys[k] = len(pats)
            pats.append(_band_pattern(*k))
        pat_id[s] = keys[k]
    pat_rows = np.asarray([p[0].size - 1 for p in pats], dtype=np.int32)
    rp_sizes = np.asarray([p[0].size for p in pats], dtype=np.int64)
    ci_sizes = np.asarray([p[1].size for p in pats], dtype=np.int64)
    pat_rowptr_off = np.concatenate([[0], np.cumsum(rp_sizes)[:-1]]).astype(np.int64)
    pat_col_off = np.concatenate([[0], np.cumsum(ci_sizes)[:-1]]).astype(np.int64)
    rowptr_all = np.concatenate([p[0] for p in pats]).astype(np.int32)
    col_all = np.concatenate([p[1] for p in pats]).astype(np.int32)
    nnz_s = ci_sizes[pat_id]
    val_off = np.concatenate([[0], np.cumsum(nnz_s)]).astype(np.int64)
    row_off = np.concatenate([[0], np.cumsum(sys_rows.astype(np.int64))]).astype(np.int64)
    total = int(val_off[-1])
    values = np.empty(total)
    # per-entry row index / signed offset, per pattern, cached
    pat_geo = []
    for rp, ci in pats:
        rows = np.repeat(np.arange(rp.size - 1), np.diff(rp))
        pat_geo.append((rows, np.sign(ci - rows), ci == rows))
    for s0 in range(0, n_batch, 4096):
        s1 = min(n_batch, s0 + 4096)
        noise = 2.0 * rng.random(int(val_off[s1] - val_off[s0])) - 1.0
        for s in range(s0, s1):
            rows, sg, dg = pat_geo[pat_id[s]]
            lo, hi = val_off[s] - val_off[s0], val_off[s + 1] - val_off[s0]
            w = -(1.0 + 0.3 * skew[s] * sg) * (1.0 + 0.1 * noise[lo:hi])
            w[dg] = 0.0
            absw = np.bincount(rows, weights=np.abs(w), minlength=int(sys_rows[s]))
            w[dg] = dominance * absw
            values[val_off[s]:val_off[s + 1]] = w
    b = 2.0 * rng.random(int(row_off[-1])) - 1.0
    return VarBatch(sys_rows, pat_id, pat_rows, pat_rowptr_off, pat_col_off,
                    rowptr_all, col_all, row_off, val_off, values, b,
                    np.zeros_like(b), {"seed": seed})


# --------------------------------------------------------------------------
# Drifting time-step sequence on the chemistry pattern (learned warm start).
# --------------------------------------------------------------------------
def chem_trajectory(n_batch: int = 1 << 16, n: int = 54, steps: int = 64,
                    fill: float = 0.35, gamma0: float = 1e-6, drift: float = 0.01,
                    seed: int = 0, b_drift: float = 0.0) -> Iterator[Batch]:
    """Yield ``steps`` batches ``A_t = I - gamma_t J_t``.

    ``gamma_t = gamma_{t-1} (1 + drift U(-1,1))`` per system and
    ``J_t = J_{t-1} o (1 + drift U(-1,1))`` per stored entry.  ``b`` is fixed
    per system when ``b_drift = 0``; otherwise ``b_t = b_{t-1} o (1 + b_drift
    U(-1,1))`` per component (a right-hand side that moves along the
    sequence).  Draw order: pattern; ``J_0`` as (sign, exponent) pairs
    ``(B, nnz, 2)``; ``b (B, n)``; then for every ``t >= 1``: ``rng.random(B)``
    for gamma, ``rng.random((B, nnz))`` for J, and with ``b_drift > 0``
    ``rng.random((B, n))`` for b.  Each yielded batch owns its arrays.
    """
    rng = np.random.default_rng(seed)
    row_ptr, col_idx = chem_pattern(n, fill, rng=rng)
    nnz = col_idx.size
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    is_diag = rows == col_idx
    J = np.empty((n_batch, nnz))
    for s in range(0, n_batch, _CHUNK):
        e = min(n_batch, s + _CHUNK)
        J[s:e] = _log_uniform_signed(rng.random((e - s, nnz, 2)), -3.0, 3.0)
    b = 2.0 * _uniform(rng, (n_batch, n)) - 1.0
    gam = np.full(n_batch, gamma0)
    for t in range(steps):
        if t > 0:
            gam = gam * (1.0 + drift * (2.0 * rng.random(n_batch) - 1.0))
            J *= 1.0 + drift * (2.0 * _uniform(rng, (n_batch, nnz)) - 1.0)
            if b_drift > 0.0:
                b = b * (1.0 + b_drift * (2.0 * _uniform(rng, (n_batch, n)) - 1.0))
        values = -gam[:, None] * J
        values[:, is_diag] += 1.0
        yield Batch("chem_trajectory", n, row_ptr, col_idx, values, b.copy(),
                    np.zeros((n_batch, n)), {"seed": seed, "t": t, "b_drift": b_drift})


# --------------------------------------------------------------------------
# Initial weights of the learned-initial-guess network.
# --------------------------------------------------------------------------
def mlp_init(n: int, hidden: int = 256, seed: int = 0, gain: float = 1.0) -> np.ndarray:
    """Flat FP32 parameter vector (W1 [3n][h], b1, W2 [h][h], b2, W3 [h][n], b3):
    weights ``gain * N(0, 2 / fan_in)`` (He normal), biases zero.  Draw order:
    W1, W2, W3, each as one ``rng.standard_normal`` call."""
    rng = np.random.default_rng(seed)
    F = 3 * n
    parts = []
    for fan_in, fan_out in ((F, hidden), (hidden, hidden), (hidden, n)):
        w = rng.standard_normal((fan_in, fan_out)) * (gain * np.sqrt(2.0 / fan_in))
        parts += [w.ravel(), np.zeros(fan_out)]
    return np.concatenate(parts).astype(np.float32)
