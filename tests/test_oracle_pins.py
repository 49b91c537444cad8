"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test fixes the oracle to mathematics or to an independent implementation:
exact integer arithmetic, closed forms, textbook optimality properties checked
by brute force on tiny systems, dense LU, and scipy's own CG/BiCGSTAB run for a
fixed number of iterations.  A dropped term, a wrong sign or a transposed
operand in any solver step fails at least one of them.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
from paper_2308_08417_amd import workloads as W

EPS = np.finfo(np.float64).eps


def rand_pattern(rng, n, fill, diag=True, empty_rows=()):
    mask = rng.random((n, n)) < fill
    if diag:
        np.fill_diagonal(mask, True)
    for r in empty_rows:
        mask[r, :] = False
    rows, cols = np.nonzero(mask)
    rp = np.zeros(n + 1, np.int32)
    np.add.at(rp, rows + 1, 1)
    return np.cumsum(rp).astype(np.int32), cols.astype(np.int32)


def csr_dense(n, rp, ci, vals):
    A = np.zeros((n, n), dtype=vals.dtype)
    rows = np.repeat(np.arange(n), np.diff(rp))
    A[rows, ci] = vals
    return A


def batch_from_dense(As, bs):
    """Shared pattern = union of nonzeros (plus diagonal); CSR values per system."""
    n = As.shape[1]
    mask = np.any(As != 0, axis=0) | np.eye(n, dtype=bool)
    rows, cols = np.nonzero(mask)
    rp = np.zeros(n + 1, np.int32)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    vals = As[:, rows, cols]
    return O.Pattern(n, rp, cols.astype(np.int32)), np.ascontiguousarray(vals), np.ascontiguousarray(bs)


# --------------------------------------------------------------- SpMV / ELL
@pytest.mark.parametrize("n,fill,empty", [(1, 1.0, ()), (7, 0.4, (3,)), (64, 0.3, ()), (97, 0.1, (0, 96))])
def test_spmv_integer_exact(n, fill, empty):
    rng = np.random.default_rng(n)
    rp, ci = rand_pattern(rng, n, fill, empty_rows=empty)
    P = O.Pattern(n, rp, ci)
    B = 5
    vals = rng.integers(-1024, 1025, size=(B, P.nnz)).astype(np.float64)
    x = rng.integers(-1024, 1025, size=(B, n)).astype(np.float64)
    y = O.batch_spmv(P, vals, x)
    for s in range(B):  # every product and sum is exact in FP64 at these sizes
        A = csr_dense(n, rp, ci, vals[s].astype(np.int64))
        assert np.array_equal(y[s], (A @ x[s].astype(np.int64)).astype(np.float64))
    ev = O.csr_values_to_ell(P, vals)
    assert np.array_equal(O.batch_spmv(P, ev, x, fmt=O.ELL), y)


def test_ell_layout_reconstructs_matrix():
    rng = np.random.default_rng(3)
    n = 23
    rp, ci = rand_pattern(rng, n, 0.3, empty_rows=(5,))
    P = O.Pattern(n, rp, ci)
    assert P.width == int(np.diff(rp).max())
    vals = rng.random((2, P.nnz))
    ev = O.csr_values_to_ell(P, vals).reshape(2, P.width, n)
    ec = P.ell_col.reshape(P.width, n)
    for s in range(2):
        A = np.zeros((n, n))
        for sl in range(P.width):
            for i in range(n):
                if ec[sl, i] >= 0:
                    A[i, ec[sl, i]] += ev[s, sl, i]
                else:
                    assert ev[s, sl, i] == 0.0
        assert np.array_equal(A, csr_dense(n, rp, ci, vals[s]))
    # padding only at the end of each row
    for i in range(n):
        col = ec[:, i]
        k = int(np.sum(col >= 0))
        assert np.all(col[:k] >= 0) and np.all(col[k:] == -1)


def test_storage_formulas(golden_dir):
    """Sec. 3.1 storage list on the Tab. 3 shapes: CSR stores B*nnz values plus
    (n+1)+nnz indexes; ELL stores B*W*n values (the padded count) plus W*n indexes."""
    import json, os
    g = json.load(open(os.path.join(golden_dir, "tab3_shapes.json")))
    B = g["batch"]
    for e in g["inputs"]:
        n, nnz = e["n"], e["nnz"]
        rng = np.random.default_rng(0)
        # a pattern with exactly nnz entries, full diagonal
        off = rng.permutation(n * n - n)[: nnz - n]
        mask = np.eye(n, dtype=bool)
        idx = np.flatnonzero(~np.eye(n, dtype=bool).ravel())[off]
        mask.ravel()[idx] = True
        rows, cols = np.nonzero(mask)
        rp = np.zeros(n + 1, np.int32)
        np.add.at(rp, rows + 1, 1)
        rp = np.cumsum(rp).astype(np.int32)
        P = O.Pattern(n, rp, cols.astype(np.int32))
        assert P.nnz == nnz
        csr_vals, csr_idx = B * nnz, (n + 1) + nnz
        ell_vals, ell_idx = B * P.width * n, P.width * n
        assert csr_vals == B * e["nnz"] and csr_idx == n + 1 + e["nnz"]
        assert ell_vals >= csr_vals and ell_idx == P.ell_col.size


# --------------------------------------------------------------- dot / Jacobi
def test_dot_against_fsum():
    rng = np.random.default_rng(1)
    for n in (1, 10, 1000):
        a, b = rng.standard_normal(n), rng.standard_normal(n)
        exact = math.fsum(a * b)  # products of doubles are exact in fsum's sense only up to rounding
        ref = math.fsum([float(x) * float(y) for x, y in zip(a, b)])
        bound = n * EPS * float(np.sum(np.abs(a * b))) + 1e-300
        assert abs(O.dot(a, b) - ref) <= bound
        assert abs(exact - ref) <= bound
    ai = rng.integers(-2**20, 2**20, 500).astype(np.float64)
    bi = rng.integers(-2**20, 2**20, 500).astype(np.float64)
    assert O.dot(ai, bi) == float(np.dot(ai.astype(np.int64), bi.astype(np.int64)))


def test_jacobi_closed_form():
    n = 6
    rp = np.array([0, 2, 3, 4, 5, 6, 7], np.int32)
    ci = np.array([0, 1, 2, 3, 4, 0, 5], np.int32)  # row 1: no diagonal stored; row 5 has col 0
    P = O.Pattern(n, rp, ci)
    vals = np.array([[4.0, 1.0, 3.0, 0.0, -8.0, 2.0, 0.5]])
    d = O.jacobi(P, vals)[0]
    # row0 a=4, row1 absent->1, row2 col2? row 2 stores col 3 -> absent -> 1
    assert d[0] == 0.25 and d[1] == 1.0
    assert d[2] == 1.0 and d[3] == 1.0 and d[4] == 1.0  # rows 2..4 store off-diagonals only
    assert d[5] == 2.0
    ev = O.csr_values_to_ell(P, vals)
    assert np.array_equal(O.jacobi(P, ev, fmt=O.ELL), O.jacobi(P, vals))


# --------------------------------------------------------------- dense LU
def test_dense_lu_matches_lapack():
    rng = np.random.default_rng(2)
    for n in (1, 2, 5, 33):
        A = rng.standard_normal((n, n)) + n * np.eye(n) * 0.1
        A[0, 0] = 0.0 if n > 1 else 1.0  # forces a row swap
        b = rng.standard_normal(n)
        x = O.dense_solve(A, b)
        xr = scipy.linalg.solve(A, b)
        k = np.linalg.cond(A)
        assert np.linalg.norm(x - xr) <= 1e3 * k * EPS * np.linalg.norm(xr)
    with pytest.raises(np.linalg.LinAlgError):
        O.dense_solve(np.zeros((3, 3)), np.ones(3))


# --------------------------------------------------------------- closed forms
@pytest.mark.parametrize("solver", [O.CG, O.BICGSTAB, O.GMRES])
def test_diagonal_system_one_iteration(solver):
    """With scalar Jacobi a diagonal A gives M A = I: one iteration, x = b / a."""
    rng = np.random.default_rng(4)
    n, B = 9, 4
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    P = O.Pattern(n, rp, ci)
    vals = 1.0 + 9.0 * rng.random((B, n))
    b = rng.standard_normal((B, n))
    x, it, res, st = O.batch_solve(P, vals, b, solver=solver)
    assert np.all(st == O.CONVERGED) and np.all(it == 1)
    assert np.allclose(x, b / vals, rtol=4 * EPS, atol=0)


@pytest.mark.parametrize("solver", [O.CG, O.BICGSTAB, O.GMRES])
def test_one_by_one(solver):
    P = O.Pattern(1, np.array([0, 1], np.int32), np.array([0], np.int32))
    vals = np.array([[3.0], [-0.5], [7.25]])
    b = np.array([[1.0], [2.0], [-3.0]])
    for prec in (O.PREC_NONE, O.PREC_JACOBI):
        x, it, res, st = O.batch_solve(P, vals, b, solver=solver, precond=prec)
        assert np.all(it == 1) and np.all(st == O.CONVERGED)
        assert np.allclose(x, b / vals, rtol=2 * EPS, atol=0)


@pytest.mark.parametrize("solver", [O.CG, O.BICGSTAB, O.GMRES])
def test_distinct_eigenvalues_bound(solver):
    """Without preconditioning, Krylov methods on a diagonalisable A with k distinct
    eigenvalues terminate within k steps (exact arithmetic; k steps + rounding here)."""
    n = 40
    rp = np.arange(n + 1, dtype=np.int32)
    ci = np.arange(n, dtype=np.int32)
    P = O.Pattern(n, rp, ci)
    rng = np.random.default_rng(5)
    for k, eig in ((2, [1.0, 2.0]), (3, [1.0, 2.5, 4.0])):
        vals = np.asarray([eig[i % k] for i in range(n)])[None, :]
        b = rng.standard_normal((1, n))
        x, it, res, st = O.batch_solve(P, vals, b, solver=solver, precond=O.PREC_NONE)
        assert st[0] == O.CONVERGED and it[0] <= k


def test_cg_laplacian_eigenvector_rhs():
    """1D Laplacian tridiag(-1,2,-1): eigenvectors sin(j pi i/(n+1)).  A right-hand
    side in the span of 3 eigenvectors makes CG terminate within 3 iterations."""
    n = 31
    rp, ci, vals = [0], [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                ci.append(j)
                vals.append(2.0 if i == j else -1.0)
        rp.append(len(ci))
    P = O.Pattern(n, np.array(rp, np.int32), np.array(ci, np.int32))
    i = np.arange(1, n + 1)
    b = sum(c * np.sin(j * np.pi * i / (n + 1)) for c, j in ((1.0, 1), (0.5, 7), (-2.0, 20)))
    x, it, res, st = O.batch_solve(P, np.array([vals]), b[None, :], solver=O.CG,
                                   precond=O.PREC_NONE)
    assert st[0] == O.CONVERGED and it[0] <= 3
    lam = lambda j: 2 - 2 * np.cos(j * np.pi / (n + 1))
    xe = sum(c / lam(j) * np.sin(j * np.pi * i / (n + 1)) for c, j in ((1.0, 1), (0.5, 7), (-2.0, 20)))
    assert np.linalg.norm(x[0] - xe) <= 1e-9 * np.linalg.norm(xe)


def test_identity_one_half_step():
    n = 17
    rp = np.arange(n + 1, dtype=np.int32)
    P = O.Pattern(n, rp, rp[:-1].copy())
    b = np.random.default_rng(6).standard_normal((2, n))
    x, it, res, st = O.batch_solve(P, np.ones((2, n)), b, solver=O.BICGSTAB,
                                   precond=O.PREC_NONE)
    assert np.all(it == 1) and np.array_equal(x, b)


# --------------------------------------------------------------- brute force
def tiny_spd(rng, n):
    Q = rng.standard_normal((n, n))
    return Q @ Q.T + n * np.eye(n)


def tiny_nonsym(rng, n):
    return rng.standard_normal((n, n)) + 2.5 * np.sqrt(n) * np.eye(n)


def krylov(Mop, v, k):
    """Orthonormal basis of span{v, Mop v, ..., Mop^(k-1) v} (Gram-Schmidt, twice).

    Same space as the power basis, without its ill-conditioning."""
    Q = [v / np.linalg.norm(v)]
    for _ in range(k - 1):
        w = Mop(Q[-1])
        for _ in range(2):
            for q in Q:
                w = w - (q @ w) * q
        Q.append(w / np.linalg.norm(w))
    return np.stack(Q, axis=1)


@pytest.mark.parametrize("prec", [O.PREC_NONE, O.PREC_JACOBI])
def test_cg_is_energy_minimiser(prec):
    """PCG iterate x_k minimises ||x - x*||_A over x0 + K_k(M A, M r0)."""
    rng = np.random.default_rng(7)
    n = 8
    A = tiny_spd(rng, n)
    A[np.abs(A) < 0.3] = 0.0  # some sparsity, still SPD (diagonal dominant part)
    A = (A + A.T) / 2 + n * np.eye(n)
    b = rng.standard_normal(n)
    x0 = rng.standard_normal(n) * 0.1
    P, vals, bb = batch_from_dense(A[None], b[None])
    M = np.diag(1 / np.diag(A)) if prec == O.PREC_JACOBI else np.eye(n)
    xs = np.linalg.solve(A, b)
    r0 = b - A @ x0
    for k in range(1, n):
        x, it, res, st = O.batch_solve(P, vals, bb, x0=x0[None], solver=O.CG, precond=prec,
                                       tol=1e-300, max_iter=k)
        assert it[0] == k and st[0] == O.MAX_ITER
        K = krylov(lambda v: M @ (A @ v), M @ r0, k)
        c = np.linalg.solve(K.T @ A @ K, K.T @ r0)
        xb = x0 + K @ c
        assert np.linalg.norm(x[0] - xb) <= 1e-8 * np.linalg.norm(xs)


@pytest.mark.parametrize("prec", [O.PREC_NONE, O.PREC_JACOBI])
def test_gmres_is_residual_minimiser(prec):
    """GMRES step k (no restart): x_k minimises ||b - A x|| over x0 + M K_k(A M, r0)."""
    rng = np.random.default_rng(8)
    n = 7
    A = tiny_nonsym(rng, n)
    b = rng.standard_normal(n)
    P, vals, bb = batch_from_dense(A[None], b[None])
    M = np.diag(1 / np.diag(A)) if prec == O.PREC_JACOBI else np.eye(n)
    for k in range(1, n):
        x, it, res, st = O.batch_solve(P, vals, bb, solver=O.GMRES, precond=prec,
                                       tol=1e-300, max_iter=k, restart=30)
        assert it[0] == k
        K = M @ krylov(lambda v: A @ (M @ v), b, k)
        c, *_ = np.linalg.lstsq(A @ K, b, rcond=None)
        xb = K @ c
        assert np.linalg.norm(x[0] - xb) <= 1e-9 * np.linalg.norm(xb)
        assert abs(np.linalg.norm(b - A @ x[0]) / np.linalg.norm(b) - res[0]) <= 1e-12


def test_gmres_restart_cycles_are_minimisers():
    """GMRES(m): each cycle minimises over the Krylov space of that cycle's true residual."""
    rng = np.random.default_rng(9)
    n, m = 9, 3
    A = tiny_nonsym(rng, n)
    b = rng.standard_normal(n)
    P, vals, bb = batch_from_dense(A[None], b[None])
    M = np.diag(1 / np.diag(A))
    xb = np.zeros(n)
    done = 0
    for k in (3, 6, 8):
        steps = k - done
        r = b - A @ xb
        K = M @ krylov(lambda v: A @ (M @ v), r, steps)
        c, *_ = np.linalg.lstsq(A @ K, r, rcond=None)
        xb = xb + K @ c
        done = k
        x, it, res, st = O.batch_solve(P, vals, bb, solver=O.GMRES, precond=O.PREC_JACOBI,
                                       tol=1e-300, max_iter=k, restart=m)
        assert it[0] == k
        assert np.linalg.norm(x[0] - xb) <= 1e-9 * np.linalg.norm(xb)


def test_gmres_full_dimension_converges():
    rng = np.random.default_rng(10)
    n = 12
    A = tiny_nonsym(rng, n)
    b = rng.standard_normal(n)
    P, vals, bb = batch_from_dense(A[None], b[None])
    x, it, res, st = O.batch_solve(P, vals, bb, solver=O.GMRES, restart=30)
    assert st[0] == O.CONVERGED and it[0] <= n


# --------------------------------------------------------------- independent implementations
def test_cg_matches_scipy_fixed_iterations():
    rng = np.random.default_rng(11)
    n = 30
    A = sp.diags([-1.0 * np.ones(n - 1), 2.5 + rng.random(n), -1.0 * np.ones(n - 1)], [-1, 0, 1]).toarray()
    b = rng.standard_normal(n)
    P, vals, bb = batch_from_dense(A[None], b[None])
    Minv = spla.LinearOperator((n, n), matvec=lambda v: v / np.diag(A))
    for k in (1, 2, 5, 9):
        xs, _ = spla.cg(A, b, rtol=0.0, atol=0.0, maxiter=k, M=Minv)
        x, it, *_ = O.batch_solve(P, vals, bb, solver=O.CG, tol=1e-300, max_iter=k)
        assert it[0] == k
        assert np.linalg.norm(x[0] - xs) <= 1e-12 * np.linalg.norm(xs)


def test_bicgstab_matches_scipy_fixed_iterations():
    b = W.tridiag_stencil(n_batch=3, n=32, seed=1)
    P = O.Pattern(b.n, b.row_ptr, b.col_idx)
    for s in range(3):
        A = O.to_dense(P, b.values[s])
        Minv = spla.LinearOperator(A.shape, matvec=lambda v, d=np.diag(A): v / d)
        for k in (1, 2, 4, 7):
            xs, _ = spla.bicgstab(A, b.b[s], rtol=0.0, atol=0.0, maxiter=k, M=Minv)
            x, it, *_ = O.batch_solve(P, b.values[s:s + 1], b.b[s:s + 1], solver=O.BICGSTAB,
                                      tol=1e-300, max_iter=k)
            assert it[0] == k
            assert np.linalg.norm(x[0] - xs) <= 1e-12 * np.linalg.norm(xs)


# --------------------------------------------------------------- final results
@pytest.mark.parametrize("solver", [O.BICGSTAB, O.GMRES])
@pytest.mark.parametrize("gen", ["tridiag", "chem", "collision"])
def test_solution_matches_dense_lu(solver, gen):
    if gen == "tridiag":
        bt = W.tridiag_stencil(n_batch=16)
    elif gen == "chem":
        bt = W.chem_jacobian(n_batch=16)
    else:
        bt = W.collision_stencil(n_batch=3)
    P = O.Pattern(bt.n, bt.row_ptr, bt.col_idx)
    tol = 1e-10
    x, it, res, st = O.batch_solve(P, bt.values, bt.b, solver=solver, tol=tol, max_iter=1000)
    assert np.all(st == O.CONVERGED)
    assert np.all(res <= tol)
    for s in range(bt.n_batch):
        A = O.to_dense(P, bt.values[s])
        xs = O.dense_solve(A, bt.b[s])
        kappa = np.linalg.cond(A)
        rr = np.linalg.norm(bt.b[s] - A @ x[s]) / np.linalg.norm(bt.b[s])
        assert abs(rr - res[s]) <= 1e-13
        assert np.linalg.norm(x[s] - xs) <= 1.01 * kappa * tol * np.linalg.norm(xs) + 1e-14


def test_cg_spd_batch_matches_dense():
    bt = W.tridiag_stencil(n_batch=8, n=50, seed=3)
    # symmetrise: use the lower off-diagonal for both sides
    P = O.Pattern(bt.n, bt.row_ptr, bt.col_idx)
    vals = bt.values.copy()
    for s in range(8):
        A = O.to_dense(P, vals[s])
        A = np.tril(A) + np.tril(A, -1).T
        vals[s] = A[np.repeat(np.arange(bt.n), np.diff(bt.row_ptr)), bt.col_idx]
    x, it, res, st = O.batch_solve(P, vals, bt.b, solver=O.CG)
    assert np.all(st == O.CONVERGED) and np.all(res <= 1e-10)
    for s in range(8):
        A = O.to_dense(P, vals[s])
        xs = np.linalg.solve(A, bt.b[s])
        assert np.linalg.norm(x[s] - xs) <= 2 * np.linalg.cond(A) * 1e-10 * np.linalg.norm(xs)


def test_csr_and_ell_solves_identical():
    bt = W.chem_jacobian(n_batch=64)
    P = O.Pattern(bt.n, bt.row_ptr, bt.col_idx)
    ev = O.csr_values_to_ell(P, bt.values)
    for solver in (O.CG, O.BICGSTAB, O.GMRES):
        a = O.batch_solve(P, bt.values, bt.b, solver=solver)
        e = O.batch_solve(P, ev, bt.b, fmt=O.ELL, solver=solver)
        for u, v in zip(a, e):
            assert np.array_equal(u, v)


# --------------------------------------------------------------- status codes
def small_batch():
    bt = W.tridiag_stencil(n_batch=4, n=8)
    return O.Pattern(bt.n, bt.row_ptr, bt.col_idx), bt


@pytest.mark.parametrize("solver", [O.CG, O.BICGSTAB, O.GMRES])
def test_status_codes(solver):
    P, bt = small_batch()
    # b = 0 -> x = 0, converged, 0 iterations
    x, it, res, st = O.batch_solve(P, bt.values, np.zeros_like(bt.b), x0=np.ones_like(bt.b),
                                   solver=solver)
    assert np.all(x == 0) and np.all(it == 0) and np.all(st == O.CONVERGED) and np.all(res == 0)
    # max_iter = 0 -> MAX_ITER, x untouched
    x, it, res, st = O.batch_solve(P, bt.values, bt.b, solver=solver, max_iter=0)
    assert np.all(st == O.MAX_ITER) and np.all(it == 0) and np.all(x == 0)
    # unreachable tolerance
    x, it, res, st = O.batch_solve(P, bt.values, bt.b, solver=solver, tol=1e-30, max_iter=25)
    assert np.all(st == O.MAX_ITER) and np.all(it == 25)
    # exact initial guess -> 0 iterations
    xs = np.stack([np.linalg.solve(O.to_dense(P, bt.values[s]), bt.b[s]) for s in range(4)])
    x, it, res, st = O.batch_solve(P, bt.values, bt.b, x0=xs, solver=solver, tol=1e-8)
    assert np.all(it == 0) and np.all(st == O.CONVERGED)
    # NaN in one system only affects that system
    v = bt.values.copy()
    v[1, 3] = np.nan
    x, it, res, st = O.batch_solve(P, v, bt.b, solver=solver)
    assert st[1] == O.NONFINITE and np.all(st[[0, 2, 3]] == O.CONVERGED)
    bb = bt.b.copy()
    bb[2, 0] = np.inf
    x, it, res, st = O.batch_solve(P, bt.values, bb, solver=solver)
    assert st[2] == O.NONFINITE and it[2] == 0
    # zero matrix -> breakdown
    x, it, res, st = O.batch_solve(P, np.zeros_like(bt.values), bt.b, solver=solver)
    assert np.all(st == O.BREAKDOWN)


# --------------------------------------------------------------- restart from the true residual
# Reading P2: when the recurrence residual passes the test but the true
# residual b - A x does not, the method starts again from x as if it were a new
# initial guess (BiCGSTAB resets its shadow residual, rho0 = alpha = omega = 1
# and p = v = 0; CG rebuilds z, p and rho from the true residual).  So a solve
# that restarts at iteration k must equal, bit for bit, a fresh solve started
# from its iterate x_k with the remaining budget, its count offset by k.  x_k
# itself is the iterate a solve with max_iter = k returns (it ends there with
# MAX_ITER).  A reset that is forgotten (a stale r^, rho0, alpha, omega, p, v or
# z) makes the continued solve differ from the fresh one.
def restart_cases():
    bt8 = W.tridiag_stencil(n_batch=4, n=8, seed=0)
    sp_rng = np.random.default_rng(5)
    n = 12
    As = []
    for _ in range(3):
        M = sp_rng.standard_normal((n, n))
        As.append(M @ M.T + n * np.eye(n))          # SPD, kappa of a few
    Pd, vd, bd = batch_from_dense(np.stack(As), sp_rng.standard_normal((3, n)))
    P8 = O.Pattern(bt8.n, bt8.row_ptr, bt8.col_idx)
    return [
        ("bicgstab_tridiag", P8, bt8.values, bt8.b, O.BICGSTAB, O.PREC_JACOBI, 1e-30, 25),
        ("bicgstab_none", P8, bt8.values, bt8.b, O.BICGSTAB, O.PREC_NONE, 1e-30, 40),
        ("cg_tridiag", P8, bt8.values, bt8.b, O.CG, O.PREC_JACOBI, 1e-20, 120),
        ("cg_spd_dense", Pd, vd, bd, O.CG, O.PREC_NONE, 1e-22, 150),
    ]


@pytest.mark.parametrize("case", restart_cases(), ids=lambda c: c[0])
def test_restart_equals_fresh_solve(case):
    name, P, vals, b, solver, prec, tol, max_iter = case
    x, it, res, st, log = O.batch_solve_log(P, vals, b, solver=solver, precond=prec, tol=tol,
                                            max_iter=max_iter)
    assert np.all(log[:, 0] >= 1), f"{name}: every system must restart at least once"
    checked = 0
    differs_off_restart = 0
    for s in range(b.shape[0]):
        for k in log[s, 1:1 + min(int(log[s, 0]), 3)]:
            k = int(k)
            one = slice(s, s + 1)
            xk, ik, _, sk = O.batch_solve(P, vals[one], b[one], solver=solver, precond=prec,
                                          tol=tol, max_iter=k)
            assert sk[0] == O.MAX_ITER and ik[0] == k
            xf, itf, rf, sf = O.batch_solve(P, vals[one], b[one], x0=xk, solver=solver,
                                            precond=prec, tol=tol, max_iter=max_iter - k)
            assert np.array_equal(xf[0], x[s]), f"{name} system {s}: restart at {k} differs"
            assert itf[0] + k == it[s] and sf[0] == st[s] and rf[0] == res[s]
            checked += 1
            # one iteration past the restart point the Krylov state is not fresh:
            # a solve restarted there by hand takes a different path
            if k + 1 < it[s]:
                xo, _, _, _ = O.batch_solve(P, vals[one], b[one], solver=solver, precond=prec,
                                            tol=tol, max_iter=k + 1)
                xg, _, _, _ = O.batch_solve(P, vals[one], b[one], x0=xo, solver=solver,
                                            precond=prec, tol=tol, max_iter=max_iter - k - 1)
                differs_off_restart += int(not np.array_equal(xg[0], x[s]))
    assert checked >= b.shape[0]
    assert differs_off_restart >= 1


# --------------------------------------------------------------- absolute stop criterion
# Tab. 2 lists an absolute and a relative stop criterion.  Absolute: stop when
# ||r||_2 <= tol and report ||b - A x||_2; relative: ||r||_2 <= tol ||b||_2 and
# report ||b - A x||_2 / ||b||_2.
def signed_ones_batch(rng, B=24):
    bt = W.chem_jacobian(n_batch=B, n=40, seed=11)
    # entries +-1: ||b||^2 = n exactly, so ||b|| = sqrt(n) on both sides to the bit
    b = np.where(rng.random(bt.b.shape) < 0.5, -1.0, 1.0)
    return O.Pattern(bt.n, bt.row_ptr, bt.col_idx), bt, b


@pytest.mark.parametrize("solver", [O.CG, O.BICGSTAB, O.GMRES])
def test_absolute_equals_relative_at_scaled_tol(solver):
    rng = np.random.default_rng(3)
    P, bt, b = signed_ones_batch(rng)
    tol = 1e-9
    rel = O.batch_solve(P, bt.values, b, solver=solver, tol=tol, max_iter=60)
    ab = O.batch_solve(P, bt.values, b, solver=solver, tol=tol * math.sqrt(bt.n), max_iter=60,
                       absolute=True)
    for u, v in zip(rel[:2] + rel[3:], ab[:2] + ab[3:]):     # x, iters, status
        assert np.array_equal(u, v)
    assert np.allclose(ab[2], rel[2] * math.sqrt(bt.n), rtol=4 * EPS, atol=0)


@pytest.mark.parametrize("solver", [O.BICGSTAB, O.GMRES])
def test_absolute_criterion_follows_the_scale_of_b(solver):
    """Scaling b by 2^10 scales every iterate exactly: the relative criterion
    takes the same steps, the absolute one (same tol) needs more, and its
    converged x meet ||b - A x|| <= tol by an independent dense evaluation."""
    bt = W.chem_jacobian(n_batch=16, n=54, seed=2)
    P = O.Pattern(bt.n, bt.row_ptr, bt.col_idx)
    tol = 1e-9
    b2 = bt.b * 1024.0
    r1 = O.batch_solve(P, bt.values, bt.b, solver=solver, tol=tol)
    r2 = O.batch_solve(P, bt.values, b2, solver=solver, tol=tol)
    assert np.array_equal(r1[1], r2[1]) and np.array_equal(r1[0] * 1024.0, r2[0])
    a1 = O.batch_solve(P, bt.values, bt.b, solver=solver, tol=tol, absolute=True)
    a2 = O.batch_solve(P, bt.values, b2, solver=solver, tol=tol, absolute=True)
    assert np.all(a2[1] >= a1[1]) and np.sum(a2[1]) > np.sum(a1[1])
    w = int(np.diff(bt.row_ptr).max())
    for (x, it, res, st), bb in ((a1, bt.b), (a2, b2)):
        assert np.all(st == O.CONVERGED)
        for s in range(bt.n_batch):
            A = O.to_dense(P, bt.values[s])
            tr = np.linalg.norm(bb[s] - A @ x[s])
            # both sides round b - A x within (w+2) eps (|b| + |A||x|) per component
            bound = 2 * (w + 2) * EPS * (np.linalg.norm(bb[s]) + np.linalg.norm(np.abs(A) @ np.abs(x[s])))
            assert res[s] <= tol and tr <= tol + bound
            assert abs(res[s] - tr) <= bound


# --------------------------------------------------------------- block Jacobi
# Blocks of bs consecutive rows; the inverse of each diagonal block by
# Gauss-Jordan elimination without pivoting; a zero pivot makes the block the
# identity.
def dense_blocks(P, v, bs):
    A = O.to_dense(P, v)
    n = A.shape[0]
    return [A[b0:b0 + bs, b0:b0 + bs] for b0 in range(0, n, bs)]


@pytest.mark.parametrize("bs", [2, 4, 8, 16])
def test_block_jacobi_inverse_matches_numpy(bs):
    bt = W.chem_jacobian(n_batch=3, n=54, seed=5)       # 54 = ragged last block for bs 4, 8, 16
    P = O.Pattern(bt.n, bt.row_ptr, bt.col_idx)
    inv = O.block_jacobi(P, bt.values, bs)
    inv_e = O.block_jacobi(P, O.csr_values_to_ell(P, bt.values), bs, fmt=O.ELL)
    assert np.array_equal(inv, inv_e)
    for s in range(bt.n_batch):
        for bi, D in enumerate(dense_blocks(P, bt.values[s], bs)):
            m = D.shape[0]
            ref = np.linalg.inv(D)
            got = inv[s, bi * bs: bi * bs + m, :m]
            assert np.allclose(got, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())
            assert np.all(inv[s, bi * bs: bi * bs + m, m:] == 0)


@pytest.mark.parametrize("solver", [O.CG, O.BICGSTAB, O.GMRES])
def test_block_size_one_is_scalar_jacobi(solver):
    bt = W.chem_jacobian(n_batch=20, n=40, seed=6) if solver != O.CG else W.tridiag_stencil(20, n=40)
    P = O.Pattern(bt.n, bt.row_ptr, bt.col_idx)
    a = O.batch_solve(P, bt.values, bt.b, solver=solver, precond=O.PREC_JACOBI)
    b = O.batch_solve(P, bt.values, bt.b, solver=solver, precond=O.PREC_BLOCK_JACOBI, block_size=1)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


@pytest.mark.parametrize("solver", [O.CG, O.BICGSTAB, O.GMRES])
def test_block_jacobi_exact_on_block_diagonal(solver):
    """A block-diagonal matrix with the preconditioner's blocks: M = A^{-1},
    so the first step solves the system."""
    rng = np.random.default_rng(9)
    n, bs, B = 24, 4, 6
    As = np.zeros((B, n, n))
    for b0 in range(0, n, bs):
        M = rng.random((B, bs, bs)) - 0.5
        if solver == O.CG:
            M = M @ np.transpose(M, (0, 2, 1)) + bs * np.eye(bs)
        else:
            M = M + bs * np.eye(bs)
        As[:, b0:b0 + bs, b0:b0 + bs] = M
    P, vals, b = batch_from_dense(As, rng.random((B, n)) - 0.5)
    x, it, res, st = O.batch_solve(P, vals, b, solver=solver, precond=O.PREC_BLOCK_JACOBI,
                                   block_size=bs, tol=1e-12)
    assert np.all(st == O.CONVERGED) and np.all(it == 1)
    for s in range(B):
        assert np.allclose(x[s], np.linalg.solve(As[s], b[s]), rtol=1e-10, atol=1e-12)


def test_block_jacobi_zero_pivot_gives_identity():
    """[[0, 1], [1, 0]] is invertible but has a zero first pivot without
    pivoting: that block becomes the identity; the other block is inverted."""
    A = np.array([[0.0, 1, 0, 0], [1, 0, 0, 0], [0, 0, 2, 1], [0, 0, 1, 3]])
    P, vals, _ = batch_from_dense(A[None], np.zeros((1, 4)))
    inv = O.block_jacobi(P, vals, 2)[0]
    assert np.array_equal(inv[:2], np.eye(2))
    assert np.allclose(inv[2:], np.linalg.inv(A[2:, 2:]), rtol=1e-15)


# ------------------------------------------------------------------ ILU(0), trsv
def ilu_case(rng, n, fill, B=3, dom=1.5):
    """Random pattern with a full diagonal, values U(-1, 1), diagonal dominant
    by rows and columns (so LU without pivoting is stable and partial pivoting
    keeps the diagonal)."""
    mask = rng.random((n, n)) < fill
    np.fill_diagonal(mask, True)
    As = np.where(mask[None], rng.random((B, n, n)) * 2 - 1, 0.0)
    for s in range(B):
        off = np.abs(As[s]).sum(1) + np.abs(As[s]).sum(0)
        As[s][np.diag_indices(n)] = dom * off + 1.0
    rows, cols = np.nonzero(mask)
    rp = np.concatenate([[0], np.cumsum(mask.sum(1))]).astype(np.int32)
    P = O.Pattern(n, rp, cols.astype(np.int32))
    return P, mask, As, np.ascontiguousarray(As[:, rows, cols])


def test_ilu0_full_pattern_is_lu():
    """On a full pattern ILU(0) is LU without pivoting: with column dominance
    scipy's partially pivoted LU keeps the identity permutation and must give
    the same factors."""
    rng = np.random.default_rng(21)
    P, mask, As, vals = ilu_case(rng, 12, 1.0)
    lu, ok = O.ilu0(P, vals)
    assert ok.all()
    for s in range(As.shape[0]):
        Pm, L, U = scipy.linalg.lu(As[s])
        assert np.array_equal(Pm, np.eye(12))
        assert np.allclose(np.tril(lu[s], -1), L - np.eye(12), rtol=1e-13, atol=1e-15)
        assert np.allclose(np.triu(lu[s]), U, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("n,fill", [(9, 0.3), (40, 0.15), (64, 0.35)])
def test_ilu0_matches_a_on_the_pattern(n, fill):
    """The defining property of ILU(0): (L U)_ij = a_ij for every (i, j) of the
    pattern, and L, U vanish off it.  A dropped or misplaced update breaks it."""
    rng = np.random.default_rng(22 + n)
    P, mask, As, vals = ilu_case(rng, n, fill)
    lu, ok = O.ilu0(P, vals)
    assert ok.all()
    for s in range(As.shape[0]):
        F = lu[s]
        assert np.all(F[~mask] == 0)
        L, U = np.tril(F, -1) + np.eye(n), np.triu(F)
        prod = L @ U
        scale = np.abs(L) @ np.abs(U)
        assert np.all(np.abs(prod - As[s])[mask] <= 8 * n * EPS * scale[mask])
    # ELL storage gives the same factors
    lu_e, _ = O.ilu0(P, O.csr_values_to_ell(P, vals), fmt=O.ELL)
    assert np.array_equal(lu, lu_e)


@pytest.mark.parametrize("col", [False, True])
def test_ilu0_apply_solves_lu(col):
    """z = (L U)^{-1} v: L (U z) reproduces v, with the row- and with the
    column-oriented backward substitution."""
    rng = np.random.default_rng(23)
    P, mask, As, vals = ilu_case(rng, 30, 0.2)
    lu, _ = O.ilu0(P, vals)
    v = rng.random((3, 30)) - 0.5
    z = O.ilu0_apply(P, vals, lu, v, col=col)
    for s in range(3):
        L, U = np.tril(lu[s], -1) + np.eye(30), np.triu(lu[s])
        assert np.allclose(L @ (U @ z[s]), v[s], rtol=1e-12, atol=1e-14)
        assert np.allclose(z[s], scipy.linalg.solve_triangular(
            U, scipy.linalg.solve_triangular(L, v[s], lower=True, unit_diagonal=True)),
            rtol=1e-12, atol=1e-14)


def test_ilu0_backward_orders_differ_only_in_rounding():
    """The two backward orders are the same operations: with at most one term
    per row above the diagonal (a bidiagonal U) they agree bit for bit, and
    where rows hold several terms they differ in the last bits only."""
    bt = W.tridiag_stencil(n_batch=6, n=40, seed=8)
    P = O.Pattern(bt.n, bt.row_ptr, bt.col_idx)
    lu, ok = O.ilu0(P, bt.values)
    v = np.random.default_rng(2).random((6, 40)) - 0.5
    assert ok.all()
    assert np.array_equal(O.ilu0_apply(P, bt.values, lu, v), O.ilu0_apply(P, bt.values, lu, v, col=True))
    x1 = O.batch_solve(P, bt.values, bt.b, precond=O.PREC_ILU, tol=1e-12)
    x2 = O.batch_solve(P, bt.values, bt.b, precond=O.PREC_ILU_COL, tol=1e-12)
    for a, b in zip(x1, x2):
        assert np.array_equal(a, b)
    rng = np.random.default_rng(31)
    P2, mask, As, vals = ilu_case(rng, 40, 0.3)
    lu2, _ = O.ilu0(P2, vals)
    w = rng.random((len(vals), 40)) - 0.5
    za, zb = O.ilu0_apply(P2, vals, lu2, w), O.ilu0_apply(P2, vals, lu2, w, col=True)
    assert not np.array_equal(za, zb)
    assert np.allclose(za, zb, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("solver", [O.BICGSTAB, O.GMRES])
def test_ilu0_exact_on_tridiagonal(solver):
    """A tridiagonal pattern is closed under elimination: ILU(0) is the exact LU,
    M = A^{-1}, and the first step solves the system."""
    bt = W.tridiag_stencil(n_batch=8, n=50, seed=3)
    P = O.Pattern(bt.n, bt.row_ptr, bt.col_idx)
    x, it, res, st = O.batch_solve(P, bt.values, bt.b, solver=solver, precond=O.PREC_ILU,
                                   tol=1e-12)
    assert np.all(st == O.CONVERGED) and np.all(it == 1)
    A = csr_dense(bt.n, bt.row_ptr, bt.col_idx, bt.values[0])
    assert np.allclose(x[0], np.linalg.solve(A, bt.b[0]), rtol=1e-11, atol=1e-13)


def test_ilu0_zero_pivot_runs_unpreconditioned():
    """A zero pivot (a_00 = 0) makes M the identity: the result is bit-identical
    to the unpreconditioned solve."""
    rng = np.random.default_rng(24)
    P, mask, As, vals = ilu_case(rng, 20, 0.3)
    d0 = np.flatnonzero(P.col_idx[P.row_ptr[0]:P.row_ptr[1]] == 0)[0] + P.row_ptr[0]
    vals = vals.copy()
    vals[:, d0] = 0.0
    _, ok = O.ilu0(P, vals)
    assert not ok.any()
    b = rng.random((3, 20)) - 0.5
    a = O.batch_solve(P, vals, b, solver=O.GMRES, precond=O.PREC_ILU)
    c = O.batch_solve(P, vals, b, solver=O.GMRES, precond=O.PREC_NONE)
    for u, v in zip(a, c):
        assert np.array_equal(u, v)


@pytest.mark.parametrize("lower", [True, False])
def test_trsv_matches_scipy(lower):
    """BatchTrsv: the triangle of A (diagonal included) solved by substitution
    against scipy's triangular solver; entries of the other triangle are
    ignored."""
    rng = np.random.default_rng(25)
    P, mask, As, vals = ilu_case(rng, 33, 0.25)
    b = rng.random((3, 33)) - 0.5
    x, it, res, st = O.batch_solve(P, vals, b, solver=O.TRSV_LOWER if lower else O.TRSV_UPPER)
    assert np.all(st == O.CONVERGED) and np.all(it == 0)
    for s in range(3):
        T = np.tril(As[s]) if lower else np.triu(As[s])
        ref = scipy.linalg.solve_triangular(T, b[s], lower=lower)
        assert np.allclose(x[s], ref, rtol=1e-12, atol=1e-14)
        assert res[s] <= 1e-14


def test_trsv_zero_diagonal_breaks_down():
    rng = np.random.default_rng(26)
    P, mask, As, vals = ilu_case(rng, 10, 0.3)
    d5 = np.flatnonzero(P.col_idx[P.row_ptr[5]:P.row_ptr[6]] == 5)[0] + P.row_ptr[5]
    vals = vals.copy()
    vals[1, d5] = 0.0
    b = rng.random((3, 10)) - 0.5
    x, it, res, st = O.batch_solve(P, vals, b, solver=O.TRSV_LOWER)
    assert list(st) == [O.CONVERGED, O.BREAKDOWN, O.CONVERGED]
    assert np.all(x[1] == 0) and res[1] == 1.0
