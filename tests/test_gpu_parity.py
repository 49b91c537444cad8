"""GPU parity: the fused HIP solver against the FP64 CPU oracle, through the C ABI.

Bar (per system): status equal; for converged systems the true relative residual
of the GPU's x, recomputed by the oracle, is <= tol; ||x - x_oracle|| /
||x_oracle|| <= 1e-8; |iters - iters_oracle| <= 2.  Layout work (ELL pattern and
value conversion) must match the oracle bit for bit.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2308_08417_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2308_08417_amd import batchsolve as bs  # noqa: E402

SOLVER_O = {bs.CG: O.CG, bs.BICGSTAB: O.BICGSTAB, bs.GMRES: O.GMRES, bs.TRSV_LOWER: O.TRSV_LOWER,
            bs.TRSV_UPPER: O.TRSV_UPPER}
XTOL, ITOL = 1e-8, 2


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bs.lib()
    return torch.device("cuda:0")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


class Case:
    def __init__(self, batch: W.Batch):
        self.batch = batch
        self.P = bs.Pattern.from_csr(batch.row_ptr, batch.col_idx)
        self.OP = O.Pattern(batch.n, batch.row_ptr, batch.col_idx)
        self.vals = dev(batch.values)
        self._ell = None

    def values(self, fmt):
        if fmt == bs.CSR:
            return self.vals
        if self._ell is None:
            B = self.batch.n_batch
            self._ell = torch.empty((B, self.P.ell_width * self.batch.n), dtype=torch.float64,
                                    device="cuda:0")
            bs.bs_values_csr_to_ell(self.P.handle, self.vals, self._ell)
        return self._ell

    def oracle_values(self, fmt):
        return self.batch.values if fmt == bs.CSR else O.csr_values_to_ell(self.OP, self.batch.values)

    def gpu(self, fmt, solver, precond=bs.PREC_JACOBI, tol=1e-10, max_iter=500, x0=None,
            b=None, values=None, extra_flags=0, **opt):
        say(f"  gpu: {self.batch.name} n={self.batch.n} B={self.batch.n_batch} fmt={fmt} "
            f"solver={solver} prec={precond} opt={opt}")
        bb = dev(self.batch.b if b is None else b)
        flags = 0
        if x0 is None:
            x = torch.zeros_like(bb)
            flags = bs.FLAG_X0_ZERO
        else:
            x = dev(x0)
        opts = bs.make_options(flags=flags | extra_flags, **opt)
        B = bb.shape[0]
        iters = torch.full((B,), -7, dtype=torch.int32, device="cuda:0")
        resid = torch.full((B,), -7.0, dtype=torch.float64, device="cuda:0")
        status = torch.full((B,), -7, dtype=torch.int32, device="cuda:0")
        v = self.values(fmt) if values is None else values
        bs.bs_batch_solve(fmt, self.P.handle, v, bb, x, solver, precond, tol, max_iter, iters,
                          resid, status, opts)
        torch.cuda.synchronize()
        return x.cpu().numpy(), iters.cpu().numpy(), resid.cpu().numpy(), status.cpu().numpy()

    def oracle(self, fmt, solver, precond=bs.PREC_JACOBI, tol=1e-10, max_iter=500, x0=None,
               b=None, values=None, restart=30, block_size=8):
        v = self.oracle_values(fmt) if values is None else values
        return O.batch_solve(self.OP, v, self.batch.b if b is None else b, x0=x0,
                             fmt=O.CSR if fmt == bs.CSR else O.ELL, solver=SOLVER_O[solver],
                             precond=precond, tol=tol, max_iter=max_iter, restart=restart,
                             block_size=block_size)


def check(case, g, o, tol=1e-10, fmt=bs.CSR, b=None, values=None, xtol=XTOL, itol=ITOL):
    xg, ig, rg, sg = g
    xo, io, ro, so = o
    assert np.array_equal(sg, so), f"status mismatch at {np.flatnonzero(sg != so)[:10]}"
    conv = so == O.CONVERGED
    v = case.oracle_values(fmt) if values is None else values
    bb = case.batch.b if b is None else b
    rt = O.true_residual(case.OP, v, bb, xg, fmt=O.CSR if fmt == bs.CSR else O.ELL)
    assert np.all(rt[conv] <= tol), f"true residual {rt[conv].max()}"
    assert np.all(rg[conv] <= tol)
    # The GPU-reported residual is the true residual of its x: both sides round
    # each component of b - A x within (w+2) eps (|b| + |A||x|) (w = longest
    # row), so the two relative norms differ by at most twice that bound.
    fin = np.isfinite(rt) & np.isfinite(rg)
    ofmt = O.CSR if fmt == bs.CSR else O.ELL
    absAx = O.batch_spmv(case.OP, np.abs(v), np.abs(np.nan_to_num(xg)), fmt=ofmt)
    nb = np.linalg.norm(bb, axis=1)
    w = int(np.diff(case.batch.row_ptr).max())
    with np.errstate(invalid="ignore", over="ignore"):
        bound = 2 * (w + 2) * np.finfo(float).eps * (nb + np.linalg.norm(absAx, axis=1))
        bound = bound / np.where(nb > 0, nb, 1.0) + 1e-12 * rt
    assert np.all(np.abs(rg - rt)[fin] <= bound[fin]), "reported residual disagrees with the oracle's"
    nx = np.linalg.norm(xo, axis=1)
    err = np.linalg.norm(xg - xo, axis=1) / np.where(nx > 0, nx, 1.0)
    assert np.all(err[conv] <= xtol), f"x error {err[conv].max()}"
    d = np.abs(ig.astype(np.int64) - io)
    assert np.all(d <= itol), f"iteration mismatch {d.max()} at {np.argmax(d)}: {ig[np.argmax(d)]} vs {io[np.argmax(d)]}"
    return err, d


# ------------------------------------------------------------------ layout
def test_ell_layout_bit_exact():
    bt = W.chem_jacobian(n_batch=37)
    c = Case(bt)
    assert np.array_equal(bs.bs_pattern_ell_cols(c.P.handle), c.OP.ell_col)
    assert c.P.ell_width == c.OP.width
    ev = c.values(bs.ELL).cpu().numpy()
    assert np.array_equal(ev, O.csr_values_to_ell(c.OP, bt.values))


# ------------------------------------------------------------------ configurations
@pytest.mark.parametrize("fmt", [bs.CSR, bs.ELL])
@pytest.mark.parametrize("solver", [bs.BICGSTAB, bs.GMRES])
def test_tridiag_stencil(fmt, solver):
    c = Case(W.tridiag_stencil(n_batch=64, n=32, seed=0))
    g = c.gpu(fmt, solver, max_iter=200)
    o = c.oracle(fmt, solver, max_iter=200)
    check(c, g, o, fmt=fmt)
    assert np.all(g[3] == bs.CONVERGED)


def symmetric_tridiag(B, n, seed):
    bt = W.tridiag_stencil(n_batch=B, n=n, seed=seed)
    rows = np.repeat(np.arange(n), np.diff(bt.row_ptr))
    lower = {}
    for k, (i, j) in enumerate(zip(rows, bt.col_idx)):
        if j < i:
            lower[(i, j)] = k
    v = bt.values.copy()
    for k, (i, j) in enumerate(zip(rows, bt.col_idx)):
        if j > i:
            v[:, k] = bt.values[:, lower[(j, i)]]
    bt.values = v
    return bt


@pytest.mark.parametrize("fmt", [bs.CSR, bs.ELL])
@pytest.mark.parametrize("n", [32, 100, 700])
def test_cg_spd(fmt, n):
    c = Case(symmetric_tridiag(48, n, seed=n))
    g = c.gpu(fmt, bs.CG, max_iter=1000)
    o = c.oracle(fmt, bs.CG, max_iter=1000)
    check(c, g, o, fmt=fmt)
    assert np.all(g[3] == bs.CONVERGED)


@pytest.mark.parametrize("fmt", [bs.CSR, bs.ELL])
@pytest.mark.parametrize("solver", [bs.BICGSTAB, bs.GMRES, bs.CG])
def test_chem_jacobian_small(fmt, solver):
    c = Case(W.chem_jacobian(n_batch=3000))  # ragged against any team count
    g = c.gpu(fmt, solver)
    o = c.oracle(fmt, solver)
    check(c, g, o, fmt=fmt)
    assert np.all(g[3] == bs.CONVERGED)


@pytest.mark.parametrize("fmt", [bs.CSR, bs.ELL])
@pytest.mark.parametrize("solver", [bs.BICGSTAB, bs.GMRES])
def test_collision_stencil(fmt, solver):
    c = Case(W.collision_stencil(n_batch=40))
    g = c.gpu(fmt, solver, max_iter=1000)
    o = c.oracle(fmt, solver, max_iter=1000)
    check(c, g, o, fmt=fmt)
    assert np.all(g[3] == bs.CONVERGED)


@pytest.mark.parametrize("name", list(W.MECHANISMS))
def test_mechanism_shapes(name):
    """The five reacting-flow shapes of Tab. 3 (22..144 rows, 29..90 % fill):
    BiCGSTAB + scalar Jacobi in BatchCsr, as the paper runs them, and in
    BatchEll; GMRES(30) in BatchCsr; at gamma 1e-6 (2..3 iterations) and 3e-4
    (8..14).  The batch holds each distinct system twice and then some, as
    the paper replicates a few cells' matrices: a copy returns its original's
    bits."""
    u = W.MECHANISMS[name][0]
    for gamma in (1e-6, 3e-4):
        c = Case(W.mechanism_batch(name, n_batch=2 * u + 7, gamma=gamma, seed=3))
        for fmt, solver in ((bs.CSR, bs.BICGSTAB), (bs.ELL, bs.BICGSTAB), (bs.CSR, bs.GMRES)):
            g = c.gpu(fmt, solver)
            o = c.oracle(fmt, solver)
            check(c, g, o, fmt=fmt)
            assert np.all(g[3] == bs.CONVERGED)
            for k in range(4):
                assert np.array_equal(g[k][u:2 * u], g[k][:u])


@pytest.mark.parametrize("gen,solver,x0", [("isooctane", bs.BICGSTAB, False),
                                           ("isooctane", bs.BICGSTAB, True),
                                           ("isooctane", bs.GMRES, False),
                                           ("chem300", bs.BICGSTAB, True)])
def test_group_staging_rounds(gen, solver, x0):
    """Multi-wave teams with rows of 32 slots or more copy the next system's CSR
    values into LDS while solving the current one: batches of several times
    the resident groups (every group takes several systems in turn), odd nnz
    (blocks at both 16-byte phases), with and without an initial guess; and
    two right-hand sides per matrix, bit-identical to the replicated batch."""
    bt = {"isooctane": lambda: W.mechanism_batch("isooctane", n_batch=1300, gamma=3e-4, seed=31),
          "chem300": lambda: W.chem_jacobian(900, n=300, fill=0.03, seed=32)}[gen]()
    p = bs.bs_plan(bs.CSR, bt.n, bt.nnz, int(np.diff(bt.row_ptr).max()), solver)
    assert p["team"] > 64 and p["slots"] >= 32 and p["stage_values"] == 2
    c = Case(bt)
    xs = np.random.default_rng(33).standard_normal(bt.b.shape) if x0 else None
    g = c.gpu(bs.CSR, solver, x0=xs)
    o = c.oracle(bs.CSR, solver, x0=xs)
    check(c, g, o)
    assert np.all(g[3] == bs.CONVERGED)
    if x0 or solver != bs.BICGSTAB:
        return
    k, B = 2, 700
    sub = bt.subset(np.arange(B))
    b = 2 * np.random.default_rng(34).random((B * k, bt.n)) - 1
    cs = Case(sub)
    x = torch.zeros((B * k, bt.n), dtype=torch.float64, device="cuda:0")
    it = torch.empty(B * k, dtype=torch.int32, device="cuda:0")
    rs = torch.empty(B * k, dtype=torch.float64, device="cuda:0")
    st = torch.empty(B * k, dtype=torch.int32, device="cuda:0")
    say(f"  staged multi-rhs {gen}")
    bs.bs_batch_solve(bs.CSR, cs.P.handle, cs.values(bs.CSR), dev(b), x, solver, bs.PREC_JACOBI,
                      1e-10, 500, it, rs, st, bs.make_options(flags=bs.FLAG_X0_ZERO, n_rhs=k))
    torch.cuda.synchronize()
    gm = (x.cpu().numpy(), it.cpu().numpy(), rs.cpu().numpy(), st.cpu().numpy())
    rep = W.Batch(bt.name + "_rep", bt.n, bt.row_ptr, bt.col_idx, np.repeat(sub.values, k, axis=0),
                  b, np.zeros_like(b))
    cr = Case(rep)
    gr = cr.gpu(bs.CSR, solver)
    for u, v in zip(gm, gr):
        assert np.array_equal(u, v)
    check(cr, gm, cr.oracle(bs.CSR, solver))


def symmetric_dense_ish(B, n, fill, seed):
    """SPD systems on a symmetric random pattern: off-diagonal pairs a_ij = a_ji
    ~ -U(0.5, 1.5) where the upper-triangle draw is below ``fill`` (mirrored),
    a_ii = 1.1 * (sum of |a_ij| of its row) + U(0, 1); b ~ U(-1, 1)."""
    rng = np.random.default_rng(seed)
    up = np.triu(rng.random((n, n)) < fill, 1)
    mask = up | up.T | np.eye(n, dtype=bool)
    rows, cols = np.nonzero(mask)
    rp = np.zeros(n + 1, np.int32)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    vals = np.zeros((B, rows.size))
    w = -(0.5 + rng.random((B, n, n)))
    w = np.triu(w, 1)
    w = w + np.transpose(w, (0, 2, 1))
    full = np.where(mask[None, :, :], w, 0.0)
    diag = 1.1 * np.abs(full).sum(axis=2) + rng.random((B, n))
    full[:, np.arange(n), np.arange(n)] = diag
    vals[:] = full[:, rows, cols]
    b = 2 * rng.random((B, n)) - 1
    return W.Batch("spd_dense_ish", n, rp, cols.astype(np.int32), vals, b, np.zeros((B, n)))


def test_group_staging_cg():
    """CG through the multi-wave CSR staging: SPD systems of 200 rows with 10..34
    entries per row (56 register slots, 256-lane teams), more systems than
    resident groups."""
    bt = symmetric_dense_ish(700, 200, 0.1, seed=35)
    p = bs.bs_plan(bs.CSR, bt.n, bt.nnz, int(np.diff(bt.row_ptr).max()), bs.CG)
    assert p["team"] == 256 and p["slots"] >= 32 and p["stage_values"] == 2
    c = Case(bt)
    g = c.gpu(bs.CSR, bs.CG, max_iter=1000)
    o = c.oracle(bs.CSR, bs.CG, max_iter=1000)
    check(c, g, o)
    assert np.all(g[3] == bs.CONVERGED)


@pytest.mark.parametrize("team", [128, 256, 512])
def test_forced_wider_teams(team):
    """A system spread over more lanes (several waves) gives the same result."""
    c = Case(W.chem_jacobian(n_batch=257))
    g = c.gpu(bs.CSR, bs.BICGSTAB, team=team)
    o = c.oracle(bs.CSR, bs.BICGSTAB)
    check(c, g, o)


@pytest.mark.parametrize("n,r", [(300, 2), (1000, 1), (1500, 2), (2048, 2), (2000, 4)])
def test_large_systems_rows_per_lane(n, r):
    bt = W.tridiag_stencil(n_batch=6, n=n, seed=n)
    c = Case(bt)
    for solver in (bs.BICGSTAB, bs.CG):
        if solver == bs.CG:
            c = Case(symmetric_tridiag(6, n, seed=n))
        g = c.gpu(bs.ELL, solver, max_iter=2000, rows_per_lane=r)
        o = c.oracle(bs.ELL, solver, max_iter=2000)
        check(c, g, o, fmt=bs.ELL)


@pytest.mark.parametrize("n", [1, 5, 16, 17, 31, 33, 63, 65, 129])
@pytest.mark.parametrize("solver", [bs.BICGSTAB, bs.GMRES, bs.CG])
def test_odd_sizes_and_ragged_batches(n, solver):
    B = 61
    bt = symmetric_tridiag(B, n, seed=3 * n + 1) if solver == bs.CG else W.tridiag_stencil(B, n, seed=n)
    c = Case(bt)
    g = c.gpu(bs.CSR, solver)
    o = c.oracle(bs.CSR, solver)
    check(c, g, o)


# ------------------------------------------------------------------ options and edge cases
@pytest.mark.parametrize("solver", [bs.BICGSTAB, bs.GMRES, bs.CG])
def test_edge_cases(solver):
    base = symmetric_tridiag(8, 24, seed=5) if solver == bs.CG else W.tridiag_stencil(8, 24, seed=5)
    c = Case(base)
    bt = base
    # nonzero initial guess, exact initial guess, b = 0, NaN values, Inf in b
    x0 = np.random.default_rng(1).standard_normal(bt.b.shape)
    xs = np.stack([np.linalg.solve(O.to_dense(c.OP, bt.values[s]), bt.b[s]) for s in range(8)])
    x0[1] = xs[1]
    b = bt.b.copy()
    b[2] = 0.0
    b[3, 4] = np.inf
    vals = bt.values.copy()
    vals[4, 7] = np.nan
    vd = dev(vals)
    g = c.gpu(bs.CSR, solver, x0=x0, b=b, values=vd, tol=1e-8)
    o = c.oracle(bs.CSR, solver, x0=x0, b=b, values=vals, tol=1e-8)
    check(c, g, o, tol=1e-8, b=b, values=vals)
    assert g[3][2] == bs.CONVERGED and g[1][2] == 0 and np.all(g[0][2] == 0.0)
    assert g[3][3] == bs.NONFINITE and g[3][4] == bs.NONFINITE
    assert g[1][1] == 0
    # no iterations allowed
    g = c.gpu(bs.CSR, solver, max_iter=0)
    assert np.all(g[3] == bs.MAX_ITER) and np.all(g[1] == 0) and np.all(g[0] == 0)
    # unreachable tolerance: exactly max_iter iterations
    g = c.gpu(bs.CSR, solver, tol=1e-30, max_iter=13)
    o = c.oracle(bs.CSR, solver, tol=1e-30, max_iter=13)
    assert np.all(g[3] == bs.MAX_ITER) and np.all(g[1] == 13) and np.array_equal(g[1], o[1])
    # zero matrix: breakdown
    z = np.zeros_like(bt.values)
    g = c.gpu(bs.CSR, solver, values=dev(z))
    o = c.oracle(bs.CSR, solver, values=z)
    assert np.all(g[3] == bs.BREAKDOWN) and np.array_equal(g[1], o[1])
    # no preconditioner
    g = c.gpu(bs.CSR, solver, precond=bs.PREC_NONE)
    o = c.oracle(bs.CSR, solver, precond=bs.PREC_NONE)
    check(c, g, o)


def test_gmres_restart_lengths():
    c = Case(W.collision_stencil(n_batch=12, nx=12, ny=10))
    for m in (1, 4, 11, 30):
        g = c.gpu(bs.CSR, bs.GMRES, max_iter=2000, restart=m)
        o = c.oracle(bs.CSR, bs.GMRES, max_iter=2000, restart=m)
        check(c, g, o)


def test_deterministic():
    c = Case(W.chem_jacobian(n_batch=2000))
    a = c.gpu(bs.ELL, bs.BICGSTAB)
    b = c.gpu(bs.ELL, bs.BICGSTAB)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


# ------------------------------------------------------------------ mixed precision
@pytest.mark.parametrize("solver", [bs.BICGSTAB, bs.GMRES])
@pytest.mark.parametrize("gen", ["tridiag", "chem", "collision"])
@pytest.mark.parametrize("fmt", [bs.CSR, bs.ELL])
def test_mixed_precision_meets_fp64_tolerance(gen, fmt, solver):
    bt = {"tridiag": lambda: W.tridiag_stencil(64),
          "chem": lambda: W.chem_jacobian(2048),
          "collision": lambda: W.collision_stencil(24)}[gen]()
    c = Case(bt)
    outer = torch.zeros(bt.n_batch, dtype=torch.int32, device="cuda:0")
    g = c.gpu(fmt, solver, max_iter=2000, precision=bs.MIXED, outer_iters=outer)
    o = c.oracle(fmt, solver, max_iter=2000)
    assert np.all(g[3] == bs.CONVERGED)
    # iteration counts of the mixed form are not those of the FP64 method
    err, _ = check(c, g, o, fmt=fmt, itol=10**9)
    say(f"  mixed {solver} {gen}: max x error vs FP64 oracle {err.max():.2e}, "
        f"inner iters mean {g[1].mean():.2f} (fp64 {o[1].mean():.2f}), "
        f"outer mean {outer.float().mean().item():.2f}")
    assert outer.min().item() >= 1


@pytest.mark.parametrize("dominance", [1.05, 1.02])
def test_gmres_weaker_dominance(dominance):
    """Teams of a wave or more orthogonalise by block Gram-Schmidt (blocks of
    four); the oracle uses modified Gram-Schmidt.  On less dominant stencils
    (up to 347 steps, a dozen restarts) the two must still agree."""
    c = Case(W.collision_stencil(n_batch=16, dominance=dominance, seed=3))
    g = c.gpu(bs.CSR, bs.GMRES, max_iter=5000, restart=30)
    o = c.oracle(bs.CSR, bs.GMRES, max_iter=5000, restart=30)
    err, d = check(c, g, o)
    say(f"  dominance {dominance}: iters {o[1].min()}..{o[1].max()}, max |diff| {d.max()}, "
        f"x err {err.max():.2e}")


def test_mixed_gmres_short_restarts():
    """Mixed GMRES with short cycles: every cycle is one refinement step, so the
    outer count grows as the restart length falls, and the answer still meets the
    FP64 tolerance."""
    c = Case(W.collision_stencil(n_batch=12, nx=12, ny=10))
    prev = None
    for m in (30, 8, 3):
        outer = torch.zeros(12, dtype=torch.int32, device="cuda:0")
        g = c.gpu(bs.CSR, bs.GMRES, max_iter=4000, restart=m, precision=bs.MIXED,
                  outer_iters=outer)
        o = c.oracle(bs.CSR, bs.GMRES, max_iter=4000, restart=m)
        assert np.all(g[3] == bs.CONVERGED)
        check(c, g, o, itol=10**9)
        mean = outer.float().mean().item()
        say(f"  restart {m}: outer mean {mean:.2f}, inner mean {g[1].mean():.2f}")
        if prev is not None:
            assert mean >= prev
        prev = mean


def test_mixed_cg_unsupported():
    c = Case(W.tridiag_stencil(8))
    with pytest.raises(bs.BatchSolveError) as e:
        c.gpu(bs.CSR, bs.CG, precision=bs.MIXED)
    assert e.value.code == bs.ERR_UNSUPPORTED


# ------------------------------------------------------------------ bank-aware layout
def spd_on_pattern(n, n_batch, seed):
    """SPD systems on a symmetrised random pattern: symmetric off-diagonal
    entries U(-1, 1), diagonal = 1 + sum of the row's |off-diagonal|."""
    rng = np.random.default_rng(seed)
    mask = rng.random((n, n)) < 0.2
    mask = mask | mask.T
    np.fill_diagonal(mask, True)
    rows, cols = np.nonzero(mask)
    row_ptr = np.concatenate([[0], np.cumsum(mask.sum(1))]).astype(np.int32)
    col_idx = cols.astype(np.int32)
    vals = np.empty((n_batch, col_idx.size))
    for s in range(n_batch):
        M = np.triu(2 * rng.random((n, n)) - 1, 1)
        M = (M + M.T) * mask
        np.fill_diagonal(M, 1 + np.abs(M).sum(1))
        vals[s] = M[rows, cols]
    b = 2 * rng.random((n_batch, n)) - 1
    return W.Batch("spd_pattern", n, row_ptr, col_idx, vals, b, np.zeros_like(b))


@pytest.mark.parametrize("solver,prec", [(bs.BICGSTAB, bs.FP64), (bs.GMRES, bs.FP64),
                                         (bs.BICGSTAB, bs.MIXED), (bs.GMRES, bs.MIXED)])
def test_bank_layout_parity(solver, prec):
    """The pattern's layout (lanes, buffer elements, windows permuted) and the
    plain layout both meet the oracle; 3001 systems leave a ragged last round."""
    bt = W.chem_jacobian(n_batch=3001, n=54, seed=0)
    c = Case(bt)
    lay = bs.bs_pattern_layout(c.P.handle)
    assert lay is not None and lay[0] == 28
    assert sorted(lay[1][lay[1] >= 0].tolist()) == list(range(54))
    rng = np.random.default_rng(5)
    x0 = None if prec == bs.MIXED else rng.standard_normal(bt.b.shape)
    itol = ITOL if prec == bs.FP64 else 10**9
    o = c.oracle(bs.CSR, solver, x0=x0)
    for flags in (0, bs.FLAG_PLAIN_LAYOUT):
        g = c.gpu(bs.CSR, solver, x0=x0, extra_flags=flags, precision=prec)
        check(c, g, o, itol=itol)


def test_bank_layout_cg_spd():
    bt = spd_on_pattern(48, 700, seed=2)
    c = Case(bt)
    lay = bs.bs_pattern_layout(c.P.handle)
    assert lay is not None
    o = c.oracle(bs.CSR, bs.CG)
    for flags in (0, bs.FLAG_PLAIN_LAYOUT):
        g = c.gpu(bs.CSR, bs.CG, extra_flags=flags)
        check(c, g, o)


# ------------------------------------------------------------------ full size
def test_chem_jacobian_full_size_sampled():
    """2^17 systems in the benchmark's launch shape: every system's residual is
    checked by the oracle, and a random sample is re-solved by the oracle."""
    bt = W.chem_jacobian(n_batch=1 << 17)
    c = Case(bt)
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(bt.n_batch, 1024, replace=False))
    for fmt in (bs.CSR, bs.ELL):
        g = c.gpu(fmt, bs.BICGSTAB)
        assert np.all(g[3] == bs.CONVERGED)
        v = c.oracle_values(fmt)
        rt = O.true_residual(c.OP, v, bt.b, g[0], fmt=O.CSR if fmt == bs.CSR else O.ELL)
        assert np.all(rt <= 1e-10)
        sub = bt.subset(idx)
        o = O.batch_solve(c.OP, v[idx], sub.b, fmt=O.CSR if fmt == bs.CSR else O.ELL,
                          solver=O.BICGSTAB, tol=1e-10, max_iter=500)
        xg = g[0][idx]
        err = np.linalg.norm(xg - o[0], axis=1) / np.linalg.norm(o[0], axis=1)
        assert np.all(err <= XTOL)
        assert np.all(np.abs(g[1][idx] - o[1]) <= ITOL)


@pytest.mark.parametrize("solver,prec,fmt", [(bs.BICGSTAB, bs.FP64, bs.CSR),
                                             (bs.BICGSTAB, bs.FP64, bs.ELL),
                                             (bs.BICGSTAB, bs.MIXED, bs.CSR),
                                             (bs.GMRES, bs.FP64, bs.CSR),
                                             (bs.GMRES, bs.MIXED, bs.CSR)])
def test_collision_full_size_sampled(solver, prec, fmt):
    """The nine-point collision batch at its benchmark size (4096 systems,
    n = 992, one 1024-lane workgroup each), in the launch shape the benchmark
    times: every system converges with the oracle's true residual of its x
    <= 1e-10, and a random sample of 48 systems is re-solved by the oracle
    (FP64: the full bar; mixed: x within the FP64 bar)."""
    bt = W.collision_stencil(4096)
    c = Case(bt)
    g = c.gpu(fmt, solver, max_iter=2000, precision=prec)
    assert np.all(g[3] == bs.CONVERGED)
    v = c.oracle_values(fmt)
    ofmt = O.CSR if fmt == bs.CSR else O.ELL
    rt = O.true_residual(c.OP, v, bt.b, g[0], fmt=ofmt)
    assert np.all(rt <= 1e-10)
    idx = np.sort(np.random.default_rng(1).choice(bt.n_batch, 48, replace=False))
    o = O.batch_solve(c.OP, v[idx], bt.subset(idx).b, fmt=ofmt,
                      solver=O.BICGSTAB if solver == bs.BICGSTAB else O.GMRES, tol=1e-10,
                      max_iter=2000)
    err = np.linalg.norm(g[0][idx] - o[0], axis=1) / np.linalg.norm(o[0], axis=1)
    assert np.all(err <= XTOL)
    if prec == bs.FP64:
        assert np.all(np.abs(g[1][idx] - o[1]) <= ITOL)


# ------------------------------------------------------------------ Tab. 2 completions
def dense_batch(n, B, seed, spd=False):
    """Dense diagonally dominant systems: off-diagonals U(-1, 1) (symmetric for
    spd), diagonal 1 + sum of the row's |off-diagonal|; b ~ U(-1, 1)."""
    rng = np.random.default_rng(seed)
    M = 2 * rng.random((B, n, n)) - 1
    if spd:
        M = np.triu(M, 1)
        M = M + np.transpose(M, (0, 2, 1))
    idx = np.arange(n)
    M[:, idx, idx] = 0.0
    M[:, idx, idx] = 1 + np.abs(M).sum(axis=2)
    b = 2 * rng.random((B, n)) - 1
    rp = (np.arange(n + 1) * n).astype(np.int32)
    ci = np.tile(np.arange(n, dtype=np.int32), n)
    return W.Batch("dense", n, rp, ci, np.ascontiguousarray(M.reshape(B, n * n)), b, np.zeros_like(b))


@pytest.mark.parametrize("n", [16, 40, 64])
@pytest.mark.parametrize("solver", [bs.CG, bs.BICGSTAB, bs.GMRES])
def test_batch_dense(n, solver):
    """BatchDense: [B][n][n] row-major values on the full pattern; the oracle
    solves the same numbers as CSR over the full pattern (the dense product)."""
    bt = dense_batch(n, 300, seed=n, spd=(solver == bs.CG))
    c = Case(bt)
    P = bs.Pattern.dense(n)
    assert P.nnz == n * n and P.max_row_nnz == n
    vals = dev(bt.values)
    say(f"  dense n={n} solver={solver}")
    B = bt.n_batch
    x = torch.zeros((B, n), dtype=torch.float64, device="cuda:0")
    it = torch.empty(B, dtype=torch.int32, device="cuda:0")
    rs = torch.empty(B, dtype=torch.float64, device="cuda:0")
    st = torch.empty(B, dtype=torch.int32, device="cuda:0")
    bs.bs_batch_solve(bs.DENSE, P.handle, vals, dev(bt.b), x, solver, bs.PREC_JACOBI, 1e-10, 500,
                      it, rs, st, bs.make_options(flags=bs.FLAG_X0_ZERO))
    torch.cuda.synchronize()
    g = (x.cpu().numpy(), it.cpu().numpy(), rs.cpu().numpy(), st.cpu().numpy())
    o = c.oracle(bs.CSR, solver)
    check(c, g, o)
    # a dense batch needs the full pattern
    tri = W.tridiag_stencil(1, n=n)
    Pt = bs.Pattern.from_csr(tri.row_ptr, tri.col_idx)
    with pytest.raises(bs.BatchSolveError) as e:
        bs.bs_batch_solve(bs.DENSE, Pt.handle, vals, dev(bt.b), x, solver, bs.PREC_JACOBI, 1e-10,
                          500, it, rs, st)
    assert e.value.code == bs.ERR_PATTERN


def check_absolute(case, g, o, tol, b, itol=ITOL, fmt=bs.CSR):
    xg, ig, rg, sg = g
    xo, io, ro, so = o
    assert np.array_equal(sg, so)
    conv = so == O.CONVERGED
    v = case.oracle_values(fmt)
    ofmt = O.CSR if fmt == bs.CSR else O.ELL
    r = b - O.batch_spmv(case.OP, v, xg, fmt=ofmt)
    rt = np.linalg.norm(r, axis=1)
    absAx = O.batch_spmv(case.OP, np.abs(v), np.abs(xg), fmt=ofmt)
    w = int(np.diff(case.batch.row_ptr).max())
    bound = 2 * (w + 2) * np.finfo(float).eps * (np.linalg.norm(b, axis=1) + np.linalg.norm(absAx, axis=1))
    assert np.all(rt[conv] <= tol + bound[conv]) and np.all(rg[conv] <= tol)
    assert np.all(np.abs(rg - rt) <= bound + 1e-12 * rt)
    nx = np.linalg.norm(xo, axis=1)
    err = np.linalg.norm(xg - xo, axis=1) / np.where(nx > 0, nx, 1.0)
    assert np.all(err[conv] <= XTOL)
    assert np.all(np.abs(ig.astype(np.int64) - io) <= itol)


@pytest.mark.parametrize("solver,prec", [(bs.BICGSTAB, bs.FP64), (bs.GMRES, bs.FP64),
                                         (bs.BICGSTAB, bs.MIXED), (bs.GMRES, bs.MIXED)])
def test_absolute_criterion(solver, prec):
    """Absolute stop criterion (Tab. 2): b scaled by 2^10 so that it stops
    later than the relative one; GPU against the oracle's absolute solve."""
    bt = W.chem_jacobian(n_batch=2000, n=54, seed=4)
    c = Case(bt)
    b = bt.b * 1024.0
    tol = 1e-8
    g = c.gpu(bs.CSR, solver, tol=tol, b=b, extra_flags=bs.FLAG_ABS_TOL, precision=prec)
    o = O.batch_solve(c.OP, bt.values, b, fmt=O.CSR, solver=SOLVER_O[solver], tol=tol,
                      max_iter=500, absolute=True)
    rel = O.batch_solve(c.OP, bt.values, b, fmt=O.CSR, solver=SOLVER_O[solver], tol=tol,
                        max_iter=500)
    assert o[1].sum() > rel[1].sum()
    check_absolute(c, g, o, tol, b, itol=ITOL if prec == bs.FP64 else 10**9)


def test_absolute_criterion_cg_and_ell():
    bt = W.tridiag_stencil(n_batch=500, n=48)
    c = Case(bt)
    b = bt.b * 4096.0
    tol = 1e-9
    o = O.batch_solve(c.OP, bt.values, b, fmt=O.CSR, solver=O.CG, tol=tol, absolute=True)
    g = c.gpu(bs.CSR, bs.CG, tol=tol, b=b, extra_flags=bs.FLAG_ABS_TOL)
    check_absolute(c, g, o, tol, b)
    oe = O.batch_solve(c.OP, c.oracle_values(bs.ELL), b, fmt=O.ELL, solver=O.BICGSTAB, tol=tol,
                       absolute=True)
    ge = c.gpu(bs.ELL, bs.BICGSTAB, tol=tol, b=b, extra_flags=bs.FLAG_ABS_TOL)
    check_absolute(c, ge, oe, tol, b, fmt=bs.ELL)


# ------------------------------------------------------------------ block Jacobi
@pytest.mark.parametrize("bsz", [2, 4, 8])
@pytest.mark.parametrize("solver", [bs.BICGSTAB, bs.GMRES])
@pytest.mark.parametrize("gen", ["chem", "collision", "small"])
def test_block_jacobi(gen, solver, bsz):
    """Block-Jacobi preconditioner (blocks of bsz rows, the last one ragged
    where bsz does not divide n) against the oracle: one-wave teams with the
    bank-aware layout (n = 54), 1024-lane teams (n = 992), 32-lane teams sharing
    a wave (n = 20).  GMRES on 1024-lane teams keeps its basis in LDS and has
    no room for the block region: refused."""
    bt = {"chem": lambda: W.chem_jacobian(1500, n=54, seed=8),
          "collision": lambda: W.collision_stencil(24),
          "small": lambda: W.chem_jacobian(700, n=20, seed=9)}[gen]()
    c = Case(bt)
    if gen == "collision" and solver == bs.GMRES:
        with pytest.raises(bs.BatchSolveError) as e:
            c.gpu(bs.CSR, solver, precond=bs.PREC_BLOCK_JACOBI, block_size=bsz)
        assert e.value.code == bs.ERR_UNSUPPORTED
        return
    for fmt in (bs.CSR, bs.ELL):
        g = c.gpu(fmt, solver, precond=bs.PREC_BLOCK_JACOBI, block_size=bsz, max_iter=2000)
        o = c.oracle(fmt, solver, precond=bs.PREC_BLOCK_JACOBI, block_size=bsz, max_iter=2000)
        check(c, g, o, fmt=fmt)


def spd_band(n, n_batch, seed):
    """SPD pentadiagonal systems: a_ij = a_ji = -(1 + 0.5 U(0, 1)) for
    0 < |i - j| <= 2, a_ii = 1.1 sum_j |a_ij| + 0.1."""
    rng = np.random.default_rng(seed)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    mask = np.abs(i - j) <= 2
    rows, cols = np.nonzero(mask)
    row_ptr = np.concatenate([[0], np.cumsum(mask.sum(1))]).astype(np.int32)
    vals = np.empty((n_batch, rows.size))
    for s in range(n_batch):
        M = np.triu(-(1.0 + 0.5 * rng.random((n, n))), 1) * mask
        M = M + M.T
        np.fill_diagonal(M, 1.1 * np.abs(M).sum(1) + 0.1)
        vals[s] = M[rows, cols]
    b = 2 * rng.random((n_batch, n)) - 1
    return W.Batch("spd_band", n, row_ptr, cols.astype(np.int32), vals, b, np.zeros_like(b))


def test_block_jacobi_cg_and_rows_per_lane():
    """CG on SPD systems (one wave per system, then 1024-lane teams of eleven
    waves, where CG applies the preconditioner right after setting it up), and
    two rows per lane (n = 1500: 1024-lane teams)."""
    bt = spd_on_pattern(48, 400, seed=4)
    c = Case(bt)
    g = c.gpu(bs.CSR, bs.CG, precond=bs.PREC_BLOCK_JACOBI, block_size=4)
    o = c.oracle(bs.CSR, bs.CG, precond=bs.PREC_BLOCK_JACOBI, block_size=4)
    check(c, g, o)
    cb = Case(spd_band(700, 30, seed=5))
    for bsz in (2, 8):
        g = cb.gpu(bs.CSR, bs.CG, precond=bs.PREC_BLOCK_JACOBI, block_size=bsz)
        o = cb.oracle(bs.CSR, bs.CG, precond=bs.PREC_BLOCK_JACOBI, block_size=bsz)
        check(cb, g, o)
    c2 = Case(W.tridiag_stencil(n_batch=40, n=1500))
    g = c2.gpu(bs.CSR, bs.BICGSTAB, precond=bs.PREC_BLOCK_JACOBI, block_size=4, max_iter=3000)
    o = c2.oracle(bs.CSR, bs.BICGSTAB, precond=bs.PREC_BLOCK_JACOBI, block_size=4, max_iter=3000)
    check(c2, g, o)
    # two rows per lane of 1024-lane teams: blocks of 8 exceed a compute unit's LDS
    with pytest.raises(bs.BatchSolveError) as e:
        c2.gpu(bs.CSR, bs.BICGSTAB, precond=bs.PREC_BLOCK_JACOBI, block_size=8)
    assert e.value.code == bs.ERR_UNSUPPORTED


def test_block_jacobi_zero_pivot_and_errors():
    """A block whose first pivot is zero becomes the identity on both sides;
    mixed precision with block Jacobi is refused; block sizes other than 2, 4
    and 8 are invalid."""
    bt = W.tridiag_stencil(n_batch=50, n=40)
    v = bt.values.copy()
    v[:, 0] = 0.0        # a_00 = 0 in every system
    c = Case(bt)
    g = c.gpu(bs.CSR, bs.BICGSTAB, precond=bs.PREC_BLOCK_JACOBI, block_size=4, values=dev(v))
    o = c.oracle(bs.CSR, bs.BICGSTAB, precond=bs.PREC_BLOCK_JACOBI, block_size=4, values=v)
    check(c, g, o, values=v)
    with pytest.raises(bs.BatchSolveError) as e:
        c.gpu(bs.CSR, bs.BICGSTAB, precond=bs.PREC_BLOCK_JACOBI, precision=bs.MIXED)
    assert e.value.code == bs.ERR_UNSUPPORTED
    for bad in (3, 16, -2):
        with pytest.raises(bs.BatchSolveError) as e:
            c.gpu(bs.CSR, bs.BICGSTAB, precond=bs.PREC_BLOCK_JACOBI, block_size=bad)
        assert e.value.code == bs.ERR_INVALID_ARG


def full_pattern_batch(bt: W.Batch) -> W.Batch:
    """The same systems on the full pattern (every entry stored, zeros included)."""
    n = bt.n
    rows = np.repeat(np.arange(n), np.diff(bt.row_ptr))
    D = np.zeros((bt.n_batch, n, n))
    D[:, rows, bt.col_idx] = bt.values
    rp = (np.arange(n + 1) * n).astype(np.int32)
    ci = np.tile(np.arange(n), n).astype(np.int32)
    return W.Batch(bt.name + "_dense", n, rp, ci, D.reshape(bt.n_batch, n * n), bt.b, bt.x0)


@pytest.mark.parametrize("solver", [bs.BICGSTAB, bs.GMRES])
@pytest.mark.parametrize("gen", ["chem", "stiff", "small", "tridiag", "dense"])
def test_ilu(gen, solver):
    """ILU(0) against the oracle: the chemistry pattern (n = 54, 28 slots), a
    stiffer chemistry batch (gamma = 1e-3, a dozen or more iterations), n = 20,
    a tridiagonal pattern and a full pattern (ILU(0) is the exact LU there: one
    iteration), CSR and ELL."""
    bt = {"chem": lambda: W.chem_jacobian(1200, n=54, seed=13),
          "stiff": lambda: W.chem_jacobian(600, n=54, gamma=1e-3, seed=14),
          "small": lambda: W.chem_jacobian(900, n=20, seed=15),
          "tridiag": lambda: W.tridiag_stencil(n_batch=300, n=64, seed=16),
          "dense": lambda: full_pattern_batch(W.chem_jacobian(200, n=30, gamma=1e-3, seed=17))}[gen]()
    c = Case(bt)
    for fmt in (bs.CSR, bs.ELL):
        g = c.gpu(fmt, solver, precond=bs.PREC_ILU, max_iter=1000)
        o = c.oracle(fmt, solver, precond=bs.PREC_ILU, max_iter=1000)
        assert np.all(o[3] == O.CONVERGED)
        # Both sides divide by the pivots; the GPU's sweeps use FMAs and it
        # sums the backward sweep column by column.  How far such rounding
        # alone moves a count is measured on the oracle itself: its row- and
        # column-oriented backward substitutions (the same operations in
        # another order) give per system spread = |k_row - k_col|, and the bar
        # is 2 plus that spread (2 wherever the orders agree).
        oc = c.oracle(fmt, solver, precond=O.PREC_ILU_COL, max_iter=1000)
        assert np.array_equal(oc[3], o[3])
        spread = np.abs(oc[1].astype(np.int64) - o[1])
        say(f"  oracle order spread: max {spread.max()}, systems with spread > 0: "
            f"{int((spread > 0).sum())} of {len(spread)}")
        check(c, g, o, fmt=fmt, itol=ITOL + spread)
        if gen in ("tridiag", "dense"):
            assert np.all(g[1] == 1)


def test_ilu_zero_pivot_and_errors():
    """A zero first pivot makes M the identity on both sides (the solve runs
    unpreconditioned); CG, mixed precision and systems of more than 1024 rows
    are refused."""
    bt = W.tridiag_stencil(n_batch=200, n=40, seed=18)
    v = bt.values.copy()
    v[:, 0] = 0.0        # a_00 = 0 in every system (still invertible)
    c = Case(bt)
    for solver in (bs.BICGSTAB, bs.GMRES):
        g = c.gpu(bs.CSR, solver, precond=bs.PREC_ILU, values=dev(v))
        o = c.oracle(bs.CSR, solver, precond=bs.PREC_ILU, values=v)
        u = c.oracle(bs.CSR, solver, precond=bs.PREC_NONE, values=v)
        assert np.all(o[3] == O.CONVERGED) and np.array_equal(o[1], u[1])
        check(c, g, o, values=v)
    for solver, opt in ((bs.CG, {}), (bs.BICGSTAB, {"precision": bs.MIXED})):
        with pytest.raises(bs.BatchSolveError) as e:
            c.gpu(bs.CSR, solver, precond=bs.PREC_ILU, **opt)
        assert e.value.code == bs.ERR_UNSUPPORTED
    big = Case(W.tridiag_stencil(n_batch=4, n=1025))
    with pytest.raises(bs.BatchSolveError) as e:
        big.gpu(bs.CSR, bs.BICGSTAB, precond=bs.PREC_ILU)
    assert e.value.code == bs.ERR_UNSUPPORTED


@pytest.mark.parametrize("lower", [True, False])
@pytest.mark.parametrize("gen", ["chem", "small", "full"])
def test_trsv(gen, lower):
    """BatchTrsv against the oracle: the triangle of the chemistry matrices
    (n = 54), n = 20, and a full pattern, CSR and ELL: x, the residual of the
    triangle, zero iterations."""
    bt = {"chem": lambda: W.chem_jacobian(1000, n=54, gamma=1e-3, seed=21),
          "small": lambda: W.chem_jacobian(700, n=20, gamma=1e-3, seed=22),
          "full": lambda: full_pattern_batch(W.chem_jacobian(300, n=40, gamma=1e-3, seed=23))}[gen]()
    c = Case(bt)
    solver = bs.TRSV_LOWER if lower else bs.TRSV_UPPER
    for fmt in (bs.CSR, bs.ELL):
        xg, ig, rg, sg = c.gpu(fmt, solver, precond=bs.PREC_NONE)
        xo, io, ro, so = c.oracle(fmt, solver, precond=bs.PREC_NONE)
        assert np.all(so == O.CONVERGED) and np.array_equal(sg, so)
        assert np.all(ig == 0) and np.all(io == 0)
        nx = np.linalg.norm(xo, axis=1)
        assert np.all(np.linalg.norm(xg - xo, axis=1) <= 1e-12 * nx)
        assert np.all(rg <= 1e-13) and np.all(np.abs(rg - ro) <= 1e-13)


def test_trsv_breakdown_and_errors():
    """A zero diagonal entry: BREAKDOWN with x = 0 and residual 1 (relative), as
    in the oracle; b = 0 gives x = 0; mixed precision and systems of more than
    1024 rows are refused."""
    bt = W.chem_jacobian(200, n=30, seed=24)
    d5 = int(np.flatnonzero(bt.col_idx[bt.row_ptr[5]:bt.row_ptr[6]] == 5)[0]) + int(bt.row_ptr[5])
    v = bt.values.copy()
    v[7, d5] = 0.0
    b = bt.b.copy()
    b[9] = 0.0
    c = Case(bt)
    for solver in (bs.TRSV_LOWER, bs.TRSV_UPPER):
        xg, ig, rg, sg = c.gpu(bs.CSR, solver, precond=bs.PREC_NONE, values=dev(v), b=b)
        xo, io, ro, so = c.oracle(bs.CSR, solver, precond=bs.PREC_NONE, values=v, b=b)
        assert np.array_equal(sg, so)
        assert sg[7] == bs.BREAKDOWN and np.all(xg[7] == 0) and rg[7] == 1.0
        assert sg[9] == bs.CONVERGED and np.all(xg[9] == 0) and rg[9] == 0.0
        ok = sg == bs.CONVERGED
        assert np.allclose(xg[ok], xo[ok], rtol=1e-12, atol=1e-14)
    with pytest.raises(bs.BatchSolveError) as e:
        c.gpu(bs.CSR, bs.TRSV_LOWER, precond=bs.PREC_NONE, precision=bs.MIXED)
    assert e.value.code == bs.ERR_UNSUPPORTED
    big = Case(W.tridiag_stencil(n_batch=4, n=1025))
    with pytest.raises(bs.BatchSolveError) as e:
        big.gpu(bs.CSR, bs.TRSV_UPPER, precond=bs.PREC_NONE)
    assert e.value.code == bs.ERR_UNSUPPORTED


# ILU(0) and BatchTrsv beyond one wave: sparse factors, level-scheduled sweeps.
def shuffled_rows(bt: W.Batch, seed: int) -> W.Batch:
    """The same systems with the entries of every row stored in a random order."""
    rng = np.random.default_rng(seed)
    col = bt.col_idx.copy()
    vals = bt.values.copy()
    for i in range(bt.n):
        a, e = int(bt.row_ptr[i]), int(bt.row_ptr[i + 1])
        p = a + rng.permutation(e - a)
        col[a:e] = bt.col_idx[p]
        vals[:, a:e] = bt.values[:, p]
    return W.Batch(bt.name + "_shuffled", bt.n, bt.row_ptr, col, vals, bt.b, bt.x0)


MW_GENS = {
    # 9-point stencil, 16 x 12 grid: n = 192 (256-lane teams), 31 lower levels
    "stencil192": lambda: W.collision_stencil(48, nx=16, ny=12, seed=41),
    # the 992-row stencil of the collision batch (1024-lane teams)
    "stencil992": lambda: W.collision_stencil(16, nx=32, ny=31, seed=42),
    # chemistry-like, n = 144 (rows of up to ~30 entries, condition numbers up
    # to 4e4) and n = 300 (rows of up to 14).  At gamma = 1e-3 one of the
    # n = 300 systems (condition 6e4) ends its first GMRES cycle 3.5 % under
    # the tolerance in the oracle: rounding alone can then leave the true
    # residual above it, and the restarted cycle gains 0.1 % per step there, so
    # that batch is taken at gamma = 3e-4 (every system ends >= 30 % under).
    "chem144": lambda: W.chem_jacobian(96, n=144, fill=0.12, gamma=1e-3, seed=43),
    "chem300": lambda: W.chem_jacobian(64, n=300, fill=0.02, gamma=3e-4, seed=44),
    # rows stored out of column order
    "shuffled": lambda: shuffled_rows(W.collision_stencil(48, nx=16, ny=12, seed=45), 46),
    # 13 x 9 grid: n = 117, not a multiple of 4 (padded LDS regions)
    "stencil117": lambda: W.collision_stencil(40, nx=13, ny=9, seed=51),
    # tridiagonal, n = 700: ILU(0) is the exact LU (one step), 700 levels
    "tridiag700": lambda: W.tridiag_stencil(n_batch=40, n=700, seed=47),
}


@pytest.mark.parametrize("solver", [bs.BICGSTAB, bs.GMRES])
@pytest.mark.parametrize("gen", list(MW_GENS))
def test_ilu_multiwave(gen, solver):
    """ILU(0) on teams of 2..16 waves against the oracle, CSR and ELL.  The GPU
    takes the oracle's row-oriented sweeps in the same order (FMAs aside), so
    the plain parity bar applies.  GMRES with ILU(0) holds its basis in
    registers, up to 512 rows; beyond that it is refused."""
    bt = MW_GENS[gen]()
    c = Case(bt)
    if solver == bs.GMRES and bt.n > 512:
        with pytest.raises(bs.BatchSolveError) as e:
            c.gpu(bs.CSR, solver, precond=bs.PREC_ILU)
        assert e.value.code == bs.ERR_UNSUPPORTED
        return
    for fmt in (bs.CSR, bs.ELL):
        g = c.gpu(fmt, solver, precond=bs.PREC_ILU, max_iter=1000)
        o = c.oracle(fmt, solver, precond=bs.PREC_ILU, max_iter=1000)
        assert np.all(o[3] == O.CONVERGED)
        j = c.oracle(fmt, solver, precond=bs.PREC_JACOBI, max_iter=1000)
        say(f"  iterations: ILU(0) gpu {g[1].mean():.1f} oracle {o[1].mean():.1f}, "
            f"Jacobi {j[1].mean():.1f}")
        check(c, g, o, fmt=fmt)
        if gen == "tridiag700":
            assert np.all(g[1] == 1)
        else:
            assert o[1].mean() < j[1].mean()


def test_ilu_multiwave_zero_pivot_and_start():
    """Multi-wave ILU(0): a zero first pivot makes M the identity on both sides
    (on the GPU bit for bit the unpreconditioned solve); a non-zero initial
    guess; the absolute criterion."""
    bt = W.collision_stencil(32, nx=16, ny=12, seed=48)
    c = Case(bt)
    v = bt.values.copy()
    v[:, 0] = 0.0
    for solver in (bs.BICGSTAB, bs.GMRES):
        g = c.gpu(bs.CSR, solver, precond=bs.PREC_ILU, values=dev(v), max_iter=1000)
        gn = c.gpu(bs.CSR, solver, precond=bs.PREC_NONE, values=dev(v), max_iter=1000)
        for a, e in zip(g, gn):
            assert np.array_equal(a, e)
        o = c.oracle(bs.CSR, solver, precond=bs.PREC_ILU, values=v, max_iter=1000)
        u = c.oracle(bs.CSR, solver, precond=bs.PREC_NONE, values=v, max_iter=1000)
        assert np.array_equal(o[1], u[1])
        # Unpreconditioned BiCGSTAB on these systems is sensitive to rounding:
        # b changed by one unit in the last place moves the oracle's own count
        # by up to 4.  The bar is 2 plus that measured spread, per system.
        spread = np.zeros(bt.n_batch, dtype=np.int64)
        for f in (1 + 2.0**-52, 1 - 2.0**-53):
            p = c.oracle(bs.CSR, solver, precond=bs.PREC_NONE, values=v, b=bt.b * f, max_iter=1000)
            spread = np.maximum(spread, np.abs(p[1].astype(np.int64) - o[1]))
        say(f"  one-ulp spread of the oracle: max {spread.max()}")
        check(c, g, o, values=v, itol=ITOL + spread)
    x0 = np.random.default_rng(49).random((bt.n_batch, bt.n))
    g = c.gpu(bs.CSR, bs.BICGSTAB, precond=bs.PREC_ILU, x0=x0)
    o = c.oracle(bs.CSR, bs.BICGSTAB, precond=bs.PREC_ILU, x0=x0)
    check(c, g, o)
    b = bt.b * 512.0
    tol = 1e-8
    g = c.gpu(bs.CSR, bs.GMRES, precond=bs.PREC_ILU, tol=tol, b=b, extra_flags=bs.FLAG_ABS_TOL)
    o = O.batch_solve(c.OP, bt.values, b, fmt=O.CSR, solver=O.GMRES, tol=tol,
                      precond=bs.PREC_ILU, max_iter=500, absolute=True)
    check_absolute(c, g, o, tol, b)


@pytest.mark.parametrize("lower", [True, False])
@pytest.mark.parametrize("gen", ["stencil192", "stencil992", "chem300", "shuffled", "stencil117"])
def test_trsv_multiwave(gen, lower):
    """BatchTrsv on teams of 2..16 waves against the oracle, CSR and ELL."""
    bt = MW_GENS[gen]()
    c = Case(bt)
    solver = bs.TRSV_LOWER if lower else bs.TRSV_UPPER
    for fmt in (bs.CSR, bs.ELL):
        xg, ig, rg, sg = c.gpu(fmt, solver, precond=bs.PREC_NONE)
        xo, io, ro, so = c.oracle(fmt, solver, precond=bs.PREC_NONE)
        assert np.all(so == O.CONVERGED) and np.array_equal(sg, so)
        assert np.all(ig == 0)
        nx = np.linalg.norm(xo, axis=1)
        assert np.all(np.linalg.norm(xg - xo, axis=1) <= 1e-12 * nx)
        assert np.all(rg <= 1e-13) and np.all(np.abs(rg - ro) <= 1e-13)


def test_trsv_multiwave_breakdown():
    """Multi-wave BatchTrsv: a zero diagonal entry is a breakdown (x = 0), b = 0
    gives x = 0, as in the oracle."""
    bt = W.collision_stencil(12, nx=16, ny=12, seed=50)
    c = Case(bt)
    r = 100
    dpos = int(np.flatnonzero(bt.col_idx[bt.row_ptr[r]:bt.row_ptr[r + 1]] == r)[0]) + int(bt.row_ptr[r])
    v = bt.values.copy()
    v[3, dpos] = 0.0
    b = bt.b.copy()
    b[5] = 0.0
    for solver in (bs.TRSV_LOWER, bs.TRSV_UPPER):
        xg, ig, rg, sg = c.gpu(bs.CSR, solver, precond=bs.PREC_NONE, values=dev(v), b=b)
        xo, io, ro, so = c.oracle(bs.CSR, solver, precond=bs.PREC_NONE, values=v, b=b)
        assert np.array_equal(sg, so)
        assert sg[3] == bs.BREAKDOWN and np.all(xg[3] == 0) and rg[3] == 1.0
        assert sg[5] == bs.CONVERGED and np.all(xg[5] == 0) and rg[5] == 0.0
        ok = sg == bs.CONVERGED
        assert np.allclose(xg[ok], xo[ok], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("solver", [bs.BICGSTAB, bs.TRSV_LOWER])
def test_multiwave_ilu_trsv_multi_rhs_and_dev(solver):
    """Multi-wave ILU(0) (BiCGSTAB) and BatchTrsv with three right-hand sides
    per matrix: bit-identical to the matrices replicated once per right-hand
    side; and through bs_batch_solve_dev (the pattern as caller-owned device
    arrays): bit-identical to the handle entry."""
    k = 3
    bt = W.collision_stencil(20, nx=16, ny=12, seed=53)
    B, n = bt.n_batch, bt.n
    b = 2 * np.random.default_rng(54).random((B * k, n)) - 1
    c = Case(bt)
    pc = bs.PREC_ILU if solver == bs.BICGSTAB else bs.PREC_NONE

    def outs(m):
        return (torch.zeros((m, n), dtype=torch.float64, device="cuda:0"),
                torch.empty(m, dtype=torch.int32, device="cuda:0"),
                torch.empty(m, dtype=torch.float64, device="cuda:0"),
                torch.empty(m, dtype=torch.int32, device="cuda:0"))

    def host(t):
        torch.cuda.synchronize()
        return tuple(u.cpu().numpy() for u in t)

    x, it, rs, st = outs(B * k)
    say(f"  multi-rhs multi-wave solver={solver}")
    bs.bs_batch_solve(bs.CSR, c.P.handle, c.vals, dev(b), x, solver, pc, 1e-10, 500, it, rs, st,
                      bs.make_options(flags=bs.FLAG_X0_ZERO, n_rhs=k))
    g = host((x, it, rs, st))
    rep = W.Batch(bt.name + "_rep", n, bt.row_ptr, bt.col_idx, np.repeat(bt.values, k, axis=0), b,
                  np.zeros_like(b))
    cr = Case(rep)
    gr = cr.gpu(bs.CSR, solver, precond=pc)
    for u, v in zip(g, gr):
        assert np.array_equal(u, v)
    o = cr.oracle(bs.CSR, solver, precond=pc)
    if solver == bs.BICGSTAB:
        check(cr, g, o)
    else:
        assert np.array_equal(g[3], o[3])
        assert np.all(np.linalg.norm(g[0] - o[0], axis=1) <= 1e-12 * np.linalg.norm(o[0], axis=1))
    # caller-owned device pattern
    x, it, rs, st = outs(B)
    bs.bs_batch_solve_dev(bs.CSR, n, dev(bt.row_ptr.astype(np.int32)), dev(bt.col_idx.astype(np.int32)),
                          c.vals, dev(bt.b), x, solver, pc, 1e-10, 500, it, rs, st,
                          bs.make_options(flags=bs.FLAG_X0_ZERO))
    gd = host((x, it, rs, st))
    gh = c.gpu(bs.CSR, solver, precond=pc)
    for u, v in zip(gd, gh):
        assert np.array_equal(u, v)


@pytest.mark.parametrize("precond,bsz", [(bs.PREC_BLOCK_JACOBI, 4), (bs.PREC_ILU, 0)])
def test_stronger_preconditioners_absolute_and_dense(precond, bsz):
    """Block Jacobi and ILU(0) under the absolute stop criterion, and through the
    BatchDense entry (the full pattern: ILU(0) is the exact LU, one step)."""
    bt = W.chem_jacobian(n_batch=1000, n=54, gamma=1e-4, seed=25)
    c = Case(bt)
    b = bt.b * 1024.0
    tol = 1e-8
    for solver in (bs.BICGSTAB, bs.GMRES):
        g = c.gpu(bs.CSR, solver, precond=precond, tol=tol, b=b, extra_flags=bs.FLAG_ABS_TOL,
                  block_size=bsz, max_iter=1000)
        o = O.batch_solve(c.OP, bt.values, b, fmt=O.CSR, solver=SOLVER_O[solver], tol=tol,
                          precond=precond, block_size=max(bsz, 1), max_iter=1000, absolute=True)
        rel = O.batch_solve(c.OP, bt.values, b, fmt=O.CSR, solver=SOLVER_O[solver], tol=tol,
                            precond=precond, block_size=max(bsz, 1), max_iter=1000)
        assert o[1].sum() > rel[1].sum()
        check_absolute(c, g, o, tol, b)
    n = 40
    db = full_pattern_batch(W.chem_jacobian(n_batch=300, n=n, gamma=1e-4, seed=26))
    cd = Case(db)
    P = bs.Pattern.dense(n)
    B = db.n_batch
    for solver in (bs.BICGSTAB, bs.GMRES):
        x = torch.zeros((B, n), dtype=torch.float64, device="cuda:0")
        it = torch.empty(B, dtype=torch.int32, device="cuda:0")
        rs = torch.empty(B, dtype=torch.float64, device="cuda:0")
        st = torch.empty(B, dtype=torch.int32, device="cuda:0")
        bs.bs_batch_solve(bs.DENSE, P.handle, dev(db.values), dev(db.b), x, solver, precond, 1e-10,
                          500, it, rs, st, bs.make_options(flags=bs.FLAG_X0_ZERO, block_size=bsz))
        torch.cuda.synchronize()
        g = (x.cpu().numpy(), it.cpu().numpy(), rs.cpu().numpy(), st.cpu().numpy())
        o = cd.oracle(bs.CSR, solver, precond=precond, block_size=max(bsz, 1))
        check(cd, g, o)
        if precond == bs.PREC_ILU:
            assert np.all(g[1] == 1)


@pytest.mark.parametrize("gen,solver,fmt", [("chem", bs.BICGSTAB, bs.CSR), ("chem", bs.GMRES, bs.ELL),
                                            ("small", bs.BICGSTAB, bs.CSR),
                                            ("collision", bs.BICGSTAB, bs.CSR)])
def test_multi_rhs(gen, solver, fmt):
    """Three right-hand sides per matrix (n_rhs = 3): bit-identical to solving
    the matrices replicated once per right-hand side, and within the parity bar
    of the oracle.  One team per wave with staged values (n = 54), two teams
    per wave (n = 20), 1024-lane teams (n = 992)."""
    k = 3
    bt = {"chem": lambda: W.chem_jacobian(400, n=54, seed=27),
          "small": lambda: W.chem_jacobian(500, n=20, seed=28),
          "collision": lambda: W.collision_stencil(12)}[gen]()
    B, n = bt.n_batch, bt.n
    rng = np.random.default_rng(29)
    b = 2 * rng.random((B * k, n)) - 1
    c = Case(bt)
    x = torch.zeros((B * k, n), dtype=torch.float64, device="cuda:0")
    it = torch.empty(B * k, dtype=torch.int32, device="cuda:0")
    rs = torch.empty(B * k, dtype=torch.float64, device="cuda:0")
    st = torch.empty(B * k, dtype=torch.int32, device="cuda:0")
    say(f"  multi-rhs {gen} solver={solver} fmt={fmt}")
    bs.bs_batch_solve(fmt, c.P.handle, c.values(fmt), dev(b), x, solver, bs.PREC_JACOBI, 1e-10,
                      1000, it, rs, st, bs.make_options(flags=bs.FLAG_X0_ZERO, n_rhs=k))
    torch.cuda.synchronize()
    g = (x.cpu().numpy(), it.cpu().numpy(), rs.cpu().numpy(), st.cpu().numpy())
    rep = W.Batch(bt.name + "_rep", n, bt.row_ptr, bt.col_idx, np.repeat(bt.values, k, axis=0), b,
                  np.zeros_like(b))
    cr = Case(rep)
    gr = cr.gpu(fmt, solver, max_iter=1000)
    for u, v in zip(g, gr):
        assert np.array_equal(u, v)
    o = cr.oracle(fmt, solver, max_iter=1000)
    check(cr, g, o, fmt=fmt)


def test_multi_rhs_errors():
    bt = W.chem_jacobian(10, n=54, seed=30)
    c = Case(bt)
    with pytest.raises(bs.BatchSolveError) as e:
        c.gpu(bs.CSR, bs.BICGSTAB, n_rhs=-1)
    assert e.value.code == bs.ERR_INVALID_ARG
    with pytest.raises(ValueError):
        c.gpu(bs.CSR, bs.BICGSTAB, n_rhs=3)      # 10 rows of b: not a multiple of 3


# ------------------------------------------------------------------ spill tier
def long_row_batch(B, seed):
    """n = 144 chemistry-like Jacobians at fill 0.5: rows of up to ~90 entries,
    beyond the 64 register slots of the register kernels."""
    return W.chem_jacobian(B, n=144, fill=0.5, seed=seed)


@pytest.mark.parametrize("fmt", [bs.CSR, bs.ELL])
@pytest.mark.parametrize("solver", [bs.BICGSTAB, bs.CG, bs.GMRES])
def test_streamed_long_rows(fmt, solver):
    """Rows longer than the register slots take the streamed placement (the
    rows stay in HBM and are read at every product): BiCGSTAB on the long-row
    chemistry batch and CG on SPD systems of a symmetrised random pattern
    (n = 200), CSR and ELL values, against the oracle."""
    bt = long_row_batch(300, 41) if solver != bs.CG else spd_on_pattern(200, 120, 42)
    assert np.diff(bt.row_ptr).max() > bs.MAX_ROW_NNZ
    p = bs.bs_plan(fmt, bt.n, int(bt.row_ptr[-1]), int(np.diff(bt.row_ptr).max()), solver)
    assert p["slots"] == 0
    c = Case(bt)
    g = c.gpu(fmt, solver, max_iter=1000)
    check(c, g, c.oracle(fmt, solver, max_iter=1000), fmt=fmt)
    # no preconditioner, and a nonzero initial guess
    x0 = np.random.default_rng(43).standard_normal(bt.b.shape)
    g = c.gpu(fmt, solver, precond=bs.PREC_NONE, x0=x0, max_iter=1000)
    check(c, g, c.oracle(fmt, solver, precond=bs.PREC_NONE, x0=x0, max_iter=1000), fmt=fmt)


def spd_grid9(nx, ny, n_batch, seed):
    """SPD systems on the nine-point pattern: a_ij = a_ji = -(1 + 0.5 U(0, 1))
    for neighbours, a_ii = 1.1 sum_j |a_ij| + 0.1."""
    rp, ci, _, _ = W.grid9_pattern(nx, ny)
    n = nx * ny
    rows = np.repeat(np.arange(n), np.diff(rp))
    _, pair = np.unique(np.minimum(rows, ci) * n + np.maximum(rows, ci), return_inverse=True)
    off = rows != ci
    rng = np.random.default_rng(seed)
    vals = np.empty((n_batch, ci.size))
    for s in range(n_batch):
        v = -(1.0 + 0.5 * rng.random(pair.max() + 1))[pair] * off
        d = np.zeros(n)
        np.add.at(d, rows, np.abs(v))
        v[~off] = 1.1 * d[rows[~off]] + 0.1
        vals[s] = v
    b = 2 * rng.random((n_batch, n)) - 1
    return W.Batch("spd_grid9", n, rp, ci, vals, b, np.zeros_like(b))


@pytest.mark.parametrize("fmt", [bs.CSR, bs.ELL])
@pytest.mark.parametrize("solver", [bs.BICGSTAB, bs.CG])
def test_streamed_two_rows_per_lane(fmt, solver):
    """Systems of 1025..2048 rows whose rows are longer than the 8 register
    slots of the 2-row shapes take the streamed placement on workgroups of
    1024 lanes x 2 rows: nine-point stencils of 40 x 40 (n = 1600) and 64 x 32
    (n = 2048), nonsymmetric for BiCGSTAB and SPD for CG, against the oracle;
    mixed GMRES there is refused."""
    for nx, ny, B in ((40, 40, 24), (64, 32, 9)):
        bt = (W.collision_stencil(B, nx=nx, ny=ny, seed=nx) if solver == bs.BICGSTAB
              else spd_grid9(nx, ny, B, nx))
        p = bs.bs_plan(fmt, bt.n, int(bt.row_ptr[-1]), 9, solver)
        assert p["slots"] == 0 and p["group_size"] == 1024 and p["rows_per_lane"] == 2
        c = Case(bt)
        g = c.gpu(fmt, solver, max_iter=2000)
        check(c, g, c.oracle(fmt, solver, max_iter=2000), fmt=fmt)
    if solver == bs.BICGSTAB:
        # mixed precision: x within the FP64 bar of the FP64 oracle
        g = c.gpu(fmt, solver, max_iter=2000, precision=bs.MIXED)
        check(c, g, c.oracle(fmt, solver, max_iter=2000), fmt=fmt, itol=10**9)
        with pytest.raises(bs.BatchSolveError) as e:
            c.gpu(fmt, bs.GMRES, precision=bs.MIXED)
        assert e.value.code == bs.ERR_UNSUPPORTED


@pytest.mark.parametrize("fmt", [bs.CSR, bs.ELL])
def test_streamed_gmres_beyond_1024_rows(fmt):
    """GMRES on systems of 1025..2048 rows (streamed rows on 1024-lane x
    2-row workgroups, the basis in device memory): nine-point stencils of
    n = 1600 and 2048 against the oracle with GMRES(30) restarts, restart 10
    without a preconditioner from a nonzero start, and a max_iter stop."""
    for nx, ny, B in ((40, 40, 16), (64, 32, 6)):
        bt = W.collision_stencil(B, nx=nx, ny=ny, seed=nx + 1)
        p = bs.bs_plan(fmt, bt.n, int(bt.row_ptr[-1]), 9, bs.GMRES)
        assert p["slots"] == 0 and p["rows_per_lane"] == 2 and p["group_size"] == 1024
        c = Case(bt)
        g = c.gpu(fmt, bs.GMRES, max_iter=2000)
        o = c.oracle(fmt, bs.GMRES, max_iter=2000)
        assert o[1].max() > 30  # restarts happen
        check(c, g, o, fmt=fmt)
    x0 = np.random.default_rng(61).standard_normal(bt.b.shape)
    g = c.gpu(fmt, bs.GMRES, precond=bs.PREC_NONE, x0=x0, restart=10, max_iter=3000)
    check(c, g, c.oracle(fmt, bs.GMRES, precond=bs.PREC_NONE, x0=x0, restart=10, max_iter=3000),
          fmt=fmt)
    g = c.gpu(fmt, bs.GMRES, max_iter=20)
    o = c.oracle(fmt, bs.GMRES, max_iter=20)
    assert np.all(o[3] == O.MAX_ITER) and np.array_equal(g[3], o[3]) and np.all(g[1] == 20)
    assert np.allclose(g[2], o[2], rtol=1e-6)


@pytest.mark.parametrize("solver", [bs.BICGSTAB, bs.GMRES])
def test_streamed_2048_options_and_edges(solver):
    """The 1024-lane x 2-row streamed paths (BiCGSTAB; GMRES with its basis in
    device memory) with the options of the register kernels: two right-hand
    sides per matrix (bit-identical to the replicated batch), a second initial
    guess (the smaller residual wins), b = 0, NaN in b, max_iter = 0, and the
    oracle's statuses on a system without a preconditioner."""
    bt = W.collision_stencil(6, nx=40, ny=40, seed=62)
    c = Case(bt)
    B, n, k = bt.n_batch, bt.n, 2
    b = 2 * np.random.default_rng(63).random((B * k, n)) - 1
    x = torch.zeros((B * k, n), dtype=torch.float64, device="cuda:0")
    it = torch.empty(B * k, dtype=torch.int32, device="cuda:0")
    rs = torch.empty(B * k, dtype=torch.float64, device="cuda:0")
    st = torch.empty(B * k, dtype=torch.int32, device="cuda:0")
    say(f"  2048-row streamed options solver={solver}")
    bs.bs_batch_solve(bs.CSR, c.P.handle, c.vals, dev(b), x, solver, bs.PREC_JACOBI, 1e-10,
                      2000, it, rs, st, bs.make_options(flags=bs.FLAG_X0_ZERO, n_rhs=k))
    torch.cuda.synchronize()
    g = (x.cpu().numpy(), it.cpu().numpy(), rs.cpu().numpy(), st.cpu().numpy())
    rep = W.Batch("rep", n, bt.row_ptr, bt.col_idx, np.repeat(bt.values, k, axis=0), b,
                  np.zeros_like(b))
    cr = Case(rep)
    for u, v in zip(g, cr.gpu(bs.CSR, solver, max_iter=2000)):
        assert np.array_equal(u, v)
    check(cr, g, cr.oracle(bs.CSR, solver, max_iter=2000))
    # a second initial guess: x0 = 0 against the oracle's solution
    xo = c.oracle(bs.CSR, solver, max_iter=2000)[0]
    used = torch.full((B,), -1, dtype=torch.int32, device="cuda:0")
    g = c.gpu(bs.CSR, solver, x0=np.zeros_like(bt.b), x_alt=dev(xo), alt_used=used)
    assert np.all(used.cpu().numpy() == 1) and np.all(g[3] == bs.CONVERGED)
    assert np.all(g[1] <= 1)
    # b = 0, NaN in b, max_iter = 0
    bb = bt.b.copy()
    bb[2] = 0.0
    bb[4, 7] = np.nan
    g = c.gpu(bs.CSR, solver, b=bb)
    o = c.oracle(bs.CSR, solver, b=bb)
    assert np.array_equal(g[3], o[3])
    assert g[3][2] == bs.CONVERGED and np.all(g[0][2] == 0.0) and g[3][4] == bs.NONFINITE
    g = c.gpu(bs.CSR, solver, max_iter=0)
    assert np.all(g[3] == bs.MAX_ITER) and np.all(g[1] == 0)


@pytest.mark.parametrize("n", [65, 100, 300])
@pytest.mark.parametrize("solver", [bs.CG, bs.BICGSTAB, bs.GMRES])
def test_streamed_dense(n, solver):
    """BatchDense beyond 64 rows: the full pattern's rows are streamed."""
    bt = dense_batch(n, 48, seed=n + 1, spd=(solver == bs.CG))
    c = Case(bt)
    P = bs.Pattern.dense(n)
    B = bt.n_batch
    x = torch.zeros((B, n), dtype=torch.float64, device="cuda:0")
    it = torch.empty(B, dtype=torch.int32, device="cuda:0")
    rs = torch.empty(B, dtype=torch.float64, device="cuda:0")
    st = torch.empty(B, dtype=torch.int32, device="cuda:0")
    say(f"  streamed dense n={n} solver={solver}")
    bs.bs_batch_solve(bs.DENSE, P.handle, dev(bt.values), dev(bt.b), x, solver, bs.PREC_JACOBI,
                      1e-10, 500, it, rs, st, bs.make_options(flags=bs.FLAG_X0_ZERO))
    torch.cuda.synchronize()
    g = (x.cpu().numpy(), it.cpu().numpy(), rs.cpu().numpy(), st.cpu().numpy())
    check(c, g, c.oracle(bs.CSR, solver))


def test_streamed_mixed_multi_rhs_and_alt():
    """The streamed placement with the options of the register kernels: mixed
    precision (x within the FP64 bar), several right-hand sides per matrix
    (bit-identical to the replicated batch), a second initial guess (the
    smaller residual wins), and the edge cases (b = 0, NaN, max_iter = 0)."""
    bt = long_row_batch(200, 44)
    c = Case(bt)
    outer = torch.zeros(bt.n_batch, dtype=torch.int32, device="cuda:0")
    g = c.gpu(bs.CSR, bs.BICGSTAB, max_iter=2000, precision=bs.MIXED, outer_iters=outer)
    assert np.all(g[3] == bs.CONVERGED) and outer.min().item() >= 1
    check(c, g, c.oracle(bs.CSR, bs.BICGSTAB, max_iter=2000), itol=10**9)
    # several right-hand sides
    k = 2
    B, n = bt.n_batch, bt.n
    b = 2 * np.random.default_rng(45).random((B * k, n)) - 1
    x = torch.zeros((B * k, n), dtype=torch.float64, device="cuda:0")
    it = torch.empty(B * k, dtype=torch.int32, device="cuda:0")
    rs = torch.empty(B * k, dtype=torch.float64, device="cuda:0")
    st = torch.empty(B * k, dtype=torch.int32, device="cuda:0")
    bs.bs_batch_solve(bs.CSR, c.P.handle, c.vals, dev(b), x, bs.BICGSTAB, bs.PREC_JACOBI, 1e-10,
                      1000, it, rs, st, bs.make_options(flags=bs.FLAG_X0_ZERO, n_rhs=k))
    torch.cuda.synchronize()
    g = (x.cpu().numpy(), it.cpu().numpy(), rs.cpu().numpy(), st.cpu().numpy())
    rep = W.Batch("long_rep", n, bt.row_ptr, bt.col_idx, np.repeat(bt.values, k, axis=0), b,
                  np.zeros_like(b))
    cr = Case(rep)
    for u, v in zip(g, cr.gpu(bs.CSR, bs.BICGSTAB, max_iter=1000)):
        assert np.array_equal(u, v)
    check(cr, g, cr.oracle(bs.CSR, bs.BICGSTAB, max_iter=1000))
    # a second initial guess: x0 = 0 against the oracle's solution
    xo = c.oracle(bs.CSR, bs.BICGSTAB)[0]
    alt = dev(xo)
    used = torch.full((B,), -1, dtype=torch.int32, device="cuda:0")
    x0 = np.zeros_like(bt.b)
    g = c.gpu(bs.CSR, bs.BICGSTAB, x0=x0, x_alt=alt, alt_used=used)
    assert np.all(used.cpu().numpy() == 1) and np.all(g[3] == bs.CONVERGED)
    assert np.all(g[1] <= 1)
    # edge cases
    bb = bt.b.copy()
    bb[3] = 0.0
    bb[5, 7] = np.nan
    g = c.gpu(bs.CSR, bs.BICGSTAB, b=bb)
    assert g[3][3] == bs.CONVERGED and np.all(g[0][3] == 0.0) and g[3][5] == bs.NONFINITE
    g = c.gpu(bs.CSR, bs.BICGSTAB, max_iter=0)
    assert np.all(g[3] == bs.MAX_ITER) and np.all(g[1] == 0)
    # what the streamed placement does not take
    for solver, prec in ((bs.GMRES, bs.PREC_BLOCK_JACOBI), (bs.BICGSTAB, bs.PREC_BLOCK_JACOBI),
                         (bs.BICGSTAB, bs.PREC_ILU)):
        with pytest.raises(bs.BatchSolveError) as e:
            c.gpu(bs.CSR, solver, precond=prec)
        assert e.value.code == bs.ERR_UNSUPPORTED


# ------------------------------------------------------------------ pattern in device memory
@pytest.mark.parametrize("fmt", [bs.CSR, bs.ELL, bs.DENSE])
def test_batch_solve_dev_matches_handle(fmt):
    """bs_batch_solve_dev, the shared pattern as caller-owned device arrays,
    gives the bits of bs_batch_solve on a pattern handle (same kernels), on the
    first call (arrays read and validated) and on a cached one; a pattern
    rewritten in place is read again under a new structure_generation."""
    bt = W.chem_jacobian(300, n=54, seed=51) if fmt != bs.DENSE else dense_batch(40, 200, seed=52)
    c = Case(bt)
    n, B = bt.n, bt.n_batch
    if fmt == bs.DENSE:
        P = bs.Pattern.dense(n)
        vals, rp, ci, w = dev(bt.values), None, None, 0
    elif fmt == bs.CSR:
        P = c.P
        vals, rp, ci, w = c.vals, dev(bt.row_ptr.astype(np.int32)), dev(bt.col_idx.astype(np.int32)), 0
    else:
        P = c.P
        vals = c.values(bs.ELL)
        w = P.ell_width
        ci = dev(np.asarray(bs.bs_pattern_ell_cols(P.handle), np.int32))
        rp = None

    def run(gen=0, handle=False):
        x = torch.zeros((B, n), dtype=torch.float64, device="cuda:0")
        it = torch.empty(B, dtype=torch.int32, device="cuda:0")
        rs = torch.empty(B, dtype=torch.float64, device="cuda:0")
        st = torch.empty(B, dtype=torch.int32, device="cuda:0")
        opts = bs.make_options(flags=bs.FLAG_X0_ZERO, structure_generation=gen)
        if handle:
            bs.bs_batch_solve(fmt, P.handle, vals, dev(bt.b), x, bs.BICGSTAB, bs.PREC_JACOBI,
                              1e-10, 500, it, rs, st, opts)
        else:
            bs.bs_batch_solve_dev(fmt, n, rp, ci, vals, dev(bt.b), x, bs.BICGSTAB,
                                  bs.PREC_JACOBI, 1e-10, 500, it, rs, st, opts, ell_width=w)
        torch.cuda.synchronize()
        return x.cpu().numpy(), it.cpu().numpy(), rs.cpu().numpy(), st.cpu().numpy()

    ref = run(handle=True)
    for g in (run(), run()):
        for u, v in zip(ref, g):
            assert np.array_equal(u, v)
    check(c, ref, c.oracle(bs.CSR if fmt == bs.DENSE else fmt, bs.BICGSTAB), fmt=fmt if fmt != bs.DENSE else bs.CSR)
    if fmt == bs.CSR:
        # a column repeated in a row, written in place: refused under a new
        # generation (the old pattern stays cached under the old one)
        bad = bt.col_idx.astype(np.int32).copy()
        bad[1] = bad[0]
        ci.copy_(dev(bad))
        with pytest.raises(bs.BatchSolveError) as e:
            run(gen=1)
        assert e.value.code == bs.ERR_PATTERN
        for u, v in zip(ref, run(gen=0)):
            assert np.array_equal(u, v)


def test_streamed_gmres_restarts_and_mixed():
    """GMRES in the streamed placement: restart lengths 30, 8 and 3 (FP64, the
    oracle's step counts within the bar) and the mixed form (every system
    converged, x within the FP64 bar), with a nonzero initial guess."""
    bt = long_row_batch(96, 46)
    c = Case(bt)
    for m in (30, 8, 3):
        g = c.gpu(bs.CSR, bs.GMRES, restart=m, max_iter=1000)
        check(c, g, c.oracle(bs.CSR, bs.GMRES, restart=m, max_iter=1000))
    x0 = np.random.default_rng(47).standard_normal(bt.b.shape)
    g = c.gpu(bs.CSR, bs.GMRES, x0=x0, max_iter=1000)
    check(c, g, c.oracle(bs.CSR, bs.GMRES, x0=x0, max_iter=1000))
    g = c.gpu(bs.ELL, bs.GMRES, max_iter=2000, precision=bs.MIXED)
    assert np.all(g[3] == bs.CONVERGED)
    check(c, g, c.oracle(bs.ELL, bs.GMRES, max_iter=2000), fmt=bs.ELL, itol=10**9)
