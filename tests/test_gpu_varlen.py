"""GPU parity of the uneven-batch path (systems of different sizes and patterns
in one persistent launch) against the FP64 CPU oracle, through the C ABI.

The oracle solves each pattern's systems as one fixed-size batch; the bar per
system is that of the fixed-size parity tests (status equal, true residual of
the GPU's x <= tol, x within 1e-8 of the oracle's, iterations within 2).
"""
import os
import sys
from types import SimpleNamespace

import numpy as np
import pytest

import oracle as O
from paper_2308_08417_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2308_08417_amd import batchsolve as bs  # noqa: E402

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_gpu_parity import check, dev, say  # noqa: E402

SOLVER_O = {bs.CG: O.CG, bs.BICGSTAB: O.BICGSTAB}


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bs.lib()


def symmetric_values(vb: W.VarBatch, seed: int) -> np.ndarray:
    """SPD values on symmetric band patterns: a_ij = a_ji = -(1 + 0.5 u) with u
    drawn per unordered pair, a_ii = 1.1 sum_j |a_ij| + 0.1 (strictly dominant)."""
    rng = np.random.default_rng(seed)
    vals = np.empty_like(vb.values)
    for s in range(vb.n_batch):
        rp, ci, _, _, _ = vb.system(s)
        n = rp.size - 1
        rows = np.repeat(np.arange(n), np.diff(rp))
        lo, hi = np.minimum(rows, ci), np.maximum(rows, ci)
        u = rng.random(n * 8).reshape(n, 8)
        w = -(1.0 + 0.5 * u[lo, np.minimum(hi - lo, 7)])
        diag = rows == ci
        w[diag] = 0.0
        w[diag] = 1.1 * np.bincount(rows, weights=np.abs(w), minlength=n) + 0.1
        vals[vb.val_off[s]:vb.val_off[s + 1]] = w
    return vals


class VCase:
    """An uneven batch on the device plus its per-pattern oracle groups."""

    def __init__(self, vb: W.VarBatch, values=None):
        self.vb = vb
        self.values = vb.values if values is None else values
        self.h = bs.VarBatch(vb.pat_rows, vb.pat_rowptr_off, vb.rowptr_all, vb.pat_col_off,
                             vb.col_all, vb.pat_id)
        self.dv = dev(self.values)
        self.db = dev(vb.b)

    def outputs(self):
        B = self.vb.n_batch
        x = torch.full((self.vb.b.size,), np.nan, dtype=torch.float64, device="cuda:0")
        it = torch.full((B,), -7, dtype=torch.int32, device="cuda:0")
        rs = torch.full((B,), -7.0, dtype=torch.float64, device="cuda:0")
        st = torch.full((B,), -7, dtype=torch.int32, device="cuda:0")
        return x, it, rs, st

    def gpu(self, solver, precond=bs.PREC_JACOBI, tol=1e-10, max_iter=1000, values=None, b=None,
            x0=None, **opt):
        say(f"  varlen gpu: B={self.vb.n_batch} rows={self.vb.b.size} solver={solver} "
            f"prec={precond} tol={tol} max_iter={max_iter} opt={opt}")
        x, it, rs, st = self.outputs()
        flags = bs.FLAG_X0_ZERO
        if x0 is not None:
            x.copy_(dev(x0))
            flags = 0
        opts = bs.make_options(flags=flags, **opt)
        bs.bs_varbatch_solve(self.h.handle, self.dv if values is None else values,
                             self.db if b is None else b, x, solver, precond, tol, max_iter, it,
                             rs, st, opts)
        torch.cuda.synchronize()
        return x.cpu().numpy(), it.cpu().numpy(), rs.cpu().numpy(), st.cpu().numpy()

    def groups(self):
        vb = self.vb
        for p in range(len(vb.pat_rows)):
            sys_ = np.flatnonzero(vb.pat_id == p)
            if sys_.size == 0:
                continue
            n = int(vb.pat_rows[p])
            rp = vb.rowptr_all[vb.pat_rowptr_off[p]: vb.pat_rowptr_off[p] + n + 1]
            ci = vb.col_all[vb.pat_col_off[p]: vb.pat_col_off[p] + rp[-1]]
            rows = (vb.row_off[sys_][:, None] + np.arange(n)).ravel()
            vals = (vb.val_off[sys_][:, None] + np.arange(rp[-1])).ravel()
            yield sys_, n, rp, ci, rows, vals

    def check(self, g, solver, precond=bs.PREC_JACOBI, tol=1e-10, max_iter=1000, values=None,
              b=None, x0=None, itol=2, block_size=8):
        xg, ig, rg, sg = g
        V = self.values if values is None else values
        Bv = self.vb.b if b is None else b
        for sys_, n, rp, ci, rows, vals in self.groups():
            OP = O.Pattern(n, rp, ci)
            v = V[vals].reshape(sys_.size, -1)
            bb = Bv[rows].reshape(sys_.size, n)
            xx = None if x0 is None else x0[rows].reshape(sys_.size, n)
            o = O.batch_solve(OP, v, bb, x0=xx, solver=SOLVER_O[solver], precond=precond,
                              tol=tol, max_iter=max_iter, block_size=block_size)
            case = SimpleNamespace(batch=SimpleNamespace(b=bb, row_ptr=rp), OP=OP,
                                   oracle_values=lambda fmt, v=v: v)
            gg = (xg[rows].reshape(sys_.size, n), ig[sys_], rg[sys_], sg[sys_])
            check(case, gg, o, tol=tol, itol=itol)


def test_absolute_criterion_uneven():
    """Absolute stop criterion (Tab. 2) in the uneven path: b scaled by 2^10;
    the oracle solves each pattern's systems with the absolute criterion."""
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from test_gpu_parity import check_absolute
    c = VCase(W.uneven_banded(300, 16, 1024, seed=7))
    b = c.vb.b * 1024.0
    tol = 1e-8
    x, it, rs, st = c.outputs()
    bs.bs_varbatch_solve(c.h.handle, c.dv, dev(b), x, bs.BICGSTAB, bs.PREC_JACOBI, tol, 1000, it,
                         rs, st, bs.make_options(flags=bs.FLAG_X0_ZERO | bs.FLAG_ABS_TOL))
    torch.cuda.synchronize()
    xg, ig, rg, sg = x.cpu().numpy(), it.cpu().numpy(), rs.cpu().numpy(), st.cpu().numpy()
    assert np.all(sg == bs.CONVERGED)
    for sys_, n, rp, ci, rows, vals in c.groups():
        OP = O.Pattern(n, rp, ci)
        v = c.values[vals].reshape(sys_.size, -1)
        bb = b[rows].reshape(sys_.size, n)
        o = O.batch_solve(OP, v, bb, solver=O.BICGSTAB, tol=tol, max_iter=1000, absolute=True)
        case = SimpleNamespace(batch=SimpleNamespace(b=bb, row_ptr=rp), OP=OP,
                               oracle_values=lambda fmt, v=v: v)
        gg = (xg[rows].reshape(sys_.size, n), ig[sys_], rg[sys_], sg[sys_])
        check_absolute(case, gg, o, tol, bb)


def test_ilu_uneven_refused():
    """ILU(0) runs on the fixed-size path only (its factors and levels belong to
    one shared pattern), and the uneven path takes one right-hand side per
    system: both are refused."""
    c = VCase(W.uneven_banded(20, 16, 200, seed=19))
    with pytest.raises(bs.BatchSolveError) as e:
        c.gpu(bs.BICGSTAB, precond=bs.PREC_ILU)
    assert e.value.code == bs.ERR_UNSUPPORTED
    with pytest.raises(bs.BatchSolveError) as e:
        c.gpu(bs.BICGSTAB, n_rhs=2)
    assert e.value.code == bs.ERR_UNSUPPORTED


@pytest.mark.parametrize("bsz", [2, 8])
def test_block_jacobi_uneven(bsz):
    """Block Jacobi in the uneven path: BiCGSTAB on every team size, CG on SPD
    bands; fewer iterations than scalar Jacobi on these banded systems."""
    c = VCase(W.uneven_banded(300, 16, 1024, seed=11))
    g = c.gpu(bs.BICGSTAB, precond=bs.PREC_BLOCK_JACOBI, block_size=bsz)
    assert np.all(g[3] == bs.CONVERGED)
    c.check(g, bs.BICGSTAB, precond=bs.PREC_BLOCK_JACOBI, block_size=bsz)
    if bsz == 8:
        g1 = c.gpu(bs.BICGSTAB)
        assert g[1].mean() < 0.8 * g1[1].mean()
    vb = W.uneven_banded(200, 16, 1024, w_min=5, w_max=5, seed=12)
    cs = VCase(vb, symmetric_values(vb, seed=12))
    g = cs.gpu(bs.CG, precond=bs.PREC_BLOCK_JACOBI, block_size=bsz)
    assert np.all(g[3] == bs.CONVERGED)
    cs.check(g, bs.CG, precond=bs.PREC_BLOCK_JACOBI, block_size=bsz)


def test_bicgstab_mixed_sizes():
    """Every team size 64..1024 in one launch (n from 16 to 1024)."""
    c = VCase(W.uneven_banded(400, 16, 1024, seed=1))
    g = c.gpu(bs.BICGSTAB)
    assert np.all(g[3] == bs.CONVERGED)
    c.check(g, bs.BICGSTAB)


def test_cg_spd_mixed_sizes():
    vb = W.uneven_banded(300, 16, 1024, w_min=5, w_max=5, seed=2)   # symmetric bands
    c = VCase(vb, symmetric_values(vb, seed=2))
    g = c.gpu(bs.CG)
    assert np.all(g[3] == bs.CONVERGED)
    c.check(g, bs.CG)


def test_small_systems_many_per_task():
    """Teams of one wave: 16 systems per task; a ragged last task."""
    c = VCase(W.uneven_banded(1000 + 13, 16, 64, seed=3))
    g = c.gpu(bs.BICGSTAB, precond=bs.PREC_NONE)
    c.check(g, bs.BICGSTAB, precond=bs.PREC_NONE)


@pytest.mark.parametrize("shape", [0, 1, 2])
def test_policies(shape):
    """Every workgroup shape (1024 x 1, 512 x 2, 256 x 4 rows per lane) and
    queue order meets the oracle.  The queue order changes who solves a system,
    not the arithmetic: orders 0 and 2 give the same bits, and so does order 1
    (teams twice as wide) with one row per lane; with R rows per lane a wider
    team moves rows between lanes, which reorders the sums."""
    c = VCase(W.uneven_banded(500, 16, 1024, seed=4))
    ref = None
    for order in (0, 2, 1):
        p = 3 * shape + order
        bs.bs_varbatch_set_policy(c.h.handle, p)
        q = c.h.query()
        assert q["policy"] == p and q["n_tasks"] >= 1
        g = c.gpu(bs.BICGSTAB)
        if ref is None:
            ref = g
            c.check(g, bs.BICGSTAB)
        elif order == 2 or shape == 0:
            for u, v in zip(ref, g):
                assert np.array_equal(u, v), f"policy {p} differs"
        else:
            c.check(g, bs.BICGSTAB)
    with pytest.raises(bs.BatchSolveError):
        bs.bs_varbatch_set_policy(c.h.handle, 18)


def test_mixed_precision_uneven():
    c = VCase(W.uneven_banded(300, 16, 1024, seed=5))
    outer = torch.zeros(c.vb.n_batch, dtype=torch.int32, device="cuda:0")
    g = c.gpu(bs.BICGSTAB, max_iter=2000, precision=bs.MIXED, outer_iters=outer)
    assert np.all(g[3] == bs.CONVERGED)
    c.check(g, bs.BICGSTAB, max_iter=2000, itol=10**9)
    assert outer.min().item() >= 1


def test_edge_cases_uneven():
    vb = W.uneven_banded(40, 16, 200, seed=6)
    c = VCase(vb)
    x0 = np.random.default_rng(1).standard_normal(vb.b.shape)
    b = vb.b.copy()
    b[vb.row_off[2]:vb.row_off[3]] = 0.0        # b = 0: converged, x = 0
    b[vb.row_off[5] + 3] = np.inf               # Inf in b
    vals = vb.values.copy()
    vals[vb.val_off[7] + 4] = np.nan            # NaN in A
    g = c.gpu(bs.BICGSTAB, values=dev(vals), b=dev(b), x0=x0, tol=1e-8)
    c.check(g, bs.BICGSTAB, values=vals, b=b, x0=x0, tol=1e-8)
    assert g[3][2] == bs.CONVERGED and g[1][2] == 0
    assert np.all(g[0][vb.row_off[2]:vb.row_off[3]] == 0.0)
    assert g[3][5] == bs.NONFINITE and g[3][7] == bs.NONFINITE
    g = c.gpu(bs.BICGSTAB, max_iter=0)
    assert np.all(g[3] == bs.MAX_ITER) and np.all(g[1] == 0) and np.all(g[0] == 0)
    g = c.gpu(bs.BICGSTAB, tol=1e-30, max_iter=9)
    assert np.all(g[3] == bs.MAX_ITER) and np.all(g[1] == 9)


def test_single_row_systems():
    """n = 1 (x = b / a exactly for these values) in a batch of three."""
    one = (np.array([0, 1], np.int32), np.array([0], np.int32))
    h = bs.VarBatch([1], [0], one[0], [0], one[1], [0, 0, 0])
    vals = dev(np.array([2.0, -4.0, 0.5]))
    b = dev(np.array([1.0, 2.0, 3.0]))
    x = torch.empty(3, dtype=torch.float64, device="cuda:0")
    it = torch.empty(3, dtype=torch.int32, device="cuda:0")
    rs = torch.empty(3, dtype=torch.float64, device="cuda:0")
    st = torch.empty(3, dtype=torch.int32, device="cuda:0")
    for solver in (bs.BICGSTAB, bs.CG):
        say(f"  n=1 solver={solver}")
        bs.bs_varbatch_solve(h.handle, vals, b, x, solver, bs.PREC_JACOBI, 1e-10, 10, it, rs, st,
                             bs.make_options(flags=bs.FLAG_X0_ZERO))
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy(), [0.5, -0.5, 6.0])
        assert np.all(st.cpu().numpy() == bs.CONVERGED)


@pytest.mark.parametrize("policy", [0, 4, 8, 13, "split"])
def test_graph_replay_matches_eager(policy):
    """The captured graph (counter reset kernel + solve, or the launches of a
    per-class plan) replayed several times, with eager work and synchronisation
    between replays, equals the eager solve bit for bit each time."""
    c = VCase(W.uneven_banded(300, 16, 1024, seed=7))
    if policy == "split":
        bs.bs_varbatch_set_plan(c.h.handle, [0, 4, 8, 9, 7])
        policy = 0
    else:
        bs.bs_varbatch_set_policy(c.h.handle, policy)
    eager = c.gpu(bs.BICGSTAB)
    x, it, rs, st = c.outputs()
    bs.bs_varbatch_capture(c.h.handle, c.dv, c.db, x, bs.BICGSTAB, bs.PREC_JACOBI, 1e-10, 1000,
                           it, rs, st, bs.make_options(flags=bs.FLAG_X0_ZERO))
    for rep in range(4):
        x.fill_(np.nan)
        it.fill_(-7)
        rs.fill_(-7.0)
        st.fill_(-7)
        torch.cuda.synchronize()
        say(f"  replay {rep}")
        bs.bs_varbatch_replay(c.h.handle)
        torch.cuda.synchronize()
        for u, v in zip(eager, (x.cpu().numpy(), it.cpu().numpy(), rs.cpu().numpy(),
                                st.cpu().numpy())):
            assert np.array_equal(u, v), f"replay {rep} differs from the eager solve"
    # a policy change drops the graph
    bs.bs_varbatch_set_policy(c.h.handle, (policy + 1) % 18)
    with pytest.raises(bs.BatchSolveError):
        bs.bs_varbatch_replay(c.h.handle)


def test_tune_and_cache(tmp_path):
    c = VCase(W.uneven_banded(600, 16, 1024, seed=8))
    x, it, rs, st = c.outputs()
    cache = str(tmp_path / "tune.txt")
    rep = bs.bs_varbatch_tune(c.h.handle, c.dv, c.db, x, bs.BICGSTAB, bs.PREC_JACOBI, 1e-10,
                              1000, it, rs, st, bs.make_options(flags=bs.FLAG_X0_ZERO), reps=2,
                              cache_path=cache)
    torch.cuda.synchronize()
    say(f"  tune: {rep}")
    assert rep.startswith("policy=") and "times_ms=" in rep and "classes=" in rep
    tok = rep.split()[0].split("=")[1]
    pol, codes = bs.bs_varbatch_get_plan(c.h.handle)
    if tok.startswith("split:"):
        assert pol == -1 and codes == [int(v) for v in tok[6:].split(",")]
    else:
        assert pol == int(tok) and c.h.query()["policy"] == pol
    times = rep.split()[1].split("=")[1].split(",")
    assert len(times) == 18 and all(t != "-" for t in times)   # every policy runs BiCGSTAB/Jacobi
    # one choice per populated size class, each named by shape, walk and placement
    classes = rep.split()[2].split("=", 1)[1].split(",")
    populated = {int(np.searchsorted([64, 128, 256, 512, 1024], n)) for n in c.vb.sys_rows}
    assert {int(e.split(":")[0]) for e in classes} == populated
    # the outputs are those of an eager solve with the chosen plan
    chosen = c.gpu(bs.BICGSTAB)
    assert np.array_equal(x.cpu().numpy(), chosen[0])
    c.check(chosen, bs.BICGSTAB)
    assert open(cache).read().count("\n") == 1
    rep2 = bs.bs_varbatch_tune(c.h.handle, c.dv, c.db, x, bs.BICGSTAB, bs.PREC_JACOBI, 1e-10,
                               1000, it, rs, st, bs.make_options(flags=bs.FLAG_X0_ZERO), reps=2,
                               cache_path=cache)
    assert "cached" in rep2 and rep2.startswith(f"policy={tok}")
    assert bs.bs_varbatch_get_plan(c.h.handle) == (pol, codes)
    # tuning from a nonzero x0 restarts every timed solve from it
    x0 = np.random.default_rng(2).standard_normal(c.vb.b.shape)
    ref = c.gpu(bs.BICGSTAB, x0=x0)
    x.copy_(dev(x0))
    bs.bs_varbatch_tune(c.h.handle, c.dv, c.db, x, bs.BICGSTAB, bs.PREC_JACOBI, 1e-10, 1000, it,
                        rs, st, bs.make_options(), reps=1)
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy(), ref[0]) and np.array_equal(it.cpu().numpy(), ref[1])


def test_uneven_full_size_sampled():
    """100k systems, n in [16, 1024], bands of width 5..9, in the benchmark's
    launch shape: every system converges with a true residual <= 1e-10 (checked
    by the oracle per pattern), and a random sample is re-solved by the oracle."""
    vb = W.uneven_banded(100_000, 16, 1024, seed=0)
    c = VCase(vb)
    g = c.gpu(bs.BICGSTAB)
    assert np.all(g[3] == bs.CONVERGED)
    rng = np.random.default_rng(0)
    pick = set(rng.choice(vb.n_batch, 300, replace=False).tolist())
    worst = 0.0
    for sys_, n, rp, ci, rows, vals in c.groups():
        OP = O.Pattern(n, rp, ci)
        v = vb.values[vals].reshape(sys_.size, -1)
        bb = vb.b[rows].reshape(sys_.size, n)
        xg = g[0][rows].reshape(sys_.size, n)
        rt = O.true_residual(OP, v, bb, xg)
        worst = max(worst, float(rt.max()))
        sel = np.array([i for i, s in enumerate(sys_) if s in pick], dtype=np.int64)
        if sel.size:
            o = O.batch_solve(OP, v[sel], bb[sel], solver=O.BICGSTAB, tol=1e-10, max_iter=1000)
            err = np.linalg.norm(xg[sel] - o[0], axis=1) / np.linalg.norm(o[0], axis=1)
            assert np.all(err <= 1e-8)
            assert np.all(np.abs(g[1][sys_[sel]] - o[1]) <= 2)
    say(f"  uneven full size: worst true residual {worst:.2e}")
    assert worst <= 1e-10


# ------------------------------------------------------------------ ELL input, placements, plans
def ell_handle(vb: W.VarBatch, extra_slots: int = 2):
    """The batch as ELL patterns (two padding slots beyond the longest row); the
    padding values are NaN, so a kernel that read one would poison its system."""
    pr, pw, pco, ca, pid, vals = vb.ell(extra_slots=extra_slots, pad_value=np.nan)
    return bs.VarBatch(pr, pw, pco, ca, pid, ell=True), dev(vals)


def handle_solve(c: VCase, h, values, solver=bs.BICGSTAB, precond=bs.PREC_JACOBI, **opt):
    x, it, rs, st = c.outputs()
    bs.bs_varbatch_solve(h.handle, values, c.db, x, solver, precond, 1e-10, 1000, it, rs, st,
                         bs.make_options(flags=bs.FLAG_X0_ZERO, **opt))
    torch.cuda.synchronize()
    return x.cpu().numpy(), it.cpu().numpy(), rs.cpu().numpy(), st.cpu().numpy()


def same(u, v, what):
    for a_, b_ in zip(u, v):
        assert np.array_equal(a_, b_), what


@pytest.mark.parametrize("policy", [0, 4, 8, 9, 13, 17])
def test_ell_input_matches_csr(policy):
    """An uneven batch given as ELL patterns (BatchEll) is solved with the bits
    of the same batch given as CSR: the slot-major walk takes a row's entries in
    the order of its CSR walk, in registers (policies 0..8) and streamed
    (9..17) alike."""
    vb = W.uneven_banded(400, 16, 1024, seed=21)
    c = VCase(vb)
    bs.bs_varbatch_set_policy(c.h.handle, policy)
    ref = c.gpu(bs.BICGSTAB)
    if policy in (0, 9, 17):
        c.check(ref, bs.BICGSTAB)
    h, dv = ell_handle(vb)
    assert h.total_values == int(sum(vb.ell(2)[1][vb.pat_id] * vb.pat_rows[vb.pat_id]))
    bs.bs_varbatch_set_policy(h.handle, policy)
    same(ref, handle_solve(c, h, dv), f"ELL input, policy {policy}")


@pytest.mark.parametrize("fmt", ["csr", "ell"])
def test_class_plans(fmt):
    """Per-class launches.  Within one workgroup shape the four choices
    (CSR or ELL walk, rows in registers or streamed) add a row's entries in the
    same order, so every uniform plan of a shape gives the bits of the single
    launch of that shape; a plan that mixes choices across classes gives, class
    by class, the bits of the uniform plan of each class's shape."""
    vb = W.uneven_banded(500, 16, 1024, seed=22)
    c = VCase(vb)
    if fmt == "csr":
        h, dv = c.h, c.dv
    else:
        h, dv = ell_handle(vb)
    by_shape = {}
    for shape in range(3):
        bs.bs_varbatch_set_policy(h.handle, 3 * shape)
        ref = handle_solve(c, h, dv)
        c.check(ref, bs.BICGSTAB)
        by_shape[shape] = ref
        for walk in range(2):
            for place in range(2):
                code = shape + 3 * walk + 6 * place
                bs.bs_varbatch_set_plan(h.handle, [code] * 5)
                assert bs.bs_varbatch_get_plan(h.handle) == (-1, [code] * 5)
                assert h.query()["policy"] == -1
                same(ref, handle_solve(c, h, dv), f"{fmt}: uniform plan {code}")
    codes = [0, 4, 8, 9, 7]     # class c takes shape codes[c] % 3
    bs.bs_varbatch_set_plan(h.handle, codes)
    g = handle_solve(c, h, dv)
    cls = np.searchsorted([64, 128, 256, 512, 1024], vb.sys_rows)
    for s in range(vb.n_batch):
        ref = by_shape[codes[cls[s]] % 3]
        r0, r1 = vb.row_off[s], vb.row_off[s + 1]
        assert np.array_equal(g[0][r0:r1], ref[0][r0:r1]), f"system {s}"
        assert g[1][s] == ref[1][s] and g[2][s] == ref[2][s] and g[3][s] == ref[3][s]
    with pytest.raises(bs.BatchSolveError) as e:
        bs.bs_varbatch_set_plan(h.handle, [0, 1, 2, 12, 0])
    assert e.value.code == bs.ERR_INVALID_ARG
    assert bs.bs_varbatch_get_plan(h.handle) == (-1, codes)


def test_mixed_precision_plans():
    """Mixed-precision BiCGSTAB under a per-class plan that streams some
    classes: every system converges and meets the FP64 oracle's x."""
    c = VCase(W.uneven_banded(300, 16, 1024, seed=23))
    bs.bs_varbatch_set_plan(c.h.handle, [6, 10, 2, 11, 7])
    g = c.gpu(bs.BICGSTAB, max_iter=2000, precision=bs.MIXED)
    assert np.all(g[3] == bs.CONVERGED)
    c.check(g, bs.BICGSTAB, max_iter=2000, itol=10**9)


def test_long_rows_streamed():
    """Rows of 21..41 entries: beyond what the register placement holds.  The
    handle starts on the streamed placement; register policies are refused at
    solve time; streamed single launches, per-class plans, ELL input and the
    caller-owned entry point all meet the oracle (CG on SPD values too)."""
    vb = W.uneven_banded(160, 16, 400, w_min=21, w_max=41, seed=24)
    c = VCase(vb)
    assert c.h.query()["policy"] == 9
    g = c.gpu(bs.BICGSTAB)
    c.check(g, bs.BICGSTAB)
    bs.bs_varbatch_set_policy(c.h.handle, 0)
    with pytest.raises(bs.BatchSolveError) as e:
        c.gpu(bs.BICGSTAB)
    assert e.value.code == bs.ERR_UNSUPPORTED
    bs.bs_varbatch_set_plan(c.h.handle, [9, 10, 11, 9, 9])
    c.check(c.gpu(bs.BICGSTAB), bs.BICGSTAB)
    h, dv = ell_handle(vb, extra_slots=1)
    bs.bs_varbatch_set_policy(h.handle, 16)
    c.check(handle_solve(c, h, dv), bs.BICGSTAB)
    arrs = varlen_arrays(vb)
    ws = torch.empty(bs.bs_varlen_workspace_size(vb.n_batch), dtype=torch.uint8, device="cuda:0")
    bs.bs_varbatch_set_policy(c.h.handle, 12)
    same(c.gpu(bs.BICGSTAB), varlen_solve(c, arrs, ws), "caller-owned default (policy 12)")
    with pytest.raises(bs.BatchSolveError) as e:
        varlen_solve(c, arrs, ws, varlen_policy=1)
    assert e.value.code == bs.ERR_UNSUPPORTED
    vs = W.uneven_banded(120, 16, 300, w_min=25, w_max=25, seed=25)   # symmetric bands
    cs = VCase(vs, values=symmetric_values(vs, 5))
    cs.check(cs.gpu(bs.CG), bs.CG)


# ------------------------------------------------------------------ caller-owned arrays
def varlen_arrays(vb: W.VarBatch):
    """The structure of an uneven batch as the device tensors the caller owns."""
    n_rows = np.asarray(vb.pat_rows)[vb.pat_id].astype(np.int32)
    return dict(sys_rows=dev(n_rows), row_off=dev(np.asarray(vb.row_off, np.int64)),
                val_off=dev(np.asarray(vb.val_off, np.int64)),
                pat_id=dev(np.asarray(vb.pat_id, np.int32)),
                pat_rowptr_off=dev(np.asarray(vb.pat_rowptr_off, np.int64)),
                pat_col_off=dev(np.asarray(vb.pat_col_off, np.int64)),
                rowptr_all=dev(np.asarray(vb.rowptr_all, np.int32)),
                col_all=dev(np.asarray(vb.col_all, np.int32)))


def varlen_solve(c: VCase, arrs, ws, solver=bs.BICGSTAB, precond=bs.PREC_JACOBI, tol=1e-10,
                 max_iter=1000, **opt):
    x, it, rs, st = c.outputs()
    opts = bs.make_options(flags=bs.FLAG_X0_ZERO, **opt)
    bs.bs_batch_solve_varlen(**arrs, values=c.dv, b=c.db, x=x, solver=solver, precond=precond,
                             tol=tol, max_iter=max_iter, iters=it, resid=rs, status=st, opts=opts,
                             ws=ws)
    torch.cuda.synchronize()
    return x.cpu().numpy(), it.cpu().numpy(), rs.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("policy", [3, 0, 8, 12, 16])
def test_varlen_caller_arrays_match_handle(policy):
    """bs_batch_solve_varlen on caller-owned device arrays gives, for the same
    queue policy, the bits of the handle API's solve; both meet the oracle's
    bar.  A second call (cached structure, workspace reused) gives the same
    bits again, and so does a fresh workspace."""
    vb = W.uneven_banded(400, 16, 1024, seed=31)
    c = VCase(vb)
    arrs = varlen_arrays(vb)
    B = vb.n_batch
    ws = torch.empty(bs.bs_varlen_workspace_size(B), dtype=torch.uint8, device="cuda:0")
    bs.bs_varbatch_set_policy(c.h.handle, policy)
    h = c.gpu(bs.BICGSTAB)
    g1 = varlen_solve(c, arrs, ws, varlen_policy=policy + 1)
    g2 = varlen_solve(c, arrs, ws, varlen_policy=policy + 1)
    ws2 = torch.empty_like(ws)
    g3 = varlen_solve(c, arrs, ws2, varlen_policy=policy + 1)
    for g in (g1, g2, g3):
        for a_, b_ in zip(g, h):
            assert np.array_equal(a_, b_, equal_nan=True)
    c.check(g1, bs.BICGSTAB)


def test_varlen_generation_and_errors():
    """Changing the structure in place takes a new generation number (the
    library then re-reads and re-validates it); inconsistent or malformed
    structure arrays and a short workspace are refused before any launch."""
    vb = W.uneven_banded(120, 16, 300, seed=32)
    c = VCase(vb)
    arrs = varlen_arrays(vb)
    B = vb.n_batch
    ws = torch.empty(bs.bs_varlen_workspace_size(B), dtype=torch.uint8, device="cuda:0")
    g = varlen_solve(c, arrs, ws, structure_generation=1)
    c.check(g, bs.BICGSTAB)
    # CG on the same structure, another generation (re-read): the oracle's bar
    vb2 = W.uneven_banded(120, 16, 300, w_min=5, w_max=5, seed=33)   # symmetric bands
    c2 = VCase(vb2, values=symmetric_values(vb2, 4))
    arrs2 = varlen_arrays(vb2)
    g2 = varlen_solve(c2, arrs2, ws, solver=bs.CG, structure_generation=2)
    c2.check(g2, bs.CG)

    def refused(codes, **change):
        a = dict(arrs)
        a.update(change)
        with pytest.raises(bs.BatchSolveError) as e:
            varlen_solve(c, a, ws, structure_generation=10 + len(change))
        assert e.value.code in codes

    bad_rows = varlen_arrays(vb)["sys_rows"].clone()
    bad_rows[5] += 1
    # one row more than its pattern: the offsets disagree with the rows, or
    # (a pattern only this system uses) its row_ptr read one entry too far is
    # no longer nondecreasing
    refused((bs.ERR_INVALID_ARG, bs.ERR_PATTERN), sys_rows=bad_rows)
    bad_pat = arrs["pat_id"].clone()
    bad_pat[0] = len(vb.pat_rows)                       # no such pattern
    refused((bs.ERR_PATTERN,), pat_id=bad_pat)
    bad_off = arrs["val_off"].clone()
    bad_off[3] += 1                                     # values of system 2 one short
    refused((bs.ERR_INVALID_ARG,), val_off=bad_off)
    bad_col = arrs["col_all"].clone()
    bad_col[1] = bad_col[0]                             # a column twice in a row
    refused((bs.ERR_PATTERN,), col_all=bad_col)
    small = torch.empty(bs.bs_varlen_workspace_size(B) - 256, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(ValueError):
        varlen_solve(c, arrs, small)
    # past the binding's check, the library refuses the short workspace itself
    x, it, rs, st = c.outputs()
    rc = bs.lib().bs_batch_solve_varlen(
        B, arrs["sys_rows"].data_ptr(), arrs["row_off"].data_ptr(), arrs["val_off"].data_ptr(),
        len(vb.pat_rows), arrs["pat_id"].data_ptr(), arrs["pat_rowptr_off"].data_ptr(),
        arrs["pat_col_off"].data_ptr(), arrs["rowptr_all"].data_ptr(), arrs["col_all"].data_ptr(),
        c.dv.data_ptr(), c.db.data_ptr(), x.data_ptr(), bs.BICGSTAB, bs.PREC_JACOBI, 1e-10, 100,
        it.data_ptr(), rs.data_ptr(), st.data_ptr(), None, small.data_ptr(), small.numel(), None)
    assert rc == bs.ERR_INVALID_ARG
