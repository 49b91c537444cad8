"""Host-side tests of the C ABI: the library loads, exports every declared entry
point, and its pure host logic (pattern validation, storage counts, planner,
error strings) behaves as documented.  No kernel is launched."""
import ctypes as C
import json
import os
import re

import numpy as np
import pytest

from paper_2308_08417_amd import batchsolve as bs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(bs_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(bs.LIB_PATH):
        pytest.fail("libbatchsolve.so is not built (run __graft_entry__.build())")
    return bs.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n


def test_error_strings(L):
    for code in (bs.OK, bs.ERR_INVALID_ARG, bs.ERR_PATTERN, bs.ERR_UNSUPPORTED, bs.ERR_HIP,
                 bs.ERR_NO_DEVICE, -99):
        assert isinstance(bs.bs_error_string(code), str) and bs.bs_error_string(code)


def test_storage_counts_tab3(L, golden_dir):
    g = json.load(open(os.path.join(golden_dir, "tab3_shapes.json")))
    B = g["batch"]
    for e in g["inputs"]:
        n, nnz = e["n"], e["nnz"]
        assert bs.bs_matrix_storage(bs.CSR, B, n, nnz, 0) == (B * nnz, n + 1 + nnz)
        w = 40
        assert bs.bs_matrix_storage(bs.ELL, B, n, nnz, w) == (B * w * n, w * n)
    with pytest.raises(bs.BatchSolveError):
        bs.bs_matrix_storage(7, 1, 1, 1, 1)


def test_mechanism_stand_ins_match_tab3(L, golden_dir):
    """The Tab. 3 stand-ins have the table's rows, stored entries and count of
    distinct systems (the golden file restates the table), a full diagonal
    and ascending columns; every system repeats its distinct original (the
    paper's replicated cells); each plans onto a register kernel."""
    from paper_2308_08417_amd import workloads as W
    g = json.load(open(os.path.join(golden_dir, "tab3_shapes.json")))
    assert sorted(e["name"] for e in g["inputs"]) == sorted(W.MECHANISMS)
    for e in g["inputs"]:
        u = e["unique"]
        bt = W.mechanism_batch(e["name"], n_batch=3 * u + 1, seed=1)
        assert (bt.n, bt.nnz, bt.meta["unique"]) == (e["n"], e["nnz"], u)
        rows = np.repeat(np.arange(bt.n), np.diff(bt.row_ptr))
        assert np.sum(rows == bt.col_idx) == bt.n
        assert np.all((np.diff(bt.col_idx) > 0) | (np.diff(rows) > 0))
        assert np.array_equal(bt.values[2 * u:3 * u], bt.values[:u])
        assert np.array_equal(bt.b[u:2 * u], bt.b[:u]) and np.array_equal(bt.values[3 * u], bt.values[0])
        assert not np.array_equal(bt.values[0], bt.values[1])
        p = bs.bs_plan(bs.CSR, bt.n, bt.nnz, int(np.diff(bt.row_ptr).max()), bs.BICGSTAB)
        assert p["slots"] >= np.diff(bt.row_ptr).max() and p["team"] >= min(bt.n, 64)


def tri(n):
    rp, ci = [0], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                ci.append(j)
        rp.append(len(ci))
    return np.array(rp, np.int32), np.array(ci, np.int32)


def create_code(fn, *args):
    try:
        fn(*args)
        return bs.OK
    except bs.BatchSolveError as e:
        return e.code


def test_pattern_validation(L):
    rp, ci = tri(8)
    bad_start = rp.copy(); bad_start[0] = 1
    assert create_code(bs.bs_pattern_create_csr, bad_start, ci) == bs.ERR_PATTERN
    bad_mono = rp.copy(); bad_mono[3] = bad_mono[4] + 1
    assert create_code(bs.bs_pattern_create_csr, bad_mono, ci) == bs.ERR_PATTERN
    bad_col = ci.copy(); bad_col[2] = 8
    assert create_code(bs.bs_pattern_create_csr, rp, bad_col) == bs.ERR_PATTERN
    neg_col = ci.copy(); neg_col[2] = -1
    assert create_code(bs.bs_pattern_create_csr, rp, neg_col) == bs.ERR_PATTERN
    dup = ci.copy(); dup[3] = dup[2]   # row 1 = (0,1,2) -> (0,0,2)
    assert create_code(bs.bs_pattern_create_csr, rp, dup) == bs.ERR_PATTERN
    # ELL: padding before a stored entry
    n = 4
    ell = np.array([[0, 1, 2, 3], [-1, 0, 1, 2], [1, -1, -1, -1]], np.int32).ravel()
    assert create_code(bs.bs_pattern_create_ell, n, ell) == bs.ERR_PATTERN
    ell_oob = np.array([[0, 1, 2, 4]], np.int32).ravel()
    assert create_code(bs.bs_pattern_create_ell, n, ell_oob) == bs.ERR_PATTERN
    # invalid arguments
    assert L.bs_pattern_create_csr(0, 0, None, None, None) == bs.ERR_INVALID_ARG
    assert L.bs_batch_solve(0, 1, 4, None, None, None, None, 1, 1, 1e-10, 10, None, None, None,
                            None, None) == bs.ERR_INVALID_ARG


def test_valid_pattern_needs_device(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present; covered by the GPU tests")
    rp, ci = tri(5)
    assert create_code(bs.bs_pattern_create_csr, rp, ci) == bs.ERR_NO_DEVICE


@pytest.mark.parametrize("n", [1, 16, 17, 32, 33, 54, 64, 65, 128, 300, 992, 1024, 1025, 2048, 4096])
def test_plan_covers_rows(L, n):
    """Sec. 3.6 work-group rule: at least one lane per row, a power of two that
    is a multiple of the 16-lane DPP row (or the whole wave), slots >= longest row."""
    for solver in (bs.CG, bs.BICGSTAB, bs.GMRES):
        maxrow = min(n, 9 if n <= 1024 else 5)
        try:
            p = bs.bs_plan(bs.ELL, n, n * maxrow, maxrow, solver)
        except bs.BatchSolveError as e:
            assert e.code == bs.ERR_UNSUPPORTED
            assert n > bs.MAX_ROWS
            continue
        assert p["team"] * p["rows_per_lane"] >= n
        assert p["team"] in (16, 32, 64, 128, 256, 512, 1024)
        if solver == bs.GMRES and n > 1024:
            # streamed rows, the basis in device memory
            assert p["slots"] == 0 and p["rows_per_lane"] == 2 and p["group_size"] == 1024
            assert p["lds_bytes"] <= 64 * 1024
            continue
        assert p["slots"] >= maxrow
        assert p["group_size"] % 64 == 0 and p["group_size"] == max(p["team"], 64)
        assert p["systems_per_group"] * p["team"] == p["group_size"]
        # smallest team for one row per lane
        if n <= 1024:
            assert p["rows_per_lane"] == 1 and (p["team"] == 16 or p["team"] // 2 < n)
        # 160 KiB of LDS per compute unit; 1024-lane GMRES teams keep 16 FP64
        # basis vectors there
        assert p["lds_bytes"] <= 160 * 1024
        if solver == bs.GMRES and p["group_size"] == 1024:
            assert p["lds_bytes"] >= 16 * 1024 * 8
        else:
            assert p["lds_bytes"] <= 64 * 1024


def test_plan_stage_and_limits(L):
    p = bs.bs_plan(bs.CSR, 54, 1042, 28, bs.BICGSTAB)
    # the narrowest compiled slot count that holds the longest row (28)
    assert p["team"] == 64 and p["slots"] == 28 and p["stage_values"] == 1
    assert p["lds_bytes"] >= 1042 * 8
    # single-wave groups prefetch each system's values and b into LDS
    p = bs.bs_plan(bs.ELL, 54, 1042, 28, bs.BICGSTAB)
    assert p["stage_values"] == 1 and p["lds_bytes"] >= (28 * 54 + 54) * 8
    # multi-wave teams read ELL values (slot-major: coalesced) straight from HBM
    p = bs.bs_plan(bs.ELL, 992, 8554, 9, bs.BICGSTAB)
    assert p["group_size"] == 1024 and p["stage_values"] == 0
    # and CSR values of short rows straight from HBM too
    p = bs.bs_plan(bs.CSR, 992, 8554, 9, bs.BICGSTAB)
    assert p["group_size"] == 1024 and p["slots"] == 12 and p["stage_values"] == 0
    # rows of 32 slots or more: the whole group copies each system's CSR values
    # into LDS, beside the vectors
    p = bs.bs_plan(bs.CSR, 144, 6135, 54, bs.BICGSTAB)
    assert p["group_size"] == 256 and p["slots"] == 56 and p["stage_values"] == 2
    assert p["lds_bytes"] >= 6135 * 8 + 2 * 257 * 8
    p = bs.bs_plan(bs.CSR, 300, 2700, 20, bs.CG)
    assert p["slots"] == 32 and p["stage_values"] == 2
    p = bs.bs_plan(bs.CSR, 300, 2700, 16, bs.CG)
    assert p["slots"] == 16 and p["stage_values"] == 0
    # rows beyond the register slots: the streamed placement (spill tier),
    # workgroups of 512 lanes x 2 rows, no register slots, no staging
    p = bs.bs_plan(bs.CSR, 54, 1042, 65, bs.BICGSTAB)
    assert p["slots"] == 0 and p["group_size"] == 512 and p["rows_per_lane"] == 2
    assert p["team"] == 64 and p["systems_per_group"] == 8 and p["stage_values"] == 0
    p = bs.bs_plan(bs.DENSE, 1000, 0, 0, bs.CG)
    assert p["slots"] == 0 and p["team"] == 512 and p["systems_per_group"] == 1
    p = bs.bs_plan(bs.CSR, 144, 6135, 80, bs.BICGSTAB, bs.make_options(precision=bs.MIXED))
    assert p["slots"] == 0 and p["team"] == 128
    # GMRES streams on 1024-lane workgroups, one system each, one row per lane
    p = bs.bs_plan(bs.CSR, 54, 1042, 65, bs.GMRES)
    assert p["slots"] == 0 and p["team"] == 1024 and p["rows_per_lane"] == 1
    assert p["systems_per_group"] == 1 and p["lds_bytes"] <= 160 * 1024
    # ... which takes neither block Jacobi / ILU(0), nor mixed CG, nor a forced
    # shape, nor more than 2048 rows (GMRES: 1024)
    for solver, opts, prec in ((bs.BICGSTAB, bs.make_options(block_size=4), bs.PREC_BLOCK_JACOBI),
                               (bs.BICGSTAB, None, bs.PREC_ILU),
                               (bs.CG, bs.make_options(precision=bs.MIXED), bs.PREC_JACOBI),
                               (bs.BICGSTAB, bs.make_options(team=128), bs.PREC_JACOBI)):
        with pytest.raises(bs.BatchSolveError) as e:
            bs.bs_plan_precond(bs.CSR, 54, 1042, 65, solver, prec, opts)
        assert e.value.code == bs.ERR_UNSUPPORTED, (solver, prec)
    p = bs.bs_plan(bs.DENSE, 1025, 0, 0, bs.CG)
    assert p["slots"] == 0 and p["team"] == 1024 and p["rows_per_lane"] == 2
    with pytest.raises(bs.BatchSolveError) as e:
        bs.bs_plan(bs.DENSE, 2049, 0, 0, bs.CG)
    assert e.value.code == bs.ERR_UNSUPPORTED
    with pytest.raises(bs.BatchSolveError) as e:
        bs.bs_plan(bs.CSR, 5000, 15000, 3, bs.BICGSTAB)
    assert e.value.code == bs.ERR_UNSUPPORTED
    with pytest.raises(bs.BatchSolveError) as e:
        bs.bs_plan(bs.CSR, 54, 1042, 28, bs.BICGSTAB, bs.make_options(team=48))
    assert e.value.code == bs.ERR_INVALID_ARG
    p = bs.bs_plan(bs.CSR, 54, 1042, 28, bs.BICGSTAB, bs.make_options(team=128))
    assert p["team"] == 128 and p["systems_per_group"] == 1
    p = bs.bs_plan(bs.CSR, 54, 1042, 28, bs.BICGSTAB, bs.make_options(precision=bs.MIXED))
    assert p["team"] == 64
    with pytest.raises(bs.BatchSolveError):
        bs.bs_plan(bs.CSR, 54, 1042, 28, bs.CG, bs.make_options(precision=bs.MIXED))


def test_plan_streamed_two_rows(L):
    """1025..2048 rows: register shapes of 2 rows x 8 slots where the rows fit,
    else the streamed placement on 1024-lane x 2-row workgroups (CG, BiCGSTAB,
    and GMRES in FP64 with its basis in device memory); every solver stops at
    2048 rows, mixed GMRES at 1024."""
    p = bs.bs_plan(bs.CSR, 1600, 8000, 5, bs.BICGSTAB)
    assert p["slots"] == 8 and p["team"] == 1024 and p["rows_per_lane"] == 2
    for solver in (bs.CG, bs.BICGSTAB, bs.GMRES):
        for n in (1025, 1600, 2048):
            p = bs.bs_plan(bs.CSR, n, 9 * n, 9, solver)
            assert p["slots"] == 0 and p["team"] == 1024 and p["rows_per_lane"] == 2, (solver, n)
            assert p["group_size"] == 1024 and p["systems_per_group"] == 1
        p = bs.bs_plan(bs.CSR, 1600, 1600 * 9, 9, solver, bs.make_options(precision=bs.MIXED)) \
            if solver == bs.BICGSTAB else p
        assert p["slots"] == 0
    for solver, n in ((bs.GMRES, 2049), (bs.BICGSTAB, 2049), (bs.CG, 2049)):
        with pytest.raises(bs.BatchSolveError) as e:
            bs.bs_plan(bs.CSR, n, 9 * n, 9, solver)
        assert e.value.code == bs.ERR_UNSUPPORTED, (solver, n)
    with pytest.raises(bs.BatchSolveError) as e:
        bs.bs_plan(bs.CSR, 1600, 9 * 1600, 9, bs.GMRES, bs.make_options(precision=bs.MIXED))
    assert e.value.code == bs.ERR_UNSUPPORTED


def test_plan_ilu_trsv_teams(L):
    """ILU(0) and BatchTrsv take one row per lane: one wave up to 64 rows, else
    the smallest power-of-two team of at least n lanes (sparse factors in LDS);
    GMRES with ILU(0) stops at 512 rows, where its basis leaves registers."""
    p = bs.bs_plan_precond(bs.CSR, 54, 1042, 28, bs.BICGSTAB, bs.PREC_ILU)
    assert p["team"] == 64 and p["slots"] == 28 and p["stage_values"] == 0
    p = bs.bs_plan_precond(bs.CSR, 992, 8554, 9, bs.BICGSTAB, bs.PREC_ILU)
    assert p["team"] == 1024 and p["rows_per_lane"] == 1 and p["slots"] == 12
    # sparse factors (8 B per entry) with the sweep vector, pivots and levels
    assert 8 * 8554 + 20 * 992 <= p["lds_bytes"] <= 160 * 1024
    p = bs.bs_plan_precond(bs.ELL, 192, 1600, 9, bs.GMRES, bs.PREC_ILU)
    assert p["team"] == 256 and p["group_size"] == 256 and p["systems_per_group"] == 1
    p = bs.bs_plan(bs.CSR, 300, 900, 3, bs.TRSV_LOWER)
    assert p["team"] == 512 and p["slots"] == 4
    p = bs.bs_plan(bs.CSR, 1000, 2998, 3, bs.TRSV_UPPER)
    assert p["team"] == 1024
    p = bs.bs_plan_precond(bs.CSR, 100, 300, 3, bs.BICGSTAB, bs.PREC_ILU, bs.make_options(team=512))
    assert p["team"] == 512
    for args in ((bs.CSR, 992, 8554, 9, bs.GMRES, bs.PREC_ILU, None),
                 (bs.CSR, 1025, 3073, 3, bs.BICGSTAB, bs.PREC_ILU, None),
                 (bs.CSR, 1025, 3073, 3, bs.TRSV_LOWER, bs.PREC_NONE, None),
                 (bs.CSR, 200, 600, 3, bs.BICGSTAB, bs.PREC_ILU, bs.make_options(team=128)),
                 (bs.CSR, 40, 120, 3, bs.BICGSTAB, bs.PREC_ILU, bs.make_options(team=32)),
                 (bs.CSR, 200, 600, 3, bs.BICGSTAB, bs.PREC_ILU, bs.make_options(rows_per_lane=2))):
        with pytest.raises(bs.BatchSolveError) as e:
            bs.bs_plan_precond(*args)
        assert e.value.code == bs.ERR_UNSUPPORTED, args


def varbatch_parts(pats, sys_pat):
    """Concatenate CSR patterns the way bs_varbatch_create takes them."""
    rows, rpo, cpo, rpa, ca = [], [], [], [], []
    for rp, ci in pats:
        rows.append(len(rp) - 1)
        rpo.append(sum(len(x) for x in rpa))
        cpo.append(sum(len(x) for x in ca))
        rpa.append(np.asarray(rp, np.int32))
        ca.append(np.asarray(ci, np.int32))
    return (rows, rpo, np.concatenate(rpa), cpo, np.concatenate(ca), np.asarray(sys_pat, np.int32))


def test_varbatch_validation(L):
    rp, ci = tri(8)
    good = varbatch_parts([(rp, ci), tri(3)], [0, 1, 1, 0])
    # pattern checks as for a single CSR pattern
    bad_col = ci.copy(); bad_col[4] = 9
    assert create_code(bs.bs_varbatch_create, *varbatch_parts([(rp, bad_col)], [0])) == bs.ERR_PATTERN
    dup = ci.copy(); dup[3] = dup[2]
    assert create_code(bs.bs_varbatch_create, *varbatch_parts([(rp, dup)], [0])) == bs.ERR_PATTERN
    # a system naming a pattern that does not exist
    assert create_code(bs.bs_varbatch_create, *varbatch_parts([(rp, ci)], [0, 1])) == bs.ERR_PATTERN
    assert create_code(bs.bs_varbatch_create, *varbatch_parts([(rp, ci)], [-1])) == bs.ERR_PATTERN
    # beyond the kernels' limits: more than 1024 rows.  Rows longer than 16
    # entries are accepted (the streamed placement holds them).
    assert create_code(bs.bs_varbatch_create, *varbatch_parts([tri(1025)], [0])) == bs.ERR_UNSUPPORTED
    n = 20
    dense = (np.arange(n + 1, dtype=np.int32) * n, np.tile(np.arange(n, dtype=np.int32), n))
    assert L.bs_varbatch_create(-1, 0, None, None, None, None, None, None, None) == bs.ERR_INVALID_ARG
    assert L.bs_varbatch_query(None, None, None, None, None) == bs.ERR_INVALID_ARG
    assert L.bs_varbatch_set_policy(None, 0) == bs.ERR_INVALID_ARG
    assert L.bs_varbatch_set_plan(None, None) == bs.ERR_INVALID_ARG
    assert L.bs_varbatch_get_plan(None, None, None) == bs.ERR_INVALID_ARG
    assert L.bs_varbatch_replay(None, None) == bs.ERR_INVALID_ARG
    assert L.bs_varbatch_destroy(None) == bs.OK
    import torch
    if not torch.cuda.is_available():
        assert create_code(bs.bs_varbatch_create, *good) == bs.ERR_NO_DEVICE
        assert create_code(bs.bs_varbatch_create, *varbatch_parts([dense], [0])) == bs.ERR_NO_DEVICE


def ell_parts(pats, sys_pat):
    """Concatenate ELL patterns (slot-major [w][n] column arrays)."""
    rows = [c.shape[1] for c in pats]
    widths = [c.shape[0] for c in pats]
    offs = np.cumsum([0] + [c.size for c in pats])[:-1]
    cols = np.concatenate([c.ravel() for c in pats]).astype(np.int32)
    return rows, widths, offs, cols, np.asarray(sys_pat, np.int32)


def test_varbatch_ell_validation(L):
    """ELL patterns of the uneven batch: columns in range, once per row, and
    padding (-1) only after a row's stored entries."""
    good = np.array([[0, 1, 2], [1, 2, -1], [-1, -1, -1]], np.int32)  # rows {0,1}, {1,2}, {2}
    after = good.copy(); after[0, 2] = -1; after[1, 2] = 2              # entry after padding
    assert create_code(bs.bs_varbatch_create_ell, *ell_parts([after], [0])) == bs.ERR_PATTERN
    out = good.copy(); out[1, 0] = 3
    assert create_code(bs.bs_varbatch_create_ell, *ell_parts([out], [0])) == bs.ERR_PATTERN
    dup = good.copy(); dup[1, 0] = 0
    assert create_code(bs.bs_varbatch_create_ell, *ell_parts([dup], [0])) == bs.ERR_PATTERN
    neg = good.copy(); neg[0, 1] = -2
    assert create_code(bs.bs_varbatch_create_ell, *ell_parts([neg], [0])) == bs.ERR_PATTERN
    assert create_code(bs.bs_varbatch_create_ell, *ell_parts([good], [1])) == bs.ERR_PATTERN
    rows, widths, offs, cols, sp = ell_parts([good], [0])
    assert create_code(bs.bs_varbatch_create_ell, rows, [-1], offs, cols, sp) == bs.ERR_INVALID_ARG
    assert create_code(bs.bs_varbatch_create_ell, [1025], [0], [0], np.zeros(1, np.int32),
                       [0]) == bs.ERR_UNSUPPORTED
    assert L.bs_varbatch_create_ell(-1, 0, None, None, None, None, None, None) == bs.ERR_INVALID_ARG
    import torch
    if not torch.cuda.is_available():
        assert create_code(bs.bs_varbatch_create_ell, *ell_parts([good], [0, 0])) == bs.ERR_NO_DEVICE
    with pytest.raises(ValueError):
        bs.bs_varbatch_set_plan(0, [0, 0, 0])


def test_varbatch_generator_layout():
    """The uneven generator's concatenated layout is what bs_varbatch_create reads."""
    from paper_2308_08417_amd import workloads as w
    vb = w.uneven_banded(200, 16, 300, seed=3)
    assert vb.row_off[-1] == vb.b.size == vb.x0.size
    assert vb.val_off[-1] == vb.values.size
    for s in (0, 57, 199):
        p = vb.pat_id[s]
        n = vb.pat_rows[p]
        assert vb.sys_rows[s] == n and 16 <= n <= 300
        rp = vb.rowptr_all[vb.pat_rowptr_off[p]: vb.pat_rowptr_off[p] + n + 1]
        assert vb.val_off[s + 1] - vb.val_off[s] == rp[-1]
        assert np.diff(rp).max() <= 9


def test_dense_format_host(L):
    """BatchDense (Sec. 3.1 storage list, Tab. 2): n^2 values per matrix and no
    indexes; planned as the full pattern in CSR order; rows over 64 entries
    cannot be held in registers and take the streamed placement."""
    assert bs.bs_matrix_storage(bs.DENSE, 1000, 54, 0, 0) == (1000 * 54 * 54, 0)
    p = bs.bs_plan(bs.DENSE, 54, 0, 0, bs.BICGSTAB)
    assert p["team"] == 64 and p["slots"] == 56  # the fewest compiled slots holding 54
    p = bs.bs_plan(bs.DENSE, 16, 0, 0, bs.GMRES)
    assert p["team"] == 16 and p["slots"] >= 16
    p = bs.bs_plan(bs.DENSE, 65, 0, 0, bs.CG)
    assert p["slots"] == 0 and p["team"] == 64 and p["rows_per_lane"] == 2
    p = bs.bs_plan(bs.DENSE, 65, 0, 0, bs.GMRES)
    assert p["slots"] == 0 and p["team"] == 1024
    p = bs.bs_plan(bs.DENSE, 1025, 0, 0, bs.GMRES)
    assert p["slots"] == 0 and p["team"] == 1024 and p["rows_per_lane"] == 2
    with pytest.raises(bs.BatchSolveError) as e:
        bs.bs_plan(bs.DENSE, 2049, 0, 0, bs.GMRES)
    assert e.value.code == bs.ERR_UNSUPPORTED
    h = C.c_void_p()
    assert L.bs_pattern_create_dense(0, C.byref(h)) == bs.ERR_INVALID_ARG
    assert L.bs_pattern_create_dense(8, None) == bs.ERR_INVALID_ARG


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of bs_options and bs_plan_info have the header's size
    and field offsets (a C program built with gcc against include/batchsolve.h)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    fields = [f[0] for f in bs.bs_options._fields_]
    pfields = [f[0] for f in bs.bs_plan_info._fields_]
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "batchsolve.h"',
           "int main(void) {", '  printf("%zu %zu\\n", sizeof(bs_options), sizeof(bs_plan_info));']
    src += [f'  printf("%zu\\n", offsetof(bs_options, {f}));' for f in fields]
    src += [f'  printf("%zu\\n", offsetof(bs_plan_info, {f}));' for f in pfields]
    src += ["  return 0;", "}"]
    c = tmp_path / "abi.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "abi"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(root, "include"), str(c), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    vals = [int(v) for v in out]
    assert vals[0] == C.sizeof(bs.bs_options) and vals[1] == C.sizeof(bs.bs_plan_info)
    offs = vals[2:]
    assert offs[:len(fields)] == [getattr(bs.bs_options, f).offset for f in fields]
    assert offs[len(fields):] == [getattr(bs.bs_plan_info, f).offset for f in pfields]


def test_workspace_sizes(L):
    """bs_workspace_size: the fused fixed-size solve takes no workspace.
    bs_varlen_workspace_size: the counter, up to one task per system (16 bytes)
    and the queue order (4 bytes per system), each region 256-byte aligned."""
    assert bs.bs_workspace_size(bs.CSR, 1 << 17, 54, 0, bs.BICGSTAB) == 0
    assert bs.bs_varlen_workspace_size(-1) == 0
    for B in (0, 1, 100, 100_000):
        want = 256 + (-(-(B + 1) * 16 // 256)) * 256 + (-(-(B + 1) * 4 // 256)) * 256
        assert bs.bs_varlen_workspace_size(B) == want


def test_batch_solve_dev_validation(L):
    """bs_batch_solve_dev refuses a missing or inconsistent device pattern
    before it touches a device; n_batch = 0 is a no-op."""
    import ctypes as C
    pd = bs.bs_pattern_dev(None, None, 0, 0)
    args = lambda fmt, nb, n, pat: (fmt, nb, n, pat, None, None, None, bs.BICGSTAB, bs.PREC_JACOBI,
                                    1e-10, 10, None, None, None, None, None, 0, None)
    assert L.bs_batch_solve_dev(*args(bs.CSR, 4, 8, None)) == bs.ERR_INVALID_ARG
    assert L.bs_batch_solve_dev(*args(bs.CSR, 4, 8, C.byref(pd))) == bs.ERR_INVALID_ARG
    bad = bs.bs_pattern_dev(None, 1 << 20, 30, 4)          # ELL: nnz != width * n
    assert L.bs_batch_solve_dev(*args(bs.ELL, 4, 8, C.byref(bad))) == bs.ERR_INVALID_ARG
    assert L.bs_batch_solve_dev(*args(bs.CSR, 4, 0, C.byref(pd))) == bs.ERR_INVALID_ARG
    assert L.bs_batch_solve_dev(*args(bs.DENSE, -1, 8, None)) == bs.ERR_INVALID_ARG
    assert L.bs_batch_solve_dev(*args(bs.DENSE, 0, 8, None)) == bs.OK
    assert L.bs_batch_solve_dev(*args(7, 4, 8, None)) == bs.ERR_INVALID_ARG
