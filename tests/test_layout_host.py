"""Bank-aware layout of one-wave teams (host only, no device).

The layout permutes lanes, buffer elements and CSR windows; the solve's
parity with it is checked on the GPU.  Here: the layout is valid (a
permutation, windows that hold their rows, distinct elements), deterministic,
never worse than the plain layout under the cost model, and its reported
costs agree with an independent evaluation of the model below:
per 32-lane half and register slot, the bank pair ((element) mod 32) that
serves the most distinct 8-byte elements, weighted 5 for gathers and vector
writes against 1 for the register copy of the staged values.
"""
import numpy as np
import pytest

from paper_2308_08417_amd import batchsolve as bs
from paper_2308_08417_amd import workloads as W


@pytest.fixture(scope="module")
def L():
    return bs.lib()


def model_cost(rp, ci, nz, lane_row, lane_win, col_pos):
    n = rp.size - 1
    total_g = total_w = total_c = 0
    for h in range(2):
        lanes = range(32 * h, 32 * h + 32)
        rows = [lane_row[l] for l in lanes if lane_row[l] >= 0]
        wins = {lane_win[l] for l in lanes if lane_row[l] >= 0}
        for k in range(nz):
            elems = set()
            for l in lanes:
                i = lane_row[l]
                if i < 0:
                    elems.add(64)
                    continue
                p = lane_win[l] + k
                elems.add(col_pos[ci[p]] if rp[i] <= p < rp[i + 1] else 64)
            total_g += max(np.bincount([e % 32 for e in elems], minlength=32))
        total_w += max(np.bincount([col_pos[i] % 32 for i in rows], minlength=32))
        total_c += nz * max(np.bincount([w % 32 for w in wins], minlength=32))
    return 5 * (total_g + total_w) + total_c


def plain(rp, nz):
    n = rp.size - 1
    nnz = int(rp[-1])
    lane_row = np.array([i if i < n else -1 for i in range(64)])
    lane_win = np.array([max(0, min(rp[i], nnz - nz)) if i < n else 0 for i in range(64)])
    return lane_row, lane_win, np.arange(n)


def check_valid(rp, ci, nz, lay):
    n = rp.size - 1
    nnz = int(rp[-1])
    lr, lw, cp = lay["lane_row"], lay["lane_win"], lay["col_pos"]
    assert sorted(lr[lr >= 0].tolist()) == list(range(n))
    assert np.all((lr >= -1) & (lr < n))
    for l in range(64):
        if lr[l] >= 0:
            i = lr[l]
            assert max(0, rp[i + 1] - nz) <= lw[l] <= min(rp[i], nnz - nz)
        else:
            half = range(32 * (l // 32), 32 * (l // 32) + 32)
            assert any(lr[m] >= 0 and lw[m] == lw[l] for m in half)
    assert np.unique(cp).size == n and np.all((cp >= 0) & (cp < 64))


@pytest.mark.parametrize("seed", [0, 3])
def test_chem_pattern_layout(L, seed):
    bt = W.chem_jacobian(n_batch=1, n=54, seed=seed)
    rp, ci = bt.row_ptr, bt.col_idx
    nz = 28 if np.diff(rp).max() <= 28 else 32
    lay = bs.bs_wave_layout(rp, ci, nz)
    check_valid(rp, ci, nz, lay)
    assert lay["cost"] == model_cost(rp, ci, nz, lay["lane_row"], lay["lane_win"], lay["col_pos"])
    assert lay["plain_cost"] == model_cost(rp, ci, nz, *plain(rp, nz))
    # the random chemistry pattern has many columns 32 apart read together
    assert lay["cost"] < 0.85 * lay["plain_cost"]
    again = bs.bs_wave_layout(rp, ci, nz)
    for k in ("lane_row", "lane_win", "col_pos"):
        assert np.array_equal(lay[k], again[k])


def test_zero_steps_is_plain(L):
    bt = W.chem_jacobian(n_batch=1, n=40, seed=1)
    rp, ci = bt.row_ptr, bt.col_idx
    nz = 32
    lay = bs.bs_wave_layout(rp, ci, nz, steps=0)
    lr, lw, cp = plain(rp, nz)
    assert np.array_equal(lay["lane_row"][:40], lr[:40]) and np.all(lay["lane_row"][40:] == -1)
    assert np.array_equal(lay["lane_win"][:40], lw[:40])
    assert np.array_equal(lay["col_pos"], cp)
    assert lay["cost"] == lay["plain_cost"]


def test_banded_layout_valid(L):
    # a tridiagonal pattern: the plain layout already reads neighbours, the
    # layout must stay valid and not cost more
    n = 64
    rows = [[j for j in (i - 1, i, i + 1) if 0 <= j < n] for i in range(n)]
    rp = np.cumsum([0] + [len(r) for r in rows]).astype(np.int32)
    ci = np.concatenate(rows).astype(np.int32)
    lay = bs.bs_wave_layout(rp, ci, 4)
    check_valid(rp, ci, 4, lay)
    assert lay["cost"] <= lay["plain_cost"]
    assert lay["cost"] == model_cost(rp, ci, 4, lay["lane_row"], lay["lane_win"], lay["col_pos"])


def test_layout_errors(L):
    rp = np.array([0, 1, 2], np.int32)
    ci = np.array([0, 1], np.int32)
    with pytest.raises(bs.BatchSolveError) as e:
        bs.bs_wave_layout(rp, ci, 1)          # 2 rows: not a one-wave size
    assert e.value.code == bs.ERR_UNSUPPORTED
    bt = W.chem_jacobian(n_batch=1, n=54, seed=0)
    with pytest.raises(bs.BatchSolveError) as e:
        bs.bs_wave_layout(bt.row_ptr, bt.col_idx, 16)   # rows longer than 16 slots
    assert e.value.code == bs.ERR_UNSUPPORTED
    bad = bt.col_idx.copy()
    bad[1] = bad[0]                            # duplicate column in row 0
    with pytest.raises(bs.BatchSolveError) as e:
        bs.bs_wave_layout(bt.row_ptr, bad, 28)
    assert e.value.code == bs.ERR_PATTERN
