"""Host-only tests of the Python binding's argument checks: a tensor of the
wrong element type or count must raise before its raw pointer reaches the
library (the kernels trust both, so a short or float32 buffer would be read or
written past its end).  CPU tensors stand in for device ones; no kernel runs."""
import pytest

torch = pytest.importorskip("torch")

from paper_2308_08417_amd import batchsolve as bs  # noqa: E402


def solve_args(B=6, n=5, nnz=13, width=4, k=1, fmt=bs.CSR):
    stored = {bs.CSR: nnz, bs.ELL: width * n, bs.DENSE: n * n}[fmt]
    return dict(values=torch.zeros(B * stored, dtype=torch.float64),
                b=torch.zeros((B * k, n), dtype=torch.float64),
                x=torch.zeros((B * k, n), dtype=torch.float64),
                iters=torch.zeros(B * k, dtype=torch.int32),
                resid=torch.zeros(B * k, dtype=torch.float64),
                status=torch.zeros(B * k, dtype=torch.int32))


@pytest.mark.parametrize("fmt", [bs.CSR, bs.ELL, bs.DENSE])
def test_solve_args_accept_the_documented_shapes(fmt):
    a = solve_args(fmt=fmt)
    assert bs.check_solve_args(fmt, 5, 13, 4, **a) == (6, 6)


@pytest.mark.parametrize("name,bad,msg", [
    ("values", torch.zeros(6 * 13, dtype=torch.float32), "dtype"),
    ("values", torch.zeros(6 * 13 - 1, dtype=torch.float64), "elements"),
    ("x", torch.zeros((6, 5), dtype=torch.float32), "dtype"),
    ("x", torch.zeros((5, 5), dtype=torch.float64), "elements"),
    ("iters", torch.zeros(6, dtype=torch.int64), "dtype"),
    ("resid", torch.zeros(5, dtype=torch.float64), "elements"),
    ("status", torch.zeros(7, dtype=torch.int32), "elements"),
    ("b", torch.zeros((6, 4), dtype=torch.float64), "b:"),
])
def test_solve_args_reject_wrong_dtype_or_size(name, bad, msg):
    a = solve_args()
    a[name] = bad
    with pytest.raises(ValueError, match=msg):
        bs.check_solve_args(bs.CSR, 5, 13, 4, **a)


def test_solve_args_several_right_hand_sides():
    a = solve_args(B=3, k=4)
    o = bs.bs_options()
    o.n_rhs = 4
    assert bs.check_solve_args(bs.CSR, 5, 13, 4, opts=o, **a) == (3, 12)
    a["values"] = torch.zeros(12 * 13, dtype=torch.float64)  # one matrix per solve: too many
    with pytest.raises(ValueError, match="elements"):
        bs.check_solve_args(bs.CSR, 5, 13, 4, opts=o, **a)


def test_solve_args_check_option_tensors():
    a = solve_args()
    o = bs.bs_options()
    o._keep = (None, torch.zeros((6, 4), dtype=torch.float64), None)  # x_alt one column short
    o.x_alt = 1
    with pytest.raises(ValueError, match="x_alt"):
        bs.check_solve_args(bs.CSR, 5, 13, 4, opts=o, **a)
    o._keep = (torch.zeros(6, dtype=torch.float32), None, None)
    o.x_alt = 0
    o.outer_iters = 1
    with pytest.raises(ValueError, match="outer_iters"):
        bs.check_solve_args(bs.CSR, 5, 13, 4, opts=o, **a)
    raw = bs.bs_options()
    raw.alt_used = 1  # a raw pointer the binding cannot size
    with pytest.raises(ValueError, match="make_options"):
        bs.check_solve_args(bs.CSR, 5, 13, 4, opts=raw, **a)


def test_varbatch_args():
    ok = dict(values=torch.zeros(40, dtype=torch.float64), b=torch.zeros(12, dtype=torch.float64),
              x=torch.zeros(12, dtype=torch.float64), iters=torch.zeros(3, dtype=torch.int32),
              resid=torch.zeros(3, dtype=torch.float64))
    bs.check_varbatch_args(40, 12, 3, **ok)
    for name, bad in (("values", torch.zeros(39, dtype=torch.float64)),
                      ("b", torch.zeros(12, dtype=torch.float32)),
                      ("iters", torch.zeros(4, dtype=torch.int32))):
        a = dict(ok)
        a[name] = bad
        with pytest.raises(ValueError):
            bs.check_varbatch_args(40, 12, 3, **a)


def test_warm_start_args():
    n, nnz, B = 4, 9, 5
    f32, f64 = torch.float32, torch.float64
    bs.check_ws_args(n, nnz, B, values=torch.zeros(B * nnz, dtype=f64),
                     b=torch.zeros((B, n), dtype=f64), x_prev=torch.zeros((B, n), dtype=f64),
                     feat=torch.zeros((B, 3 * n), dtype=f32), delta=torch.zeros((B, n), dtype=f32))
    with pytest.raises(ValueError, match="feat"):
        bs.check_ws_args(n, nnz, B, feat=torch.zeros((B, 3 * n), dtype=f64))
    with pytest.raises(ValueError, match="values"):
        bs.check_ws_args(n, nnz, B, values=torch.zeros(B * nnz - 1, dtype=f64))
    with pytest.raises(ValueError, match="rows"):
        bs.check_ws_args(n, nnz, B, rows=torch.zeros(B - 1, dtype=torch.int32))
    bs.check_ws_args(n, nnz, B, rows=torch.zeros(B + 3, dtype=torch.int32))  # longer list: ok


def test_solve_leaves_the_callers_options_alone(monkeypatch):
    seen = []
    monkeypatch.setattr(bs, "bs_batch_solve", lambda *a, **k: seen.append(a[12]))

    class P:
        handle = 1

    o = bs.bs_options()
    o.flags = bs.FLAG_ABS_TOL
    b = torch.zeros((3, 4), dtype=torch.float64)
    bs.solve(P(), torch.zeros(12, dtype=torch.float64), b, opts=o)
    assert o.flags == bs.FLAG_ABS_TOL  # unchanged
    assert seen[0].flags == bs.FLAG_ABS_TOL | bs.FLAG_X0_ZERO
    bs.solve(P(), torch.zeros(12, dtype=torch.float64), b)
    assert seen[1].flags == bs.FLAG_X0_ZERO
