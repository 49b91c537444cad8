"""The allocation-free training step (bs_ws_train_step_noalloc) against the
allocating one (bs_ws_train_step), through the C ABI: two models from the same
parameters take the same steps, one through each entry point; after every step
their parameters, Adam state (through the next step) and losses agree bit for
bit.  Two calls in a row, the second with a smaller (ragged) minibatch; a step
beyond the static workspace is refused."""
import numpy as np
import pytest

from paper_2308_08417_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2308_08417_amd import batchsolve as bs  # noqa: E402


def test_noalloc_train_step_matches_allocating_step():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("no-alloc: training step vs allocating step, n = 54, minibatches 2048 then 1000",
          flush=True)
    bt = W.chem_jacobian(n_batch=4096, n=54, seed=41)
    n = bt.n
    rng = np.random.default_rng(3)
    M = 4096
    feat = torch.from_numpy(rng.standard_normal((M, 3 * n)).astype(np.float32)).to("cuda:0")
    delta = torch.from_numpy(rng.standard_normal((M, n)).astype(np.float32)).to("cuda:0")
    params = W.mlp_init(n, seed=5)
    a = bs.WarmStartModel(n, bt.row_ptr, bt.col_idx)
    b = bs.WarmStartModel(n, bt.row_ptr, bt.col_idx)
    for m in (a, b):
        bs.bs_ws_set_params(m.handle, params)
        bs.bs_ws_fit_scaling(m.handle, feat, delta)
    la = torch.empty(1, dtype=torch.float32, device="cuda:0")
    lb = torch.empty(1, dtype=torch.float32, device="cuda:0")
    for size, seed in ((2048, 1), (1000, 2)):
        rows = torch.from_numpy(np.random.default_rng(seed).permutation(M)[:size]
                                .astype(np.int32)).to("cuda:0")
        bs.bs_ws_train_step(a.handle, feat, delta, 1e-3, loss=la, rows=rows)
        bs.bs_ws_train_step_noalloc(b.handle, feat, delta, 1e-3, loss=lb, rows=rows)
        torch.cuda.synchronize()
        pa, pb = bs.bs_ws_get_params(a.handle), bs.bs_ws_get_params(b.handle)
        assert np.array_equal(pa, pb), f"parameters differ after a {size}-sample step"
        assert la.item() == lb.item()
        assert not np.array_equal(pa, params)  # the step changed something
    big = torch.arange(2049, dtype=torch.int32, device="cuda:0")
    with pytest.raises(bs.BatchSolveError) as e:
        bs.bs_ws_train_step_noalloc(b.handle, feat, delta, 1e-3, rows=big)
    assert e.value.code == bs.ERR_UNSUPPORTED
