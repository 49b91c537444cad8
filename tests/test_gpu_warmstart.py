"""GPU parity of the learned initial guess against the FP64 oracle
(oracle/mlp.py), through the C ABI.

The network's products run in BF16 with FP32 accumulation; the oracle is
evaluated on the same BF16-rounded weights and normalised inputs, in FP64, and
the bar is a max-norm relative error of 2e-2 per tensor (outputs, loss, each
weight and bias gradient).  Layout work (features) is bit-exact; the scaling
moments agree to FP64 summation order; the Adam step agrees to FP32 rounding.
Whatever start is used, the solve itself is judged by the FP64 residual.
"""
import os
import sys

import numpy as np
import pytest

import oracle as O
from oracle import mlp as OM
from paper_2308_08417_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2308_08417_amd import batchsolve as bs  # noqa: E402

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_gpu_parity import dev, say  # noqa: E402

BF16_TOL = 2e-2
H = 256


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bs.lib()


def maxrel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def traj():
    """Four steps of a drifting chemistry-like sequence (2048 systems, n = 54),
    solved by the oracle: the data every test below starts from."""
    steps = list(W.chem_trajectory(n_batch=2048, n=54, steps=4, seed=3))
    OP = O.Pattern(54, steps[0].row_ptr, steps[0].col_idx)
    xs = [O.batch_solve(OP, s.values, s.b, tol=1e-12, max_iter=100)[0] for s in steps]
    return steps, xs


def model_for(bt, params=None):
    m = bs.WarmStartModel(bt.n, bt.row_ptr, bt.col_idx)
    if params is not None:
        bs.bs_ws_set_params(m.handle, params)
    return m


def gpu_features(m, bt, x_prev, x_next):
    B, n = bt.b.shape
    feat = torch.empty((B, 3 * n), dtype=torch.float32, device="cuda:0")
    delta = torch.empty((B, n), dtype=torch.float32, device="cuda:0")
    bs.bs_ws_features(m.handle, dev(bt.values), dev(bt.b), dev(x_prev), feat, x_next=dev(x_next),
                      delta=delta)
    torch.cuda.synchronize()
    return feat, delta


def oracle_setup(bt, x_prev, x_next, feat_np, delta_np, params, mu, sd, sdd):
    """Oracle inputs on the GPU's own rounding: FP32 raw features, normalised in
    FP64, rounded through FP32 to BF16; BF16 weights, FP32 biases."""
    n = bt.n
    z = OM.bf16(((feat_np.astype(np.float64) - mu) / sd).astype(np.float32))
    P = OM.Params.from_flat(params.astype(np.float64), 3 * n, H, n)
    Pb = OM.Params(OM.bf16(P.W1), P.b1, OM.bf16(P.W2), P.b2, OM.bf16(P.W3), P.b3)
    tgt = (delta_np.astype(np.float64) / sdd).astype(np.float32).astype(np.float64)
    return z, Pb, tgt


def test_features_bit_exact(traj):
    steps, xs = traj
    bt = steps[1]
    m = model_for(bt)
    feat, delta = gpu_features(m, bt, xs[0], xs[1])
    d = OM.csr_diagonal(bt.n, bt.row_ptr, bt.col_idx, bt.values)
    ref = OM.features(d, bt.b, xs[0]).astype(np.float32)
    assert np.array_equal(feat.cpu().numpy(), ref)
    assert np.array_equal(delta.cpu().numpy(), (xs[1] - xs[0]).astype(np.float32))


def test_scaling_moments(traj):
    steps, xs = traj
    bt = steps[2]
    m = model_for(bt)
    feat, delta = gpu_features(m, bt, xs[1], xs[2])
    bs.bs_ws_fit_scaling(m.handle, feat, delta)
    mu, sd, sdd = bs.bs_ws_get_scaling(m.handle, bt.n)
    f = feat.cpu().numpy().astype(np.float64)
    dl = delta.cpu().numpy().astype(np.float64)
    omu, osd = OM.moments(f)
    assert np.allclose(mu, omu, rtol=1e-12, atol=1e-300)
    assert np.allclose(sd, osd, rtol=1e-10)
    assert np.allclose(sdd, OM.delta_scale(dl), rtol=1e-10)


@pytest.fixture(scope="module")
def fitted(traj):
    steps, xs = traj
    bt = steps[1]
    params = W.mlp_init(bt.n, seed=7)
    rng = np.random.default_rng(11)
    # nonzero biases so that every term of the network is exercised
    nb = params.size
    params = params.copy()
    F, n = 3 * bt.n, bt.n
    o_b1, o_b2 = F * H, F * H + H + H * H
    o_b3 = o_b2 + H + H * n
    params[o_b1:o_b1 + H] = rng.standard_normal(H).astype(np.float32) * 0.1
    params[o_b2:o_b2 + H] = rng.standard_normal(H).astype(np.float32) * 0.1
    params[o_b3:o_b3 + n] = rng.standard_normal(n).astype(np.float32) * 0.1
    assert params.size == nb
    m = model_for(bt, params)
    feat, delta = gpu_features(m, bt, xs[0], xs[1])
    bs.bs_ws_fit_scaling(m.handle, feat, delta)
    mu, sd, sdd = bs.bs_ws_get_scaling(m.handle, bt.n)
    fnp, dnp = feat.cpu().numpy(), delta.cpu().numpy()
    z, Pb, tgt = oracle_setup(bt, xs[0], xs[1], fnp, dnp, params, mu, sd, sdd)
    return dict(bt=bt, m=m, params=params, feat=feat, delta=delta, z=z, Pb=Pb, tgt=tgt, mu=mu,
                sd=sd, sdd=sdd, x_prev=xs[0], x_next=xs[1])


def test_forward_matches_oracle(fitted):
    f = fitted
    B, n = f["bt"].b.shape
    y = torch.empty((B, n), dtype=torch.float32, device="cuda:0")
    bs.bs_ws_forward(f["m"].handle, f["feat"], y)
    torch.cuda.synchronize()
    yo = OM.forward(f["Pb"], f["z"])[2]
    err = maxrel(y.cpu().numpy(), yo)
    say(f"  forward max rel error {err:.2e}")
    assert err <= BF16_TOL
    # a row list picks rows
    rows = torch.from_numpy(np.array([5, 0, 2047, 5], np.int32)).to("cuda:0")
    y2 = torch.empty((4, n), dtype=torch.float32, device="cuda:0")
    bs.bs_ws_forward(f["m"].handle, f["feat"], y2, rows=rows)
    torch.cuda.synchronize()
    assert np.array_equal(y2.cpu().numpy(), y.cpu().numpy()[[5, 0, 2047, 5]])


def test_gradient_matches_oracle(fitted):
    f = fitted
    m = f["m"]
    grad = torch.empty(m.param_count, dtype=torch.float32, device="cuda:0")
    loss = torch.empty(1, dtype=torch.float32, device="cuda:0")
    bs.bs_ws_grad(m.handle, f["feat"], f["delta"], grad, loss)
    torch.cuda.synchronize()
    L, g = OM.grad(f["Pb"], f["z"], f["tgt"])
    n = f["bt"].n
    gg = OM.Params.from_flat(grad.cpu().numpy().astype(np.float64), 3 * n, H, n)
    errs = {k: maxrel(getattr(gg, k), getattr(g, k)) for k in OM.Params.ORDER}
    lerr = abs(loss.item() - L) / L
    say(f"  loss {loss.item():.6e} vs {L:.6e} (rel {lerr:.1e}); grad max rel errors {errs}")
    assert lerr <= BF16_TOL
    for k, e in errs.items():
        assert e <= BF16_TOL, f"{k}: {e}"
    # deterministic: the same call gives the same bits
    grad2 = torch.empty_like(grad)
    bs.bs_ws_grad(m.handle, f["feat"], f["delta"], grad2, loss)
    torch.cuda.synchronize()
    assert torch.equal(grad, grad2)


def test_gradient_ragged_minibatch(fitted):
    """A minibatch given by a row list whose length is not a multiple of the
    64-sample tile (1000 = 15 * 64 + 40).  The rounding noise of the BF16
    products averages out as 1/sqrt(M) against the gradient, so the per-tensor
    bound is checked on minibatches of this size and up; the row-list
    indirection itself is checked exactly on a smaller one."""
    f = fitted
    m = f["m"]
    n = f["bt"].n
    grad = torch.empty(m.param_count, dtype=torch.float32, device="cuda:0")
    loss = torch.empty(1, dtype=torch.float32, device="cuda:0")
    sel = np.random.default_rng(3).choice(2048, 1000, replace=False).astype(np.int32)
    bs.bs_ws_grad(m.handle, f["feat"], f["delta"], grad, loss, rows=torch.from_numpy(sel).to("cuda:0"))
    torch.cuda.synchronize()
    L, g = OM.grad(f["Pb"], f["z"][sel], f["tgt"][sel])
    gg = OM.Params.from_flat(grad.cpu().numpy().astype(np.float64), 3 * n, H, n)
    errs = {k: maxrel(getattr(gg, k), getattr(g, k)) for k in OM.Params.ORDER}
    say(f"  1000-sample minibatch: grad max rel errors {errs}")
    for k, e in errs.items():
        assert e <= BF16_TOL, k
    assert abs(loss.item() - L) / L <= BF16_TOL
    # rows picked through the list == the same rows stored contiguously
    small = torch.from_numpy(sel[:300].copy()).to("cuda:0")
    bs.bs_ws_grad(m.handle, f["feat"], f["delta"], grad, loss, rows=small)
    g_list = grad.clone()
    l_list = loss.clone()
    feat_c = f["feat"][small.long()].contiguous()
    delta_c = f["delta"][small.long()].contiguous()
    bs.bs_ws_grad(m.handle, feat_c, delta_c, grad, loss)
    torch.cuda.synchronize()
    assert torch.equal(g_list, grad) and torch.equal(l_list, loss)


def test_adam_step_matches_oracle(fitted):
    """Two Adam steps: each moves the FP32 master weights as the oracle's Adam
    does with the GPU's gradient at the current weights."""
    f = fitted
    m = model_for(f["bt"], f["params"])
    bs.bs_ws_set_scaling(m.handle, f["mu"], f["sd"], f["sdd"])
    grad = torch.empty(m.param_count, dtype=torch.float32, device="cuda:0")
    loss = torch.empty(1, dtype=torch.float32, device="cuda:0")
    opt = OM.Adam.zeros(m.param_count)
    lr = 1e-3
    theta = f["params"].astype(np.float64)
    for step in range(2):
        bs.bs_ws_grad(m.handle, f["feat"], f["delta"], grad, loss)
        torch.cuda.synchronize()
        g = grad.cpu().numpy().astype(np.float64)
        bs.bs_ws_train_step(m.handle, f["feat"], f["delta"], lr)
        got = bs.bs_ws_get_params(m.handle).astype(np.float64)
        ref = opt.step(theta, g, lr)
        dev_ = np.max(np.abs((got - theta) - (ref - theta)))
        say(f"  Adam step {step + 1}: max deviation {dev_:.2e} (lr {lr})")
        assert dev_ <= 1e-4 * lr + 1e-6 * np.max(np.abs(theta))
        theta = got


def test_inference_matches_oracle(fitted):
    f = fitted
    bt = f["bt"]
    B, n = bt.b.shape
    x0 = torch.empty((B, n), dtype=torch.float64, device="cuda:0")
    bs.bs_ws_infer(f["m"].handle, dev(bt.values), dev(bt.b), dev(f["x_prev"]), x0)
    torch.cuda.synchronize()
    # the oracle's features straight from FP64 (the fused kernel reads the batch)
    d = OM.csr_diagonal(n, bt.row_ptr, bt.col_idx, bt.values)
    z = OM.bf16(((OM.features(d, bt.b, f["x_prev"]) - f["mu"]) / f["sd"]).astype(np.float32))
    yo = OM.forward(f["Pb"], z)[2]
    yg = (x0.cpu().numpy() - f["x_prev"]) / f["sdd"]
    err = maxrel(yg, yo)
    say(f"  inference max rel error {err:.2e}")
    assert err <= BF16_TOL


@pytest.mark.parametrize("solver", [bs.BICGSTAB, bs.CG, bs.GMRES])
def test_fallback_start_choice(traj, solver):
    """The solve keeps the start with the smaller residual: garbage in half the
    systems' x must lose to x_alt there, an exact x must win elsewhere."""
    steps, xs = traj
    bt = steps[3]
    if solver == bs.CG:  # CG needs SPD: use a symmetric tridiagonal batch instead
        from test_gpu_parity import symmetric_tridiag
        bt = symmetric_tridiag(512, 40, seed=9)
    B, n = bt.b.shape
    OP = O.Pattern(n, bt.row_ptr, bt.col_idx)
    so = {bs.BICGSTAB: O.BICGSTAB, bs.CG: O.CG, bs.GMRES: O.GMRES}[solver]
    exact = O.batch_solve(OP, bt.values, bt.b, solver=so, tol=1e-13, max_iter=300)[0]
    rng = np.random.default_rng(5)
    x_try = exact + 1e-9 * rng.standard_normal(exact.shape)
    x_try[::2] = 10.0 * rng.standard_normal(x_try[::2].shape)
    x_alt = exact + 1e-6 * rng.standard_normal(exact.shape)
    P = bs.Pattern.from_csr(bt.row_ptr, bt.col_idx)
    x = dev(x_try)
    used = torch.full((B,), -1, dtype=torch.int32, device="cuda:0")
    it = torch.empty(B, dtype=torch.int32, device="cuda:0")
    rs = torch.empty(B, dtype=torch.float64, device="cuda:0")
    st = torch.empty(B, dtype=torch.int32, device="cuda:0")
    opts = bs.make_options(x_alt=dev(x_alt), alt_used=used)
    bs.bs_batch_solve(bs.CSR, P.handle, dev(bt.values), dev(bt.b), x, solver, bs.PREC_JACOBI,
                      1e-10, 300, it, rs, st, opts)
    torch.cuda.synchronize()
    r_try = O.true_residual(OP, bt.values, bt.b, x_try)
    r_alt = O.true_residual(OP, bt.values, bt.b, x_alt)
    want = ~OM.choose_start(r_try, r_alt)
    u = used.cpu().numpy()
    assert np.array_equal(u.astype(bool), want)
    assert u[::2].all() and not u[1::2].any()
    start = np.where(want[:, None], x_alt, x_try)
    o = O.batch_solve(OP, bt.values, bt.b, x0=start, solver=so, tol=1e-10, max_iter=300)
    assert np.array_equal(st.cpu().numpy(), o[3])
    assert np.all(np.abs(it.cpu().numpy() - o[1]) <= 2)
    xg = x.cpu().numpy()
    assert np.all(O.true_residual(OP, bt.values, bt.b, xg) <= 1e-10)
    # x_alt with BS_FLAG_X0_ZERO is refused
    with pytest.raises(bs.BatchSolveError):
        bs.bs_batch_solve(bs.CSR, P.handle, dev(bt.values), dev(bt.b), x, solver, bs.PREC_JACOBI,
                          1e-10, 300, it, rs, st,
                          bs.make_options(flags=bs.FLAG_X0_ZERO, x_alt=dev(x_alt)))


def run_sequence(B, T, T_train, seed, b_drift, epochs, mb, lr=1e-3):
    """Solve a drifting chemistry-like sequence with the plain solver (x0 = 0),
    train the network on steps t < T_train, and return what the held-out steps
    need: the pattern, values, right-hand sides, solutions, the model and the
    loss after every epoch."""
    n = 54
    steps = list(W.chem_trajectory(n_batch=B, n=n, steps=T, seed=seed, b_drift=b_drift))
    bt0 = steps[0]
    P = bs.Pattern.from_csr(bt0.row_ptr, bt0.col_idx)
    it = torch.empty(B, dtype=torch.int32, device="cuda:0")
    rs = torch.empty(B, dtype=torch.float64, device="cuda:0")
    st = torch.empty(B, dtype=torch.int32, device="cuda:0")
    vals = [dev(s.values) for s in steps]
    bbs = [dev(s.b) for s in steps]
    xs = []
    for t in range(T):  # the plain solver's solutions (x0 = 0)
        x = torch.empty((B, n), dtype=torch.float64, device="cuda:0")
        bs.bs_batch_solve(bs.CSR, P.handle, vals[t], bbs[t], x, bs.BICGSTAB, bs.PREC_JACOBI,
                          1e-10, 200, it, rs, st, bs.make_options(flags=bs.FLAG_X0_ZERO))
        torch.cuda.synchronize()
        assert (st == 0).all().item()
        xs.append(x)
    m = bs.WarmStartModel(n, bt0.row_ptr, bt0.col_idx)
    bs.bs_ws_set_params(m.handle, W.mlp_init(n, seed=2))
    M = (T_train - 1) * B
    feat = torch.empty((M, 3 * n), dtype=torch.float32, device="cuda:0")
    delta = torch.empty((M, n), dtype=torch.float32, device="cuda:0")
    for t in range(1, T_train):
        sl = slice((t - 1) * B, t * B)
        bs.bs_ws_features(m.handle, vals[t], bbs[t], xs[t - 1], feat[sl], x_next=xs[t],
                          delta=delta[sl])
    bs.bs_ws_fit_scaling(m.handle, feat, delta)
    loss = torch.empty(1, dtype=torch.float32, device="cuda:0")
    rng = np.random.default_rng(4)
    losses = []
    for epoch in range(epochs):
        perm = torch.from_numpy(rng.permutation(M).astype(np.int32)).to("cuda:0")
        for i in range(0, M - mb + 1, mb):
            bs.bs_ws_train_step(m.handle, feat, delta, lr, loss=loss, rows=perm[i:i + mb])
        torch.cuda.synchronize()
        losses.append(loss.item())
    return dict(steps=steps, P=P, vals=vals, bbs=bbs, xs=xs, m=m, losses=losses, it=it, rs=rs,
                st=st, B=B, n=n)


def held_out(r, T_train, T):
    """On each held-out step: the network's loss on that step, the true residual
    of the guess and of x_{t-1} before any solve (oracle, FP64), and the
    iterations of the FP64 solve from x0 = 0, from x_{t-1}, and from the guess
    with x_{t-1} as the fallback."""
    B, n, m = r["B"], r["n"], r["m"]
    OP = O.Pattern(n, r["steps"][0].row_ptr, r["steps"][0].col_idx)
    out = {"loss": [], "r_guess": [], "r_prev": [], "it_zero": [], "it_prev": [],
           "it_learned": [], "fallback": []}
    grad = torch.empty(bs.bs_ws_param_count(m.handle), dtype=torch.float32, device="cuda:0")
    loss = torch.empty(1, dtype=torch.float32, device="cuda:0")
    for t in range(T_train, T):
        vals, bb, xp = r["vals"][t], r["bbs"][t], r["xs"][t - 1]
        feat = torch.empty((B, 3 * n), dtype=torch.float32, device="cuda:0")
        delta = torch.empty((B, n), dtype=torch.float32, device="cuda:0")
        bs.bs_ws_features(m.handle, vals, bb, xp, feat, x_next=r["xs"][t], delta=delta)
        bs.bs_ws_grad(m.handle, feat, delta, grad, loss)
        guess = torch.empty((B, n), dtype=torch.float64, device="cuda:0")
        bs.bs_ws_infer(m.handle, vals, bb, xp, guess)
        torch.cuda.synchronize()
        out["loss"].append(loss.item())
        sb = r["steps"][t]
        out["r_guess"].append(O.true_residual(OP, sb.values, sb.b, guess.cpu().numpy()))
        out["r_prev"].append(O.true_residual(OP, sb.values, sb.b, xp.cpu().numpy()))
        for kind in ("zero", "prev", "learned"):
            x = torch.empty((B, n), dtype=torch.float64, device="cuda:0")
            used = torch.empty(B, dtype=torch.int32, device="cuda:0")
            if kind == "zero":
                opts = bs.make_options(flags=bs.FLAG_X0_ZERO)
            elif kind == "prev":
                x.copy_(xp)
                opts = bs.make_options()
            else:
                x.copy_(guess)
                opts = bs.make_options(x_alt=xp, alt_used=used)
            bs.bs_batch_solve(bs.CSR, r["P"].handle, vals, bb, x, bs.BICGSTAB, bs.PREC_JACOBI,
                              1e-10, 200, r["it"], r["rs"], r["st"], opts)
            torch.cuda.synchronize()
            assert (r["st"] == 0).all().item() and (r["rs"] <= 1e-10).all().item()
            out["it_" + kind].append(r["it"].cpu().numpy())
            if kind == "learned":
                out["fallback"].append(used.cpu().numpy())
    return {k: np.concatenate(v) if k != "loss" else np.array(v) for k, v in out.items()}


def test_learned_start_beats_previous_solution():
    """A sequence whose right-hand side drifts 1% per step (besides gamma and
    J): the change of the solution follows b_t - x_{t-1}, which the features
    carry, so training must work here.  On held-out steps the network's loss
    falls well below 1 (the variance of the change it predicts), its guess has
    a smaller true residual than x_{t-1} for most systems, and the solve from
    it (x_{t-1} as the fallback) takes no more iterations than from x_{t-1}."""
    T, T_train = 18, 15
    r = run_sequence(B=4096, T=T, T_train=T_train, seed=21, b_drift=0.01, epochs=16, mb=1024)
    say(f"  training loss by epoch: {['%.4f' % v for v in r['losses']]}")
    h = held_out(r, T_train, T)
    better = float(np.mean(h["r_guess"] < h["r_prev"]))
    ratio = float(np.median(h["r_guess"] / h["r_prev"]))
    mean = {k: float(h[k].mean()) for k in ("it_zero", "it_prev", "it_learned")}
    say(f"  held-out loss {h['loss']}; guess residual below x_prev's for {100 * better:.1f}% "
        f"of systems (median ratio {ratio:.3f}); iterations {mean}; fallback "
        f"{100 * h['fallback'].mean():.1f}%")
    assert np.all(h["loss"] < 0.3)
    assert r["losses"][-1] < 0.3 * r["losses"][0]
    assert better >= 0.9 and ratio < 0.5
    assert h["fallback"].mean() <= 0.1
    assert mean["it_learned"] <= mean["it_prev"] and mean["it_learned"] <= mean["it_zero"]


def test_literal_sequence_has_no_signal_and_fallback_protects():
    """The literal sequence (b fixed; gamma and every J entry drift by fresh
    random factors): the change of the solution comes from the drift of J,
    which the features do not show, so the held-out loss stays near 1.  The
    fallback keeps each solve's start at least as good as x_{t-1}: the mean
    iterations from the learned start do not exceed those from x_{t-1}."""
    T, T_train = 12, 9
    r = run_sequence(B=4096, T=T, T_train=T_train, seed=1, b_drift=0.0, epochs=8, mb=1024)
    h = held_out(r, T_train, T)
    mean = {k: float(h[k].mean()) for k in ("it_zero", "it_prev", "it_learned")}
    say(f"  training loss by epoch: {['%.4f' % v for v in r['losses']]}; held-out loss "
        f"{h['loss']}; iterations {mean}; fallback {100 * h['fallback'].mean():.1f}%")
    assert np.all(h["loss"] > 0.5)
    start = np.minimum(h["r_guess"], h["r_prev"])
    assert np.all(start <= h["r_prev"])
    assert mean["it_learned"] <= mean["it_prev"] + 0.05


def test_packed_inference_equals_model_inference(fitted):
    """bs_ws_infer_packed on weights copied out by bs_ws_pack, with the
    diagonals handed over as an array, gives the bits of bs_ws_infer (which
    gathers the diagonal from the CSR values itself)."""
    f = fitted
    bt = f["bt"]
    B, n = bt.b.shape
    x0 = torch.empty((B, n), dtype=torch.float64, device="cuda:0")
    bs.bs_ws_infer(f["m"].handle, dev(bt.values), dev(bt.b), dev(f["x_prev"]), x0)
    w = torch.full((bs.bs_ws_packed_bytes(n),), 0xFF, dtype=torch.uint8, device="cuda:0")
    bs.bs_ws_pack(f["m"].handle, w)
    diag = dev(OM.csr_diagonal(n, bt.row_ptr, bt.col_idx, bt.values))
    x1 = torch.empty_like(x0)
    bs.bs_ws_infer_packed(w, n, diag, dev(bt.b), dev(f["x_prev"]), x1)
    torch.cuda.synchronize()
    assert torch.equal(x0, x1)
    with pytest.raises(ValueError):
        bs.bs_ws_infer_packed(w[:100], n, diag, dev(bt.b), dev(f["x_prev"]), x1)
    assert bs.bs_ws_packed_bytes(0) == 0 and bs.bs_ws_packed_bytes(65) == 0
