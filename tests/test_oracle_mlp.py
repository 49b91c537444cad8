"""Pins of the learned-warm-start oracle (oracle/mlp.py) against facts that do
not come from the oracle itself: central finite differences, a linear network
evaluated through a different association, ReLU cut-offs, Adam's closed-form
first steps, torch's own bfloat16 conversion, and moments of known data."""
import numpy as np
import pytest

from oracle import mlp as M


def small(F=7, H=5, O=3, seed=0, scale=0.5):
    rng = np.random.default_rng(seed)
    p = M.Params(rng.standard_normal((F, H)) * scale, rng.standard_normal(H) * 0.1,
                 rng.standard_normal((H, H)) * scale, rng.standard_normal(H) * 0.1,
                 rng.standard_normal((H, O)) * scale, rng.standard_normal(O) * 0.1)
    z = rng.standard_normal((11, F))
    tgt = rng.standard_normal((11, O))
    return p, z, tgt


def test_backward_matches_central_differences():
    p, z, tgt = small()
    F, H, O = p.W1.shape[0], p.W1.shape[1], p.W3.shape[1]
    L, g = M.grad(p, z, tgt)
    theta = p.flat()
    gf = g.flat()
    h = 1e-6
    num = np.empty_like(theta)
    for i in range(theta.size):
        e = np.zeros_like(theta)
        e[i] = h
        lp = M.loss(M.Params.from_flat(theta + e, F, H, O), z, tgt)
        lm = M.loss(M.Params.from_flat(theta - e, F, H, O), z, tgt)
        num[i] = (lp - lm) / (2 * h)
    assert L == pytest.approx(M.loss(p, z, tgt), rel=0, abs=0)
    err = np.abs(num - gf) / np.maximum(np.abs(num), 1e-3)
    assert err.max() < 1e-6, err.max()


def test_linear_network_reassociated():
    """With every pre-activation positive the net is affine: compare with the
    product of the weight matrices taken first."""
    rng = np.random.default_rng(1)
    F, H, O = 6, 4, 3
    p = M.Params(rng.random((F, H)), rng.random(H), rng.random((H, H)), rng.random(H),
                 rng.standard_normal((H, O)), rng.standard_normal(O))
    z = rng.random((9, F))  # positive inputs, positive first two layers
    y = M.forward(p, z)[2]
    Wc = p.W1 @ (p.W2 @ p.W3)
    bc = (p.b1 @ p.W2 + p.b2) @ p.W3 + p.b3
    assert np.allclose(y, z @ Wc + bc, rtol=1e-13, atol=1e-13)


def test_relu_cuts_negative_units():
    """A hidden unit whose pre-activation is negative for every input cannot
    influence the output, nor receive gradient."""
    p, z, tgt = small(seed=2)
    p.W1[:, 2] = 0.0
    p.b1[2] = -1.0
    y0 = M.forward(p, z)[2]
    p2 = M.Params(**{k: getattr(p, k).copy() for k in M.Params.ORDER})
    p2.W2[2, :] = 123.0
    assert np.array_equal(M.forward(p2, z)[2], y0)
    _, g = M.grad(p, z, tgt)
    assert np.all(g.W2[2, :] == 0) and np.all(g.W1[:, 2] == 0) and g.b1[2] == 0


def test_gradient_zero_at_exact_fit_and_bias_only():
    p, z, tgt = small(seed=3)
    y = M.forward(p, z)[2]
    _, g = M.grad(p, z, y)
    assert np.all(g.flat() == 0)
    # output-bias gradient of the mean squared error: 2 * mean residual / O
    L, g = M.grad(p, z, y - 1.0)
    assert L == pytest.approx(1.0)
    assert np.allclose(g.b3, 2.0 / y.shape[1])


def test_adam_first_steps_closed_form():
    """With bias correction the first two steps under a constant gradient g
    move every parameter by -lr * g / (|g| + eps)."""
    theta = np.array([1.0, -2.0, 0.5, 3.0])
    g = np.array([0.3, -4.0, 1e-3, -0.02])
    opt = M.Adam.zeros(4)
    lr = 0.01
    t1 = opt.step(theta, g, lr)
    assert np.allclose(t1, theta - lr * g / (np.abs(g) + M.ADAM_EPS), rtol=0, atol=1e-15)
    t2 = opt.step(t1, g, lr)
    assert np.allclose(t2, t1 - lr * g / (np.abs(g) + M.ADAM_EPS), rtol=0, atol=1e-15)
    # a zero gradient leaves the parameter where it is
    opt = M.Adam.zeros(1)
    assert opt.step(np.array([5.0]), np.array([0.0]), lr)[0] == 5.0


def test_bf16_against_definition_and_torch():
    torch = pytest.importorskip("torch")
    # exact cases: representable values stay, ties go to even
    one = 1.0
    assert M.bf16(one) == 1.0
    assert M.bf16(1 + 2 ** -8) == 1.0            # tie between 1 and 1+2^-7: even is 1
    assert M.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6  # tie between 1+2^-7 and 1+2^-6: even is 1+2^-6
    assert M.bf16(1 + 2 ** -7) == 1 + 2 ** -7
    assert M.bf16(-3.0) == -3.0
    assert np.isnan(M.bf16(np.nan))
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.standard_normal(5000) * 10 ** rng.uniform(-20, 20, 5000),
                        [0.0, -0.0, 65504.0, 1e-40, 3.4e38]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16(x), ref)


def test_moments_known_data():
    a = np.array([[1.0, 5.0, 2.0], [3.0, 5.0, 2.0], [5.0, 5.0, -4.0]])
    mu, sd = M.moments(a)
    assert np.allclose(mu, [3.0, 5.0, 0.0])
    assert np.allclose(sd, [np.sqrt(8 / 3), 1.0, np.sqrt(8.0)])  # zero spread -> 1


def test_features_and_diagonal():
    rp = np.array([0, 2, 3, 5])
    ci = np.array([0, 2, 0, 1, 2])   # row 1 stores no diagonal
    v = np.array([[4.0, 1.0, 7.0, 2.0, 9.0], [5.0, 0.0, 1.0, 3.0, -1.0]])
    d = M.csr_diagonal(3, rp, ci, v)
    assert np.array_equal(d, [[4.0, 0.0, 9.0], [5.0, 0.0, -1.0]])
    f = M.features(d, np.ones((2, 3)), np.full((2, 3), 2.0))
    assert f.shape == (2, 9) and np.array_equal(f[:, :3], d)
    assert np.array_equal(f[:, 3:6], -np.ones((2, 3)))          # b - x_prev
    assert np.array_equal(f[:, 6:], np.full((2, 3), 2.0))


def test_predict_and_choice():
    p, _, _ = small(F=6, H=4, O=2, seed=5)
    p.W3[:] = 0.0
    p.b3[:] = [1.0, -2.0]
    x0 = M.predict_x0(p, np.zeros(6), np.ones(6), np.array([0.5, 0.25]),
                      np.ones((3, 2)), np.ones((3, 2)), np.full((3, 2), 10.0))
    assert np.array_equal(x0, np.tile([10.5, 9.5], (3, 1)))
    assert list(M.choose_start([1.0, 2.0, 3.0], [1.0, 1.0, 4.0])) == [True, False, True]
