"""FP64 oracle of the learned initial guess -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may use
this module; the product path never does.

The learned warm start predicts the change of the solution between two time
steps of a sequence of related batches.  For system s at step t:

  features   f = [diag(A_t), b_t - x_{t-1}, x_{t-1}]            (3n values)
  normalised z = (f - mu_f) / sigma_f   (per component, training-set moments)
  network    h1 = relu(z W1 + b1), h2 = relu(h1 W2 + b2), y = h2 W3 + b3
  guess      x0 = x_{t-1} + sigma_d * y
  target     y* = (x_t - x_{t-1}) / sigma_d

with sigma_d the per-component standard deviation of x_t - x_{t-1} over the
training set.  The features carry the information of (diag(A_t), b_t,
x_{t-1}); the middle block is the difference b_t - x_{t-1}, formed in FP64
before any rounding, because the change of the solution from one step to the
next is of the order of that difference, which is far below the precision a
bfloat16 input keeps of b_t and x_{t-1} themselves.  Loss: mean squared error over samples and components.  Training
uses Adam (Kingma and Ba 2015) with beta1 = 0.9, beta2 = 0.999, eps = 1e-8.
The guess is kept only if its residual is not larger than that of x_{t-1}.

Everything here is plain NumPy in float64; `bf16` rounds to bfloat16 from the
format's definition (round to nearest, ties to even) so that a test can feed
the same rounded weights and inputs to this oracle and to the GPU kernels.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

BETA1, BETA2, ADAM_EPS = 0.9, 0.999, 1e-8
STD_FLOOR = 1e-30  # a component with zero spread is left unscaled


# ------------------------------------------------------------------ bfloat16
def bf16(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64.

    bfloat16 keeps the sign, the 8 exponent bits and the top 7 mantissa bits of
    an IEEE float32; rounding adds half of the dropped range, plus one if the
    kept part is odd (ties to even), then truncates.  NaN stays NaN.
    """
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


# ------------------------------------------------------------------ model
@dataclass
class Params:
    W1: np.ndarray  # [F, H]
    b1: np.ndarray  # [H]
    W2: np.ndarray  # [H, H]
    b2: np.ndarray  # [H]
    W3: np.ndarray  # [H, O]
    b3: np.ndarray  # [O]

    ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")

    def flat(self) -> np.ndarray:
        return np.concatenate([getattr(self, k).ravel() for k in self.ORDER])

    @classmethod
    def from_flat(cls, v, F: int, H: int, O: int) -> "Params":
        v = np.asarray(v, dtype=np.float64)
        shapes = {"W1": (F, H), "b1": (H,), "W2": (H, H), "b2": (H,), "W3": (H, O), "b3": (O,)}
        out, i = {}, 0
        for k in cls.ORDER:
            size = int(np.prod(shapes[k]))
            out[k] = v[i:i + size].reshape(shapes[k]).copy()
            i += size
        assert i == v.size, "parameter vector length does not match the shapes"
        return cls(**out)

    def map(self, fn) -> "Params":
        return Params(**{k: fn(getattr(self, k)) for k in self.ORDER})


def param_count(F: int, H: int, O: int) -> int:
    return F * H + H + H * H + H + H * O + O


def features(diag, b, x_prev) -> np.ndarray:
    """[diag(A), b - x_prev, x_prev] per system: arrays [B, n] -> [B, 3n]."""
    xp = np.asarray(x_prev, np.float64)
    return np.concatenate([np.asarray(diag, np.float64), np.asarray(b, np.float64) - xp, xp],
                          axis=1)


def csr_diagonal(n: int, row_ptr, col_idx, values) -> np.ndarray:
    """A[i, i] of every system (0 where the pattern stores no diagonal)."""
    rp = np.asarray(row_ptr)
    ci = np.asarray(col_idx)
    v = np.asarray(values, np.float64)
    d = np.zeros((v.shape[0], n))
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            if ci[k] == i:
                d[:, i] = v[:, k]
    return d


def moments(a) -> tuple[np.ndarray, np.ndarray]:
    """Per-column mean and (population) standard deviation; a zero spread
    becomes 1 so that the column is only shifted."""
    a = np.asarray(a, np.float64)
    mu = a.mean(axis=0)
    sd = np.sqrt(((a - mu) ** 2).mean(axis=0))
    return mu, np.where(sd > STD_FLOOR, sd, 1.0)


def delta_scale(delta) -> np.ndarray:
    """Per-component standard deviation of x_t - x_{t-1} (about its mean)."""
    return moments(delta)[1]


def forward(p: Params, z) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Returns (h1, h2, y) for normalised features z [M, F]."""
    z = np.asarray(z, np.float64)
    h1 = np.maximum(z @ p.W1 + p.b1, 0.0)
    h2 = np.maximum(h1 @ p.W2 + p.b2, 0.0)
    y = h2 @ p.W3 + p.b3
    return h1, h2, y


def loss(p: Params, z, target) -> float:
    y = forward(p, z)[2]
    return float(np.mean((y - target) ** 2))


def grad(p: Params, z, target) -> tuple[float, Params]:
    """Loss and its gradient with respect to every parameter (backpropagation
    through the three layers; the ReLU derivative is taken as 0 at 0)."""
    z = np.asarray(z, np.float64)
    h1, h2, y = forward(p, z)
    M, O = y.shape
    dy = 2.0 * (y - target) / (M * O)
    dW3 = h2.T @ dy
    db3 = dy.sum(axis=0)
    dz2 = (dy @ p.W3.T) * (h2 > 0)
    dW2 = h1.T @ dz2
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ p.W2.T) * (h1 > 0)
    dW1 = z.T @ dz1
    db1 = dz1.sum(axis=0)
    return float(np.mean((y - target) ** 2)), Params(dW1, db1, dW2, db2, dW3, db3)


@dataclass
class Adam:
    m: np.ndarray
    v: np.ndarray
    t: int = 0

    @classmethod
    def zeros(cls, n: int) -> "Adam":
        return cls(np.zeros(n), np.zeros(n), 0)

    def step(self, theta: np.ndarray, g: np.ndarray, lr: float) -> np.ndarray:
        """One Adam update of the flat parameter vector; returns the new one."""
        self.t += 1
        self.m = BETA1 * self.m + (1 - BETA1) * g
        self.v = BETA2 * self.v + (1 - BETA2) * g * g
        mhat = self.m / (1 - BETA1 ** self.t)
        vhat = self.v / (1 - BETA2 ** self.t)
        return theta - lr * mhat / (np.sqrt(vhat) + ADAM_EPS)


def predict_x0(p: Params, mu_f, sd_f, sd_d, diag, b, x_prev) -> np.ndarray:
    """x0 = x_{t-1} + sigma_d * y(z)."""
    z = (features(diag, b, x_prev) - mu_f) / sd_f
    return np.asarray(x_prev, np.float64) + sd_d * forward(p, z)[2]


def choose_start(res_pred, res_prev) -> np.ndarray:
    """True where the predicted start is kept: its residual norm is not larger
    than that of the previous step's solution."""
    return np.asarray(res_pred) <= np.asarray(res_prev)
