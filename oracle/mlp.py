"""Reference network for the loss surrogate (oracle, FP64, numpy).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The surrogate is not part of the paper: it is a small fully connected
network that maps a momentum transfer and an energy (Q, w), through the 49
features of encode(), to log Im[-1/eps_LFE](Q, w), the quantity of Eq.
(eps_LFE) that the rate integral of Sec. II sweeps over a dense grid.
Architecture: widths 49 -> 256 -> 256 -> 256 -> 256 -> 1 with the SiLU activation
silu(z) = z / (1 + e^{-z}) after every hidden layer and a linear output;
mean-squared-error loss; Adam (Kingma and Ba, ICLR 2015) with bias
correction.  Every function here is generic in the widths so that small
networks can be checked by finite differences.

Parameters travel as one flat vector, per layer l = 1..L the weight matrix
W_l[n_out][n_in] (row-major) followed by the bias b_l[n_out].

Two arithmetic modes:
* exact: plain FP64 (the function and its exact gradient);
* bf16: the rounding recipe of the GPU kernels, applied to FP64 values:
  every weight matrix is rounded to bfloat16 (round to nearest even) before
  use; the hidden-layer products (layers 2..L-1 and the output layer) round
  their activation operand h to bfloat16, and the backward products round
  dz to bfloat16; the first layer's inputs (the features), the biases, the activation
  function, the loss and the bias gradients are not rounded.  The gradient
  in this mode is the straight-through one (rounding treated as identity).

Parity: forward/backward pinned by central finite differences and by an
independent autograd evaluation (tests/test_oracle_mlp.py); Adam pinned by
its closed-form first step and by a library optimiser; the bfloat16
rounding pinned against a library conversion.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

N_FREQ = 8
N_IN = 5 + 4 * N_FREQ + 12
WIDTHS = (N_IN, 256, 256, 256, 256, 1)


def n_params(widths: Sequence[int] = WIDTHS) -> int:
    return sum(widths[i + 1] * widths[i] + widths[i + 1] for i in range(len(widths) - 1))


def unpack(theta: np.ndarray, widths: Sequence[int] = WIDTHS) -> List[Tuple[np.ndarray, np.ndarray]]:
    """Flat vector -> [(W_l, b_l)], views into theta."""
    out, o = [], 0
    for i in range(len(widths) - 1):
        n_in, n_out = widths[i], widths[i + 1]
        W = theta[o:o + n_out * n_in].reshape(n_out, n_in)
        o += n_out * n_in
        b = theta[o:o + n_out]
        o += n_out
        out.append((W, b))
    assert o == len(theta)
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even) via the float32 bit
    pattern: keep the upper 16 bits after adding 0x7fff plus the lowest
    kept bit.  Non-finite inputs are not expected here."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def forward(theta: np.ndarray, X: np.ndarray, widths: Sequence[int] = WIDTHS, bf16: bool = False):
    """y[b] for inputs X[b][n_in]; returns (y, cache) with the pre-activations
    z_l and activations h_l of every layer (h_0 = X)."""
    r = bf16_round if bf16 else (lambda a: a)
    layers = unpack(np.asarray(theta, np.float64), widths)
    h = np.asarray(X, np.float64)
    hs, zs = [h], []
    L = len(layers)
    for l, (W, b) in enumerate(layers):
        Wr = r(W)
        hin = h if l == 0 else r(h)          # first layer reads the raw inputs
        z = hin @ Wr.T + b
        zs.append(z)
        if l < L - 1:
            h = silu(z)
            hs.append(h)
    y = zs[-1][:, 0]
    return y, dict(hs=hs, zs=zs)


def mse(y, t):
    d = np.asarray(y, np.float64) - np.asarray(t, np.float64)
    return float(np.mean(d * d))


def backward(theta: np.ndarray, cache, y: np.ndarray, t: np.ndarray,
             widths: Sequence[int] = WIDTHS, bf16: bool = False) -> np.ndarray:
    """Gradient of mean((y - t)^2) with respect to the flat parameters."""
    r = bf16_round if bf16 else (lambda a: a)
    layers = unpack(np.asarray(theta, np.float64), widths)
    hs, zs = cache["hs"], cache["zs"]
    B = len(y)
    L = len(layers)
    grads = [None] * L
    dz = (2.0 / B) * (np.asarray(y) - np.asarray(t))[:, None]     # output layer, [B][1]
    for l in range(L - 1, -1, -1):
        W, _ = layers[l]
        hin = hs[l] if l == 0 else r(hs[l])
        dzr = dz if l == 0 else r(dz)
        if l == L - 1:
            dzr = dz          # the output layer's dz (= dy) is FP32 on the GPU
        gW = dzr.T @ hin
        gb = dz.sum(axis=0)
        grads[l] = (gW, gb)
        if l > 0:
            dh = (dz if l == L - 1 else r(dz)) @ r(W)
            dz = dh * silu_grad(zs[l - 1])
    return pack(grads)


def loss_and_grad(theta, X, t, widths=WIDTHS, bf16=False):
    y, cache = forward(theta, X, widths, bf16)
    return mse(y, t), backward(theta, cache, y, t, widths, bf16)


class Adam:
    """Adam with bias correction; state m, v start at zero, step count at 0."""

    def __init__(self, n, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.b1, self.b2, self.eps = beta1, beta2, eps

    def step(self, theta, g, lr):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return theta - lr * mh / (np.sqrt(vh) + self.eps)


def cosine_lr(step: int, n_steps: int, lr0: float, lr1: float) -> float:
    """lr1 + (lr0 - lr1) (1 + cos(pi step / n_steps)) / 2."""
    return lr1 + 0.5 * (lr0 - lr1) * (1.0 + math.cos(math.pi * step / n_steps))


def train(theta, X, t, order, batch, lr0, lr1, widths=WIDTHS, bf16=False):
    """Mini-batch Adam: step s uses samples order[s*batch:(s+1)*batch].
    Returns (theta, per-step losses)."""
    theta = np.array(theta, np.float64)
    n_steps = len(order) // batch
    opt = Adam(len(theta))
    hist = []
    for s in range(n_steps):
        idx = order[s * batch:(s + 1) * batch]
        loss, g = loss_and_grad(theta, X[idx], t[idx], widths, bf16)
        hist.append(loss)
        theta = opt.step(theta, g, cosine_lr(s, n_steps, lr0, lr1))
    return theta, np.array(hist)


# ---------------------------------------------------------------------------
# surrogate input / output scaling
# ---------------------------------------------------------------------------
def frequencies(n: int = N_FREQ) -> np.ndarray:
    """pi 2^(j/2), j < n: the angular frequencies of the Fourier features
    (per unit of the scaled variable w/w_max or |Q|/q_max)."""
    return np.array([math.pi * (math.sqrt(2.0) if j % 2 else 1.0) * 2 ** (j // 2) for j in range(n)])


def encode(qw: np.ndarray, q_max: float, w_max: float, lattice) -> np.ndarray:
    """Features of queries qw[n] = (Qx, Qy, Qz, w) (the surrogate's own
    choice, not the paper's):
      2|Q|/q_max - 1;  Q/|Q| (zero for Q = 0);  2 w/w_max - 1;
      sin, cos of f_j w/w_max;  sin, cos of f_j |Q|/q_max  (f = frequencies());
      sin, cos of h Q.a_i for the primitive vectors a_i (rows of lattice) and
      h = 1, 2, which are unchanged by Q -> Q + any reciprocal lattice vector."""
    qw = np.asarray(qw, np.float64)
    Q, w = qw[:, :3], qw[:, 3]
    q = np.linalg.norm(Q, axis=1)
    d = np.where(q[:, None] > 0, Q / np.where(q > 0, q, 1.0)[:, None], 0.0)
    cols = [2 * q / q_max - 1, d[:, 0], d[:, 1], d[:, 2], 2 * w / w_max - 1]
    for f in frequencies():
        cols += [np.sin(f * w / w_max), np.cos(f * w / w_max)]
    for f in frequencies():
        cols += [np.sin(f * q / q_max), np.cos(f * q / q_max)]
    A = np.asarray(lattice, np.float64).reshape(3, 3)
    for i in range(3):
        ph = Q @ A[i]
        for h in (1, 2):
            cols += [np.sin(h * ph), np.cos(h * ph)]
    return np.column_stack(cols)


def target(loss: np.ndarray, mu: float, sigma: float) -> np.ndarray:
    """Standardised log of the loss, floored at 1e-30."""
    return (np.log(np.maximum(loss, 1e-30)) - mu) / sigma


def decode(ys: np.ndarray, mu: float, sigma: float, calib: float):
    """Ensemble outputs ys[K][n] -> (loss, relative-error estimate):
    exp(mu + sigma * mean) and calib * sigma * sample standard deviation."""
    ys = np.asarray(ys, np.float64)
    m = ys.mean(axis=0)
    sd = ys.std(axis=0, ddof=1) if len(ys) > 1 else np.zeros_like(m)
    return np.exp(mu + sigma * m), calib * sigma * sd
