"""CPU oracle of the learned current surrogate (TEST INFRASTRUCTURE).

The paper has no learned part.  This is a small convolutional network over
one crossbar's conductance map and inputs that predicts the relative
parasitic correction of each bit-line current,
    delta_j = (I_j - I0_j) / I0_j,   I0 = G^T V  (the ideal currents, no wire
    resistance: the limit of Sec. II.A as the segment resistance goes to 0),
trained on currents from the exact solver.  Only the test suite uses this
module; it shares nothing with the GPU library.  Arithmetic is float64.

Definitions (the GPU library implements the same definitions in float32):

* Features, 7 channels per crosspoint (i, j) of an m x n crossbar:
  log10(G_ij) + 5 (so [1e-6, 1e-4] S maps to [-1, 1]), 2 V_i, (r - 3) / 2
  for the segment resistance r (ohm), the column and row positions
  2 j / (n - 1) - 1 and 2 i / (m - 1) - 1 (0 for a single column or row), and
  two line totals that set the drops at the line ends: 1e4 times the mean
  conductance of row i, and 1e4 times the column mean of G_i'j 2 V_i' (the
  ideal current of column j over 0.5 m V).
* Network: 3 x 3 convolutions with zero padding of one crosspoint (four by
  default), 7 -> C -> ... -> C -> 2 channels, a bias per output channel, ReLU
  after all but the last.  conv(x)[o, y, x] = b[o] + sum_{c, dy, dx} w[o, c, dy, dx]
  x[c, y + dy - 1, x + dx - 1] (cross-correlation, as deep-learning
  convolutions are defined).
* Column readouts: yhat_j = mean over rows i of the last layer's channel 0
  (the correction), s_j = mean over rows of channel 1 (the error estimate).
* Loss: mean over samples and columns of e_j^2 with e = yhat - delta, plus
  lam times the mean of (s_j - t_j)^2 with t_j = (log(e_j^2 + eps) - MU) / SIG,
  the normalised log of the squared error, held constant (no gradient through
  e).  The estimate term trains only the last layer's channel-1 weights: its
  gradient does not flow into the shared layers, whose gradients are those of
  the first term alone.
* Prediction: I_j = I0_j (1 + yhat_j); relative current error estimate
  exp((SIG s_j + MU) / 2) / |1 + yhat_j| (the current error I0 |yhat - delta|
  over I).
* Optimizer: Adam with bias correction (Kingma and Ba, 2015).
"""
from __future__ import annotations

import numpy as np

N_FEATURES = 7


def features(G: np.ndarray, V: np.ndarray, r: np.ndarray) -> np.ndarray:
    """G [B][m][n] (S), V [B][m] (V), r [B] (ohm) -> X [B][7][m][n]."""
    G = np.asarray(G, dtype=np.float64)
    B, m, n = G.shape
    X = np.empty((B, N_FEATURES, m, n))
    X[:, 0] = np.log10(G) + 5.0
    X[:, 1] = 2.0 * np.asarray(V, dtype=np.float64)[:, :, None]
    X[:, 2] = ((np.asarray(r, dtype=np.float64) - 3.0) / 2.0)[:, None, None]
    X[:, 3] = (2.0 * np.arange(n) / (n - 1) - 1.0)[None, None, :] if n > 1 else 0.0
    X[:, 4] = (2.0 * np.arange(m) / (m - 1) - 1.0)[None, :, None] if m > 1 else 0.0
    X[:, 5] = 1e4 * G.mean(axis=2)[:, :, None]
    X[:, 6] = 1e4 * (G * 2.0 * np.asarray(V, dtype=np.float64)[:, :, None]).mean(axis=1)[:, None, :]
    return X


def ideal_currents(G: np.ndarray, V: np.ndarray) -> np.ndarray:
    """I0 [B][n] = G^T V per sample."""
    return np.einsum("bij,bi->bj", np.asarray(G, np.float64), np.asarray(V, np.float64))


def targets(I: np.ndarray, G: np.ndarray, V: np.ndarray) -> np.ndarray:
    """delta [B][n] = (I - I0) / I0."""
    I0 = ideal_currents(G, V)
    return (np.asarray(I, np.float64) - I0) / I0


def conv2d(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x [B][C][H][W], w [O][C][3][3], b [O] -> [B][O][H][W], zero padding 1."""
    B, C, H, W = x.shape
    xp = np.zeros((B, C, H + 2, W + 2))
    xp[:, :, 1:H + 1, 1:W + 1] = x
    y = np.zeros((B, w.shape[0], H, W)) + b[None, :, None, None]
    for dy in range(3):
        for dx in range(3):
            y += np.einsum("oc,bchw->bohw", w[:, :, dy, dx], xp[:, :, dy:dy + H, dx:dx + W])
    return y


def conv2d_grad_input(g: np.ndarray, w: np.ndarray) -> np.ndarray:
    """d(sum conv2d(x) * g)/dx: g [B][O][H][W] -> [B][C][H][W].  Output (y, x) read
    input (y + dy - 1, x + dx - 1), so input (p, q) receives g at (p - dy + 1, q - dx + 1)."""
    B, O, H, W = g.shape
    gp = np.zeros((B, O, H + 2, W + 2))
    gp[:, :, 1:H + 1, 1:W + 1] = g
    dx_ = np.zeros((B, w.shape[1], H, W))
    for dy in range(3):
        for dx in range(3):
            dx_ += np.einsum("oc,bohw->bchw", w[:, :, dy, dx], gp[:, :, 2 - dy:2 - dy + H, 2 - dx:2 - dx + W])
    return dx_


def conv2d_grad_weight(x: np.ndarray, g: np.ndarray):
    """d(sum conv2d(x) * g)/dw [O][C][3][3] and /db [O]."""
    B, C, H, W = x.shape
    xp = np.zeros((B, C, H + 2, W + 2))
    xp[:, :, 1:H + 1, 1:W + 1] = x
    gw = np.zeros((g.shape[1], C, 3, 3))
    for dy in range(3):
        for dx in range(3):
            gw[:, :, dy, dx] = np.einsum("bohw,bchw->oc", g, xp[:, :, dy:dy + H, dx:dx + W])
    return gw, g.sum(axis=(0, 2, 3))


def init_params(channels: int = 32, seed: int = 0, depth: int = 4):
    """He-initialised weights [(w, b)] of the `depth` layers, float64."""
    rng = np.random.default_rng(seed)
    dims = [N_FEATURES] + [channels] * (depth - 1) + [2]
    out = []
    for k in range(depth):
        fan_in = dims[k] * 9
        out.append((rng.normal(0.0, np.sqrt(2.0 / fan_in), (dims[k + 1], dims[k], 3, 3)), np.zeros(dims[k + 1])))
    return out


def forward(params, X):
    """Activations [X, a1, ..., Y] (a_k after ReLU; Y the last map, [B][2][m][n])."""
    acts = [X]
    for k, (w, b) in enumerate(params):
        y = conv2d(acts[-1], w, b)
        acts.append(np.maximum(y, 0.0) if k < len(params) - 1 else y)
    return acts


def readout(Y: np.ndarray) -> np.ndarray:
    """yhat [B][n] = mean over rows of Y[:, 0]."""
    return Y[:, 0].mean(axis=1)


LAM, EPS, MU, SIG = 0.1, 1e-8, -12.0, 4.0


def estimate(Y: np.ndarray) -> np.ndarray:
    """Relative current error estimate [B][n] = exp((SIG s + MU) / 2) / |1 + yhat|, s =
    mean over rows of Y[:, 1]: the error of the correction, |yhat - delta|, divided by
    the predicted current over the ideal one, I / I0 = 1 + yhat."""
    return np.exp(0.5 * (SIG * Y[:, 1].mean(axis=1) + MU)) / np.abs(1.0 + readout(Y))


def loss_and_grad(Y: np.ndarray, delta: np.ndarray, lam: float = LAM, eps: float = EPS):
    """(main loss, estimate loss, dLoss/dY) for the two column readouts."""
    B, _, m, n = Y.shape
    e = readout(Y) - delta
    s = Y[:, 1].mean(axis=1)
    t = (np.log(e * e + eps) - MU) / SIG
    dY = np.empty_like(Y)
    dY[:, 0] = (2.0 * e / (B * n * m))[:, None, :]
    dY[:, 1] = (lam * 2.0 * (s - t) / (B * n * m))[:, None, :]
    return float(np.mean(e * e)), float(np.mean((s - t) ** 2)), dY


def backward(params, acts, dY):
    """Gradients [(dw, db)] of every layer given dLoss/dY; the estimate channel's
    gradient stops at the last layer (its input gradient uses channel 0 only)."""
    last = len(params) - 1
    grads = [None] * len(params)
    g = dY
    for k in range(last, -1, -1):
        w, _ = params[k]
        grads[k] = conv2d_grad_weight(acts[k], g)
        if k == last:
            g = g.copy()
            g[:, 1] = 0.0
        if k > 0:
            g = conv2d_grad_input(g, w) * (acts[k] > 0.0)
    return grads


def adam_step(p, g, m1, m2, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t >= 1: returns (p, m1, m2)."""
    m1 = b1 * m1 + (1.0 - b1) * g
    m2 = b2 * m2 + (1.0 - b2) * g * g
    mh = m1 / (1.0 - b1 ** t)
    vh = m2 / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m1, m2


def predict(params, G, V, r):
    """Surrogate currents [B][n] and their relative error estimates [B][n]."""
    Y = forward(params, features(G, V, r))[-1]
    return ideal_currents(G, V) * (1.0 + readout(Y)), estimate(Y)
