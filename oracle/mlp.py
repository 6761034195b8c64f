"""Oracle for the learned rank predictor: a plain FP64 multilayer perceptron
32 -> 64 -> 64 -> 2 (ReLU hidden layers, linear output) with a hand-written
backward pass, mean-squared-error loss and Adam, plus the features and labels
it is trained on.

TEST INFRASTRUCTURE ONLY (see oracle/oracle.py): nothing in the product path
uses this module.  It shares no code with the HIP kernels.

The predictor is not part of the paper; it chooses, per transform-domain face,
the rank and sketch width of the randomized truncation that the paper's
compression step (Algorithm alg:strategy, step 3) needs.  Readings:
* features: log10(s_j / s_1), j = 1..32, of the singular values s of a
  32-column Gaussian sketch Y = Xhat_f Omega[:, :32] (0 when s_1 = 0, clipped
  below at -30);
* targets: (k* / 32, l* / 48), k* the exact energy rank at tau, l* the sketch
  width label; loss = mean over the batch of the sum of squared errors / 2;
* parameters, flat: W1 (64 x 32, row major), b1 (64), W2 (64 x 64), b2 (64),
  W3 (2 x 64), b3 (2): 6402 values;
* fp16=True rounds the values the kernels store in half precision (weights,
  inputs, hidden activations) to the nearest half, as the kernels do;
  arithmetic stays FP64.
"""
from __future__ import annotations

import numpy as np

NIN, NH, NOUT = 32, 64, 2
SIZES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
         ("W3", (NOUT, NH)), ("b3", (NOUT,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta: np.ndarray) -> dict:
    """Views of the flat parameter vector as the six arrays (row-major)."""
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def init_params(g: np.random.Generator) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases."""
    theta = np.zeros(NPARAMS)
    P = unpack(theta)
    for name, (fo, fi) in (("W1", (NH, NIN)), ("W2", (NH, NH)), ("W3", (NOUT, NH))):
        b = np.sqrt(6.0 / fi)
        P[name][...] = g.uniform(-b, b, size=(fo, fi))
    return theta


def _h(a, fp16):
    return a.astype(np.float16).astype(np.float64) if fp16 else a


def forward(theta: np.ndarray, X: np.ndarray, fp16: bool = False):
    """y = W3 relu(W2 relu(W1 x + b1) + b2) + b3 for every row x of X (n x 32).
    Returns (y (n x 2), cache)."""
    P = {k: _h(v, fp16) for k, v in unpack(np.asarray(theta, dtype=np.float64)).items()}
    x = _h(np.asarray(X, dtype=np.float64), fp16)
    z1 = x @ P["W1"].T + P["b1"]
    a1 = _h(np.maximum(z1, 0.0), fp16)
    z2 = a1 @ P["W2"].T + P["b2"]
    a2 = _h(np.maximum(z2, 0.0), fp16)
    y = a2 @ P["W3"].T + P["b3"]
    return y, dict(x=x, z1=z1, a1=a1, z2=z2, a2=a2, P=P)


def loss(y: np.ndarray, T: np.ndarray) -> float:
    """Mean over the rows of half the squared error."""
    return float(0.5 * np.sum((y - T) ** 2) / y.shape[0])


def backward(theta: np.ndarray, X: np.ndarray, T: np.ndarray, fp16: bool = False):
    """Gradient of loss(forward(theta, X), T) with respect to theta (flat),
    by the chain rule written out layer by layer.  Returns (loss, grad)."""
    y, c = forward(theta, X, fp16)
    n = y.shape[0]
    P = c["P"]
    dy = (y - T) / n                       # d loss / d y
    g = np.zeros(NPARAMS)
    G = unpack(g)
    G["W3"][...] = dy.T @ c["a2"]
    G["b3"][...] = dy.sum(axis=0)
    da2 = dy @ P["W3"]
    dz2 = da2 * (c["z2"] > 0)
    G["W2"][...] = dz2.T @ c["a1"]
    G["b2"][...] = dz2.sum(axis=0)
    da1 = dz2 @ P["W2"]
    dz1 = da1 * (c["z1"] > 0)
    G["W1"][...] = dz1.T @ c["x"]
    G["b1"][...] = dz1.sum(axis=0)
    return loss(y, T), g


def adam_step(theta, m, v, grad, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; step counts from 1.
    Returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def features(s: np.ndarray) -> np.ndarray:
    """log10(s_j / s_1) for the (32,) or (n, 32) singular values s (sorted
    decreasing); 0 where s_1 = 0; clipped below at -30."""
    s = np.atleast_2d(np.asarray(s, dtype=np.float64))
    s1 = s[:, :1]
    with np.errstate(divide="ignore", invalid="ignore"):
        f = np.where(s1 > 0, np.log10(np.maximum(s, 1e-300) / np.where(s1 > 0, s1, 1.0)), 0.0)
    return np.maximum(f, -30.0)


def predict_widths(y: np.ndarray, kcap: int = 32, widths=(16, 32, 40)):
    """Rank and sketch width from the outputs (k/32, l/48): round up, add one,
    and take the smallest available width >= the prediction (the largest when
    none is).  Returns (k_hat, l_hat) integer arrays."""
    y = np.atleast_2d(y)
    k = np.clip(np.ceil(y[:, 0] * 32.0).astype(int) + 1, 1, kcap)
    lw = np.ceil(y[:, 1] * 48.0).astype(int) + 1
    ws = np.array(sorted(widths))
    idx = np.searchsorted(ws, lw, side="left")
    l = ws[np.minimum(idx, len(ws) - 1)]
    return k, l


def rank_label(sigma: np.ndarray, tau: float, kcap: int = 32) -> int:
    """Rank label of a face whose singular values are prescribed (sigma,
    decreasing): its exact energy rank at tau, the smallest k <= kcap with
    sum_{j>k} s_j^2 <= tau^2 sum_j s_j^2 (the cap when none is)."""
    from . import oracle as _o
    s = np.asarray(sigma, dtype=np.float64)
    return _o.rank_energy(s, float(np.sum(s * s)), tau, kmax=kcap)
