"""Plain FP64 CPU oracle of the learned rank predictor that warm-starts the
basis size of EOD-ABE (the basis loop of Alg. 1, with the stopping test on
|T_j(l,l)|, is the method it serves; the predictor is not part of the paper).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library.

What it defines, written out plainly in NumPy FP64:

* features(diag, m, n, eps): 67 inputs from the first 64 values
  d_c = |T(c,c)| of the stopping test of Alg. 1 (the diagonal of the R factor
  of A Omega[:, :64] computed by block Gram-Schmidt), normalised by d_0 on a
  log10 scale clamped at -16 and divided by 16, then log2 m / 16,
  log2 n / 16 and log10(eps / d_0) / 16 with eps = tol ||A||_F, the
  threshold of the stopping test on the same scale (clamped like the d_c).
* the network 67 -> 256 -> 256 -> 256 -> 2 with the erf form of GELU,
  GELU(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2, after each hidden layer;
  flat parameter layout W1 (256 x 67, row-major), b1, W2 (256 x 256), b2,
  W3, b3, W4 (2 x 256), b4.
* the loss over a batch of B samples with targets t = log(1 + rank):
  (1/B) sum_b [(y_b0 - t_b)^2 + rho_tau(t_b - y_b1)], rho_tau(u) =
  max(tau u, (tau - 1) u), tau = 0.9: head 0 regresses log(1 + rank), head 1
  is its 0.9-quantile.
* its gradient by hand-written backpropagation, and one Adam step (Kingma
  and Ba, ICLR 2015: bias-corrected first and second moments).

Pins (tests/test_predictor_oracle.py): GELU identities and derivative,
closed-form networks, central finite differences of the loss for every
parameter block, the closed form of a first Adam step, the feature map on
geometric sequences.
"""
from __future__ import annotations

import math

import numpy as np

NIN, NH, NOUT = 67, 256, 2
TAU = 0.9
SHAPES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
          ("W3", (NH, NH)), ("b3", (NH,)), ("W4", (NOUT, NH)), ("b4", (NOUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p: np.ndarray) -> dict:
    """Views of the flat parameter vector, in the order of SHAPES."""
    out, off = {}, 0
    for name, shp in SHAPES:
        cnt = int(np.prod(shp))
        out[name] = p[off:off + cnt].reshape(shp)
        off += cnt
    return out


def features(diag: np.ndarray, m: int, n: int, eps: float) -> np.ndarray:
    """67 network inputs from the stopping-test values d_0..d_63 and the
    threshold eps = tol ||A||_F."""
    d = np.asarray(diag, dtype=np.float64)[:64]
    x = np.empty(NIN)
    for c in range(64):
        if d[0] > 0 and d[c] > 0:
            x[c] = max(math.log10(d[c] / d[0]), -16.0) / 16.0
        else:
            x[c] = -1.0
    x[64] = math.log2(m) / 16.0
    x[65] = math.log2(n) / 16.0
    if d[0] > 0 and eps > 0:
        x[66] = min(max(math.log10(eps / d[0]), -16.0), 16.0) / 16.0
    else:
        x[66] = -1.0
    return x


def gelu(z):
    return 0.5 * z * (1.0 + np.vectorize(math.erf)(z / math.sqrt(2.0)))


def gelu_grad(z):
    cdf = 0.5 * (1.0 + np.vectorize(math.erf)(z / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return cdf + z * pdf


def forward(p: np.ndarray, X: np.ndarray):
    """Outputs (B x 2) and the pre-activations of the hidden layers."""
    P = unpack(p)
    z1 = X @ P["W1"].T + P["b1"]
    h1 = gelu(z1)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = gelu(z2)
    z3 = h2 @ P["W3"].T + P["b3"]
    h3 = gelu(z3)
    y = h3 @ P["W4"].T + P["b4"]
    return y, (X, z1, h1, z2, h2, z3, h3)


def loss(y: np.ndarray, t: np.ndarray) -> float:
    B = y.shape[0]
    u = t - y[:, 1]
    pin = np.maximum(TAU * u, (TAU - 1.0) * u)
    return float(np.sum((y[:, 0] - t) ** 2 + pin) / B)


def loss_grad_y(y: np.ndarray, t: np.ndarray) -> np.ndarray:
    """d loss / d y (B x 2); at u = t - y1 = 0 the subgradient 1 - tau."""
    B = y.shape[0]
    g = np.zeros_like(y)
    g[:, 0] = 2.0 * (y[:, 0] - t) / B
    u = t - y[:, 1]
    g[:, 1] = np.where(u > 0, -TAU, 1.0 - TAU) / B
    return g


def grad(p: np.ndarray, X: np.ndarray, t: np.ndarray):
    """(loss, gradient of the loss with respect to the flat parameters)."""
    P = unpack(p)
    y, (X, z1, h1, z2, h2, z3, h3) = forward(p, X)
    L = loss(y, t)
    gy = loss_grad_y(y, t)
    G = {}
    G["W4"] = gy.T @ h3
    G["b4"] = gy.sum(0)
    gz3 = (gy @ P["W4"]) * gelu_grad(z3)
    G["W3"] = gz3.T @ h2
    G["b3"] = gz3.sum(0)
    gz2 = (gz3 @ P["W3"]) * gelu_grad(z2)
    G["W2"] = gz2.T @ h1
    G["b2"] = gz2.sum(0)
    gz1 = (gz2 @ P["W2"]) * gelu_grad(z1)
    G["W1"] = gz1.T @ X
    G["b1"] = gz1.sum(0)
    flat = np.concatenate([G[name].ravel() for name, _ in SHAPES])
    return L, flat


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def predicted_width(y1: float, b: int, margin: float) -> int:
    """Warm-start width d0 = b ceil((rhat (1 + margin) + 1) / b) from the
    quantile head, rhat = exp(y1) - 1 (at least one block)."""
    rhat = max(math.exp(y1) - 1.0, 0.0)
    return b * max(1, math.ceil((rhat * (1.0 + margin) + 1.0) / b))
