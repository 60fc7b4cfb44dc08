"""Pins of the FP64 oracle of the learned rank predictor (CPU only).

Each check fixes the oracle to something other than itself: identities of
the error function, networks whose output is known in closed form, central
finite differences of the loss (which use only the forward pass), the
closed form of a first Adam step, and the feature map on sequences whose
logarithms are known.
"""
import math

import numpy as np
import pytest

from oracle import predictor_oracle as P


def test_gelu_identities():
    z = np.linspace(-6.0, 6.0, 121)
    g = P.gelu(z)
    # odd part of GELU is z/2: GELU(z) - GELU(-z) = z (erf is odd)
    assert np.allclose(g - P.gelu(-z), z, atol=1e-15)
    assert P.gelu(np.array([0.0]))[0] == 0.0
    # far tails: GELU(z) -> z and -> 0 faster than the Gaussian density
    assert abs(P.gelu(np.array([10.0]))[0] - 10.0) < 1e-20
    assert abs(P.gelu(np.array([-10.0]))[0]) < 1e-20
    # GELU(1) = Phi(1) with Phi(1) = 0.8413447460685429 (normal table)
    assert abs(P.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15


def test_gelu_derivative():
    z = np.linspace(-5.0, 5.0, 41)
    h = 1e-6
    fd = (P.gelu(z + h) - P.gelu(z - h)) / (2 * h)
    assert np.allclose(P.gelu_grad(z), fd, atol=1e-9)
    assert abs(P.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-15


def test_closed_form_network():
    p = np.zeros(P.NPARAM)
    Q = P.unpack(p)
    Q["b4"][:] = [1.5, -2.0]                      # all weights zero: output = b4
    X = np.random.default_rng(0).standard_normal((5, P.NIN))
    y, _ = P.forward(p, X)
    assert np.allclose(y, [[1.5, -2.0]] * 5, atol=0)
    # one path: x_0 -> unit 0 of every layer -> output 0, each GELU on a
    # positive input 3: y0 = GELU(GELU(GELU(3 x0)))
    Q["W1"][0, 0] = 3.0
    Q["W2"][0, 0] = 1.0
    Q["W3"][0, 0] = 1.0
    Q["W4"][0, 0] = 1.0
    Q["b4"][:] = 0.0
    X = np.zeros((1, P.NIN))
    X[0, 0] = 1.0
    phi = lambda v: 0.5 * v * (1.0 + math.erf(v / math.sqrt(2.0)))
    y, _ = P.forward(p, X)
    assert abs(y[0, 0] - phi(phi(phi(3.0)))) < 1e-15 and y[0, 1] == 0.0


def test_loss_closed_form():
    y = np.array([[1.0, 2.0], [0.0, 0.5]])
    t = np.array([2.0, 1.0])
    # sample 0: (1-2)^2 + rho(0) = 1; sample 1: (0-1)^2 + rho(0.5) = 1 + 0.45
    assert abs(P.loss(y, t) - (1.0 + 1.45) / 2) < 1e-15
    # u < 0: rho(u) = (tau - 1) u = 0.1 |u|
    assert abs(P.loss(np.array([[3.0, 5.0]]), np.array([3.0])) - 0.2) < 1e-15


@pytest.mark.parametrize("block", ["W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"])
def test_gradient_central_differences(block):
    rng = np.random.default_rng(7)
    p = rng.standard_normal(P.NPARAM) * 0.1
    X = rng.standard_normal((6, P.NIN))
    y0, _ = P.forward(p, X)
    # targets away from the quantile head's kink (u = t - y1 = 0)
    t = y0[:, 1] + np.where(rng.random(6) < 0.5, 0.7, -0.7)
    _, g = P.grad(p, X, t)
    off = 0
    for name, shp in P.SHAPES:
        cnt = int(np.prod(shp))
        if name == block:
            break
        off += cnt
    idx = off + rng.choice(cnt, size=min(cnt, 12), replace=False)
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (P.loss(P.forward(pp, X)[0], t) - P.loss(P.forward(pm, X)[0], t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-6 * abs(fd), (name, i, fd, g[i])


def test_adam_first_step_closed_form():
    # first step: mhat = g, vhat = g^2, so p1 = p0 - lr g / (|g| + eps)
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    p1, m, v = P.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    # second step with the same gradient: mhat = g, vhat = g^2 again
    p2, _, _ = P.adam_step(p1, g, m, v, 2, lr=0.01)
    assert np.allclose(p2, p1 - 0.01 * g / (np.abs(g) + 1e-8), atol=1e-15)


def test_features_geometric():
    d = 10.0 ** (-0.25 * np.arange(64))           # log10(d_c / d_0) = -c/4
    x = P.features(d * 7.0, 4096, 1024, 7e-3)     # eps / d_0 = 1e-3
    assert np.allclose(x[:64], np.maximum(-0.25 * np.arange(64), -16.0) / 16.0, atol=1e-14)
    assert x[64] == 12 / 16 and x[65] == 10 / 16 and abs(x[66] + 3 / 16) < 1e-15
    d2 = 10.0 ** (-1.0 * np.arange(64))           # clamped after 16 decades
    x2 = P.features(d2, 512, 512, 1e-30)
    assert x2[20] == -1.0 and abs(x2[10] + 10 / 16) < 1e-14 and x2[66] == -1.0
    assert P.features(np.zeros(64), 8, 8, 0.5)[0] == -1.0


def test_predicted_width():
    assert P.predicted_width(math.log(1 + 100.0), 32, 0.1) == 128   # 111 -> 4 blocks
    assert P.predicted_width(math.log(1 + 0.0), 32, 0.1) == 32
    assert P.predicted_width(-5.0, 16, 0.0) == 16
