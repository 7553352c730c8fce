"""Pins of the proposal-network oracle: finite differences, closed forms,
published update rules and sampling statistics."""
import math

import numpy as np
import pytest
import scipy.stats

from oracle import mlp_oracle as M


def _rand_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    parts = []
    for k, n in M.LAYERS:
        parts.append(rng.uniform(-1, 1, size=k * n) * scale / math.sqrt(k))
        parts.append(rng.uniform(-0.1, 0.1, size=n))
    return np.concatenate(parts)


def test_param_count():
    assert M.param_count() == 154_448


def test_gelu_values_and_derivative():
    assert M.gelu(np.array(0.0)) == 0.0
    assert abs(M.gelu(np.array(10.0)) - 10.0) < 1e-12
    assert abs(M.gelu(np.array(-10.0))) < 1e-12
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(M.gelu_grad(z), fd, rtol=0, atol=1e-8)
    # tanh form at 1: 0.5 (1 + tanh(sqrt(2/pi) * 1.044715))
    assert abs(M.gelu(np.array(1.0)) - 0.5 * (1 + math.tanh(math.sqrt(2 / math.pi) * 1.044715))) < 1e-15


def test_single_component_mixture_is_gaussian():
    rng = np.random.default_rng(1)
    B = 50
    mu = rng.uniform(-0.5, 0.5, size=(B, 2))
    ls = rng.uniform(-2, 0, size=(B, 2))
    Y = np.zeros((B, M.N_COMP, 5))
    Y[:, :, 0] = 3.7                      # equal logits, identical components
    Y[:, :, 1:3] = mu[:, None, :]
    Y[:, :, 3:5] = ls[:, None, :]
    T = rng.uniform(-1, 1, size=(B, 2))
    nll, _ = M.mdn_nll(Y.reshape(B, -1), T)
    ref = np.sum(0.5 * ((T - mu) / np.exp(ls)) ** 2 + ls + 0.5 * math.log(2 * math.pi), axis=1)
    np.testing.assert_allclose(nll, ref, rtol=1e-12, atol=1e-12)


def test_mdn_gradient_and_clamp_by_finite_differences():
    rng = np.random.default_rng(2)
    B = 7
    Y = rng.normal(size=(B, M.N_OUT))
    Y.reshape(B, M.N_COMP, 5)[:, 3, 3] = -9.0    # clamped low: zero gradient
    Y.reshape(B, M.N_COMP, 5)[:, 5, 4] = 3.0     # clamped high: zero gradient
    T = rng.uniform(-1, 1, size=(B, 2))
    _, G = M.mdn_nll(Y, T)
    h = 1e-6
    for idx in rng.choice(B * M.N_OUT, size=60, replace=False):
        Yp, Ym = Y.copy().ravel(), Y.copy().ravel()
        Yp[idx] += h
        Ym[idx] -= h
        fd = (M.mdn_nll(Yp.reshape(B, -1), T)[0].sum() - M.mdn_nll(Ym.reshape(B, -1), T)[0].sum()) / (2 * h)
        assert abs(G.ravel()[idx] - fd) < 1e-6 * max(1.0, abs(fd)), idx
    assert np.all(G.reshape(B, M.N_COMP, 5)[:, 3, 3] == 0) and np.all(G.reshape(B, M.N_COMP, 5)[:, 5, 4] == 0)


def test_network_gradient_by_finite_differences():
    rng = np.random.default_rng(3)
    w = _rand_params(4)
    B = 5
    X = rng.normal(size=(B, M.N_IN))
    mean, std = rng.normal(size=M.N_IN) * 0.1, rng.uniform(0.5, 2, size=M.N_IN)
    T = rng.uniform(-1, 1, size=(B, 2))
    L0, g = M.loss_and_grad(w, X, T, mean, std)
    offs = np.cumsum([0] + [k * n + n for k, n in M.LAYERS])
    idxs = np.concatenate([rng.integers(offs[i], offs[i + 1], size=12) for i in range(4)])
    h = 1e-6
    for i in idxs:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (M.loss_and_grad(wp, X, T, mean, std)[0] - M.loss_and_grad(wm, X, T, mean, std)[0]) / (2 * h)
        assert abs(g[i] - fd) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (i, g[i], fd)


def test_adam_first_step_closed_form():
    g = np.array([0.3, -2.0, 1e-9, 0.0])
    w0 = np.array([1.0, 2.0, 3.0, 4.0])
    w1, m, v = M.adam_step(w0, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    np.testing.assert_allclose(w1, w0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_forward_hand_evaluated_sparse_network():
    """A network with one path through it, evaluated by hand.  Input 0 is 5 with
    mean 1 and standard deviation 2, so the standardised input is (5 - 1) / 2 = 2;
    W1[0, 0] = 1 gives z1 = 2; W2[0, 3] = 0.5 gives z2 = 0.5 gelu(2); W3[3, 7] = 2
    and b3[7] = 0.25 give z3 = 2 gelu(z2) + 0.25; W4[7, 11] = -1 and b4[11] = 0.1
    give y11 = 0.1 - gelu(z3).  Every other output is its bias; other inputs
    (standardised with their own mean and deviation) reach nothing."""
    def g(z):  # tanh-form GELU, written out from its definition
        return 0.5 * z * (1.0 + math.tanh(math.sqrt(2.0 / math.pi) * (z + 0.044715 * z ** 3)))

    flat = np.zeros(M.param_count())
    offs = np.cumsum([0] + [k * n + n for k, n in M.LAYERS])

    def w(layer, i, j, v):
        k, n = M.LAYERS[layer]
        flat[offs[layer] + i * n + j] = v

    def b(layer, j, v):
        k, n = M.LAYERS[layer]
        flat[offs[layer] + k * n + j] = v

    w(0, 0, 0, 1.0)
    w(1, 0, 3, 0.5)
    w(2, 3, 7, 2.0)
    b(2, 7, 0.25)
    w(3, 7, 11, -1.0)
    b(3, 11, 0.1)
    b(3, 40, -0.7)
    X = np.array([[5.0, 3.0, -2.0, 0.5, 0.0, 1.0, 2.0, -1.0]])
    mean = np.array([1.0, 0.5, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0])
    std = np.array([2.0, 4.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0])
    Y, _ = M.forward(flat, X, mean, std)
    expect = np.zeros(M.N_OUT)
    expect[11] = 0.1 - g(2.0 * g(0.5 * g(2.0)) + 0.25)
    expect[40] = -0.7
    np.testing.assert_allclose(Y[0], expect, rtol=0, atol=1e-15)


def test_adam_constant_gradient_is_bias_free():
    """Under a constant gradient g the bias-corrected moments are exactly g and
    g^2 at every step (Kingma & Ba 2015, Sec. 3: the correction removes the
    zero-initialisation bias), so each step moves w by lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 5.0])
    w0 = np.array([1.0, 2.0, 3.0, 4.0])
    w, m, v = w0.copy(), np.zeros(4), np.zeros(4)
    lr = 0.01
    for step in range(1, 6):
        w, m, v = M.adam_step(w, g, m, v, step, lr=lr)
        np.testing.assert_allclose(w, w0 - step * lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)
        np.testing.assert_allclose(m, (1.0 - 0.9 ** step) * g, rtol=1e-13)
        np.testing.assert_allclose(v, (1.0 - 0.999 ** step) * g * g, rtol=1e-12)


def test_sampler_statistics():
    Y = np.zeros((M.N_COMP, 5))
    Y[:, 0] = -30.0
    Y[7] = [10.0, 0.2, -0.3, math.log(0.1), math.log(0.05)]
    lo, hi = np.array([-0.4, -3.0]), np.array([0.4, 3.0])
    u, k = M.sample(Y.ravel(), 20000, seed=9, tick=3, loop=1, u_lo=lo, u_hi=hi)
    assert np.all(k == 7)
    un = (u - 0.5 * (lo + hi)) / (0.5 * (hi - lo))
    z0 = (un[:, 0] - 0.2) / 0.1
    z1 = (un[:, 1] + 0.3) / 0.05
    assert scipy.stats.kstest(z0, "norm").pvalue > 1e-3
    assert scipy.stats.kstest(z1, "norm").pvalue > 1e-3
    assert abs(np.corrcoef(z0, z1)[0, 1]) < 0.03


def test_sampler_component_frequencies():
    Y = np.zeros((M.N_COMP, 5))
    logits = np.linspace(-1, 1, M.N_COMP)
    Y[:, 0] = logits
    Y[:, 3:5] = -3.0
    u, k = M.sample(Y.ravel(), 40000, seed=1, tick=0, loop=0, u_lo=[-1, -1], u_hi=[1, 1])
    w = np.exp(logits) / np.exp(logits).sum()
    counts = np.bincount(k, minlength=M.N_COMP)
    chi = scipy.stats.chisquare(counts, w * counts.sum())
    assert chi.pvalue > 1e-3
    assert np.all(np.abs(u) <= 1.0)
