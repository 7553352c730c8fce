"""FP64 oracle of the learned proposal network (test infrastructure only).

TEST INFRASTRUCTURE ONLY: imported by the test suite and the cpu_baseline leg
of bench.py, never by the GPU product path; imports nothing from it.

The network proposes candidate inputs near the safe minimal-intervention
input, so that a tick can evaluate a few thousand proposals instead of an
exhaustive grid (the exhaustive sampler of Sec. IV-B stays the fallback).  Its
shape is fixed: 8 inputs (state and user input, standardised), three hidden
layers of 256 with GELU, 80 outputs read as a 16-component mixture of
diagonal Gaussians over the normalised input (logit, two means, two
log-standard-deviations per component).

Readings (none of this is in the paper): GELU in its tanh form; log sigma
clamped to [-7, 2]; targets are the chosen input mapped to [-1, 1] per
dimension; the loss is the mean mixture negative log-likelihood; Adam with
bias correction.
"""
from __future__ import annotations

import math

import numpy as np

from .mpmi_oracle import hash_counter

N_IN, N_HID, N_COMP = 8, 256, 16
N_OUT = 5 * N_COMP
LAYERS = [(N_IN, N_HID), (N_HID, N_HID), (N_HID, N_HID), (N_HID, N_OUT)]
LOGSIG_MIN, LOGSIG_MAX = -7.0, 2.0
GELU_C = math.sqrt(2.0 / math.pi)
GELU_A = 0.044715
LOG_2PI = math.log(2.0 * math.pi)


def param_count() -> int:
    return sum(k * n + n for k, n in LAYERS)


def unpack(flat: np.ndarray):
    """Flat parameter vector -> [(W (k, n), b (n,)), ...] in layer order (W row-major, then b)."""
    out, o = [], 0
    for k, n in LAYERS:
        W = flat[o:o + k * n].reshape(k, n)
        o += k * n
        b = flat[o:o + n]
        o += n
        out.append((W, b))
    return out


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(GELU_C * (z + GELU_A * z ** 3)))


def gelu_grad(z):
    t = np.tanh(GELU_C * (z + GELU_A * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * GELU_C * (1.0 + 3.0 * GELU_A * z * z)


def forward(flat, X, mean, std):
    """Returns (Y (B, 80), cache) for inputs X (B, 8); inputs standardised by (mean, std)."""
    p = unpack(np.asarray(flat, np.float64))
    h = (np.asarray(X, np.float64) - mean) / std
    cache = [h]
    for i, (W, b) in enumerate(p):
        z = h @ W + b
        if i < len(p) - 1:
            cache.append(z)
            h = gelu(z)
            cache.append(h)
        else:
            cache.append(z)
            h = z
    return h, cache


def split_head(Y):
    """Y (B, 80) -> logits (B, 16), mu (B, 16, 2), raw log sigma (B, 16, 2)."""
    Y = Y.reshape(-1, N_COMP, 5)
    return Y[:, :, 0], Y[:, :, 1:3], Y[:, :, 3:5]


def mdn_nll(Y, T):
    """Per-sample negative log-likelihood of targets T (B, 2) and dNLL/dY (B, 80)."""
    logit, mu, ls_raw = split_head(Y)
    ls = np.clip(ls_raw, LOGSIG_MIN, LOGSIG_MAX)
    inside = (ls_raw > LOGSIG_MIN) & (ls_raw < LOGSIG_MAX)
    sig = np.exp(ls)
    d = (T[:, None, :] - mu) / sig                       # (B, K, 2)
    logN = -np.sum(0.5 * d * d + ls + 0.5 * LOG_2PI, axis=2)
    m = np.max(logit, axis=1, keepdims=True)
    logpi = logit - m - np.log(np.sum(np.exp(logit - m), axis=1, keepdims=True))
    a = logpi + logN
    am = np.max(a, axis=1, keepdims=True)
    lse = am[:, 0] + np.log(np.sum(np.exp(a - am), axis=1))
    nll = -lse
    gamma = np.exp(a - lse[:, None])                     # responsibilities
    pi = np.exp(logpi)
    g_logit = pi - gamma
    g_mu = -gamma[:, :, None] * d / sig
    g_ls = gamma[:, :, None] * (1.0 - d * d) * inside
    G = np.concatenate([g_logit[:, :, None], g_mu, g_ls], axis=2).reshape(-1, N_OUT)
    return nll, G


def loss_and_grad(flat, X, T, mean, std):
    """Mean NLL over the batch and its gradient with respect to the flat parameters."""
    p = unpack(np.asarray(flat, np.float64))
    Y, cache = forward(flat, X, mean, std)
    nll, G = mdn_nll(Y, np.asarray(T, np.float64))
    B = X.shape[0]
    dz = G / B
    grads = []
    # cache = [h0, z1, h1, z2, h2, z3, h3, z4]
    for i in range(len(p) - 1, -1, -1):
        W, _ = p[i]
        h_prev = cache[2 * i]
        gW = h_prev.T @ dz
        gb = dz.sum(axis=0)
        grads.append((gW, gb))
        if i > 0:
            dh = dz @ W.T
            dz = dh * gelu_grad(cache[2 * i - 1])
    grads.reverse()
    flat_g = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return float(nll.mean()), flat_g


def adam_step(w, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; step counts from 1."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def sample(Y_row, P, seed, tick, loop, u_lo, u_hi):
    """P proposals from one mixture head Y_row (80,), as an array (P, 2) of FP32 numbers.

    Proposal p draws three counter-based uniforms (slots 0, 1, 2 of
    hash(seed, tick, loop, p, slot)): r0 picks the component whose cumulative
    mixture weight first exceeds it (weights computed in FP32), r1 in (0, 1]
    and r2 in [0, 1) give two standard normals by the Box-Muller transform;
    the normalised draw mu + sigma z is clipped to [-1, 1] and mapped to the
    input box.
    """
    logit, mu, ls_raw = split_head(np.asarray(Y_row, np.float64)[None])
    logit32 = logit[0].astype(np.float32)
    e = np.exp((logit32 - logit32.max()).astype(np.float32)).astype(np.float32)
    cdf = np.cumsum(e, dtype=np.float32)
    cdf = (cdf / cdf[-1]).astype(np.float32)
    p = np.arange(P, dtype=np.uint64)
    bits = [hash_counter(np.uint64(seed), np.uint64(tick), np.uint64(loop), p, np.uint64(s)) for s in range(3)]
    r0 = ((bits[0] >> np.uint64(40)).astype(np.float64) * 2.0 ** -24).astype(np.float32)
    r1 = ((bits[1] >> np.uint64(40)).astype(np.float64) + 1.0) * 2.0 ** -24
    r2 = (bits[2] >> np.uint64(40)).astype(np.float64) * 2.0 ** -24
    k = np.minimum(np.sum(cdf[None, :] <= r0[:, None], axis=1), N_COMP - 1)
    rad = np.sqrt(-2.0 * np.log(r1))
    z = np.stack([rad * np.cos(2.0 * math.pi * r2), rad * np.sin(2.0 * math.pi * r2)], axis=1)
    sig = np.exp(np.clip(ls_raw[0], LOGSIG_MIN, LOGSIG_MAX))
    un = np.clip(mu[0][k] + sig[k] * z, -1.0, 1.0)
    lo, hi = np.asarray(u_lo, np.float64), np.asarray(u_hi, np.float64)
    u = 0.5 * (lo + hi) + 0.5 * (hi - lo) * un
    return u.astype(np.float32).astype(np.float64), k
