"""Learned proposal for the race car: labels, training and serving.

* Labels: for random (state, user input) pairs, the minimal-intervention input
  u* chosen by the exhaustive tick over a 256 x 256 grid with H = 60 (the
  method itself generates its training data).  Pairs are served 4,096 at a
  time as loops of one many-loop launch.
* Training: mini-batch Adam on the mean mixture negative log-likelihood of u*
  (mapped to [-1, 1]^2), every step in the library's kernels (mlp_grad +
  mlp_adam); host code only orders the batches.
* Serving: mpmi_proposal_tick -- network, 2,048 proposals, fused tick over
  them plus the user's input, exhaustive fallback when nothing is safe.

Every computation runs in libmpmi; this module moves tensors and keeps state.
"""
from __future__ import annotations

import os
import time

import numpy as np
import torch

from . import mpmi

ASSET = os.path.join(os.path.dirname(os.path.abspath(__file__)), "assets", "proposal_net.npz")


class ProposalNet:
    """Parameters (FP32 master + BF16 copy), Adam state and input standardisation, on the device."""

    def __init__(self, ctx: mpmi.Context, flat: np.ndarray, mean: np.ndarray, std: np.ndarray, step: int = 0,
                 m: np.ndarray | None = None, v: np.ndarray | None = None):
        dev = ctx.device
        self.ctx = ctx
        self.w32 = torch.tensor(np.asarray(flat, np.float32), device=dev)
        self.w16 = self.w32.to(torch.bfloat16)
        self.m = torch.zeros_like(self.w32) if m is None else torch.tensor(np.asarray(m, np.float32), device=dev)
        self.v = torch.zeros_like(self.w32) if v is None else torch.tensor(np.asarray(v, np.float32), device=dev)
        self.mean = torch.tensor(np.asarray(mean, np.float32), device=dev)
        self.std = torch.tensor(np.asarray(std, np.float32), device=dev)
        self.step = step

    def tensors(self) -> dict:
        return dict(w16=self.w16, w32=self.w32, mean=self.mean, std=self.std)

    def save(self, path: str, with_adam: bool = False):
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        extra = dict(m=self.m.cpu().numpy(), v=self.v.cpu().numpy()) if with_adam else {}
        np.savez(path, flat=self.w32.cpu().numpy(), mean=self.mean.cpu().numpy(), std=self.std.cpu().numpy(),
                 step=np.array(self.step), **extra)

    @classmethod
    def load(cls, ctx: mpmi.Context, path: str = ASSET) -> "ProposalNet":
        z = np.load(path, allow_pickle=False)
        return cls(ctx, z["flat"], z["mean"], z["std"], int(z["step"]),
                   z["m"] if "m" in z.files else None, z["v"] if "v" in z.files else None)


def normalise(u: np.ndarray, lo, hi) -> np.ndarray:
    lo, hi = np.asarray(lo, np.float64), np.asarray(hi, np.float64)
    return (np.asarray(u, np.float64) - 0.5 * (lo + hi)) / (0.5 * (hi - lo))


def generate_labels(ctx: mpmi.Context, model: mpmi.Model, states: np.ndarray, users: np.ndarray,
                    grid=(256, 256), horizon: int = 60, chunk: int = 4096, log=None, precision: int = mpmi.PREC_FP32,
                    with_index: bool = False):
    """u* (n, 2), status (n,) and n_safe (n,) for every (state, user input) pair,
    from exhaustive ticks served as the loops of one many-loop launch (and the
    chosen candidate's index (n,) with with_index)."""
    n = states.shape[0]
    chunk = min(chunk, n, mpmi.MAX_LOOPS)
    dev = ctx.device
    xb = torch.zeros((chunk, 6), dtype=torch.float32, device=dev)
    ub = torch.zeros((chunk, 2), dtype=torch.float32, device=dev)
    ob = torch.zeros((chunk, mpmi.SELECTION_BYTES), dtype=torch.uint8, device=dev)
    N = int(grid[0] * grid[1])
    loops = [dict(model=model, x_t=xb[i], u_user=ub[i], out=ob[i], n_cand=N, horizon=horizon,
                  gen=mpmi.GEN_GRID, grid=list(grid)) for i in range(chunk)]
    multi = mpmi.Multi(ctx, loops, block=256, precision=precision)
    u_star = np.zeros((n, 2))
    status = np.zeros(n, np.int32)
    n_safe = np.zeros(n, np.int64)
    idx = np.zeros(n, np.int64)
    t0 = time.perf_counter()
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        k = e - s
        xb[:k] = torch.tensor(states[s:e], dtype=torch.float32, device=dev)
        ub[:k] = torch.tensor(users[s:e], dtype=torch.float32, device=dev)
        if k < chunk:  # pad the last chunk with the first pair (results discarded)
            xb[k:] = xb[0]
            ub[k:] = ub[0]
        multi.tick()
        rec = ob.cpu().numpy()
        raw = rec.view(np.int32).reshape(chunk, -1)
        flt = rec.view(np.float32).reshape(chunk, -1)
        idx[s:e] = raw[:k, 0]
        status[s:e] = raw[:k, 1]
        n_safe[s:e] = raw[:k, 2]
        u_star[s:e] = flt[:k, 4:6]
        if log and (s // chunk) % 32 == 0:
            log(f"labels {e}/{n} ({time.perf_counter() - t0:.1f} s)")
    multi.close()
    return (u_star, status, n_safe, idx) if with_index else (u_star, status, n_safe)


def train(ctx: mpmi.Context, net: ProposalNet, X: np.ndarray, T: np.ndarray, epochs: int, batch: int = 4096,
          lr: float = 1e-3, seed: int = 6, log=None):
    """Mini-batch Adam over (X, T); returns the mean loss of every epoch."""
    dev = ctx.device
    Xd = torch.tensor(np.asarray(X, np.float32), device=dev)
    Td = torch.tensor(np.asarray(T, np.float32), device=dev)
    n = Xd.shape[0]
    work = mpmi.mlp_workspace(ctx, batch)
    grad = torch.empty(mpmi.MLP_PARAMS, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    rng = np.random.default_rng(seed)
    losses = []
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(n), device=dev)
        acc = torch.zeros(1, dtype=torch.float32, device=dev)
        nb = n // batch
        for b in range(nb):
            idx = perm[b * batch:(b + 1) * batch]
            xb = Xd.index_select(0, idx).contiguous()
            tb = Td.index_select(0, idx).contiguous()
            mpmi.mlp_grad(ctx, net.w16, net.w32, net.mean, net.std, xb, tb, work=work, grad=grad, loss=loss)
            net.step += 1
            mpmi.mlp_adam(ctx, net.w32, net.w16, net.m, net.v, grad, net.step, lr)
            acc += loss
        losses.append(float(acc.item()) / max(1, nb))
        if log:
            log(f"epoch {ep + 1}/{epochs}: mean NLL {losses[-1]:.4f}")
    return losses


class LearnedTicker:
    """Serves learned-proposal ticks for one race-car model."""

    def __init__(self, ctx: mpmi.Context, model: mpmi.Model, net: ProposalNet, proposals: int = 2048,
                 horizon: int = 60, fallback_grid=(128, 128), seed: int = 8, loop: int = 1, fallback_loop: int = 2,
                 lanes_per_cand: int = 1, block: int = 0, precision: int = mpmi.PREC_FP32):
        self.ctx, self.model, self.net = ctx, model, net
        self.P, self.H = proposals, horizon
        self.lanes, self.block = lanes_per_cand, block
        self.precision = precision
        self.fallback = mpmi.tick_desc(int(fallback_grid[0] * fallback_grid[1]), horizon, gen=mpmi.GEN_GRID,
                                       grid=list(fallback_grid), loop=fallback_loop, precision=precision)
        self.seed, self.loop = seed, loop
        self.cand = torch.empty((1, 2, proposals), dtype=torch.float32, device=ctx.device)
        self.head = torch.empty(mpmi.MLP_OUT, dtype=torch.float32, device=ctx.device)
        self.work = mpmi.mlp_workspace(ctx, 1)

    def tick(self, x_t, u_user, tick: int, out=None, stream=None):
        prop = mpmi.tick_desc(self.P, self.H, gen=mpmi.GEN_EXPLICIT, seed=self.seed, tick=tick, loop=self.loop,
                              precision=self.precision)
        prop.lanes_per_cand, prop.block = self.lanes, self.block
        return mpmi.mpmi_proposal_tick(self.ctx, self.model, self.net.tensors(), x_t, u_user, prop, self.fallback,
                                       self.cand, self.work, out=out, head_out=self.head, stream=stream)
