"""FP64 CPU oracle for the minimal-intervention shared-control hot path.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously correct
definition that the GPU library is checked against.  Only the test suite,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it; the GPU product path never does, and this module imports nothing
from the GPU package.

It follows Algorithm 2 (MPMI-SC, Sec. IV-C) step by step, in FP64 NumPy:

* candidates: N samples of the input box (equally spaced grid, Sec. IV-B, or
  uniform draws, Alg. 2 first step); candidate 0 is the user's own input,
  which Alg. 1's pass-through rule (Sec. III-D) requires to be returned
  whenever it is safe;
* prediction: x_p <- f(x_p, xi(i)), f being the learned Koopman model
  (Sec. IV-A): lift (x, u) through the basis psi, multiply by K, keep the
  state columns;
* predictive safety (Sec. IV-B, inflated barrier of Sec. V-C-1): every
  predicted state is checked and the rollout stops at the first violation;
* selection: the safe candidate of least cost, cost = distance to the user's
  input (Alg. 2 selection step; Euclidean per Sec. IV-D).

Readings where the paper is silent (each listed in the design notes):
horizon = H integer steps, states x_1..x_H are checked; candidate inputs are
held over the horizon or piecewise constant over S equal segments; cost is the
squared Euclidean distance after dividing input j by its half-range, taken on
the first segment; ties go to the lowest index; when nothing is safe the
candidate with the latest first violation (then least cost, then lowest index)
is returned with status NO_SAFE; process noise (Alg. 2's z_i) is Gaussian with
a per-component standard deviation, zero unless a system states one, drawn
from the counter generator through Box-Muller; the fit is least squares on
RMS-scaled columns (EDMD, Sec. IV-A's Koopman citation).

Every function here is pinned by a test of tests/test_oracle_pins.py against
something other than this module: basis values written out by hand; the
linear plant's closed form (fit, rollout with and without noise, selection
interval); brute-force enumeration; published SplitMix64 vectors; hand-derived
uniform draws, grid points and track margins (nonzero phases included);
library least squares and the residual's orthogonality; the Sec. IV-D
printed values; zero intervention and mask monotonicity.  The basis
selection (selection_problem, group_shrink, sparse_admm, select_basis) is
pinned in tests/test_selection_pins.py: hand-computed shrinkage, the
closed-form solution of an orthonormal design, the optimality conditions of
the convex problem, the least-squares limit, the zero solution above the
critical penalty, and a planted support with its polished coefficients.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

STATUS_OK = 0
STATUS_NO_SAFE = 1

# ----------------------------------------------------------------------------
# Systems: basis family + safety set + input box
# ----------------------------------------------------------------------------
@dataclass
class System:
    """What the oracle needs to know about one controlled system.

    kind        'linear' (psi = [x; u]), 'balance_bot' or 'race_car'
    n, m        state and input dimensions
    box         list of (state index, bound, inflation): |x[idx]| < bound - inflation
    track       None, or dict(r0, half, amp[4], freq[4], phase[4], infl): the
                radial gap |rho - r_c(phi)| < half - infl, with rho, phi the
                polar coordinates of (x[0], x[1])
    u_lo, u_hi  input box (FP32 numbers)
    noise       per-component standard deviations of the process noise added
                to every predicted state (Alg. 2's z_i), or None
    """

    kind: str
    n: int
    m: int
    box: list = field(default_factory=list)
    track: Optional[dict] = None
    u_lo: np.ndarray = None
    u_hi: np.ndarray = None
    noise: Optional[np.ndarray] = None

    def __post_init__(self):
        self.u_lo = np.asarray(np.float32(self.u_lo), np.float64).reshape(-1)
        self.u_hi = np.asarray(np.float32(self.u_hi), np.float64).reshape(-1)

    @property
    def dim(self) -> int:
        return basis_dim(self.kind, self.n, self.m)

    @property
    def half_range(self) -> np.ndarray:
        return 0.5 * (self.u_hi - self.u_lo)


@dataclass(frozen=True)
class Basis:
    """A basis given as data (Sec. IV-A: the functions of state the Koopman
    operator acts on, here chosen by the caller): atoms are (kind, k) with
    kind 'one', 'var', 'sin' or 'cos' of component k of w = [x; u]; feature f
    is the product of atoms feats[f][0] and feats[f][1]."""

    atoms: tuple
    feats: tuple

    def atom_values(self, W: np.ndarray) -> list:
        out = []
        for kind, k in self.atoms:
            if kind == "one":
                out.append(np.ones(W.shape[0]))
            elif kind == "var":
                out.append(W[:, k])
            elif kind == "sin":
                out.append(np.sin(W[:, k]))
            elif kind == "cos":
                out.append(np.cos(W[:, k]))
            else:
                raise ValueError(kind)
        return out

    def lift(self, W: np.ndarray) -> np.ndarray:
        at = self.atom_values(W)
        return np.stack([at[a] * at[b] for a, b in self.feats], axis=1)


def basis_dim(kind, n: int, m: int) -> int:
    if isinstance(kind, Basis):
        return len(kind.feats)
    if kind == "linear":
        return n + m
    if kind == "balance_bot":
        return 21
    if kind == "race_car":
        return 64
    raise ValueError(kind)


# ----------------------------------------------------------------------------
# Basis psi(x, u)  (Sec. IV-A: the Koopman operator acts on functions of the
# state; here the functions are fixed families written out explicitly)
# ----------------------------------------------------------------------------
def lift(kind: str, X: np.ndarray, U: np.ndarray) -> np.ndarray:
    """Rows psi(x_t, u_t) for rows of X (T, n) and U (T, m); returns (T, D)."""
    X = np.asarray(X, np.float64)
    U = np.asarray(U, np.float64)
    if X.ndim == 1:
        X = X[None]
    if U.ndim == 1:
        U = U[None]
    W = np.concatenate([X, U], axis=1)  # w = [x; u]
    T = W.shape[0]
    if isinstance(kind, Basis):
        return kind.lift(W)
    if kind == "linear":
        return W.copy()
    if kind == "balance_bot":
        # [1, w_0..w_4, w_k*w_l for 0 <= k <= l <= 4 in row order]
        cols = [np.ones(T)]
        cols += [W[:, k] for k in range(5)]
        for k in range(5):
            for l in range(k, 5):
                cols.append(W[:, k] * W[:, l])
        return np.stack(cols, axis=1)
    if kind == "race_car":
        # w = [x, y, psi, vx, vy, r, delta, a]
        x, y, psi, vx, vy, r, delta, a = (W[:, k] for k in range(8))
        sp, cp = np.sin(psi), np.cos(psi)
        sd, cd = np.sin(delta), np.cos(delta)
        cols = [np.ones(T)]
        cols += [W[:, k] for k in range(8)]
        for k in range(8):
            for l in range(k, 8):
                cols.append(W[:, k] * W[:, l])
        cols += [sp, cp, sd, cd]
        cols += [sp * vx, sp * vy, sp * r, sp * a]
        cols += [cp * vx, cp * vy, cp * r, cp * a]
        cols += [sd * vx, sd * vy, sd * r]
        cols += [cd * vx, cd * vy, cd * r]
        cols += [a * sd]
        return np.stack(cols, axis=1)
    raise ValueError(kind)


# ----------------------------------------------------------------------------
# Fit (Sec. IV-A: K learned from data; EDMD least squares)
# ----------------------------------------------------------------------------
def fit(kind: str, X, U, Y, ridge: float = 0.0):
    """K_x = argmin ||Psi K - Y||_F (+ ridge ||scaled K||^2), returned as (D, n).

    Columns of Psi are divided by their RMS before solving; K is scaled back.
    Returns (K, info) with info = dict(cond, resid_rms, scale).
    """
    Psi = lift(kind, X, U)
    Y = np.asarray(Y, np.float64)
    scale = np.sqrt(np.mean(Psi * Psi, axis=0))
    scale[scale == 0.0] = 1.0
    Ps = Psi / scale
    A, B = Ps, Y
    if ridge > 0.0:
        D = Ps.shape[1]
        A = np.vstack([Ps, np.sqrt(ridge) * np.eye(D)])
        B = np.vstack([Y, np.zeros((D, Y.shape[1]))])
    Ks, _, _, sv = np.linalg.lstsq(A, B, rcond=None)
    K = Ks / scale[:, None]
    resid = Y - Psi @ K
    info = dict(cond=float(sv[0] / sv[-1]) if sv[-1] > 0 else np.inf,
                resid_rms=np.sqrt(np.mean(resid * resid, axis=0)), scale=scale)
    return K, info


def predict(kind: str, K: np.ndarray, X, U) -> np.ndarray:
    """One prediction step f(x, u) = psi(x, u)^T K for each row."""
    return lift(kind, X, U) @ K


def state_columns(kind: str, n: int) -> np.ndarray:
    """Features of psi that are the state components themselves (psi holds w
    = [x; u] linearly): linear -> 0..n-1, balance bot and race car -> 1..n
    (after the constant feature)."""
    if isinstance(kind, Basis):
        # the features that are w_j itself (VAR j times ONE, either order)
        cols = []
        for j in range(n):
            hit = [f for f, (a, b) in enumerate(kind.feats)
                   if {kind.atoms[a], kind.atoms[b]} in ({("var", j), ("one", 0)},)
                   or (kind.atoms[a] == ("var", j) and kind.atoms[b][0] == "one")
                   or (kind.atoms[b] == ("var", j) and kind.atoms[a][0] == "one")]
            if not hit:
                raise ValueError(f"the basis has no feature equal to x_{j}")
            cols.append(hit[0])
        return np.array(cols)
    first = 0 if kind == "linear" else 1
    return np.arange(first, first + n)


def fit_lifted(kind: str, X, U, Y, ridge: float = 0.0):
    """The full lifted operator of Sec. IV-A's linear representation: K (D, D)
    with psi(x_{t+1}, u_t) ~ psi(x_t, u_t) K, in the least-squares sense on
    RMS-scaled columns, as fit() does for the state columns.  The input is
    held over the step, as a candidate's input is held over the horizon, so
    the lifted state z = psi(x, u) of a constant-input rollout advances by
    z <- z K (one matrix-vector product per step; a batch of candidates, one
    matrix-matrix product).  Returns (K, info) like fit()."""
    X, U, Y = (np.asarray(a, np.float64) for a in (X, U, Y))
    Psi = lift(kind, X, U)
    Target = lift(kind, Y, U)
    scale = np.sqrt(np.mean(Psi * Psi, axis=0))
    scale[scale == 0.0] = 1.0
    Ps = Psi / scale
    A, B = Ps, Target
    if ridge > 0.0:
        D = Ps.shape[1]
        A = np.vstack([Ps, np.sqrt(ridge) * np.eye(D)])
        B = np.vstack([Target, np.zeros((D, Target.shape[1]))])
    Ks, _, _, sv = np.linalg.lstsq(A, B, rcond=None)
    K = Ks / scale[:, None]
    resid = Target - Psi @ K
    info = dict(cond=float(sv[0] / sv[-1]) if sv[-1] > 0 else np.inf,
                resid_rms=np.sqrt(np.mean(resid * resid, axis=0)), scale=scale)
    return K, info


# ----------------------------------------------------------------------------
# Safety (Sec. IV-B "geometric safety checks", Sec. V-C-1 inflated barrier)
# ----------------------------------------------------------------------------
def centre_radius(track: dict, phi):
    return track["r0"] + sum(a * np.sin(f * phi + p)
                             for a, f, p in zip(track["amp"], track["freq"], track["phase"]))


def margins(sys: System, X: np.ndarray) -> np.ndarray:
    """Per-constraint margins (bound - inflation) - |g(x)| for rows of X, shape (T, C).

    Box constraints come first in the given order, then the track.  A state is
    safe iff every margin is > 0 (a NaN margin is not > 0).
    """
    X = np.atleast_2d(np.asarray(X, np.float64))
    out = []
    for idx, bound, infl in sys.box:
        out.append((bound - infl) - np.abs(X[:, idx]))
    if sys.track is not None:
        tr = sys.track
        with np.errstate(invalid="ignore"):
            rho = np.hypot(X[:, 0], X[:, 1])
            phi = np.arctan2(X[:, 1], X[:, 0])
            out.append((tr["half"] - tr["infl"]) - np.abs(rho - centre_radius(tr, phi)))
    if not out:
        return np.zeros((X.shape[0], 0))
    return np.stack(out, axis=1)


def is_safe(sys: System, X: np.ndarray) -> np.ndarray:
    with np.errstate(invalid="ignore"):
        return np.all(margins(sys, X) > 0.0, axis=1)


# ----------------------------------------------------------------------------
# Candidate inputs (Sec. IV-B; Alg. 2 sampling step)
# ----------------------------------------------------------------------------
_M64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15


def mix64(z):
    """SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014), on uint64 arrays."""
    z = np.asarray(z, np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def splitmix64_sequence(seed: int, count: int):
    """The plain SplitMix64 generator: state += gamma; output mix64(state)."""
    out = []
    s = seed & _M64
    for _ in range(count):
        s = (s + GOLDEN_GAMMA) & _M64
        out.append(int(mix64(np.uint64(s))))
    return out


def hash_counter(seed, tick, loop, index, slot):
    """Counter-based draw: h = seed; for each word w: h = mix64((h ^ w) + gamma)."""
    h = np.asarray(seed, np.uint64)
    with np.errstate(over="ignore"):
        for w in (tick, loop, index, slot):
            h = mix64((h ^ np.asarray(w, np.uint64)) + np.uint64(GOLDEN_GAMMA))
    return h


def unit_from_bits(h):
    """Top 24 bits of a 64-bit draw as a float in [0, 1) (exact in FP32)."""
    return (np.asarray(h, np.uint64) >> np.uint64(40)).astype(np.float64) * 2.0 ** -24


def _to_f32(v):
    return np.asarray(v, np.float64).astype(np.float32).astype(np.float64)


def grid_candidates(sys: System, grid) -> np.ndarray:
    """Cell-centred grid over the input box, as an array (N, m) of FP32 numbers.

    Grid index k = k_0 + G_0 (k_1 + G_1 (...)) (dimension 0 fastest); value of
    dimension j is lo_j + (k_j + 1/2) * ((hi_j - lo_j) / G_j), evaluated in
    FP64 in that order and rounded to FP32.
    """
    grid = [int(g) for g in grid]
    N = int(np.prod(grid))
    k = np.arange(N)
    cols = []
    for j, G in enumerate(grid):
        kj = k % G
        k = k // G
        step = (sys.u_hi[j] - sys.u_lo[j]) / G
        cols.append(_to_f32(sys.u_lo[j] + (kj + 0.5) * step))
    return np.stack(cols, axis=1)


def uniform_value(lo, hi, h):
    """The input value a 64-bit draw h stands for on [lo, hi): lo + (hi - lo) * r
    with r = unit_from_bits(h), in FP64, rounded to FP32."""
    return _to_f32(np.asarray(lo, np.float64) + (np.asarray(hi, np.float64) - np.asarray(lo, np.float64))
                   * unit_from_bits(h))


def uniform_candidates(sys: System, N: int, S: int, seed: int, tick: int, loop: int) -> np.ndarray:
    """N random candidates of S segments: array (N, S, m) of FP32 numbers.

    Candidate i (1-based), segment g, input j takes uniform_value(lo_j, hi_j,
    hash(seed, tick, loop, i, g*m + j)).
    """
    i = np.arange(1, N + 1, dtype=np.uint64)[:, None, None]
    g = np.arange(S, dtype=np.uint64)[None, :, None]
    j = np.arange(sys.m, dtype=np.uint64)[None, None, :]
    slot = g * np.uint64(sys.m) + j
    h = hash_counter(np.uint64(seed), np.uint64(tick), np.uint64(loop), i, slot)
    return uniform_value(sys.u_lo, sys.u_hi, h)


def with_user(cand: np.ndarray, u_h, S: int) -> np.ndarray:
    """Prepend candidate 0 = the user's input held over all S segments -> (N+1, S, m)."""
    cand = np.asarray(cand, np.float64)
    if cand.ndim == 2:
        cand = np.repeat(cand[:, None, :], S, axis=1)
    u0 = np.broadcast_to(np.asarray(u_h, np.float64).reshape(1, 1, -1), (1, S, cand.shape[2]))
    return np.concatenate([u0, cand], axis=0)


NOISE_SLOT = 65536


def process_noise(seed, tick, loop, idx, s: int, n: int) -> np.ndarray:
    """Standard normals (len(idx), n) for step s of candidates idx.

    Components 2q, 2q+1 come from one draw h = hash(seed, tick, loop, i,
    65536 + 4 (s - 1) + q): u1 = ((h >> 40) + 1) 2^-24, u2 = ((h >> 16) &
    0xFFFFFF) 2^-24, and the Box-Muller pair sqrt(-2 ln u1) (cos, sin)(2 pi u2).
    """
    idx = np.asarray(idx, np.uint64)
    out = np.zeros((idx.size, n))
    for q in range((n + 1) // 2):
        h = hash_counter(np.uint64(seed), np.uint64(tick), np.uint64(loop), idx,
                         np.uint64(NOISE_SLOT + 4 * (s - 1) + q))
        u1 = ((h >> np.uint64(40)).astype(np.float64) + 1.0) * 2.0 ** -24
        u2 = ((h >> np.uint64(16)) & np.uint64(0xFFFFFF)).astype(np.float64) * 2.0 ** -24
        r = np.sqrt(-2.0 * np.log(u1))
        out[:, 2 * q] = r * np.cos(2.0 * np.pi * u2)
        if 2 * q + 1 < n:
            out[:, 2 * q + 1] = r * np.sin(2.0 * np.pi * u2)
    return out


def segment_of_step(s: int, S: int, H: int) -> int:
    """Segment used at prediction step s (1..H): floor((s - 1) * S / H)."""
    return ((s - 1) * S) // H


# ----------------------------------------------------------------------------
# Prediction with early exit (Alg. 2 inner loop)
# ----------------------------------------------------------------------------
def rollout(sys: System, K: np.ndarray, x0, cand: np.ndarray, H: int, early_exit: bool = True,
            noise_key=None, index=None):
    """Roll every candidate forward H steps from x0.

    cand: (Nc, S, m).  Returns (traj, fv): traj (H, Nc, n) with NaN where a
    rollout had already stopped, and fv (Nc,) the first step (1..H) whose
    predicted state is unsafe, or H + 1 if every state was safe.  With
    early_exit=False every step is predicted (fv is unchanged).  If the system
    has process noise, noise_key = (seed, tick, loop) and index (candidate
    numbers of the rows, default 0..Nc-1) select the draws.
    """
    cand = np.asarray(cand, np.float64)
    Nc, S, _ = cand.shape
    K = np.asarray(K, np.float64)
    x = np.tile(np.asarray(x0, np.float64).reshape(1, -1), (Nc, 1))
    traj = np.full((H, Nc, sys.n), np.nan)
    fv = np.full(Nc, H + 1, dtype=np.int64)
    alive = np.ones(Nc, dtype=bool)
    for s in range(1, H + 1):
        g = segment_of_step(s, S, H)
        idx = np.nonzero(alive)[0] if early_exit else np.arange(Nc)
        if idx.size == 0:
            break
        with np.errstate(over="ignore", invalid="ignore"):
            x[idx] = predict(sys.kind, K, x[idx], cand[idx, g, :])
            if sys.noise is not None and np.any(np.asarray(sys.noise) > 0):
                rows = np.arange(Nc) if index is None else np.asarray(index)
                z = process_noise(*noise_key, rows[idx], s, sys.n)
                x[idx] = x[idx] + np.asarray(sys.noise, np.float64)[None, :sys.n] * z
        traj[s - 1, idx] = x[idx]
        bad = idx[~is_safe(sys, x[idx])]
        newly = bad[fv[bad] == H + 1]
        fv[newly] = s
        alive[bad] = False
    return traj, fv


def rollout_lifted(sys: System, K: np.ndarray, x0, cand: np.ndarray, H: int, early_exit: bool = True):
    """Constant-input rollouts in the lifted space (Sec. IV-A: predicting with
    the Koopman representation is a matrix-vector product per step, and a
    batch of trajectories a matrix-matrix product).  Z holds one lifted state
    z = psi(x0, u_i) per candidate (rows); each step Z <- Z K with the full
    lifted operator K (D, D) of fit_lifted; the predicted state is read off
    the state columns of Z.  cand: (Nc, 1, m), one segment.  Safety, first
    violations and early exit as in rollout(): returns (traj (H, Nc, n),
    fv (Nc,))."""
    cand = np.asarray(cand, np.float64)
    Nc, S, _ = cand.shape
    if S != 1:
        raise ValueError("lifted rollouts hold each candidate's input over the horizon (one segment)")
    K = np.asarray(K, np.float64)
    cols = state_columns(sys.kind, sys.n)
    Z = lift(sys.kind, np.tile(np.asarray(x0, np.float64).reshape(1, -1), (Nc, 1)), cand[:, 0, :])
    traj = np.full((H, Nc, sys.n), np.nan)
    fv = np.full(Nc, H + 1, dtype=np.int64)
    alive = np.ones(Nc, dtype=bool)
    for s in range(1, H + 1):
        idx = np.nonzero(alive)[0] if early_exit else np.arange(Nc)
        if idx.size == 0:
            break
        with np.errstate(over="ignore", invalid="ignore"):
            Z[idx] = Z[idx] @ K
        x = Z[idx][:, cols]
        traj[s - 1, idx] = x
        bad = idx[~is_safe(sys, x)]
        newly = bad[fv[bad] == H + 1]
        fv[newly] = s
        alive[bad] = False
    return traj, fv


def tick_lifted(sys: System, K, x_t, u_h, cand: np.ndarray, H: int) -> dict:
    """One MPMI-SC tick whose predictions come from the lifted rollout."""
    traj, fv = rollout_lifted(sys, K, x_t, cand, H, early_exit=True)
    out = select(sys, cand, fv, H, u_h)
    out["fv"] = fv
    return out


# ----------------------------------------------------------------------------
# Cost and selection (Alg. 2 selection step; Sec. III-D pass-through; Sec. IV-D)
# ----------------------------------------------------------------------------
def cost(sys: System, cand: np.ndarray, u_h) -> np.ndarray:
    """Squared distance of each candidate's first-segment input to u_h, input j
    divided by its half-range h_j."""
    d = (np.asarray(cand, np.float64)[:, 0, :] - np.asarray(u_h, np.float64).reshape(1, -1)) / sys.half_range
    return np.sum(d * d, axis=1)


def select(sys: System, cand: np.ndarray, fv: np.ndarray, H: int, u_h) -> dict:
    """Minimal-intervention choice over the candidates whose rollout stayed safe.

    Safe set = {i : fv_i = H + 1}.  If it is non-empty: the lexicographic
    minimum of (cost_i, i), status OK.  Otherwise: the lexicographic maximum of
    (fv_i, -cost_i, -i), status NO_SAFE.  n_safe counts safe candidates other
    than candidate 0.
    """
    c = cost(sys, cand, u_h)
    fv = np.asarray(fv)
    idx_all = np.arange(fv.size)
    safe = fv == H + 1
    if safe.any():
        cand_idx = idx_all[safe]
        order = np.lexsort((cand_idx, c[safe]))
        i = int(cand_idx[order[0]])
        status = STATUS_OK
    else:
        order = np.lexsort((idx_all, c, -fv))
        i = int(order[0])
        status = STATUS_NO_SAFE
    u_r = np.asarray(cand, np.float64)[i, 0, :]
    return dict(idx=i, status=status, n_safe=int(safe[1:].sum()), u_r=u_r, cost=float(c[i]),
                deviation=float(np.linalg.norm(u_r - np.asarray(u_h, np.float64).reshape(-1))))


def tick(sys: System, K, x_t, u_h, cand: np.ndarray, H: int, noise_key=None) -> dict:
    """One MPMI-SC control tick over an explicit candidate set (N+1, S, m)."""
    traj, fv = rollout(sys, K, x_t, cand, H, early_exit=True, noise_key=noise_key)
    out = select(sys, cand, fv, H, u_h)
    out["fv"] = fv
    return out


# ----------------------------------------------------------------------------
# Sec. IV-D deviation bound
# ----------------------------------------------------------------------------
def deviation_bound(lebesgue_measure: float, N: int) -> float:
    """lambda*(U) / (2 N): half the spacing of N equally spaced 1-D samples."""
    return lebesgue_measure / (2.0 * N)


# ----------------------------------------------------------------------------
# Basis selection (Sec. IV-A and Sec. V-C-3: a library of random basis
# functions is reduced to the ones most relevant to the dynamics by the
# sparsity-promoting method of Jovanovic, Schmid and Nichols (2014))
# ----------------------------------------------------------------------------
def selection_problem(library, X, U, Y):
    """The quadratic data term of the selection on scaled columns.

    Psi_s = Psi / s (s the RMS of each library function over the T rows) and
    Y_s = Y / s_y (s_y the RMS of each state component); with K the (L, n)
    coefficients of the scaled problem,
        J(K) = ||Psi_s K - Y_s||^2 / T = tr(K^T G K) - 2 tr(K^T A) + c,
    G = Psi_s^T Psi_s / T, A = Psi_s^T Y_s / T.  Returns (G, A, s, s_y)."""
    X, U, Y = (np.asarray(a, np.float64) for a in (X, U, Y))
    Psi = lift(library, X, U)
    T = Psi.shape[0]
    s = np.sqrt(np.sum(Psi * Psi, axis=0) / T)
    s[s == 0.0] = 1.0
    sy = np.sqrt(np.sum(Y * Y, axis=0) / T)
    sy[sy == 0.0] = 1.0
    Ps, Ys = Psi / s, Y / sy
    return Ps.T @ Ps / T, Ps.T @ Ys / T, s, sy


def group_shrink(V: np.ndarray, kappa: float) -> np.ndarray:
    """Row-wise block soft threshold: row v -> max(0, 1 - kappa / ||v||) v
    (a row of norm <= kappa becomes exactly zero; for one column this is the
    scalar soft threshold sign(v) max(|v| - kappa, 0))."""
    norms = np.sqrt(np.sum(V * V, axis=1))
    with np.errstate(divide="ignore", invalid="ignore"):
        f = np.where(norms > kappa, 1.0 - kappa / norms, 0.0)
    return V * f[:, None]


def sparse_admm(G, A, gamma: float, rho: float, iters: int):
    """ADMM of the sparsity-promoting problem, in the three steps of
    Jovanovic et al. (2014), Sec. III, with a basis function's row of
    coefficients as the unit that is kept or dropped:
        minimise  J(K) + gamma * sum_f ||B_f||   subject to  K = B,
    augmented Lagrangian with multiplier Lam and penalty rho; from
    B = Lam = 0, each iteration
        K   <- (G + rho/2 I)^-1 (A + rho/2 (B - Lam / rho))   (J's minimiser plus the penalty)
        B'  <- group_shrink(K + Lam / rho, gamma / rho)        (the sparsity step)
        Lam <- Lam + rho (K - B')
    and reports the primal residual ||K - B'||_F and the dual residual
    rho ||B' - B||_F of the last iteration.  A fixed number of iterations
    (no data-dependent stop).  Returns (B, K, Lam, (primal, dual))."""
    G = np.asarray(G, np.float64)
    A = np.asarray(A, np.float64)
    L, n = A.shape
    Mreg = G + 0.5 * rho * np.eye(L)
    B = np.zeros((L, n))
    Lam = np.zeros((L, n))
    K = np.zeros((L, n))
    prim = dual = 0.0
    for _ in range(iters):
        K = np.linalg.solve(Mreg, A + 0.5 * rho * (B - Lam / rho))
        Bn = group_shrink(K + Lam / rho, gamma / rho)
        Lam = Lam + rho * (K - Bn)
        prim = float(np.sqrt(np.sum((K - Bn) ** 2)))
        dual = float(rho * np.sqrt(np.sum((Bn - B) ** 2)))
        B = Bn
    return B, K, Lam, (prim, dual)


def select_basis(library, X, U, Y, gamma: float, rho: float = 1.0, iters: int = 500):
    """Basis selection followed by the polishing step of Jovanovic et al.:
    the support S = {f : B_f != 0} of the sparse solution, then the plain
    least-squares fit (fit()) on the selected functions alone.  Returns
    dict(support, B (unscaled: B_s * s_y / s), K_polished (|S|, n) or None,
    basis (the selected Basis) or None, residuals)."""
    G, A, s, sy = selection_problem(library, X, U, Y)
    B, _, _, res = sparse_admm(G, A, gamma, rho, iters)
    support = np.nonzero(np.any(B != 0.0, axis=1))[0]
    out = dict(support=support, B=B * sy[None, :] / s[:, None], residuals=res, K_polished=None, basis=None)
    if support.size:
        sel = Basis(atoms=library.atoms, feats=tuple(library.feats[f] for f in support))
        out["basis"] = sel
        out["K_polished"] = fit(sel, X, U, Y)[0]
    return out
