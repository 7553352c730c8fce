"""Seeded synthetic workloads for the shared-control hot path.

This module produces *inputs only*: plant transitions used to fit the Koopman
model, control-tick states and user inputs, track geometry parameters and the
per-loop sizes of the many-loop serving workload.  It holds none of the
method's own arithmetic (lifting, prediction, safety, selection): both the
GPU library and the FP64 oracle consume what it produces, and each implements
the method on its own.

The paper's simulators (a PyBullet balance bot and the Box2D race car of the
"Simulated Environments" subsection of Sec. V) are not available, so two
classic plants of the same shape stand in for them:

* balance bot  -> frictionless cart-pole, state [p, p_dot, theta, theta_dot],
  one input force u in [-5, 5] N, dt = 0.01 s;
* race car     -> dynamic bicycle with saturated linear tyres, state
  [x, y, psi, v_x, v_y, r], inputs [delta, a] in [-0.4, 0.4] x [-3, 3],
  dt = 1/60 s, driving on a closed track whose centreline radius is
  30 m plus four random-phase sinusoids.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------
# Cart-pole ("balance bot")
# ----------------------------------------------------------------------------
CARTPOLE = dict(m_cart=1.0, m_pole=0.2, l=0.5, g=9.81, dt=0.01)
BB_U_LO, BB_U_HI = -5.0, 5.0


def cartpole_deriv(x: np.ndarray, u: np.ndarray, prm: dict = CARTPOLE) -> np.ndarray:
    """Time derivative of the frictionless cart-pole, rows of x = [p, pd, th, thd].

    Classic rigid-body equations (Barto, Sutton & Anderson 1983, with the sign
    correction of Florian 2007); l is the pivot-to-centre-of-mass length.
    """
    mc, mp, l, g = prm["m_cart"], prm["m_pole"], prm["l"], prm["g"]
    x = np.atleast_2d(x)
    u = np.asarray(u, dtype=np.float64).reshape(-1)
    pd, th, thd = x[:, 1], x[:, 2], x[:, 3]
    s, c = np.sin(th), np.cos(th)
    mt = mc + mp
    tmp = (u + mp * l * thd * thd * s) / mt
    thdd = (g * s - c * tmp) / (l * (4.0 / 3.0 - mp * c * c / mt))
    pdd = tmp - mp * l * thdd * c / mt
    return np.stack([pd, pdd, thd, thdd], axis=1)


def rk4(deriv, x, u, dt):
    k1 = deriv(x, u)
    k2 = deriv(x + 0.5 * dt * k1, u)
    k3 = deriv(x + 0.5 * dt * k2, u)
    k4 = deriv(x + dt * k3, u)
    return x + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def cartpole_step(x, u, dt=CARTPOLE["dt"]):
    return rk4(cartpole_deriv, np.atleast_2d(np.asarray(x, np.float64)), u, dt)


def balance_bot_transitions(T: int = 5000, seed: int = 0):
    """T transitions of the cart-pole under u ~ U[-5, 5] (one trajectory with resets).

    Episodes start with every state component in [-0.05, 0.05] and reset when
    |theta| > 0.8 rad or |p| > 3 m.  Returns X (T, 4), U (T, 1), Y (T, 4), FP64.
    """
    rng = np.random.default_rng(seed)
    X = np.empty((T, 4))
    U = np.empty((T, 1))
    Y = np.empty((T, 4))
    x = rng.uniform(-0.05, 0.05, size=4)
    for t in range(T):
        u = rng.uniform(BB_U_LO, BB_U_HI)
        y = cartpole_step(x, np.array([u]))[0]
        X[t], U[t, 0], Y[t] = x, u, y
        x = y
        if abs(x[2]) > 0.8 or abs(x[0]) > 3.0:
            x = rng.uniform(-0.05, 0.05, size=4)
    return X, U, Y


def balance_bot_states(n: int, seed: int = 1):
    """n held-out cart-pole states strictly inside the safe box |p| < 2, |theta| < 0.5.

    States are visited by random-input episodes (as in the fit data, but from
    another seed) and kept when |theta| < 0.4 and |p| < 1.8.
    """
    rng = np.random.default_rng(seed)
    out = []
    x = rng.uniform(-0.05, 0.05, size=4)
    while len(out) < n:
        x = cartpole_step(x, np.array([rng.uniform(BB_U_LO, BB_U_HI)]))[0]
        if abs(x[2]) > 0.8 or abs(x[0]) > 3.0:
            x = rng.uniform(-0.05, 0.05, size=4)
            continue
        if abs(x[2]) < 0.4 and abs(x[0]) < 1.8 and rng.uniform() < 0.25:
            out.append(x.copy())
    return np.array(out)


def uniform_user(n: int, lo, hi, seed: int = 2):
    """n user inputs drawn uniformly from the input box, shape (n, m)."""
    lo = np.atleast_1d(np.asarray(lo, np.float64))
    hi = np.atleast_1d(np.asarray(hi, np.float64))
    rng = np.random.default_rng(seed)
    return lo + (hi - lo) * rng.uniform(size=(n, lo.size))


class AR1User:
    """User input as an AR(1) walk u_t = clip(rho*u_{t-1} + sigma*eta_t, lo, hi)."""

    def __init__(self, lo, hi, rho=0.95, sigma=1.0, seed=2, u0=None):
        self.lo = np.atleast_1d(np.asarray(lo, np.float64))
        self.hi = np.atleast_1d(np.asarray(hi, np.float64))
        self.rho, self.sigma = rho, np.broadcast_to(np.asarray(sigma, np.float64), self.lo.shape)
        self.rng = np.random.default_rng(seed)
        self.u = np.zeros_like(self.lo) if u0 is None else np.asarray(u0, np.float64).copy()

    def next(self):
        eta = self.rng.standard_normal(self.lo.shape)
        self.u = np.clip(self.rho * self.u + self.sigma * eta, self.lo, self.hi)
        return self.u.copy()


# ----------------------------------------------------------------------------
# Dynamic bicycle ("race car") and its track
# ----------------------------------------------------------------------------
BICYCLE = dict(m=1500.0, Iz=2500.0, lf=1.2, lr=1.4, Cf=5.0e4, Cr=5.0e4, mu=1.0, g=9.81, dt=1.0 / 60.0)
RC_U_LO = np.array([-0.4, -3.0])
RC_U_HI = np.array([0.4, 3.0])


def bicycle_deriv(x: np.ndarray, u: np.ndarray, prm: dict = BICYCLE) -> np.ndarray:
    """Time derivative of the dynamic bicycle, rows of x = [x, y, psi, vx, vy, r], u = [delta, a].

    Linear tyres on slip angles computed with max(vx, 1 m/s), each lateral force
    saturated at mu*F_z (so the car can skid out).
    """
    m, Iz, lf, lr = prm["m"], prm["Iz"], prm["lf"], prm["lr"]
    Cf, Cr, mu, g = prm["Cf"], prm["Cr"], prm["mu"], prm["g"]
    x = np.atleast_2d(x)
    u = np.atleast_2d(u)
    psi, vx, vy, r = x[:, 2], x[:, 3], x[:, 4], x[:, 5]
    delta, a = u[:, 0], u[:, 1]
    vxs = np.maximum(vx, 1.0)
    alpha_f = delta - np.arctan((vy + lf * r) / vxs)
    alpha_r = -np.arctan((vy - lr * r) / vxs)
    fzf = m * g * lr / (lf + lr)
    fzr = m * g * lf / (lf + lr)
    Fyf = np.clip(Cf * alpha_f, -mu * fzf, mu * fzf)
    Fyr = np.clip(Cr * alpha_r, -mu * fzr, mu * fzr)
    cps, sps = np.cos(psi), np.sin(psi)
    cd, sd = np.cos(delta), np.sin(delta)
    return np.stack([
        vx * cps - vy * sps,
        vx * sps + vy * cps,
        r,
        a - Fyf * sd / m + vy * r,
        (Fyf * cd + Fyr) / m - vx * r,
        (lf * Fyf * cd - lr * Fyr) / Iz,
    ], axis=1)


def bicycle_step(x, u, dt=BICYCLE["dt"]):
    y = rk4(bicycle_deriv, np.atleast_2d(np.asarray(x, np.float64)), np.atleast_2d(u), dt)
    y[:, 3] = np.maximum(y[:, 3], 0.0)
    return y


@dataclass
class Track:
    """Closed track: centreline radius r_c(phi) = r0 + sum_k amp[k] sin(freq[k] phi + phase[k])."""

    r0: float = 30.0
    half_width: float = 3.0
    amp: np.ndarray = field(default_factory=lambda: np.array([2.0, 1.0, 2.0 / 3.0, 0.5]))
    freq: np.ndarray = field(default_factory=lambda: np.array([2, 3, 4, 5]))
    phase: np.ndarray = field(default_factory=lambda: np.zeros(4))

    def centre_radius(self, phi):
        phi = np.asarray(phi, np.float64)
        return self.r0 + sum(a * np.sin(f * phi + p) for a, f, p in zip(self.amp, self.freq, self.phase))

    def centre_radius_dphi(self, phi):
        phi = np.asarray(phi, np.float64)
        return sum(a * f * np.cos(f * phi + p) for a, f, p in zip(self.amp, self.freq, self.phase))


def make_track(seed: int = 3) -> Track:
    """Track with phases ~ U[0, 2 pi) from the seed (amplitudes 2/k m, frequencies k+1)."""
    rng = np.random.default_rng(seed)
    return Track(phase=rng.uniform(0.0, 2.0 * math.pi, size=4))


def race_car_states(n: int, track: Track, seed: int = 1, offset=2.0, psi_sd=0.2,
                    vx=(5.0, 15.0), vy=(-0.5, 0.5), r=(-0.3, 0.3)):
    """n on-track race-car states: radial offset U[-offset, offset] from the centreline,
    heading = centreline tangent + N(0, psi_sd), speeds uniform in the given ranges."""
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=n)
    rho = track.centre_radius(phi) + rng.uniform(-offset, offset, size=n)
    rc = track.centre_radius(phi)
    drc = track.centre_radius_dphi(phi)
    tx = drc * np.cos(phi) - rc * np.sin(phi)
    ty = drc * np.sin(phi) + rc * np.cos(phi)
    psi = np.arctan2(ty, tx) + psi_sd * rng.standard_normal(n)
    return np.stack([
        rho * np.cos(phi), rho * np.sin(phi), psi,
        rng.uniform(*vx, size=n), rng.uniform(*vy, size=n), rng.uniform(*r, size=n),
    ], axis=1)


def race_car_transitions(T: int = 50000, seed: int = 0, track: Track | None = None):
    """T one-step transitions of the bicycle from random on-track states under
    uniform random inputs in the input box.  Returns X (T, 6), U (T, 2), Y (T, 6)."""
    track = make_track() if track is None else track
    X = race_car_states(T, track, seed=seed + 1000, offset=3.5, psi_sd=0.4,
                        vx=(2.0, 18.0), vy=(-1.5, 1.5), r=(-0.8, 0.8))
    U = uniform_user(T, RC_U_LO, RC_U_HI, seed=seed)
    Y = bicycle_step(X, U)
    return X, U, Y


# ----------------------------------------------------------------------------
# The paper's three-input race car (Sec. V-A: a desired heading, gas and brake)
# ----------------------------------------------------------------------------
# Inputs w_6.. = [h, gas, brake] on [-1, 1] x [0, 1] x [-1, 0]; the same
# bicycle with steering delta = 0.4 h rad and acceleration a = 3 (gas + brake) m/s^2.
RC3_U_LO = np.array([-1.0, 0.0, -1.0])
RC3_U_HI = np.array([1.0, 1.0, 0.0])
RC3_STEER, RC3_ACCEL = 0.4, 3.0


def race_car3_inputs(u3: np.ndarray) -> np.ndarray:
    """[h, gas, brake] rows -> the bicycle's [delta, a] rows."""
    u3 = np.atleast_2d(np.asarray(u3, np.float64))
    return np.stack([RC3_STEER * u3[:, 0], RC3_ACCEL * (u3[:, 1] + u3[:, 2])], axis=1)


def bicycle3_step(x, u3, dt=BICYCLE["dt"]):
    return bicycle_step(x, race_car3_inputs(u3), dt)


def race_car3_transitions(T: int = 50000, seed: int = 0, track: Track | None = None):
    """T one-step transitions of the three-input car from random on-track states
    under uniform random inputs in its box.  Returns X (T, 6), U (T, 3), Y (T, 6)."""
    track = make_track() if track is None else track
    X = race_car_states(T, track, seed=seed + 1000, offset=3.5, psi_sd=0.4,
                        vx=(2.0, 18.0), vy=(-1.5, 1.5), r=(-0.8, 0.8))
    U = uniform_user(T, RC3_U_LO, RC3_U_HI, seed=seed)
    return X, U, bicycle3_step(X, U)


def race_car3_basis():
    """A 64-feature basis for the three-input car as (atoms, features): atoms
    ('one' | 'var' | 'sin' | 'cos', component of w = [x, y, psi, vx, vy, r, h,
    gas, brake]); feature = product of two atoms.  1; w (9); the state
    quadratics (21); the input quadratics (6); vx, vy, r times h, and vx times
    gas and brake (5); sin/cos psi and sin/cos h (4); sin/cos psi times (vx, vy,
    r) (6) and times gas and brake (4); sin/cos h times (vx, vy, r) (6); gas and
    brake times sin h (2)."""
    atoms = [("one", 0)] + [("var", k) for k in range(9)] + [("sin", 2), ("cos", 2), ("sin", 6), ("cos", 6)]
    ONE, W, SP, CP, SH, CH = 0, list(range(1, 10)), 10, 11, 12, 13
    feats = [(ONE, ONE)] + [(W[k], ONE) for k in range(9)]
    feats += [(W[k], W[l]) for k in range(6) for l in range(k, 6)]
    feats += [(W[k], W[l]) for k in range(6, 9) for l in range(k, 9)]
    feats += [(W[3], W[6]), (W[4], W[6]), (W[5], W[6]), (W[3], W[7]), (W[3], W[8])]
    feats += [(SP, ONE), (CP, ONE), (SH, ONE), (CH, ONE)]
    feats += [(SP, W[k]) for k in (3, 4, 5)] + [(CP, W[k]) for k in (3, 4, 5)]
    feats += [(SP, W[7]), (SP, W[8]), (CP, W[7]), (CP, W[8])]
    feats += [(SH, W[k]) for k in (3, 4, 5)] + [(CH, W[k]) for k in (3, 4, 5)]
    feats += [(W[7], SH), (W[8], SH)]
    assert len(feats) == 64 and len(atoms) == 14
    return atoms, feats


def random_library(n: int, m: int, L: int, seed: int = 0):
    """A library of L candidate basis functions as (atoms, features): the
    atoms 1, w_k, sin w_k, cos w_k of w = [x; u] (k < n + m), the features the
    constant, every w_k, and L - 1 - (n + m) further products of two atoms
    drawn uniformly without replacement from the remaining unordered atom
    pairs (seeded)."""
    nw = n + m
    atoms = [("one", 0)] + [("var", k) for k in range(nw)] + [("sin", k) for k in range(nw)] + \
        [("cos", k) for k in range(nw)]
    base = [(0, 0)] + [(1 + k, 0) for k in range(nw)]
    pairs = [(a, b) for a in range(len(atoms)) for b in range(a, len(atoms))]
    rest = [p for p in pairs if p not in base and (p[1], p[0]) not in base]
    k = L - len(base)
    if k < 0 or k > len(rest):
        raise ValueError(f"a library of {L} functions does not fit {len(atoms)} atoms")
    rng = np.random.default_rng(seed)
    pick = sorted(rng.choice(len(rest), size=k, replace=False))
    return atoms, base + [rest[i] for i in pick]


# ----------------------------------------------------------------------------
# Linear plant (identity-basis checks) and many-loop sizes
# ----------------------------------------------------------------------------
def linear_plant(n: int = 4, m: int = 1, seed: int = 11, radius: float = 0.97):
    """A random stable linear plant x+ = A x + B u (spectral radius <= radius)."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    A *= radius / max(1e-12, np.max(np.abs(np.linalg.eigvals(A))))
    B = rng.standard_normal((n, m))
    return A, B


def linear_transitions(A, B, T: int = 400, seed: int = 12):
    rng = np.random.default_rng(seed)
    n, m = B.shape
    X = rng.standard_normal((T, n))
    U = rng.uniform(-1.0, 1.0, size=(T, m))
    Y = X @ A.T + U @ B.T
    return X, U, Y


def loop_sizes(n_loops: int = 64, seed: int = 5, n_lo: int = 1024, n_hi: int = 65536,
               h_lo: int = 20, h_hi: int = 60):
    """Per-loop candidate counts N_l = round(exp(U[ln n_lo, ln n_hi])) and horizons H_l ~ U{h_lo..h_hi}."""
    rng = np.random.default_rng(seed)
    N = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=n_loops))).astype(np.int64)
    H = rng.integers(h_lo, h_hi + 1, size=n_loops)
    return N, H


class ManyLoops:
    """The mixed serving workload: n_loops closed control loops, the first half
    cart-poles and the second half race cars, with candidate counts and
    horizons from loop_sizes(n_loops, seed), AR(1) users (cart-pole: sigma
    1 N, seeds 100 + i; race car: sigma (0.08 rad, 0.6 m/s^2), seeds 200 + i)
    and plants that advance with the applied inputs and restart from a fresh
    seeded state when they leave their safe set.  States and user inputs are
    padded to (n_loops, 8) and (n_loops, 4); loop i draws its candidates with
    seed 1000 + i."""

    def __init__(self, track: "Track", n_loops: int = 64, seed: int = 5):
        self.track = track
        self.n_loops = n_loops
        self.nb = n_loops // 2
        self.N, self.H = loop_sizes(n_loops, seed=seed)
        self.kinds = ["bb"] * self.nb + ["rc"] * (n_loops - self.nb)
        self.seeds = [1000 + i for i in range(n_loops)]
        self.x = np.zeros((n_loops, 8), np.float32)
        self.u = np.zeros((n_loops, 4), np.float32)
        self.x[: self.nb, :4] = balance_bot_states(self.nb, seed=1)
        self.x[self.nb:, :6] = race_car_states(n_loops - self.nb, track, seed=1)
        self.users = [AR1User([BB_U_LO], [BB_U_HI], seed=100 + i) for i in range(self.nb)] + \
                     [AR1User(RC_U_LO, RC_U_HI, sigma=[0.08, 0.6], seed=200 + i) for i in range(n_loops - self.nb)]
        self.resets = 0
        self._next_users()

    def _next_users(self):
        for i, us in enumerate(self.users):
            self.u[i, : us.lo.size] = us.next()

    def advance(self, u_applied: np.ndarray, t: int):
        """Steps every plant with its applied input (n_loops, >= 2), restarts
        those that left their safe set, and moves the users on."""
        nb = self.nb
        xb = cartpole_step(self.x[:nb, :4].astype(np.float64), u_applied[:nb, 0].astype(np.float64))
        bad = (np.abs(xb[:, 2]) > 0.5) | (np.abs(xb[:, 0]) > 2.0)
        self.resets += int(bad.sum())
        if bad.any():
            xb[bad] = balance_bot_states(int(bad.sum()), seed=7 + t)
        self.x[:nb, :4] = xb
        xr = bicycle_step(self.x[nb:, :6].astype(np.float64), u_applied[nb:, :2].astype(np.float64))
        off = np.hypot(xr[:, 0], xr[:, 1]) - self.track.centre_radius(np.arctan2(xr[:, 1], xr[:, 0]))
        badr = (np.abs(off) > 3.0) | (np.abs(xr[:, 4]) > 2.0)
        self.resets += int(badr.sum())
        if badr.any():
            xr[badr] = race_car_states(int(badr.sum()), self.track, seed=9 + t)
        self.x[nb:, :6] = xr
        self._next_users()


# ----------------------------------------------------------------------------
# Proposal-network initialisation and label states
# ----------------------------------------------------------------------------
MLP_LAYERS = [(8, 256), (256, 256), (256, 256), (256, 80)]


def mlp_init(seed: int = 6) -> np.ndarray:
    """Flat initial parameters: per layer W [in][out] ~ U(-1/sqrt(in), 1/sqrt(in)), b = 0."""
    rng = np.random.default_rng(seed)
    parts = []
    for k, n in MLP_LAYERS:
        lim = 1.0 / math.sqrt(k)
        parts.append(rng.uniform(-lim, lim, size=k * n))
        parts.append(np.zeros(n))
    return np.concatenate(parts)
