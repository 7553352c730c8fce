"""Checks of the synthetic stand-in plants (inputs of the fit and of the
closed loops) against closed forms and conservation laws."""
import math

import numpy as np

import synth


def test_cartpole_energy_conserved_without_force():
    # Frictionless cart-pole, u = 0: total mechanical energy is invariant.
    p = synth.CARTPOLE
    mc, mp, l, g = p["m_cart"], p["m_pole"], p["l"], p["g"]

    def energy(x):
        pd, th, thd = x[1], x[2], x[3]
        # pole centre of mass at (p + l sin th, l cos th); pole inertia about its centre m l^2 / 3
        vx = pd + l * thd * math.cos(th)
        vy = -l * thd * math.sin(th)
        return 0.5 * mc * pd ** 2 + 0.5 * mp * (vx ** 2 + vy ** 2) + 0.5 * (mp * l * l / 3) * thd ** 2 + \
            mp * g * l * math.cos(th)

    x = np.array([0.0, 0.3, 0.2, -0.5])
    e0 = energy(x)
    for _ in range(200):
        x = synth.cartpole_step(x, np.array([0.0]))[0]
    assert abs(energy(x) - e0) < 1e-6 * abs(e0)


def test_cartpole_momentum_response_to_force():
    # Upright pole at rest: a force F gives the system momentum F dt per step.
    p = synth.CARTPOLE
    x = np.zeros(4)
    y = synth.cartpole_step(x, np.array([2.0]))[0]
    l = p["l"]
    mom = (p["m_cart"] + p["m_pole"]) * y[1] + p["m_pole"] * l * y[3] * math.cos(y[2])
    assert abs(mom - 2.0 * p["dt"]) < 1e-9


def test_bicycle_straight_line():
    # No steering, no throttle, no lateral motion: uniform straight motion.
    x = np.array([1.0, 2.0, 0.3, 10.0, 0.0, 0.0])
    y = synth.bicycle_step(x, np.array([0.0, 0.0]))[0]
    dt = synth.BICYCLE["dt"]
    np.testing.assert_allclose(y, [1.0 + 10 * dt * math.cos(0.3), 2.0 + 10 * dt * math.sin(0.3), 0.3, 10.0, 0.0, 0.0],
                               atol=1e-12)
    # throttle only: v_x grows by a dt
    y = synth.bicycle_step(x, np.array([0.0, 2.0]))[0]
    assert abs(y[3] - (10.0 + 2.0 * dt)) < 1e-12


def test_track_states_on_track():
    tr = synth.make_track(3)
    X = synth.race_car_states(2000, tr, seed=1)
    rho = np.hypot(X[:, 0], X[:, 1])
    off = rho - tr.centre_radius(np.arctan2(X[:, 1], X[:, 0]))
    assert np.all(np.abs(off) <= 2.0 + 1e-9)
    assert np.all((X[:, 3] >= 5) & (X[:, 3] <= 15))


def test_loop_sizes_log_uniform():
    N, H = synth.loop_sizes(64, seed=5)
    assert N.min() >= 1024 and N.max() <= 65536 and H.min() >= 20 and H.max() <= 60
    assert 9000 < N.mean() < 25000
