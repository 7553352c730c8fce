"""Pins of the FP64 oracle against facts fixed outside the oracle itself.

Each test checks the oracle against a closed form, a hand-written value, a
published test vector, a brute-force enumeration or an invariant the paper
states, so that a dropped term, a wrong sign or index, or a transposed operand
anywhere in the oracle fails at least one of them.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg
from hypothesis import given, settings, strategies as st

import synth
from oracle import mpmi_oracle as o

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _bb(infl=0.0, theta=0.5, p=2.0):
    return o.System("balance_bot", 4, 1, box=[(2, theta, infl), (0, p, infl)], u_lo=[-5.0], u_hi=[5.0])


@pytest.fixture(scope="module")
def bb_model():
    X, U, Y = synth.balance_bot_transitions(5000, seed=0)
    K, info = o.fit("balance_bot", X, U, Y)
    return K, info, (X, U, Y)


# ---------------------------------------------------------------- basis ------
def test_basis_golden_points():
    with open(os.path.join(GOLDEN, "basis_points.txt")) as f:
        rows = [l for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        kind, w, expect = (s.strip() for s in row.split("|"))
        w = np.array([float(v) for v in w.split()])
        expect = np.array([float(v) for v in expect.split()])
        n = 4 if kind == "balance_bot" else 6
        base = "race_car" if kind.startswith("race_car") else kind
        psi = o.lift(base, w[None, :n], w[None, n:])[0]
        if kind == "race_car_tail":
            psi = psi[-19:]
        assert psi.shape == expect.shape
        np.testing.assert_allclose(psi, expect, rtol=0, atol=1e-12)
    assert o.basis_dim("balance_bot", 4, 1) == 21 and o.basis_dim("race_car", 6, 2) == 64


# ----------------------------------------------------- P1: linear closed form --
def _linear_case(seed=11):
    A, B = synth.linear_plant(4, 1, seed=seed)
    X, U, Y = synth.linear_transitions(A, B, T=300, seed=seed + 1)
    return A, B, X, U, Y


def test_identity_basis_fit_recovers_linear_plant():
    A, B, X, U, Y = _linear_case()
    K, info = o.fit("linear", X, U, Y)
    np.testing.assert_allclose(K, np.vstack([A.T, B.T]), rtol=0, atol=1e-11)
    assert np.all(info["resid_rms"] < 1e-12)


def _affine_in_u(A, B, x0, H):
    """x_s(u) = a_s + b_s u for constant u (closed form A^s x0 + sum_{j<s} A^j B u)."""
    out = []
    for s in range(1, H + 1):
        a = np.linalg.matrix_power(A, s) @ x0
        b = sum(np.linalg.matrix_power(A, j) @ B[:, 0] for j in range(s))
        out.append((a, b))
    return out


def test_linear_rollout_matches_closed_form():
    A, B, X, U, Y = _linear_case()
    K = np.vstack([A.T, B.T])
    sys = o.System("linear", 4, 1, box=[], u_lo=[-1.0], u_hi=[1.0])
    x0 = np.array([0.3, -0.2, 0.5, 0.1])
    cand = o.with_user(o.grid_candidates(sys, [33]), [0.25], 1)
    H = 12
    traj, fv = o.rollout(sys, K, x0, cand, H, early_exit=False)
    for s, (a, b) in enumerate(_affine_in_u(A, B, x0, H), start=1):
        expect = a[None, :] + np.outer(cand[:, 0, 0], b)
        np.testing.assert_allclose(traj[s - 1], expect, rtol=1e-12, atol=1e-12)
    # u = 0 gives A^s x0
    traj0, _ = o.rollout(sys, K, x0, np.zeros((1, 1, 1)), H, early_exit=False)
    np.testing.assert_allclose(traj0[H - 1, 0], np.linalg.matrix_power(A, H) @ x0, rtol=1e-12, atol=1e-13)
    assert np.all(fv == H + 1)  # no constraints: everything safe


@pytest.mark.parametrize("seed,u_h", [(11, 0.9), (13, -0.7), (17, 0.05), (19, 0.6), (23, -0.95)])
def test_linear_selection_matches_closed_form_interval(seed, u_h):
    """Each predicted state is affine in a constant u, so the safe inputs form an
    open interval (L, R); the choice is u_h when inside, else the grid point in
    (L, R) nearest u_h."""
    A, B, _, _, _ = _linear_case(seed)
    K = np.vstack([A.T, B.T])
    H = 10
    x0 = np.array([0.2, -0.1, 0.15, 0.05])
    bounds = [(0, 0.6), (2, 0.5)]
    sys = o.System("linear", 4, 1, box=[(i, c, 0.0) for i, c in bounds], u_lo=[-1.0], u_hi=[1.0])
    L, R = -np.inf, np.inf
    for a, b in _affine_in_u(A, B, x0, H):
        for i, c in bounds:
            if b[i] == 0.0:
                if abs(a[i]) >= c:
                    L, R = np.inf, -np.inf
                continue
            lo, hi = sorted([(-c - a[i]) / b[i], (c - a[i]) / b[i]])
            L, R = max(L, lo), min(R, hi)
    grid = o.grid_candidates(sys, [200])
    cand = o.with_user(grid, [u_h], 1)
    res = o.tick(sys, K, x0, [u_h], cand, H)
    u = cand[:, 0, 0]
    inside = (u > L) & (u < R)
    far = (np.abs(u - L) > 1e-9) & (np.abs(u - R) > 1e-9)
    np.testing.assert_array_equal((res["fv"] == H + 1)[far], inside[far])
    if L < u_h < R:
        assert res["idx"] == 0 and res["status"] == o.STATUS_OK
    elif inside[1:].any():
        gi = np.nonzero(inside[1:])[0] + 1
        best = gi[np.argmin(np.abs(u[gi] - u_h))]
        assert res["idx"] == best and res["status"] == o.STATUS_OK
    else:
        assert res["status"] == o.STATUS_NO_SAFE


# --------------------------------------------------------- P2: brute force --
def _brute_force(sys, K, x0, cand, H, u_h):
    Nc, S, m = cand.shape
    fvs, costs = [], []
    for i in range(Nc):
        x = np.array(x0, dtype=np.float64)
        first = H + 1
        for s in range(1, H + 1):
            g = ((s - 1) * S) // H
            x = o.predict(sys.kind, K, x[None], cand[i, g][None])[0]
            ok = True
            for idx, bound, infl in sys.box:
                if not (abs(x[idx]) < bound - infl):
                    ok = False
            if not ok and first == H + 1:
                first = s
        fvs.append(first)
        c = 0.0
        for j in range(m):
            d = (cand[i, 0, j] - u_h[j]) / (0.5 * (sys.u_hi[j] - sys.u_lo[j]))
            c += d * d
        costs.append(c)
    order = sorted(range(Nc), key=lambda i: (costs[i], i))
    safe = [i for i in order if fvs[i] == H + 1]
    if safe:
        return safe[0], o.STATUS_OK, fvs
    order = sorted(range(Nc), key=lambda i: (-fvs[i], costs[i], i))
    return order[0], o.STATUS_NO_SAFE, fvs


@pytest.mark.parametrize("seed", range(8))
def test_bruteforce_tiny(bb_model, seed):
    K = bb_model[0]
    rng = np.random.default_rng(100 + seed)
    sys = _bb(theta=0.12, p=0.5)
    H = int(rng.integers(2, 6))
    S = int(rng.integers(1, 3))
    N = int(rng.integers(4, 16))
    x0 = np.array([rng.uniform(-0.3, 0.3), rng.uniform(-1, 1), rng.uniform(-0.1, 0.1), rng.uniform(-1, 1)])
    u_h = rng.uniform(-5, 5, size=1)
    cand = o.with_user(o.uniform_candidates(sys, N, S, seed, 0, 0), u_h, S)
    res = o.tick(sys, K, x0, u_h, cand, H)
    idx, status, fvs = _brute_force(sys, K, x0, cand, H, u_h)
    assert res["idx"] == idx and res["status"] == status
    np.testing.assert_array_equal(res["fv"], fvs)


# --------------------------------------------------- P3: zero intervention --
@settings(max_examples=25, deadline=None)
@given(seed=st.integers(0, 10_000), u=st.floats(-5, 5))
def test_zero_intervention(bb_model, seed, u):
    K = bb_model[0]
    sys = _bb(theta=0.3)
    x0 = synth.balance_bot_states(1, seed=seed)[0]
    cand = o.with_user(o.grid_candidates(sys, [64]), [u], 1)
    res = o.tick(sys, K, x0, [u], cand, 20)
    if res["fv"][0] == 21:
        assert res["idx"] == 0 and res["u_r"][0] == np.float64(u) and res["deviation"] == 0.0


# ---------------------------------------------------- P4: mask monotone ------
@settings(max_examples=15, deadline=None)
@given(seed=st.integers(0, 10_000), r1=st.floats(0.0, 0.2), dr=st.floats(0.0, 0.2))
def test_mask_monotone_in_inflation(bb_model, seed, r1, dr):
    K = bb_model[0]
    x0 = synth.balance_bot_states(1, seed=seed)[0]
    cand = o.with_user(o.uniform_candidates(_bb(), 128, 5, seed, 1, 0), [0.0], 5)
    _, fv1 = o.rollout(_bb(infl=r1), K, x0, cand, 50)
    _, fv2 = o.rollout(_bb(infl=r1 + dr), K, x0, cand, 50)
    assert np.all(fv2 <= fv1)


# -------------------------------------------------------------- P5: fit -----
def test_fit_exact_nonlinear_model():
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, size=(400, 4))
    U = rng.uniform(-5, 5, size=(400, 1))
    K_true = rng.standard_normal((21, 4))
    Y = o.lift("balance_bot", X, U) @ K_true
    K, _ = o.fit("balance_bot", X, U, Y)
    np.testing.assert_allclose(K, K_true, rtol=0, atol=1e-9)


def test_fit_residual_orthogonal_and_normal_equations(bb_model):
    K, info, (X, U, Y) = bb_model
    Psi = o.lift("balance_bot", X, U)
    G = Psi.T @ (Y - Psi @ K)
    assert np.max(np.abs(G)) < 1e-9 * np.linalg.norm(Psi) * np.linalg.norm(Y)
    s = np.sqrt(np.mean(Psi ** 2, axis=0))
    Ps = Psi / s
    c = scipy.linalg.cho_factor(Ps.T @ Ps)
    Kn = scipy.linalg.cho_solve(c, Ps.T @ Y) / s[:, None]
    np.testing.assert_allclose(K, Kn, rtol=0, atol=1e-7 * np.max(np.abs(K)))
    assert 1.0 < info["cond"] < 1e6


def test_fit_ridge_closed_form(bb_model):
    _, _, (X, U, Y) = bb_model
    lam = 3.0
    K, _ = o.fit("balance_bot", X, U, Y, ridge=lam)
    Psi = o.lift("balance_bot", X, U)
    s = np.sqrt(np.mean(Psi ** 2, axis=0))
    Ps = Psi / s
    Kr = np.linalg.solve(Ps.T @ Ps + lam * np.eye(21), Ps.T @ Y) / s[:, None]
    np.testing.assert_allclose(K, Kr, rtol=0, atol=1e-8 * np.max(np.abs(K)))


def test_fit_race_car_residual_orthogonal():
    X, U, Y = synth.race_car_transitions(3000, seed=0)
    K, info = o.fit("race_car", X, U, Y)
    Psi = o.lift("race_car", X, U)
    s = np.sqrt(np.mean(Psi ** 2, axis=0))
    G = (Psi / s).T @ (Y - Psi @ K)
    assert np.max(np.abs(G)) < 1e-7 * np.linalg.norm(Psi / s) * np.linalg.norm(Y)


# ------------------------------------------------------ P6/P7: Eq. 2 bound --
def test_eq2_printed_values():
    assert o.deviation_bound(2.0, 10_000) == pytest.approx(1e-4, rel=1e-12)
    assert round(o.deviation_bound(4.0, 10_120), 4) == 0.0002
    assert o.deviation_bound(10.0, 1024) == 0.0048828125


@pytest.mark.parametrize("seed", [11, 13, 17, 19, 23, 29])
def test_grid_resolution_bound(seed):
    A, B, _, _, _ = _linear_case(seed)
    K = np.vstack([A.T, B.T])
    sys = o.System("linear", 4, 1, box=[(0, 0.6, 0.0), (2, 0.5, 0.0)], u_lo=[-1.0], u_hi=[1.0])
    x0 = np.array([0.2, -0.1, 0.15, 0.05])
    N = 256
    grid = o.grid_candidates(sys, [N])[:, None, :]
    _, fv = o.rollout(sys, K, x0, grid, 10)
    safe_u = grid[fv == 11, 0, 0]
    if safe_u.size < 2:
        pytest.skip("empty safe set for this plant")
    lam = 2.0
    rng = np.random.default_rng(seed)
    for u_h in rng.uniform(-1, 1, size=40):
        res = o.select(sys, grid, fv, 10, [u_h])
        inside = safe_u.min() - lam / (2 * N) <= u_h <= safe_u.max() + lam / (2 * N)
        if inside:
            assert abs(res["u_r"][0] - u_h) <= lam / (2 * N) + 1e-12
        else:
            proj = np.clip(u_h, safe_u.min() - lam / (2 * N), safe_u.max() + lam / (2 * N))
            assert abs(res["u_r"][0] - proj) < lam / N


# ------------------------------------------------------- candidates / RNG --
def test_splitmix64_published_vectors():
    with open(os.path.join(GOLDEN, "splitmix64_vectors.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    for row in rows:
        seed, outs = int(row[0]), [int(v) for v in row[1:]]
        assert o.splitmix64_sequence(seed, 3) == outs


def test_counter_hash_is_chained_splitmix():
    # hash(seed, a, b, c, d) with all words zero equals SplitMix64 applied four
    # times to a state of 0 that is re-fed its own output.
    h = 0
    for _ in range(4):
        h = int(o.mix64(np.uint64((h + o.GOLDEN_GAMMA) & ((1 << 64) - 1))))
    assert int(o.hash_counter(0, 0, 0, 0, 0)) == h
    assert int(o.hash_counter(0, 0, 0, 0, 0)) != int(o.hash_counter(0, 0, 0, 1, 0))


def _golden_splitmix(seed):
    with open(os.path.join(GOLDEN, "splitmix64_vectors.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    return [int(v) for v in {int(r[0]): r[1:] for r in rows}[seed]]


def test_counter_hash_chain_from_published_vectors():
    """The chained hash h <- mix((h ^ w) + gamma) steered through the published
    seed-0 stream: with seed ^ tick = 0 the first round is mix(gamma) = out1; a
    loop word of out1 ^ gamma makes the second mix(2 gamma) = out2; an index
    word of out2 ^ (2 gamma) makes the third out3; a slot word of out3 brings
    the fourth back to mix(gamma) = out1."""
    out1, out2, out3 = _golden_splitmix(0)
    g = o.GOLDEN_GAMMA
    two_g = (2 * g) & ((1 << 64) - 1)
    h = o.hash_counter(np.uint64(12345), np.uint64(12345), np.uint64(out1 ^ g), np.uint64(out2 ^ two_g),
                       np.uint64(out3))
    assert int(h) == out1
    # one round less: the slot word zero gives mix(out3 + gamma) instead
    assert int(o.hash_counter(np.uint64(7), np.uint64(7), np.uint64(out1 ^ g), np.uint64(out2 ^ two_g),
                              np.uint64(0))) != out1


def test_uniform_value_hand_derived():
    """A draw's top 24 bits are the fraction of the box: out1 of the published
    seed-0 stream is 16294208416658607535, whose top 24 bits are 14819496, so
    on [-5, 5) it stands for -5 + 10 * 14819496 / 2^24 = 3.833107948303223
    (FP32 3.8331079483032227).  A draw of 0 is the lower end, the largest
    draw one 2^-24 step short of the upper end."""
    out1 = _golden_splitmix(0)[0]
    assert out1 >> 40 == 14819496
    assert o.uniform_value(-5.0, 5.0, np.uint64(out1)) == np.float64(np.float32(3.8331079483032227))
    assert o.uniform_value(-0.4, 0.4, np.uint64(0)) == np.float64(np.float32(-0.4))
    top = o.uniform_value(-3.0, 3.0, np.uint64((1 << 64) - 1))
    assert top == np.float64(np.float32(-3.0 + 6.0 * (1.0 - 2.0 ** -24))) and top < 3.0


def test_uniform_candidates_follow_their_draws():
    """Candidate (i, g, j) is the value of draw hash(seed, tick, loop, i, g m + j)
    (i from 1); the value map is increasing, so sorting the draws sorts the
    candidates, and the extreme draws land next to the box ends."""
    sys = o.System("race_car", 6, 2, u_lo=[-0.4, -3.0], u_hi=[0.4, 3.0])
    N, S = 3000, 3
    c = o.uniform_candidates(sys, N, S, seed=4, tick=7, loop=2)
    for i, g, j in ((1, 0, 0), (1, 0, 1), (17, 2, 1), (N, 1, 0)):
        h = o.hash_counter(np.uint64(4), np.uint64(7), np.uint64(2), np.uint64(i), np.uint64(g * 2 + j))
        assert c[i - 1, g, j] == o.uniform_value(sys.u_lo[j], sys.u_hi[j], h)
    for j in range(2):
        h = o.hash_counter(np.uint64(4), np.uint64(7), np.uint64(2), np.arange(1, N + 1, dtype=np.uint64),
                           np.uint64(j))
        vals = c[:, 0, j][np.argsort(h >> np.uint64(40), kind="stable")]
        assert np.all(np.diff(vals) >= 0)
        span = sys.u_hi[j] - sys.u_lo[j]
        assert vals[0] - sys.u_lo[j] < 0.01 * span and sys.u_hi[j] - vals[-1] < 0.01 * span


def test_uniform_candidates_in_box_and_unbiased():
    sys = o.System("race_car", 6, 2, u_lo=[-0.4, -3.0], u_hi=[0.4, 3.0])
    c = o.uniform_candidates(sys, 20000, 3, seed=4, tick=7, loop=2)
    assert c.shape == (20000, 3, 2)
    assert np.all(c >= sys.u_lo) and np.all(c < sys.u_hi + 1e-6)
    mean = c.mean(axis=(0, 1))
    assert np.all(np.abs(mean - 0.5 * (sys.u_lo + sys.u_hi)) < 0.02 * (sys.u_hi - sys.u_lo))
    assert np.all(c == c.astype(np.float32).astype(np.float64))


def test_grid_candidates_closed_form():
    sys = o.System("linear", 1, 1, u_lo=[-5.0], u_hi=[5.0])
    np.testing.assert_array_equal(o.grid_candidates(sys, [4])[:, 0], [-3.75, -1.25, 1.25, 3.75])
    sys2 = o.System("race_car", 6, 2, u_lo=[-0.4, -3.0], u_hi=[0.4, 3.0])
    g = o.grid_candidates(sys2, [2, 3])
    np.testing.assert_allclose(g, [[np.float32(-0.2), -2], [np.float32(0.2), -2], [np.float32(-0.2), 0],
                                   [np.float32(0.2), 0], [np.float32(-0.2), 2], [np.float32(0.2), 2]], rtol=0, atol=1e-7)


def test_segments():
    assert [o.segment_of_step(s, 5, 50) for s in (1, 10, 11, 20, 21, 50)] == [0, 0, 1, 1, 2, 4]
    assert all(o.segment_of_step(s, 1, 20) == 0 for s in range(1, 21))


# ------------------------------------------------------------- safety ------
def test_margins_hand_cases():
    sys = _bb()
    m = o.margins(sys, np.array([[1.5, 0.0, 0.3, 0.0], [0.0, 0.0, -0.6, 0.0]]))
    np.testing.assert_allclose(m, [[0.2, 0.5], [-0.1, 2.0]], atol=1e-15)
    assert list(o.is_safe(sys, np.array([[1.5, 0, 0.3, 0], [0, 0, -0.6, 0], [np.nan, 0, 0, 0]]))) == [True, False, False]
    tr = dict(r0=30.0, half=3.0, amp=[2.0, 1.0, 2 / 3, 0.5], freq=[2, 3, 4, 5], phase=[0.0] * 4, infl=0.5)
    rc = o.System("race_car", 6, 2, box=[(4, 2.0, 0.0)], track=tr, u_lo=[-0.4, -3.0], u_hi=[0.4, 3.0])
    x = np.array([[31.0, 0.0, 0, 0, 1.0, 0], [0.0, 29.0, 0, 0, 0, 0], [0.0, 0.0, 0, 0, 0, 0]])
    # phi = 0: r_c = 30 -> gap 1, margin 2.5 - 1 = 1.5; phi = pi/2: sin(k pi/2 * ...)
    rc_half_pi = 30 + 2 * math.sin(math.pi) + math.sin(1.5 * math.pi) + (2 / 3) * math.sin(2 * math.pi) + 0.5 * math.sin(2.5 * math.pi)
    m = o.margins(rc, x)
    np.testing.assert_allclose(m[:, 0], [1.0, 2.0, 2.0])
    np.testing.assert_allclose(m[:, 1], [1.5, 2.5 - abs(29.0 - rc_half_pi), 2.5 - 30.0], atol=1e-12)


def test_track_margins_with_phases():
    """Phases shift each sinusoid: r_c(phi) = 30 + 2 sin(2 phi + pi/2) + sin(3 phi + pi).
    At phi = 0 that is 30 + 2 + 0 = 32; at phi = pi/2 it is 30 + 2 sin(3 pi/2)
    + sin(5 pi/2) = 29; at phi = pi, 30 + 2 - 0 = 32 again."""
    tr = dict(r0=30.0, half=3.0, amp=[2.0, 1.0, 0.0, 0.0], freq=[2, 3, 4, 5],
              phase=[math.pi / 2, math.pi, 0.0, 0.0], infl=0.5)
    rc = o.System("race_car", 6, 2, box=[], track=tr, u_lo=[-0.4, -3.0], u_hi=[0.4, 3.0])
    x = np.array([[32.5, 0.0, 0, 0, 0, 0], [0.0, 29.0, 0, 0, 0, 0], [0.0, 30.0, 0, 0, 0, 0],
                  [-31.0, 0.0, 0, 0, 0, 0]])
    np.testing.assert_allclose(o.centre_radius(tr, np.array([0.0, math.pi / 2, math.pi])), [32.0, 29.0, 32.0],
                               atol=1e-12)
    # margins (3 - 0.5) - |rho - r_c|: gaps 0.5, 0, 1, 1
    np.testing.assert_allclose(o.margins(rc, x)[:, 0], [2.0, 2.5, 1.5, 1.5], atol=1e-12)


def test_no_safe_fallback_rule():
    sys = _bb()
    cand = np.array([[[0.0]], [[1.0]], [[-1.0]], [[2.0]]])
    fv = np.array([3, 5, 5, 4])
    r = o.select(sys, cand, fv, 10, [0.0])
    assert r["status"] == o.STATUS_NO_SAFE and r["idx"] == 1 and r["n_safe"] == 0
    fv = np.array([3, 11, 11, 11])
    r = o.select(sys, cand, fv, 10, [0.0])
    assert r["status"] == o.STATUS_OK and r["idx"] == 1 and r["n_safe"] == 3


# ------------------------------------------------------- process noise (Alg. 2 z_i) --
def test_process_noise_is_standard_normal():
    z = o.process_noise(3, 4, 5, np.arange(1, 20001), 7, 6)
    assert z.shape == (20000, 6)
    for j in range(6):
        assert scipy.stats.kstest(z[:, j], "norm").pvalue > 1e-3
    c = np.corrcoef(z.T)
    assert np.max(np.abs(c - np.eye(6))) < 0.03
    # different steps and candidates give different draws
    assert not np.allclose(o.process_noise(3, 4, 5, [1], 1, 6), o.process_noise(3, 4, 5, [1], 2, 6))


def test_noisy_linear_rollout_closed_form():
    """x_s = A x_{s-1} + B u + sigma z_s, so x_s = A^s x0 + sum_j A^j B u + sum_k A^{s-k} sigma z_k."""
    A, B, _, _, _ = _linear_case()
    K = np.vstack([A.T, B.T])
    sig = np.array([0.1, 0.02, 0.05, 0.3])
    sys = o.System("linear", 4, 1, box=[], u_lo=[-1.0], u_hi=[1.0], noise=sig)
    x0 = np.array([0.3, -0.2, 0.5, 0.1])
    cand = o.with_user(o.grid_candidates(sys, [9]), [0.25], 1)
    H = 8
    traj, _ = o.rollout(sys, K, x0, cand, H, early_exit=False, noise_key=(11, 12, 13))
    zs = [o.process_noise(11, 12, 13, np.arange(cand.shape[0]), s, 4) for s in range(1, H + 1)]
    for s in range(1, H + 1):
        exp = (np.linalg.matrix_power(A, s) @ x0)[None, :] + \
            np.outer(cand[:, 0, 0], sum(np.linalg.matrix_power(A, j) @ B[:, 0] for j in range(s)))
        for k in range(1, s + 1):
            exp = exp + (zs[k - 1] * sig[None, :]) @ np.linalg.matrix_power(A, s - k).T
        np.testing.assert_allclose(traj[s - 1], exp, rtol=1e-11, atol=1e-12)
    # zero noise reproduces the deterministic rollout
    sys0 = o.System("linear", 4, 1, box=[], u_lo=[-1.0], u_hi=[1.0], noise=np.zeros(4))
    t0, _ = o.rollout(sys0, K, x0, cand, H, early_exit=False, noise_key=(11, 12, 13))
    t1, _ = o.rollout(o.System("linear", 4, 1, box=[], u_lo=[-1.0], u_hi=[1.0]), K, x0, cand, H, early_exit=False)
    np.testing.assert_array_equal(t0, t1)


# ------------------------------------------- lifted (whole-horizon) form ------
def test_lifted_fit_identity_basis_is_the_plant_with_the_input_held():
    """With psi = [x; u] and the input held over a step, psi(x', u) = psi(x, u) K
    has the exact solution K = [[A^T, 0], [B^T, I]] (rows: x then u)."""
    A, B, X, U, Y = _linear_case()
    K, info = o.fit_lifted("linear", X, U, Y)
    expect = np.block([[A.T, np.zeros((4, 1))], [B.T, np.eye(1)]])
    np.testing.assert_allclose(K, expect, rtol=0, atol=1e-11)
    assert np.all(info["resid_rms"] < 1e-12)


@pytest.mark.parametrize("seed", [11, 13, 17])
def test_lifted_rollout_is_exact_for_a_linear_plant_in_the_quadratic_basis(seed):
    """The span of 1, w and all degree-2 monomials of w = [x; u] is closed under
    x' = A x + B u with u held (each product of two affine forms is again in
    the span), so the fitted lifted operator is exact and its rollout follows
    the closed form A^s x0 + sum_{j<s} A^j B u for 30 steps."""
    A, B, X, U, Y = _linear_case(seed)
    K, info = o.fit_lifted("balance_bot", X, U, Y)
    assert np.all(info["resid_rms"] < 1e-12)
    sysb = o.System("balance_bot", 4, 1, box=[], u_lo=[-1.0], u_hi=[1.0])
    x0 = np.array([0.3, -0.2, 0.5, 0.1])
    cand = o.with_user(o.grid_candidates(sysb, [9]), [0.25], 1)
    H = 30
    traj, fv = o.rollout_lifted(sysb, K, x0, cand, H, early_exit=False)
    for s, (a, b) in enumerate(_affine_in_u(A, B, x0, H), start=1):
        np.testing.assert_allclose(traj[s - 1], a[None, :] + np.outer(cand[:, 0, 0], b), rtol=0, atol=1e-10)
    assert np.all(fv == H + 1)


def test_lifted_state_columns_are_the_relift_fit(bb_model):
    """The state columns of the lifted operator solve the same least-squares
    problem as the re-lifting model's K (same rows, same targets x_{t+1}), so
    they agree, and the first predicted step of both rollouts is the same."""
    K, _, (X, U, Y) = bb_model
    KL, _ = o.fit_lifted("balance_bot", X, U, Y)
    cols = o.state_columns("balance_bot", 4)
    np.testing.assert_allclose(KL[:, cols], K, rtol=0, atol=1e-9 * np.max(np.abs(K)))
    assert list(o.state_columns("race_car", 6)) == [1, 2, 3, 4, 5, 6]
    assert list(o.state_columns("linear", 3)) == [0, 1, 2]
    sys = _bb()
    x0 = synth.balance_bot_states(1, seed=4)[0]
    cand = o.with_user(o.grid_candidates(sys, [50]), [1.0], 1)
    t1, _ = o.rollout(sys, K, x0, cand, 1, early_exit=False)
    t2, _ = o.rollout_lifted(sys, KL, x0, cand, 1, early_exit=False)
    np.testing.assert_allclose(t2, t1, rtol=0, atol=1e-9)


@pytest.mark.parametrize("seed", range(4))
def test_lifted_tick_brute_force(bb_model, seed):
    """Tiny lifted ticks against a candidate-by-candidate evaluation: z = psi(x0,
    u) as a vector, z <- z K per step, state read off the state coordinates,
    box checks, then the first safe candidate in (cost, index) order."""
    _, _, (X, U, Y) = bb_model
    KL, _ = o.fit_lifted("balance_bot", X, U, Y)
    rng = np.random.default_rng(300 + seed)
    sys = _bb(theta=0.15, p=0.6)
    H = int(rng.integers(2, 9))
    N = int(rng.integers(4, 16))
    x0 = np.array([rng.uniform(-0.3, 0.3), rng.uniform(-1, 1), rng.uniform(-0.1, 0.1), rng.uniform(-1, 1)])
    u_h = rng.uniform(-5, 5, size=1)
    cand = o.with_user(o.uniform_candidates(sys, N, 1, seed, 0, 0), u_h, 1)
    res = o.tick_lifted(sys, KL, x0, u_h, cand, H)
    fvs, costs = [], []
    for i in range(N + 1):
        u = cand[i, 0, 0]
        w = [x0[0], x0[1], x0[2], x0[3], u]
        z = np.array([1.0] + w + [w[k] * w[l] for k in range(5) for l in range(k, 5)])
        first = H + 1
        for s in range(1, H + 1):
            z = z @ KL
            p, th = z[1], z[3]
            if first == H + 1 and not (abs(th) < 0.15 and abs(p) < 0.6):
                first = s
        fvs.append(first)
        costs.append(((u - u_h[0]) / 5.0) ** 2)
    order = sorted(range(N + 1), key=lambda i: (costs[i], i))
    safe = [i for i in order if fvs[i] == H + 1]
    expect = safe[0] if safe else sorted(range(N + 1), key=lambda i: (-fvs[i], costs[i], i))[0]
    np.testing.assert_array_equal(res["fv"], fvs)
    assert res["idx"] == expect


# ------------------------------------------------------ a basis given as data --
def test_custom_basis_hand_values():
    """Atoms [1, w_0, sin w_1, cos w_2] at w = (0.5, pi/6, pi/3): features
    1*1 = 1, w_0 sin w_1 = 0.25, sin w_1 cos w_2 = 0.25, w_0^2 = 0.25 and
    cos w_2 * 1 = 0.5."""
    b = o.Basis(atoms=(("one", 0), ("var", 0), ("sin", 1), ("cos", 2)),
                feats=((0, 0), (1, 2), (2, 3), (1, 1), (3, 0)))
    psi = o.lift(b, np.array([[0.5, math.pi / 6]]), np.array([[math.pi / 3]]))[0]
    np.testing.assert_allclose(psi, [1.0, 0.25, 0.25, 0.25, 0.5], rtol=0, atol=1e-15)
    assert o.basis_dim(b, 2, 1) == 5
    with pytest.raises(ValueError):
        o.state_columns(b, 2)  # no feature is x_1 itself
    b2 = o.Basis(atoms=(("one", 0), ("var", 1), ("var", 0)), feats=((0, 0), (2, 0), (0, 1)))
    assert list(o.state_columns(b2, 2)) == [1, 2]
