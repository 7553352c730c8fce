"""Pins of the oracle's basis selection (the sparsity-promoting ADMM of
Jovanovic, Schmid and Nichols 2014, applied to the library of random basis
functions of Sec. V-C-3) against facts that do not come from the oracle:
hand-computed shrinkage, the closed-form solution for an orthonormal design,
the optimality (KKT) conditions of the convex problem, the least-squares limit,
the all-zero solution above the critical penalty, and planted supports."""
import numpy as np
import pytest

import synth
from oracle import mpmi_oracle as o


def test_group_shrink_hand_values():
    V = np.array([[3.0, 4.0], [0.6, 0.8], [0.0, 0.0], [-6.0, 8.0]])
    out = o.group_shrink(V, 1.0)
    # norms 5, 1 (= kappa: dropped), 0, 10
    np.testing.assert_allclose(out, [[2.4, 3.2], [0.0, 0.0], [0.0, 0.0], [-5.4, 7.2]], rtol=1e-15, atol=0)
    assert np.all(out[1:3] == 0.0)
    # one column: the scalar soft threshold
    np.testing.assert_allclose(o.group_shrink(np.array([[-2.5], [0.3], [1.7]]), 0.5)[:, 0], [-2.0, 0.0, 1.2],
                               rtol=0, atol=1e-15)


def test_orthonormal_design_closed_form():
    """G = I: the problem separates per row, ||b||^2 - 2 b.a + gamma ||b||,
    whose minimiser is b = max(0, 1 - gamma / (2 ||a||)) a."""
    rng = np.random.default_rng(1)
    A = rng.normal(size=(7, 3))
    gamma = 2.0 * np.median(np.linalg.norm(A, axis=1))  # rows below the median norm drop
    B, _, _, (prim, dual) = o.sparse_admm(np.eye(7), A, gamma, rho=1.0, iters=400)
    nrm = np.linalg.norm(A, axis=1)
    want = np.maximum(0.0, 1.0 - gamma / (2.0 * nrm))[:, None] * A
    np.testing.assert_allclose(B, want, rtol=0, atol=1e-10)
    assert 0 < np.sum(np.any(want != 0, axis=1)) < 7  # some rows dropped, some kept
    assert prim < 1e-10 and dual < 1e-10


def _spd(rng, L):
    Q = rng.normal(size=(L, L))
    return Q @ Q.T / L + 0.05 * np.eye(L)


@pytest.mark.parametrize("seed", [2, 3])
def test_kkt_conditions_at_convergence(seed):
    """Optimality of J(B) + gamma sum ||B_f|| (J = tr B'GB - 2 tr B'A): for a
    kept row, 2 (GB - A)_f + gamma B_f / ||B_f|| = 0; for a dropped row,
    ||2 (GB - A)_f|| <= gamma."""
    rng = np.random.default_rng(seed)
    L, n = 9, 2
    G = _spd(rng, L)
    A = rng.normal(size=(L, n))
    gamma = 0.6 * np.max(np.linalg.norm(2 * A, axis=1))
    B, _, _, _ = o.sparse_admm(G, A, gamma, rho=1.0, iters=6000)
    grad = 2.0 * (G @ B - A)
    kept = np.any(B != 0, axis=1)
    assert 0 < kept.sum() < L
    for f in range(L):
        if kept[f]:
            r = grad[f] + gamma * B[f] / np.linalg.norm(B[f])
            assert np.linalg.norm(r) <= 1e-7 * gamma, (f, r)
        else:
            assert np.linalg.norm(grad[f]) <= gamma * (1 + 1e-7), f


def test_zero_penalty_is_least_squares():
    """gamma = 0: the iterates converge to the solution of the normal
    equations G B = A."""
    rng = np.random.default_rng(4)
    G = _spd(rng, 6)
    A = rng.normal(size=(6, 3))
    B, _, _, _ = o.sparse_admm(G, A, 0.0, rho=1.0, iters=3000)
    np.testing.assert_allclose(G @ B, A, rtol=0, atol=1e-9)


def test_penalty_above_critical_gives_zero():
    """gamma >= 2 max_f ||A_f||: B = 0 satisfies the optimality conditions
    (||2 (G 0 - A)_f|| <= gamma), and the unique minimiser is reached exactly
    (rows shrunk to zero are exactly zero)."""
    rng = np.random.default_rng(5)
    G = _spd(rng, 8)
    A = rng.normal(size=(8, 2))
    gamma = 2.0 * np.max(np.linalg.norm(A, axis=1)) * 1.01
    B, _, _, _ = o.sparse_admm(G, A, gamma, rho=1.0, iters=3000)
    assert np.all(B == 0.0)


def test_planted_support_recovered_and_polished():
    """Data made exactly by 5 functions of a 40-function random library (no
    noise; inputs and states independent, uniform on symmetric ranges; the 5
    -- x0, x2, u, x1 sin x0, sin x0 cos x1 -- have zero mean, so none of them
    is nearly a multiple of the library's near-constant functions): penalties
    from 1e-3 to 0.3 keep exactly those 5, and the polishing least squares
    returns their coefficients; a penalty above the critical one keeps none."""
    atoms, feats = synth.random_library(3, 1, 40, seed=9)
    lib = o.Basis(atoms=tuple(atoms), feats=tuple(feats))
    rng = np.random.default_rng(10)
    T = 4000
    X = rng.uniform(-1.5, 1.5, size=(T, 3))
    U = rng.uniform(-1.0, 1.0, size=(T, 1))
    S = np.array([1, 3, 4, 12, 25])
    assert [(lib.atoms[a], lib.atoms[b]) for a, b in (lib.feats[f] for f in S)] == [
        (("var", 0), ("one", 0)), (("var", 2), ("one", 0)), (("var", 3), ("one", 0)), (("var", 1), ("sin", 0)),
        (("sin", 0), ("cos", 1))]
    Ktrue = rng.normal(size=(S.size, 3))
    Y = o.lift(lib, X, U)[:, S] @ Ktrue
    for gamma in (1e-3, 3e-2, 0.3):
        r = o.select_basis(lib, X, U, Y, gamma=gamma, rho=1.0, iters=3000)
        assert list(r["support"]) == list(S), gamma
        np.testing.assert_allclose(r["K_polished"], Ktrue, rtol=0, atol=1e-9)
    G, A, _, _ = o.selection_problem(lib, X, U, Y)
    r0 = o.select_basis(lib, X, U, Y, gamma=2.0 * np.max(np.linalg.norm(A, axis=1)) * 1.01, iters=3000)
    assert r0["support"].size == 0 and r0["K_polished"] is None


def test_selection_problem_scaling():
    """G has a unit diagonal (RMS-scaled columns) and A's rows are the
    scaled correlations of each function with the scaled targets."""
    atoms, feats = synth.random_library(2, 1, 12, seed=3)
    lib = o.Basis(atoms=tuple(atoms), feats=tuple(feats))
    rng = np.random.default_rng(2)
    X, U = rng.normal(size=(500, 2)), rng.normal(size=(500, 1))
    Y = rng.normal(size=(500, 2)) * [3.0, 0.1]
    G, A, s, sy = o.selection_problem(lib, X, U, Y)
    np.testing.assert_allclose(np.diag(G), 1.0, rtol=1e-14)
    Psi = o.lift(lib, X, U)
    np.testing.assert_allclose(A[4, 1], np.mean(Psi[:, 4] * Y[:, 1]) / (s[4] * sy[1]), rtol=1e-12)


def test_random_library_shape():
    atoms, feats = synth.random_library(4, 1, 50, seed=0)
    assert len(feats) == 50 and len(set(tuple(sorted(f)) for f in feats)) == 50
    assert feats[0] == (0, 0) and [f for f in feats[1:6]] == [(1 + k, 0) for k in range(5)]
    atoms_r, feats_r = synth.random_library(6, 2, 150, seed=0)
    assert len(atoms_r) == 25 and len(feats_r) == 150
