"""GPU parity of the sparsity-promoting basis selection (koopman_select_basis)
against the FP64 oracle: the ADMM's coefficients and supports over a penalty
path, the planted support and its polished model, and the paper's library
sizes (50 random functions for the cart-pole, 150 for the race car) carried
through the polishing fit into a tick on the selected basis."""
import sys
import time

import numpy as np
import pytest
import torch

import synth
from oracle import mpmi_oracle as o
from paper_1906_02318_amd import mpmi
from tests import workloads as W
from tests.parity import check_tick

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return mpmi.Context(0)


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def oracle_path(lib, X, U, Y, gammas, rho, iters):
    """Oracle B (unscaled), supports, residuals and each row's last shrink
    argument norm relative to the threshold (for the band of ambiguous rows)."""
    G, A, s, sy = o.selection_problem(lib, X, U, Y)
    out = []
    for g in gammas:
        B, K, Lam, res = o.sparse_admm(G, A, g, rho, iters)
        lam_prev = Lam - rho * (K - B)
        V = K + lam_prev / rho
        rel = np.abs(np.linalg.norm(V, axis=1) - g / rho) / max(g / rho, 1e-300)
        out.append(dict(B=B * sy[None, :] / s[:, None], support=np.any(B != 0, axis=1), res=res, rel=rel))
    return out


def compare(tag, gpu_B, gpu_sup, gpu_res, ref, gammas):
    sizes = []
    for k, r in enumerate(ref):
        Bg = gpu_B[k]
        scale = max(np.max(np.abs(r["B"])), 1e-12)
        err = np.max(np.abs(Bg - r["B"])) / scale
        amb = r["rel"] < 1e-8
        mism = (gpu_sup[k].astype(bool) != r["support"]) & ~amb
        assert not mism.any(), f"{tag} gamma {gammas[k]}: supports differ at {np.nonzero(mism)[0]}"
        assert err <= 1e-8, f"{tag} gamma {gammas[k]}: B differs by {err:.3e} of its largest entry"
        np.testing.assert_allclose(gpu_res[k], r["res"], rtol=1e-6, atol=1e-12 * max(1.0, r["res"][0]))
        sizes.append(int(gpu_sup[k].sum()))
    log(f"[select] {tag}: supports along the path {sizes}")
    return sizes


def test_select_planted_support_and_polish(ctx):
    """The planted case of the oracle's pins (5 of 40 functions make the data
    exactly): GPU coefficients and supports equal the oracle's over a penalty
    path; the selected basis polished by koopman_fit on the GPU returns the
    planted coefficients."""
    atoms, feats = synth.random_library(3, 1, 40, seed=9)
    lib_o = o.Basis(atoms=tuple(atoms), feats=tuple(feats))
    rng = np.random.default_rng(10)
    T = 4000
    X = rng.uniform(-1.5, 1.5, size=(T, 3))
    U = rng.uniform(-1.0, 1.0, size=(T, 1))
    S = np.array([1, 3, 4, 12, 25])
    Ktrue = rng.normal(size=(S.size, 3))
    Y = o.lift(lib_o, X, U)[:, S] @ Ktrue
    G, A, _, _ = o.selection_problem(lib_o, X, U, Y)
    gcrit = 2.0 * np.max(np.linalg.norm(A, axis=1))
    gammas = [1e-3, 3e-2, 0.3, 1.01 * gcrit]
    lib = mpmi.library_desc(3, 1, atoms, feats)
    B, sup, res = mpmi.koopman_select_basis(ctx, lib, dev(X), dev(U), dev(Y), gammas, rho=1.0, iters=3000)
    ref = oracle_path(lib_o, X, U, Y, gammas, 1.0, 3000)
    sizes = compare("planted", B.cpu().numpy(), sup.cpu().numpy(), res, ref, gammas)
    assert sizes == [5, 5, 5, 0]
    assert list(np.nonzero(sup.cpu().numpy()[1])[0]) == list(S)
    sel_feats = [feats[f] for f in S]
    sysg = mpmi.custom_system(3, 1, atoms, sel_feats, [], [-1.0], [1.0])
    Kp, _ = mpmi.koopman_fit(ctx, sysg, dev(X), dev(U), dev(Y))
    np.testing.assert_allclose(Kp.cpu().numpy(), Ktrue, rtol=0, atol=1e-9)


@pytest.mark.parametrize("system", ["balance_bot", "race_car"])
def test_select_paper_library_sizes(ctx, system):
    """The paper's library sizes on the synthetic plants' transitions: 50
    random functions for the cart-pole (T = 5,000), 150 for the race car
    (T = 50,000); a 16-penalty path in one call against the oracle; the
    smallest penalty whose support fits the paper's selected count (6 / 26)
    gives the basis that koopman_fit polishes on the GPU (against the oracle's
    polishing fit), and ticks on that basis agree with the oracle."""
    if system == "balance_bot":
        n, m, L, target = 4, 1, 50, 6
        X, U, Y = W.bb_model()[2]
    else:
        n, m, L, target = 6, 2, 150, 26
        X, U, Y = W.rc_model()[2]
    atoms, feats = synth.random_library(n, m, L, seed=0)
    lib_o = o.Basis(atoms=tuple(atoms), feats=tuple(feats))
    G, A, _, _ = o.selection_problem(lib_o, X, U, Y)
    gcrit = 2.0 * np.max(np.linalg.norm(A, axis=1))
    gammas = list(gcrit * np.logspace(-4, 0, 16))
    iters = 500
    lib = mpmi.library_desc(n, m, atoms, feats)
    Xd, Ud, Yd = dev(X), dev(U), dev(Y)
    mpmi.koopman_select_basis(ctx, lib, Xd, Ud, Yd, gammas, rho=1.0, iters=iters)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B, sup, res = mpmi.koopman_select_basis(ctx, lib, Xd, Ud, Yd, gammas, rho=1.0, iters=iters)
    torch.cuda.synchronize()
    log(f"[select] {system}: {L} functions, T = {X.shape[0]:,}, {len(gammas)} penalties x {iters} ADMM iterations: "
        f"{(time.perf_counter() - t0) * 1e3:.2f} ms call to return")
    ref = oracle_path(lib_o, X, U, Y, gammas, 1.0, iters)
    sizes = compare(system, B.cpu().numpy(), sup.cpu().numpy(), res, ref, gammas)
    k = next(i for i, sz in enumerate(sizes) if 0 < sz <= target)
    S = np.nonzero(sup.cpu().numpy()[k])[0]
    sel_feats = [feats[f] for f in S]
    basis_o = o.Basis(atoms=tuple(atoms), feats=tuple(sel_feats))
    K_o, info = o.fit(basis_o, X, U, Y)
    if system == "balance_bot":
        so = W.bb_oracle_system()
        so = o.System(basis_o, 4, 1, box=so.box, u_lo=so.u_lo, u_hi=so.u_hi)
        sysg = mpmi.custom_system(4, 1, atoms, sel_feats, [(2, W.BB_THETA, 0.0), (0, W.BB_P, 0.0)], [-5.0], [5.0],
                                  eps32_box=[1e-4, 4e-4])
        grid, H, xs, us, eps = [1024], 20, synth.balance_bot_states(10, seed=1), \
            synth.uniform_user(10, [-5.0], [5.0], seed=2), [1e-4, 4e-4]
    else:
        tr = W.rc_track()
        so = o.System(basis_o, 6, 2, box=[(4, W.RC_VY, 0.0)], track=W.track_dict(tr), u_lo=synth.RC_U_LO,
                      u_hi=synth.RC_U_HI)
        sysg = mpmi.custom_system(6, 2, atoms, sel_feats, [(4, W.RC_VY, 0.0)], synth.RC_U_LO, synth.RC_U_HI,
                                  track=W.track_dict(tr), eps32_box=[3e-4], eps32_track=2e-3)
        grid, H, xs, us, eps = [64, 64], 30, synth.race_car_states(6, tr, seed=1), \
            synth.uniform_user(6, synth.RC_U_LO, synth.RC_U_HI, seed=2), [1e-3, 1e-3]
    Kg, cond = mpmi.koopman_fit(ctx, sysg, dev(X), dev(U), dev(Y))
    Kg = Kg.cpu().numpy()
    Psi = o.lift(basis_o, X, U)
    dp = np.max(np.abs(Psi @ Kg - Psi @ K_o)) / np.max(np.abs(Y))
    log(f"[select] {system}: gamma {gammas[k]:.4g} keeps {S.size} of {L} functions; polished fit cond "
        f"{cond:.3g}, prediction vs oracle {dp:.2e}, one-step residual RMS {info['resid_rms']}")
    assert dp <= 1e-8
    model = mpmi.mpmi_model_pack(ctx, sysg, dev(K_o))
    N = int(np.prod(grid))
    kinds = []
    for t in range(len(xs)):
        x, u = W.f32(xs[t]), W.f32(us[t])
        fv = torch.empty(N + 1, dtype=torch.int16, device="cuda")
        rec = mpmi.mpmi_tick(ctx, model, mpmi.tick_desc(N, H, gen=mpmi.GEN_GRID, grid=grid), dev(x, torch.float32),
                             dev(u, torch.float32), first_violation=fv)
        r = check_tick(so, K_o, x, u, o.with_user(o.grid_candidates(so, grid), u, 1), H, mpmi.decode_selection(rec),
                       fv.cpu().numpy(), eps, label=f"selected-basis tick {t}")
        kinds.append(r["kind"])
    log(f"[select] {system}: ticks on the selected basis {kinds}")
