"""GPU parity of the control tick against the FP64 oracle (MI355X only).

Every test drives the HIP path through the C ABI (Python binding) and checks
the result against the oracle on the same seeded inputs, with the rules of
tests/parity.py.
"""
import ctypes
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import mpmi_oracle as o
from paper_1906_02318_amd import mpmi
from tests import workloads as W
from tests.parity import agreed, agreement, ambiguous, check_selection, check_tick, eps64, oracle_chunk, \
    recheck64_eps, replay_job, rollout_rel_err, tally

pytestmark = pytest.mark.gpu

# eps bands for FP32 verdicts (rounding of FP32 rollouts against FP64):
# balance bot theta 1e-4 rad, p 4e-4 m; race car v_y 1e-3 m/s, track 1e-3 m.
EPS_BB = [1e-4, 4e-4]
EPS_RC = [1e-3, 1e-3]


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return mpmi.Context(0)


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def to_sm(cand64):
    """Oracle layout (Nc, S, m) -> library layout (S, m, Nc), float32."""
    return np.ascontiguousarray(np.transpose(cand64, (1, 2, 0))).astype(np.float32)


@pytest.fixture(scope="module")
def bb(ctx):
    K = W.bb_model()[0]
    return W.bb_oracle_system(), mpmi.mpmi_model_pack(ctx, mpmi.balance_bot_system(), dev(K, torch.float64)), K


@pytest.fixture(scope="module")
def rc(ctx):
    K = W.rc_model()[0]
    tr = W.track_dict(W.rc_track())
    sys_g = mpmi.race_car_system(tr)
    return W.rc_oracle_system(W.rc_track()), mpmi.mpmi_model_pack(ctx, sys_g, dev(K, torch.float64)), K


# --------------------------------------------------------------- candidates --
@pytest.mark.parametrize("case", ["bb_grid", "rc_grid", "rc_uniform", "bb_uniform_seq"])
def test_generated_candidates_bitexact(ctx, bb, rc, case):
    log(f"[gen] {case}")
    if case == "bb_grid":
        so, model, _ = bb
        desc = mpmi.tick_desc(1024, 20, gen=mpmi.GEN_GRID, grid=[1024])
        u_h = [1.2345]
        ref = o.with_user(o.grid_candidates(so, [1024]), W.f32(u_h), 1)
    elif case == "rc_grid":
        so, model, _ = rc
        desc = mpmi.tick_desc(128 * 128, 60, gen=mpmi.GEN_GRID, grid=[128, 128])
        u_h = [0.05, -1.5]
        ref = o.with_user(o.grid_candidates(so, [128, 128]), W.f32(u_h), 1)
    elif case == "rc_uniform":
        so, model, _ = rc
        desc = mpmi.tick_desc(5000, 60, gen=mpmi.GEN_UNIFORM, n_seg=3, seed=9, tick=17, loop=3)
        u_h = [-0.3, 2.0]
        ref = o.with_user(o.uniform_candidates(so, 5000, 3, 9, 17, 3), W.f32(u_h), 3)
    else:
        so, model, _ = bb
        desc = mpmi.tick_desc(10240, 50, gen=mpmi.GEN_UNIFORM, n_seg=5, seed=4, tick=123456789012, loop=0)
        u_h = [3.5]
        ref = o.with_user(o.uniform_candidates(so, 10240, 5, 4, 123456789012, 0), W.f32(u_h), 5)
    got = mpmi.mpmi_generate_candidates(ctx, model, desc, dev(u_h, torch.float32)).cpu().numpy()
    np.testing.assert_array_equal(got, to_sm(ref))


# ------------------------------------------------------------------ rollout --
@pytest.mark.parametrize("system", ["bb", "rc"])
def test_rollout_batch_parity(ctx, bb, rc, system):
    if system == "bb":
        so, model, K = bb
        H, S, N = 50, 5, 4095
        xs = synth.balance_bot_states(3, seed=21)
        floors = W.bb_floors()
    else:
        so, model, K = rc
        H, S, N = 60, 1, 2047
        xs = synth.race_car_states(3, W.rc_track(), seed=21)
        floors = W.rc_floors()
    worst = 0.0
    for t, x0 in enumerate(xs):
        x0 = W.f32(x0)
        cand = o.with_user(o.uniform_candidates(so, N, S, 31, t, 0), so.u_lo * 0.5 + so.u_hi * 0.25, S)
        cand = W.f32(cand)
        log(f"[rollout] {system} tick {t} N={N} H={H} S={S}")
        traj = mpmi.rollout_batch(ctx, model, dev(x0, torch.float32), dev(to_sm(cand), torch.float32), H)
        ref, _ = o.rollout(so, K, x0, cand, H, early_exit=False)
        err = rollout_rel_err(traj.cpu().numpy().transpose(0, 2, 1), ref, floors, comp_axis=2)
        worst = max(worst, err)
    log(f"[rollout] {system} max relative error vs FP64: {worst:.3e}")
    assert worst <= 1e-4


# --------------------------------------------------------------- safe_mask --
@pytest.mark.parametrize("system,H", [("bb", 30), ("rc", 40), ("rc", 3), ("linear", 1), ("linear", 9)])
def test_safe_mask_on_synthetic_trajectories(ctx, bb, rc, system, H):
    """The kernel loads four steps ahead of its checks: horizons that end
    inside such a group (1, 3, 9, 30) reread in-range steps and drop them.
    The linear system (n = 3 of 8 component slots) rereads component n - 1
    for the missing components."""
    rng = np.random.default_rng(77 + H)
    Nc = 3001
    if system == "bb":
        so, model, _ = bb
        n = 4
        traj = rng.normal(0.0, [1.0, 1.0, 0.25, 1.0], size=(H, Nc, n))
    elif system == "linear":
        n = 3
        so = o.System("linear", n, 1, box=[(0, float(W.f32(1.0)), 0.0), (2, float(W.f32(0.5)), float(W.f32(0.125)))],
                      u_lo=[-1.0], u_hi=[1.0])
        sys_g = mpmi.linear_system(n, 1, [(0, 1.0, 0.0), (2, 0.5, 0.125)], [-1.0], [1.0])
        K = torch.zeros((n + 1, n), dtype=torch.float64, device="cuda")
        model = mpmi.mpmi_model_pack(ctx, sys_g, K)
        traj = rng.normal(0.0, [0.45, 5.0, 0.18], size=(H, Nc, n))
    else:
        so, model, _ = rc
        n = 6
        tr = W.rc_track()
        phi = rng.uniform(0, 2 * np.pi, size=(H, Nc))
        rho = tr.centre_radius(phi) + rng.uniform(-3.3, 3.3, size=(H, Nc))
        traj = np.stack([rho * np.cos(phi), rho * np.sin(phi), rng.normal(size=(H, Nc)), rng.normal(size=(H, Nc)),
                         rng.uniform(-2.2, 2.2, size=(H, Nc)), rng.normal(size=(H, Nc))], axis=2)
    traj[:, 5, 0] = np.nan  # a NaN state is unsafe
    traj = W.f32(traj)
    log(f"[mask] {system} H={H} Nc={Nc}")
    fv, mm = mpmi.safe_mask(ctx, model, dev(np.transpose(traj, (0, 2, 1)), torch.float32))
    fv, mm = fv.cpu().numpy().astype(np.int64), mm.cpu().numpy().astype(np.float64)
    with np.errstate(invalid="ignore"):
        M = o.margins(so, traj.reshape(H * Nc, n)).reshape(H, Nc, -1)
        unsafe = ~np.all(M > 0, axis=2)
    fv_o = np.where(unsafe.any(axis=0), unsafe.argmax(axis=0) + 1, H + 1)
    Mmin = np.min(M, axis=2)
    near = np.abs(Mmin) < 2e-5
    upto = np.minimum(np.minimum(fv, fv_o), H)
    amb = np.any(near & (np.arange(1, H + 1)[:, None] <= upto[None, :]), axis=0)
    assert np.all((fv == fv_o) | amb)
    assert fv[5] == 1 and np.isnan(mm[5])
    ok = ~amb & (fv == fv_o)
    least = np.array([np.min(Mmin[: min(f, H), c]) for c, f in enumerate(fv_o)])
    fin = ok & np.isfinite(least)
    np.testing.assert_allclose(mm[fin], least[fin], rtol=0, atol=2e-5)


# ------------------------------------------------------------------ select --
@pytest.mark.parametrize("case", ["mixed", "user_safe", "none_safe", "ragged_large", "million"])
def test_select_min_intervention_parity(ctx, bb, rc, case):
    """The million case has more candidates than the launch has lanes: each
    lane scans several, the last pass ragged."""
    rng = np.random.default_rng({"mixed": 1, "user_safe": 2, "none_safe": 3, "ragged_large": 4, "million": 5}[case])
    so, model, _ = rc
    H, S = 60, 2
    Nc = {"ragged_large": 200_001, "million": 1_048_577}.get(case, 4097)
    cand = W.f32(o.with_user(o.uniform_candidates(so, Nc - 1, S, 5, 0, 0), [0.1, 0.4], S))
    fv = rng.integers(1, H + 2, size=Nc)
    if case == "user_safe":
        fv[0] = H + 1
    if case == "none_safe":
        fv = rng.integers(1, H + 1, size=Nc)
    if case == "mixed":
        fv[0] = 7
    log(f"[select] {case} Nc={Nc}")
    rec = mpmi.select_min_intervention(ctx, model, dev(to_sm(cand), torch.float32), dev(fv, torch.int16), H,
                                       dev([0.1, 0.4], torch.float32), loop=5)
    sel = mpmi.decode_selection(rec)
    ref = o.select(so, cand, fv, H, W.f32([0.1, 0.4]))
    cost = o.cost(so, cand, W.f32([0.1, 0.4]))
    assert sel["status"] == ref["status"] and sel["n_safe"] == ref["n_safe"]
    assert sel["idx"] == ref["idx"] or (fv[sel["idx"]] == fv[ref["idx"]] and
                                        abs(cost[sel["idx"]] - cost[ref["idx"]]) <= 1e-6 * cost[ref["idx"]])
    assert sel["first_violation"] == fv[sel["idx"]]
    if case == "user_safe":
        assert sel["idx"] == 0 and sel["deviation"] == 0.0 and sel["cost"] == 0.0


# ------------------------------------------------------------- fused ticks --
def run_ticks(ctx, model, so, K, xs, uhs, desc_fn, H, eps, label, cand_fn):
    kinds = {}
    for t, (x, u) in enumerate(zip(xs, uhs)):
        x, u = W.f32(x), W.f32(u)
        desc = desc_fn(t)
        fv = torch.empty(desc.n_cand + 1, dtype=torch.int16, device="cuda")
        rec = mpmi.mpmi_tick(ctx, model, desc, dev(x, torch.float32), dev(u, torch.float32), first_violation=fv)
        sel = mpmi.decode_selection(rec)
        res = check_tick(so, K, x, u, cand_fn(t, u), H, sel, fv.cpu().numpy(), eps, label=f"{label} tick {t}")
        kinds[res["kind"]] = kinds.get(res["kind"], 0) + 1
        kinds["zero_intervention"] = kinds.get("zero_intervention", 0) + int(res["zero_intervention"])
        kinds["no_safe"] = kinds.get("no_safe", 0) + int(res["status"] != o.STATUS_OK)
    log(f"[tick] {label}: {kinds}")
    return kinds


def test_tick_balance_bot_small_all_ticks(ctx, bb):
    """Cart-pole, N = 1,024 grid + u_h, H = 20: every one of 1,000 ticks."""
    so, model, K = bb
    xs = synth.balance_bot_states(1000, seed=1)
    uhs = synth.uniform_user(1000, [-5.0], [5.0], seed=2)
    grid = o.grid_candidates(so, [1024])
    kinds = run_ticks(ctx, model, so, K, xs, uhs, lambda t: mpmi.tick_desc(1024, 20, gen=mpmi.GEN_GRID, grid=[1024]),
                      20, EPS_BB, "bb N=1024 H=20", lambda t, u: o.with_user(grid, u, 1))
    assert agreed(kinds) >= 0.999 * 1000


def test_tick_balance_bot_sequences(ctx, bb):
    """Cart-pole at real-time size: N = 10,240 sequences of 5 segments, H = 50 (sampled ticks)."""
    so, model, K = bb
    T = 8
    xs = synth.balance_bot_states(T, seed=41)
    uhs = synth.uniform_user(T, [-5.0], [5.0], seed=42)
    desc_fn = lambda t: mpmi.tick_desc(10240, 50, gen=mpmi.GEN_UNIFORM, n_seg=5, seed=4, tick=t)
    cand_fn = lambda t, u: o.with_user(o.uniform_candidates(so, 10240, 5, 4, t, 0), u, 5)
    run_ticks(ctx, model, so, K, xs, uhs, desc_fn, 50, EPS_BB, "bb N=10240 S=5 H=50", cand_fn)


def test_tick_race_car(ctx, rc):
    """Race car, N = 16,384 (128 x 128 grid) + u_h, H = 60 (sampled ticks)."""
    so, model, K = rc
    T = 6
    xs = synth.race_car_states(T, W.rc_track(), seed=1)
    uhs = synth.uniform_user(T, synth.RC_U_LO, synth.RC_U_HI, seed=2)
    grid = o.grid_candidates(so, [128, 128])
    desc_fn = lambda t: mpmi.tick_desc(128 * 128, 60, gen=mpmi.GEN_GRID, grid=[128, 128])
    run_ticks(ctx, model, so, K, xs, uhs, desc_fn, 60, EPS_RC, "rc N=16384 H=60", lambda t, u: o.with_user(grid, u, 1))


def test_tick_race_car_high_harmonic_track_and_stacked_boxes(ctx, rc):
    """Race car on a track with harmonics up to the eighth (the degree-8 track
    polynomial) and three boxes, two of them on v_y (the least limit binds)
    and one on the yaw rate."""
    so0, _, K = rc
    tr = synth.Track(amp=np.array([1.0, 0.5, 0.3, 0.2]), freq=np.array([3, 5, 7, 8]),
                     phase=np.random.default_rng(11).uniform(0.0, 2 * np.pi, size=4))
    td = W.track_dict(tr)
    boxes = [(4, float(W.f32(2.0)), 0.0), (4, float(W.f32(1.2)), 0.0), (5, float(W.f32(0.5)), 0.0)]
    so = o.System("race_car", 6, 2, box=boxes, track=td, u_lo=synth.RC_U_LO, u_hi=synth.RC_U_HI)
    sys_g = mpmi._sys(mpmi.BASIS_RACE_CAR, 6, 2, boxes, synth.RC_U_LO, synth.RC_U_HI, track=td,
                      eps_box=[0.02] * 3, eps_track=0.02)
    model = mpmi.mpmi_model_pack(ctx, sys_g, dev(K, torch.float64))
    T = 6
    xs = synth.race_car_states(T, tr, seed=4, offset=1.5, vy=(-0.3, 0.3), r=(-0.2, 0.2))
    uhs = synth.uniform_user(T, synth.RC_U_LO, synth.RC_U_HI, seed=5)
    grid = o.grid_candidates(so, [96, 96])
    run_ticks(ctx, model, so, K, xs, uhs, lambda t: mpmi.tick_desc(96 * 96, 40, gen=mpmi.GEN_GRID, grid=[96, 96]), 40,
              [1e-3, 1e-3, 1e-3, 1e-3], "rc degree-8 track, stacked boxes N=9216 H=40",
              lambda t, u: o.with_user(grid, u, 1))


@pytest.mark.parametrize("N,H,gen", [(0, 20, mpmi.GEN_UNIFORM), (777, 1, mpmi.GEN_UNIFORM), (1000, 33, mpmi.GEN_UNIFORM),
                                     (63, 5, mpmi.GEN_GRID), (65, 255, mpmi.GEN_GRID)])
def test_tick_edge_sizes(ctx, bb, N, H, gen):
    so, model, K = bb
    x, u = W.f32(synth.balance_bot_states(1, seed=5)[0]), W.f32([-4.0])
    desc = mpmi.tick_desc(N, H, gen=gen, grid=[N] if gen == mpmi.GEN_GRID else None, seed=8, tick=3)
    cand = (o.with_user(o.grid_candidates(so, [N]), u, 1) if gen == mpmi.GEN_GRID
            else o.with_user(o.uniform_candidates(so, N, 1, 8, 3, 0), u, 1))
    log(f"[edge] N={N} H={H} gen={gen}")
    fv = torch.empty(N + 1, dtype=torch.int16, device="cuda")
    rec = mpmi.mpmi_tick(ctx, model, desc, dev(x, torch.float32), dev(u, torch.float32), first_violation=fv)
    sel = mpmi.decode_selection(rec)
    assert sel["n_cand"] == N + 1
    check_tick(so, K, x, u, cand, H, sel, fv.cpu().numpy(), EPS_BB, label=f"edge N={N} H={H}")


@pytest.mark.parametrize("N", [7, 600, 8191, 8192])
def test_tick_selection_across_ticket_levels(ctx, bb, N):
    """The selection does not depend on how the workgroups publish: from one
    workgroup to more than the 128 that take their ticket on the slot itself
    (N = 8,191 at 64 lanes: 128 workgroups; 8,192: 129, each sub-slot's last
    workgroup taking the slot ticket), records and first violations are
    identical across launch shapes and agree with the oracle."""
    so, model, K = bb
    x, u = W.f32(synth.balance_bot_states(1, seed=6)[0]), W.f32([2.5])
    cand = o.with_user(o.uniform_candidates(so, N, 1, 9, 4, 0), u, 1)
    recs, fvs = [], []
    for block, lanes in ((64, 1), (256, 1), (64, 2), (128, 8)):
        desc = mpmi.tick_desc(N, 30, gen=mpmi.GEN_UNIFORM, seed=9, tick=4, block=block, lanes_per_cand=lanes)
        parts = ((N + 1) * lanes + block - 1) // block
        log(f"[tickets] N={N} block={block} lanes={lanes} workgroups={parts}")
        fv = torch.empty(N + 1, dtype=torch.int16, device="cuda")
        recs.append(mpmi.mpmi_tick(ctx, model, desc, dev(x, torch.float32), dev(u, torch.float32),
                                   first_violation=fv).cpu().numpy().tobytes())
        fvs.append(fv.cpu().numpy())
    assert all(r == recs[0] for r in recs)
    assert all(np.array_equal(f, fvs[0]) for f in fvs)
    sel = mpmi.decode_selection(torch.tensor(np.frombuffer(recs[0], np.uint8)))
    check_tick(so, K, x, u, cand, 30, sel, fvs[0], EPS_BB, label=f"tickets N={N}")


def test_tick_no_safe_candidate(ctx, bb):
    """Inflation larger than the bounds: nothing is safe; the fallback rule decides."""
    so0, _, K = bb
    so = W.bb_oracle_system(infl=0.45)
    model = mpmi.mpmi_model_pack(ctx, mpmi.balance_bot_system(infl=0.45), dev(K, torch.float64))
    xs = synth.balance_bot_states(5, seed=9)
    for t, x in enumerate(xs):
        x, u = W.f32(x), W.f32([2.5])
        desc = mpmi.tick_desc(500, 30, gen=mpmi.GEN_UNIFORM, seed=1, tick=t)
        fv = torch.empty(501, dtype=torch.int16, device="cuda")
        sel = mpmi.decode_selection(mpmi.mpmi_tick(ctx, model, desc, dev(x, torch.float32), dev(u, torch.float32),
                                                   first_violation=fv))
        cand = o.with_user(o.uniform_candidates(so, 500, 1, 1, t, 0), u, 1)
        res = check_tick(so, K, x, u, cand, 30, sel, fv.cpu().numpy(), EPS_BB, label=f"no-safe {t}")
        if res["status"] == o.STATUS_NO_SAFE:
            assert sel["status"] == mpmi.NO_SAFE and sel["n_safe"] == 0


def test_tick_nan_model_is_unsafe(ctx, bb):
    _, _, K = bb
    Kn = K.copy()
    Kn[3, 2] = np.nan
    model = mpmi.mpmi_model_pack(ctx, mpmi.balance_bot_system(), dev(Kn, torch.float64))
    desc = mpmi.tick_desc(256, 10, gen=mpmi.GEN_GRID, grid=[256])
    fv = torch.empty(257, dtype=torch.int16, device="cuda")
    sel = mpmi.decode_selection(mpmi.mpmi_tick(ctx, model, desc, dev([0.1, 0, 0.05, 0], torch.float32),
                                               dev([0.0], torch.float32), first_violation=fv))
    assert sel["status"] == mpmi.NO_SAFE and np.all(fv.cpu().numpy() == 1)


def test_tick_deterministic_across_block_sizes(ctx, rc):
    so, model, K = rc
    x = W.f32(synth.race_car_states(1, W.rc_track(), seed=13)[0])
    u = W.f32([0.35, 2.9])
    recs, fvs = [], []
    for block in (64, 128, 256, 512, 1024, 0):
        desc = mpmi.tick_desc(20000, 60, gen=mpmi.GEN_UNIFORM, seed=2, tick=9, block=block)
        fv = torch.empty(20001, dtype=torch.int16, device="cuda")
        for _ in range(2):  # repeated calls reuse the slot
            rec = mpmi.mpmi_tick(ctx, model, desc, dev(x, torch.float32), dev(u, torch.float32), first_violation=fv)
            recs.append(rec.cpu().numpy().tobytes())
        fvs.append(fv.cpu().numpy())
    assert all(r == recs[0] for r in recs)
    assert all(np.array_equal(f, fvs[0]) for f in fvs)


def test_tick_trajectory_store_matches_rollout(ctx, rc):
    """The fused tick's optional trajectory output equals rollout_batch up to each first violation."""
    so, model, K = rc
    x = W.f32(synth.race_car_states(1, W.rc_track(), seed=3)[0])
    u = W.f32([0.0, 1.0])
    N, H = 4095, 60
    desc = mpmi.tick_desc(N, H, gen=mpmi.GEN_UNIFORM, seed=6, tick=1)
    fv = torch.empty(N + 1, dtype=torch.int16, device="cuda")
    traj = torch.full((H, 6, N + 1), float("nan"), device="cuda")
    mpmi.mpmi_tick(ctx, model, desc, dev(x, torch.float32), dev(u, torch.float32), first_violation=fv, traj=traj)
    cand = mpmi.mpmi_generate_candidates(ctx, model, desc, dev(u, torch.float32))
    full = mpmi.rollout_batch(ctx, model, dev(x, torch.float32), cand, H)
    fvn = fv.cpu().numpy()
    steps = np.arange(1, H + 1)[:, None]
    valid = steps <= np.minimum(fvn, H)[None, :]
    a, b = traj.cpu().numpy(), full.cpu().numpy()
    np.testing.assert_array_equal(np.where(valid[:, None, :], a, 0), np.where(valid[:, None, :], b, 0))


# --------------------------------------------------------------------- fit --
@pytest.mark.parametrize("system", ["bb", "rc", "linear"])
def test_koopman_fit_parity(ctx, system):
    if system == "bb":
        K_o, info, (X, U, Y) = W.bb_model()
        sys_g = mpmi.balance_bot_system()
    elif system == "rc":
        K_o, info, (X, U, Y) = W.rc_model()
        sys_g = mpmi.race_car_system(W.track_dict(W.rc_track()))
    else:
        A, B = synth.linear_plant(4, 1, seed=11)
        X, U, Y = synth.linear_transitions(A, B, T=300, seed=12)
        K_o, info = o.fit("linear", X, U, Y)
        sys_g = mpmi.linear_system(4, 1, [], [-1.0], [1.0])
    log(f"[fit] {system} T={X.shape[0]}")
    K, cond = mpmi.koopman_fit(ctx, sys_g, dev(X, torch.float64), dev(U, torch.float64), dev(Y, torch.float64))
    K = K.cpu().numpy()
    kind = {"bb": "balance_bot", "rc": "race_car", "linear": "linear"}[system]
    Psi = o.lift(kind, X, U)
    # The normal equations lose cond(Psi_s)^2 * eps relative accuracy; compare predictions and coefficients.
    tol = max(1e-12, 50 * info["cond"] ** 2 * 2.2e-16)
    scale = np.sqrt(np.mean(Psi ** 2, axis=0))
    dk = np.max(np.abs((K - K_o) * scale[:, None])) / np.max(np.abs(K_o * scale[:, None]))
    dp = np.max(np.abs(Psi @ K - Psi @ K_o)) / np.max(np.abs(Y))
    log(f"[fit] {system}: cond oracle {info['cond']:.4g} gpu {cond:.4g}; scaled K rel diff {dk:.3e} (tol {tol:.1e}); "
        f"prediction rel diff {dp:.3e}")
    assert dk <= tol and dp <= 1e-9
    assert abs(cond - info["cond"]) <= 1e-3 * info["cond"]
    if system == "linear":
        np.testing.assert_allclose(K, np.vstack([A.T, B.T]), rtol=0, atol=1e-10)


def test_koopman_fit_deterministic_and_single_tile(ctx):
    """Repeated fits are bit-identical (fixed-order partial sums, no atomics);
    a fit from fewer rows than one Gram tile (T = 40 < 64) matches the
    oracle."""
    K_o, info, (X, U, Y) = W.rc_model()
    sys_g = mpmi.race_car_system(W.track_dict(W.rc_track()))
    Xd, Ud, Yd = dev(X, torch.float64), dev(U, torch.float64), dev(Y, torch.float64)
    runs = [mpmi.koopman_fit(ctx, sys_g, Xd, Ud, Yd) for _ in range(3)]
    for K, cond in runs[1:]:
        assert torch.equal(K, runs[0][0]) and cond == runs[0][1]
    A, B = synth.linear_plant(4, 1, seed=21)
    X, U, Y = synth.linear_transitions(A, B, T=40, seed=22)
    K_o, info = o.fit("linear", X, U, Y)
    K, cond = mpmi.koopman_fit(ctx, mpmi.linear_system(4, 1, [], [-1.0], [1.0]), dev(X, torch.float64),
                               dev(U, torch.float64), dev(Y, torch.float64))
    log(f"[fit] T=40: cond oracle {info['cond']:.4g} gpu {cond:.4g}")
    np.testing.assert_allclose(K.cpu().numpy(), K_o, rtol=0, atol=max(1e-12, 50 * info["cond"] ** 2 * 2.2e-16))
    assert abs(cond - info["cond"]) <= 1e-3 * info["cond"]


def test_koopman_fit_singular(ctx):
    rng = np.random.default_rng(0)
    X = rng.normal(size=(200, 3))
    U = X[:, :1].copy()  # input identical to the first state feature -> rank-deficient Gram matrix
    Y = rng.normal(size=(200, 3))
    with pytest.raises(mpmi.MpmiError) as e:
        mpmi.koopman_fit(ctx, mpmi.linear_system(3, 1, [], [-1.0], [1.0]), dev(X, torch.float64),
                         dev(U, torch.float64), dev(Y, torch.float64))
    assert e.value.status == mpmi.ESINGULAR


# ----------------------------------------------------------- error paths --
def test_invalid_arguments_rejected(ctx, bb):
    _, model, _ = bb
    x, u = dev([0, 0, 0, 0], torch.float32), dev([0.0], torch.float32)
    bad = [
        mpmi.tick_desc(10, 0),                                      # H = 0
        mpmi.tick_desc(10, 256),                                    # H > max
        mpmi.tick_desc(10, 5, gen=mpmi.GEN_GRID, grid=[11]),        # grid product != N
        mpmi.tick_desc(10, 5, gen=mpmi.GEN_GRID, grid=[10], n_seg=2),
        mpmi.tick_desc(10, 5, n_seg=9, gen=mpmi.GEN_UNIFORM),
        mpmi.tick_desc(10, 5, gen=mpmi.GEN_UNIFORM, loop=5000),
        mpmi.tick_desc(10, 5, gen=mpmi.GEN_UNIFORM, block=100),
        mpmi.tick_desc(10, 5, gen=mpmi.GEN_EXPLICIT),               # no cand
        mpmi.tick_desc(-1, 5, gen=mpmi.GEN_UNIFORM),
    ]
    for d in bad:
        with pytest.raises(mpmi.MpmiError) as e:
            mpmi.mpmi_tick(ctx, model, d, x, u)
        assert e.value.status == mpmi.EINVAL
    s = mpmi.balance_bot_system()
    s.n_state = 5
    with pytest.raises(mpmi.MpmiError):
        mpmi.mpmi_model_pack(ctx, s, dev(np.zeros((21, 4)), torch.float64))


def test_closed_loop_balance_bot_decisions_replayed(ctx, bb, oracle_pool):
    """Closed loop at real-time size (N = 10,240 five-segment sequences, H = 50)
    driven by FP32_RECHECK64 ticks: the plant advances with the applied input,
    the user input is an AR(1) walk.  All 1,000 decisions are replayed by the
    oracle on the visited (x_t, u_h, candidates): the re-rolled ticks' first
    violations equal the oracle's outside the FP64 band and at least 99.9% of
    their decisions agree.  The plain FP32 tick on the same inputs is held to
    the FP32 band and its agreement is reported."""
    so, model, K = bb
    T = 1000
    x = synth.balance_bot_states(1, seed=3)[0]
    user = synth.AR1User([-5.0], [5.0], rho=0.95, sigma=1.0, seed=2)
    jobs, rechecked = [], []
    for t in range(T):
        u = W.f32(user.next())
        xt = W.f32(x)
        results = []
        for prec, name in ((mpmi.PREC_FP32_RECHECK64, "fp32+fp64"), (mpmi.PREC_FP32, "fp32")):
            desc = mpmi.tick_desc(10240, 50, gen=mpmi.GEN_UNIFORM, n_seg=5, seed=4, tick=t, precision=prec)
            fv = torch.empty(10241, dtype=torch.int16, device="cuda")
            sel = mpmi.decode_selection(mpmi.mpmi_tick(ctx, model, desc, dev(xt, torch.float32),
                                                       dev(u, torch.float32), first_violation=fv))
            eps = recheck64_eps(so, sel, EPS_BB) if prec == mpmi.PREC_FP32_RECHECK64 else EPS_BB
            results.append((sel, fv.cpu().numpy(), f"closed loop tick {t} ({name})", eps))
        rechecked.append(results[0][0]["n_recheck"])
        jobs.append((so, K, xt, u, ("uniform", 10240, 5, 4, t, 0), 50, EPS_BB, None, results))
        x = synth.cartpole_step(x, np.array([results[0][0]["u_r"][0]], np.float64))[0]
        if abs(x[2]) > 0.5 or abs(x[0]) > 2.0:
            x = synth.balance_bot_states(1, seed=100 + t)[0]
        if t % 250 == 0:
            log(f"[closed loop] GPU tick {t}")
    out = list(oracle_pool.map(replay_job, jobs, chunksize=8))
    k64, k32 = tally([r[0] for r in out]), tally([r[1] for r in out])
    log(f"[closed loop] 1,000 ticks replayed; FP32+FP64 recheck: {k64}, agreement {agreed(k64) / T:.4f}, "
        f"re-rolled per tick mean {np.mean(rechecked):.1f} max {max(rechecked)}; plain FP32: {k32}, "
        f"agreement {agreed(k32) / T:.4f}")
    assert agreed(k64) >= 0.999 * T


def test_race_car_agreement_fp32_and_bf16x3(ctx, rc, oracle_pool):
    """Race car, N = 16,384 (128 x 128 grid) + u_h, H = 60, 100 ticks (states
    seed 1, user inputs seed 2): FP32 ticks and BF16X3 ticks (shared-coefficient
    contraction on BF16 matrix cores, hi/lo split, FP32 recheck of candidates
    within 0.02 of a constraint) against one oracle replay per tick; each form
    agrees with the oracle on at least 99.9% of the ticks.  Both forms are
    deterministic (two runs, identical records)."""
    so, model, K = rc
    T = 100
    xs = synth.race_car_states(T, W.rc_track(), seed=1)
    uhs = synth.uniform_user(T, synth.RC_U_LO, synth.RC_U_HI, seed=2)
    jobs, rechecks = [], []
    for t in range(T):
        x, u = W.f32(xs[t]), W.f32(uhs[t])
        results = []
        for prec, name in ((mpmi.PREC_FP32, "fp32"), (mpmi.PREC_BF16X3, "bf16x3")):
            desc = mpmi.tick_desc(128 * 128, 60, gen=mpmi.GEN_GRID, grid=[128, 128], precision=prec)
            fv = torch.empty(128 * 128 + 1, dtype=torch.int16, device="cuda")
            rec = mpmi.mpmi_tick(ctx, model, desc, dev(x, torch.float32), dev(u, torch.float32),
                                 first_violation=fv).cpu().numpy().tobytes()
            if t < 5:
                again = mpmi.mpmi_tick(ctx, model, desc, dev(x, torch.float32), dev(u, torch.float32)).cpu()
                assert again.numpy().tobytes() == rec, f"{name} tick is not deterministic"
            sel = mpmi.decode_selection(torch.tensor(np.frombuffer(rec, np.uint8)))
            if name == "bf16x3":
                rechecks.append(sel["n_recheck"])
            results.append((sel, fv.cpu().numpy(), f"{name} tick {t}"))
        jobs.append((so, K, x, u, ("grid", [128, 128]), 60, EPS_RC, None, results))
    log(f"[rc agreement] GPU ticks done; BF16X3 rechecked per tick: mean {np.mean(rechecks):.0f}, "
        f"max {max(rechecks)}")
    out = list(oracle_pool.map(replay_job, jobs))
    for k, name in enumerate(("fp32", "bf16x3")):
        kinds = tally([r[k] for r in out])
        log(f"[rc agreement] {name}: {kinds}; agreement {agreed(kinds) / T:.4f}")
        assert agreed(kinds) >= 0.999 * T, name


def test_full_size_race_car_sampled_parity_and_properties(ctx, rc, oracle_pool):
    """Bench configuration (race car, 1024 x 1024 grid + u_h, H = 60, default
    launch shape), 3 ticks: the selection record (index, status, safe count)
    is the selection rule over the kernel's whole first-violation vector;
    first violations of ~3,000 sampled candidates (plus the chosen one)
    against the oracle; on the first tick the oracle rolls out all 1,048,577
    candidates (in slices across worker processes) and every first violation
    and the decision are compared.  Properties at full size: the mask is
    monotone under inflation and a safe user input passes unchanged."""
    so, model, K = rc
    N = 1024 * 1024
    H = 60
    rng = np.random.default_rng(21)
    xs = synth.race_car_states(3, W.rc_track(), seed=1)
    uhs = synth.uniform_user(3, synth.RC_U_LO, synth.RC_U_HI, seed=2)
    grid = o.grid_candidates(so, [1024, 1024])
    desc = mpmi.tick_desc(N, H, gen=mpmi.GEN_GRID, grid=[1024, 1024])
    model_infl = mpmi.mpmi_model_pack(ctx, mpmi.race_car_system(W.track_dict(W.rc_track(), infl=0.3), infl=0.3),
                                      dev(K, torch.float64))
    for t in range(3):
        x, u = W.f32(xs[t]), W.f32(uhs[t])
        fv = torch.empty(N + 1, dtype=torch.int16, device="cuda")
        sel = mpmi.decode_selection(mpmi.mpmi_tick(ctx, model, desc, dev(x, torch.float32), dev(u, torch.float32),
                                                   first_violation=fv))
        fvg = fv.cpu().numpy().astype(np.int64)
        full = o.with_user(grid, u, 1)
        check_selection(so, full, H, u, sel, fvg, label=f"1M tick {t}")
        idx = np.unique(np.concatenate([[0, sel["idx"]], rng.integers(1, N + 1, size=3000)]))
        cand = full[idx]
        traj, fvo = o.rollout(so, K, x, cand, H, early_exit=False)
        amb = ambiguous(so, traj, fvo, fvg[idx], EPS_RC)
        assert np.all((fvo == fvg[idx]) | amb), f"tick {t}: sampled first violations differ"
        if fvo[0] == H + 1 and not amb[0]:
            assert sel["idx"] == 0 and sel["deviation"] == 0.0
        if t == 0:
            # The same tick with the FP64 re-roll of the FP32 band, then the
            # oracle over every candidate: the FP32 verdicts agree outside the
            # FP32 band, the re-rolled ones outside the FP64 band, and the
            # re-rolled tick's decision is the oracle's.
            d64 = mpmi.tick_desc(N, H, gen=mpmi.GEN_GRID, grid=[1024, 1024], precision=mpmi.PREC_FP32_RECHECK64)
            fv64 = torch.empty(N + 1, dtype=torch.int16, device="cuda")
            sel64 = mpmi.decode_selection(mpmi.mpmi_tick(ctx, model, d64, dev(x, torch.float32),
                                                         dev(u, torch.float32), first_violation=fv64))
            fvg64 = fv64.cpu().numpy().astype(np.int64)
            check_selection(so, full, H, u, sel64, fvg64, label="1M tick 0 (FP32+FP64)")
            log("[full size] tick 0: oracle rollout of every candidate")
            step = 65536
            e64 = recheck64_eps(so, sel64, EPS_RC)
            jobs = [(so, K, x, full[a:a + step], H, [(fvg[a:a + step], EPS_RC), (fvg64[a:a + step], e64)])
                    for a in range(0, N + 1, step)]
            parts = list(oracle_pool.map(oracle_chunk, jobs))
            fv_o = np.concatenate([p[0] for p in parts])
            amb32 = np.concatenate([p[1][0] for p in parts])
            amb64 = np.concatenate([p[1][1] for p in parts])
            mism = (fv_o != fvg) & ~amb32
            assert not mism.any(), f"1M tick: {int(mism.sum())} FP32 first violations differ outside the band"
            mism64 = (fv_o != fvg64) & ~amb64
            assert not mism64.any(), f"1M tick: {int(mism64.sum())} re-rolled first violations differ"
            ag = agreement(so, full, H, u, fv_o, amb32, sel)
            ag64 = agreement(so, full, H, u, fv_o, amb64, sel64)
            log(f"[full size] tick 0 against the full oracle: FP32 {ag['kind']} (FP32 band holds "
                f"{int(amb32.sum())} candidates, oracle idx {ag['idx']}, gpu idx {ag['gpu_idx']}); FP32+FP64 "
                f"{ag64['kind']} (band candidates listed {sel64['n_recheck']}, idx {sel64['idx']})")
            assert ag64["kind"] in ("identical", "equal_cost")
            assert sel64["n_recheck"] > 0
        # monotone under inflation (same candidates, tighter set)
        fv2 = torch.empty(N + 1, dtype=torch.int16, device="cuda")
        mpmi.mpmi_tick(ctx, model_infl, desc, dev(x, torch.float32), dev(u, torch.float32), first_violation=fv2)
        assert np.all(fv2.cpu().numpy() <= fvg), f"tick {t}: mask not monotone under inflation"
        log(f"[full size] tick {t}: idx={sel['idx']} status={sel['status']} n_safe={sel['n_safe']} "
            f"sampled={idx.size} ambiguous={int(amb.sum())}")


def test_tick_maximum_candidate_count(ctx, bb):
    """The largest tick the interface allows (Nc = MPMI_MAX_CAND: a 1-D grid of
    2^25 - 2 inputs + u_h), cart-pole, H = 10: one lane and four lanes per
    candidate give identical records and first violations (the four-lane
    launch has 2^19 workgroups, so every sub-slot serves 2^16 of them); the
    record (index, status, safe count) is the selection rule over the whole
    first-violation vector; first violations of ~3,000 sampled candidates
    agree with the oracle."""
    so, model, K = bb
    N = mpmi.MAX_CAND - 1
    H = 10
    # a pole falling at 1.2 rad/s from 0.35 rad: about half the inputs keep it
    # up for 10 steps, and the user's -4 N is not one of them
    x, u = W.f32([0.0, 0.0, 0.35, 1.2]), W.f32([-4.0])
    recs, fvs = [], []
    for lanes in (1, 4):
        desc = mpmi.tick_desc(N, H, gen=mpmi.GEN_GRID, grid=[N], lanes_per_cand=lanes)
        fv = torch.empty(N + 1, dtype=torch.int16, device="cuda")
        recs.append(mpmi.mpmi_tick(ctx, model, desc, dev(x, torch.float32), dev(u, torch.float32),
                                   first_violation=fv).cpu().numpy().tobytes())
        fvs.append(fv)
    assert recs[0] == recs[1]
    assert torch.equal(fvs[0], fvs[1])
    fvg = fvs[0].cpu().numpy().astype(np.int64)
    del fvs
    sel = mpmi.decode_selection(torch.tensor(np.frombuffer(recs[0], np.uint8)))
    assert sel["n_cand"] == N + 1
    assert 0 < sel["n_safe"] < N and fvg[0] <= H  # a mixed tick: the user's input is unsafe
    assert sel["status"] == mpmi.OK and sel["idx"] != 0
    full = o.with_user(o.grid_candidates(so, [N]), u, 1)
    check_selection(so, full, H, u, sel, fvg, label="maximum size")
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([[0, sel["idx"]], rng.integers(1, N + 1, size=3000)]))
    cand = full[idx]
    del full
    traj, fvo = o.rollout(so, K, x, cand, H, early_exit=False)
    amb = ambiguous(so, traj, fvo, fvg[idx], EPS_BB)
    assert np.all((fvo == fvg[idx]) | amb)
    log(f"[max size] Nc={N + 1}: idx={sel['idx']} status={sel['status']} n_safe={sel['n_safe']} "
        f"ambiguous={int(amb.sum())}")


@pytest.mark.parametrize("system", ["bb", "rc"])
def test_tick_with_process_noise(ctx, system):
    """Alg. 2's process noise z_i: every predicted state gains sigma * z, z from
    the counter generator (same definition on both sides)."""
    if system == "bb":
        K = W.bb_model()[0]
        sig = [0.002, 0.01, 0.002, 0.02]
        so = W.bb_oracle_system()
        model = mpmi.mpmi_model_pack(ctx, mpmi.balance_bot_system(noise=sig), dev(K, torch.float64))
        xs = synth.balance_bot_states(4, seed=61)
        uhs = synth.uniform_user(4, [-5.0], [5.0], seed=62)
        N, H, S, eps = 4000, 50, 5, EPS_BB
    else:
        K = W.rc_model()[0]
        sig = [0.01, 0.01, 0.002, 0.05, 0.02, 0.005]
        so = W.rc_oracle_system(W.rc_track())
        model = mpmi.mpmi_model_pack(ctx, mpmi.race_car_system(W.track_dict(W.rc_track()), noise=sig),
                                     dev(K, torch.float64))
        xs = synth.race_car_states(4, W.rc_track(), seed=61)
        uhs = synth.uniform_user(4, synth.RC_U_LO, synth.RC_U_HI, seed=62)
        N, H, S, eps = 4000, 60, 1, EPS_RC
    so.noise = W.f32(sig)
    kinds = {}
    for t in range(4):
        x, u = W.f32(xs[t]), W.f32(uhs[t])
        desc = mpmi.tick_desc(N, H, gen=mpmi.GEN_UNIFORM, n_seg=S, seed=21, tick=t, loop=3)
        fv = torch.empty(N + 1, dtype=torch.int16, device="cuda")
        sel = mpmi.decode_selection(mpmi.mpmi_tick(ctx, model, desc, dev(x, torch.float32), dev(u, torch.float32),
                                                   first_violation=fv))
        cand = o.with_user(o.uniform_candidates(so, N, S, 21, t, 3), u, S)
        res = check_tick(so, K, x, u, cand, H, sel, fv.cpu().numpy(), eps, label=f"noisy {system} tick {t}",
                         noise_key=(21, t, 3))
        kinds[res["kind"]] = kinds.get(res["kind"], 0) + 1
    log(f"[noise] {system}: {kinds}")


def _lanes_case(ctx, bb, rc, case):
    """(model, x, u, tick-descriptor fields) of one latency-form case."""
    if case.startswith("bb"):
        _, model, K = bb
        x, u = W.f32(synth.balance_bot_states(1, seed=44)[0]), W.f32([3.0])
        base = dict(n_cand=10240, horizon=50, gen=mpmi.GEN_UNIFORM, n_seg=5, seed=4, tick=2)
        if case == "bb_short_horizon":  # more segments than steps: boundaries skip segments
            base.update(n_cand=1000, horizon=3, n_seg=5, seed=9)
        elif case == "bb_h7_s4":
            base.update(n_cand=3000, horizon=7, n_seg=4, seed=10)
        elif case == "bb_track":  # a track on (x0, x1): the degree-8 track variant of the balance bot
            tr = synth.Track(amp=np.array([0.05, 0.03]), freq=np.array([2, 6]), phase=np.array([0.3, 1.1]),
                             r0=0.3, half_width=0.4)
            sg = mpmi._sys(mpmi.BASIS_BALANCE_BOT, 4, 1, [(2, float(W.f32(0.5)), 0.0), (0, float(W.f32(2.0)), 0.0)],
                           [-5.0], [5.0], track=W.track_dict(tr), eps_box=[5e-5, 2e-4], eps_track=1e-3)
            model = mpmi.mpmi_model_pack(ctx, sg, dev(K, torch.float64))
            x = W.f32([0.25, 0.1, 0.05, -0.1])
        return model, x, u, base
    _, model, K = rc
    x, u = W.f32(synth.race_car_states(1, W.rc_track(), seed=44)[0]), W.f32([0.3, -2.0])
    base = dict(n_cand=16384, horizon=60, gen=mpmi.GEN_GRID, grid=[128, 128])
    if case == "rc_segments":
        base = dict(n_cand=8192, horizon=45, gen=mpmi.GEN_UNIFORM, n_seg=3, seed=12, tick=5)
    elif case == "rc_degree8_stacked_boxes":
        tr = synth.Track(amp=np.array([1.0, 0.5, 0.3, 0.2]), freq=np.array([3, 5, 7, 8]),
                         phase=np.random.default_rng(11).uniform(0.0, 2 * np.pi, size=4))
        boxes = [(4, float(W.f32(2.0)), 0.0), (4, float(W.f32(1.2)), 0.0), (5, float(W.f32(0.5)), 0.0)]
        sg = mpmi._sys(mpmi.BASIS_RACE_CAR, 6, 2, boxes, synth.RC_U_LO, synth.RC_U_HI, track=W.track_dict(tr),
                       eps_box=[0.02] * 3, eps_track=0.02)
        model = mpmi.mpmi_model_pack(ctx, sg, dev(K, torch.float64))
        x = W.f32(synth.race_car_states(1, tr, seed=4, offset=1.5, vy=(-0.3, 0.3), r=(-0.2, 0.2))[0])
        base = dict(n_cand=96 * 96, horizon=40, gen=mpmi.GEN_GRID, grid=[96, 96])
    elif case == "rc_no_track":  # boxes only: the track-free variant
        boxes = [(4, float(W.f32(1.0)), 0.0), (3, float(W.f32(12.0)), 0.0), (5, float(W.f32(1.5)), 0.0)]
        sg = mpmi._sys(mpmi.BASIS_RACE_CAR, 6, 2, boxes, synth.RC_U_LO, synth.RC_U_HI, eps_box=[0.02] * 3)
        model = mpmi.mpmi_model_pack(ctx, sg, dev(K, torch.float64))
    return model, x, u, base


@pytest.mark.parametrize("case", ["bb", "bb_short_horizon", "bb_h7_s4", "bb_track", "rc", "rc_segments",
                                  "rc_degree8_stacked_boxes", "rc_no_track"])
def test_tick_lanes_per_candidate_identical_and_autotuned(ctx, bb, rc, case):
    """The latency form (2, 4 or 8 lanes per candidate) performs the same FP32
    operations in the same order: selections and first violations are
    identical to the one-lane form, and the tick autotuner keeps them so.
    The cases cover each kernel instance (track polynomial of degree 5 or 8,
    no track) and segment boundaries, also with more segments than steps."""
    model, x, u, base = _lanes_case(ctx, bb, rc, case)
    N = base["n_cand"]
    log(f"[lanes] {case}: N={N} H={base['horizon']} n_seg={base.get('n_seg', 1)}")
    recs, fvs = [], []
    for lanes in (1, 2, 4, 8):
        for block in (64, 256):
            d = mpmi.tick_desc(base["n_cand"], base["horizon"], gen=base["gen"], grid=base.get("grid"),
                               n_seg=base.get("n_seg", 1), seed=base.get("seed", 0), tick=base.get("tick", 0),
                               block=block, lanes_per_cand=lanes)
            fv = torch.empty(N + 1, dtype=torch.int16, device="cuda")
            recs.append(mpmi.mpmi_tick(ctx, model, d, dev(x, torch.float32), dev(u, torch.float32),
                                       first_violation=fv).cpu().numpy().tobytes())
            fvs.append(fv.cpu().numpy())
    assert all(r == recs[0] for r in recs)
    assert all(np.array_equal(f, fvs[0]) for f in fvs)
    log(f"[lanes] {case}: safe {(fvs[0] == base['horizon'] + 1).sum()} of {N + 1}")
    if case not in ("bb", "rc"):
        return
    d = mpmi.tick_desc(base["n_cand"], base["horizon"], gen=base["gen"], grid=base.get("grid"),
                       n_seg=base.get("n_seg", 1), seed=base.get("seed", 0), tick=base.get("tick", 0))
    best = mpmi.mpmi_tick_autotune(ctx, model, d, dev(x, torch.float32), dev(u, torch.float32), reps=10)
    log(f"[autotune] {case}: {best}")
    assert best["lanes_per_cand"] in (1, 2, 4, 8) and best["block"] in (64, 128, 256, 512)
    rec = mpmi.mpmi_tick(ctx, model, d, dev(x, torch.float32), dev(u, torch.float32)).cpu().numpy().tobytes()
    assert rec == recs[0]


def test_write_rate_diagnostic(ctx):
    """The trajectory store's write ceilings and the safety check's read
    ceilings: rates finite and below the part's 8 TB/s, for rows Nc floats
    apart and for rows padded to 256-byte boundaries; misaligned buffers and
    strides below Nc are rejected."""
    Nc, rows = 262145, 60
    ld = mpmi.traj_ld(Nc)
    buf = torch.empty(rows * ld, dtype=torch.float32, device="cuda")
    r = mpmi.mpmi_write_rates(ctx, buf, Nc, rows)
    rp = mpmi.mpmi_write_rates(ctx, buf, Nc, rows, ld=ld)
    log(f"[diag] write ceilings: rows {Nc} floats apart {r}; rows {ld} floats apart {rp}")
    for q in (r, rp):
        assert 100.0 < q["pattern_GB_s"] < 8000.0 and 100.0 < q["stream_GB_s"] < 8000.0
    with pytest.raises(mpmi.MpmiError):
        mpmi.mpmi_write_rates(ctx, buf[1:], Nc - 1, rows)  # misaligned
    with pytest.raises(mpmi.MpmiError):
        mpmi.mpmi_write_rates(ctx, buf, Nc, rows, ld=Nc - 1)
    rr = mpmi.mpmi_read_rates(ctx, buf, Nc, rows, ld=ld)
    log(f"[diag] read ceilings, rows {ld} floats apart: {rr}")
    assert 100.0 < rr["pattern_GB_s"] < 8000.0 and 100.0 < rr["stream_GB_s"] < 8000.0
    with pytest.raises(mpmi.MpmiError):
        mpmi.mpmi_read_rates(ctx, buf[1:], Nc - 1, rows)  # misaligned
    with pytest.raises(mpmi.MpmiError):
        mpmi.mpmi_read_rates(ctx, buf, Nc, rows, ld=Nc - 1)


@pytest.mark.parametrize("system", ["rc", "bb", "linear"])
def test_trajectory_row_stride(ctx, bb, rc, system):
    """rollout_batch, safe_mask and the fused tick's store give the same
    states, verdicts and margins with rows N + 1 floats apart and with rows
    padded to 256-byte boundaries (columns past N + 1 untouched); a stride
    below N + 1 is rejected at the boundary.  Cart-pole with five input
    segments, race car with one, and a linear system with three of eight
    state slots."""
    if system == "linear":
        N, H, n, S = 4100, 30, 3, 2
        sys_g = mpmi.linear_system(n, 1, [(0, 1.0, 0.0), (2, 0.5, 0.125)], [-1.0], [1.0])
        A = np.array([[0.97, 0.05, 0.0], [-0.05, 0.97, 0.02], [0.0, -0.02, 0.99]])
        B = np.array([[0.0, 0.04, 0.02]])
        model = mpmi.mpmi_model_pack(ctx, sys_g, dev(np.vstack([A.T, B]), torch.float64))
        x = dev([0.3, -0.2, 0.1], torch.float32)
        u = dev([0.25], torch.float32)
    elif system == "rc":
        so, model, _ = rc
        N, H, n, S = 5000, 25, 6, 1
        x = dev(synth.race_car_states(1, W.rc_track(), seed=91)[0], torch.float32)
        u = dev([0.05, 0.4], torch.float32)
    else:
        so, model, _ = bb
        N, H, n, S = 3001, 50, 4, 5
        x = dev(synth.balance_bot_states(1, seed=92)[0], torch.float32)
        u = dev([0.7], torch.float32)
    desc = mpmi.tick_desc(N, H, gen=mpmi.GEN_UNIFORM, seed=9, tick=2, n_seg=S)
    cand = mpmi.mpmi_generate_candidates(ctx, model, desc, u)
    plain = torch.full((H, n, N + 1), float("nan"), device="cuda")
    mpmi.rollout_batch(ctx, model, x, cand, H, traj=plain)
    ld = mpmi.traj_ld(N + 1)
    assert ld % 64 == 0 and ld > N + 1
    base = torch.full((H, n, ld), -7.0, device="cuda")
    padded = base[:, :, : N + 1]
    mpmi.rollout_batch(ctx, model, x, cand, H, traj=padded)
    same = dict(rtol=0, atol=0, equal_nan=True)  # exact, a diverged state's NaN included
    torch.testing.assert_close(padded, plain, **same)
    assert bool((base[:, :, N + 1:] == -7.0).all())
    fa, ma = mpmi.safe_mask(ctx, model, plain)
    fb, mb = mpmi.safe_mask(ctx, model, padded)
    assert torch.equal(fa, fb)
    torch.testing.assert_close(mb, ma, **same)
    tb = torch.full((H, n, ld), float("nan"), device="cuda")
    fv = torch.empty(N + 1, dtype=torch.int16, device="cuda")
    mpmi.mpmi_tick(ctx, model, desc, x, u, first_violation=fv, traj=tb[:, :, : N + 1])
    assert torch.equal(fv, fa)
    steps = torch.arange(1, H + 1, device="cuda")[:, None, None]
    written = steps <= torch.clamp(fv.to(torch.int64), max=H)[None, None, :]
    torch.testing.assert_close(torch.where(written, tb[:, :, : N + 1], 0.0), torch.where(written, plain, 0.0), **same)
    st = ctx.lib.rollout_batch(ctx.handle, ctypes.c_void_p(model.ptr), mpmi.PREC_FP32, x.data_ptr(),
                               cand.data_ptr(), N + 1, S, H, base.data_ptr(), N, None)
    assert st == mpmi.EINVAL


def test_fp32_fma_rate_diagnostic(ctx):
    """The non-packed FP32 FMA ceiling the roofline is judged against: within
    the part's theoretical 78.6 TFLOP/s (256 CUs x 4 SIMDs x 16 lanes x 2 x
    2.4 GHz) and well above half of it."""
    r = mpmi.mpmi_fp32_fma_rate(ctx)
    log(f"[diag] FP32 FMA rate {r:.1f} TFLOP/s")
    assert 40.0 < r < 80.0


def test_bf16x3_rollout_state_error(ctx, rc):
    """BF16X3 predictions (rollout_batch with MPMI_PREC_BF16X3: the tick's
    step with every state stored, unchecked) against the FP64 oracle over the
    full horizon, race car, H = 60: within 2e-2 relative (floors as for FP32).
    The error of the constraint margins is what the FP32 recheck band covers:
    it stays below that band (0.02 m on the track, 0.02 m/s on v_y)."""
    so, model, K = rc
    H, N = 60, 4095
    xs = synth.race_car_states(4, W.rc_track(), seed=21)
    floors = W.rc_floors()
    worst, worst_fp32, worst_margin = 0.0, 0.0, 0.0
    for t, x0 in enumerate(xs):
        x0 = W.f32(x0)
        cand = W.f32(o.with_user(o.uniform_candidates(so, N, 1, 41, t, 0), [0.0, 0.0], 1))
        c_dev = dev(to_sm(cand), torch.float32)
        tb = mpmi.rollout_batch(ctx, model, dev(x0, torch.float32), c_dev, H, precision=mpmi.PREC_BF16X3)
        tf = mpmi.rollout_batch(ctx, model, dev(x0, torch.float32), c_dev, H)
        ref, _ = o.rollout(so, K, x0, cand, H, early_exit=False)
        got = tb.cpu().numpy().transpose(0, 2, 1).astype(np.float64)
        worst = max(worst, rollout_rel_err(got, ref, floors, comp_axis=2))
        worst_fp32 = max(worst_fp32, rollout_rel_err(tf.cpu().numpy().transpose(0, 2, 1), ref, floors, comp_axis=2))
        with np.errstate(invalid="ignore"):
            mg = o.margins(so, got.reshape(-1, 6))
            mr = o.margins(so, ref.reshape(-1, 6))
        keep = np.isfinite(mr).all(axis=1) & (np.abs(mr) < 10.0).all(axis=1)
        worst_margin = max(worst_margin, float(np.max(np.abs(mg[keep] - mr[keep]))))
    log(f"[bf16x3 states] race car H=60: max relative error vs FP64 {worst:.3e} (FP32 path {worst_fp32:.3e}); "
        f"max margin error {worst_margin:.3e} (recheck band 0.02)")
    assert worst <= 2e-2
    assert worst_margin < 0.02


def test_bf16x3_tick_size_limit(ctx, rc):
    """A BF16X3 tick takes at most 2^22 candidates, so that every
    near-boundary candidate fits the FP32 recheck list; larger ones are
    refused before anything is enqueued."""
    so, model, K = rc
    x, u = dev(W.f32(synth.race_car_states(1, W.rc_track(), seed=3)[0]), torch.float32), dev([0.0, 0.0], torch.float32)
    big = mpmi.tick_desc(1 << 22, 10, gen=mpmi.GEN_UNIFORM, precision=mpmi.PREC_BF16X3)
    with pytest.raises(mpmi.MpmiError) as e:
        mpmi.mpmi_tick(ctx, model, big, x, u)
    assert e.value.status == mpmi.EUNSUPPORTED
    ok = mpmi.tick_desc((1 << 22) - 1, 2, gen=mpmi.GEN_UNIFORM, precision=mpmi.PREC_BF16X3)
    sel = mpmi.decode_selection(mpmi.mpmi_tick(ctx, model, ok, x, u))
    assert sel["n_cand"] == 1 << 22


@pytest.mark.parametrize("system", ["bb", "rc"])
def test_safe_mask_near_bits(ctx, bb, rc, system):
    """safe_mask's near-boundary bitmask over full-horizon rollouts: against
    the oracle (set wherever some oracle margin up to the first violation is
    inside half the FP32 band, clear wherever every one is outside one and a
    half bands: the margin error is below half a band, C18-C19), and exactly
    as many candidates as the FP32_RECHECK64 tick re-rolls on the same
    candidates (the same FP32 states and margin code)."""
    so, model, K = bb if system == "bb" else rc
    sysg = model.system
    eps = np.array([sysg.eps32_box[b] for b in range(sysg.n_box)] + ([sysg.eps32_track] if sysg.has_track else []))
    if system == "bb":
        grid, H = [4096], 50  # 44 candidates inside half a band in FP64 over the 6 ticks
        xs, us = synth.balance_bot_states(6, seed=7), synth.uniform_user(6, [-5.0], [5.0], seed=8)
    else:
        grid, H = [128, 128], 60
        xs = synth.race_car_states(4, W.rc_track(), seed=7)
        us = synth.uniform_user(4, synth.RC_U_LO, synth.RC_U_HI, seed=8)
    N = int(np.prod(grid))
    total = 0
    for t in range(len(xs)):
        x, u = W.f32(xs[t]), W.f32(us[t])
        desc = mpmi.tick_desc(N, H, gen=mpmi.GEN_GRID, grid=grid, precision=mpmi.PREC_FP32_RECHECK64)
        cand = mpmi.mpmi_generate_candidates(ctx, model, desc, dev(u, torch.float32))
        traj = mpmi.rollout_batch(ctx, model, dev(x, torch.float32), cand, H)
        fv, _, nb = mpmi.safe_mask(ctx, model, traj, with_margin=False, with_near=True)
        words = nb.cpu().numpy().view(np.uint32)
        bits = ((words[:, None] >> np.arange(32, dtype=np.uint32)[None, :]) & 1).reshape(-1)[: N + 1].astype(bool)
        assert not np.any(((words[-1] >> np.uint32((N + 1) % 32)) if (N + 1) % 32 else 0))  # nothing past Nc
        sel = mpmi.decode_selection(mpmi.mpmi_tick(ctx, model, desc, dev(x, torch.float32), dev(u, torch.float32)))
        assert int(bits.sum()) == sel["n_recheck"], (t, int(bits.sum()), sel["n_recheck"])
        c64 = np.transpose(cand.cpu().numpy().astype(np.float64), (2, 0, 1))
        t64, fv_o = o.rollout(so, K, x, c64, H, early_exit=False)
        M = o.margins(so, t64.reshape(-1, so.n)).reshape(H, N + 1, -1)
        upto = np.minimum(np.minimum(fv_o, fv.cpu().numpy().astype(np.int64)), H)
        keep = (np.arange(1, H + 1)[:, None] <= upto[None, :])[:, :, None]
        inside = np.any(keep & (np.abs(M) < 0.5 * eps), axis=(0, 2))
        outside = ~np.any(keep & (np.abs(M) < 1.5 * eps), axis=(0, 2))
        assert np.all(bits[inside]), f"tick {t}: near candidates not flagged"
        assert not np.any(bits[outside]), f"tick {t}: far candidates flagged"
        total += int(bits.sum())
    log(f"[near bits] {system}: {total} flagged over {len(xs)} ticks, equal to the re-rolled counts")
    assert total > 0


@pytest.mark.parametrize("prec", [mpmi.PREC_FP32, mpmi.PREC_FP32_RECHECK64])
def test_tick_graph_replays(ctx, rc, prec):
    """A single-loop tick captured as a HIP graph (mpmi_tick_graph): three
    replays, each after writing new inputs into the captured tensors and some
    eager work, give the records and first violations of eager ticks on the
    same inputs."""
    so, model, K = rc
    N, H = 128 * 128, 60
    desc = mpmi.tick_desc(N, H, gen=mpmi.GEN_GRID, grid=[128, 128], precision=prec)
    xs = synth.race_car_states(4, W.rc_track(), seed=17)
    us = synth.uniform_user(4, synth.RC_U_LO, synth.RC_U_HI, seed=18)
    x_dev, u_dev = dev(W.f32(xs[0]), torch.float32), dev(W.f32(us[0]), torch.float32)
    fv = torch.zeros(N + 1, dtype=torch.int16, device="cuda")
    g = mpmi.TickGraph(ctx, model, desc, x_dev, u_dev, first_violation=fv)
    try:
        for r in range(1, 4):
            x_dev.copy_(dev(W.f32(xs[r]), torch.float32))
            u_dev.copy_(dev(W.f32(us[r]), torch.float32))
            junk = torch.randn(1 << 20, device="cuda").sum()
            rec = g.launch().clone()
            fv_g = fv.clone()
            torch.cuda.synchronize()
            del junk
            fv_e = torch.zeros(N + 1, dtype=torch.int16, device="cuda")
            ref = mpmi.mpmi_tick(ctx, model, desc, x_dev, u_dev, first_violation=fv_e)
            torch.cuda.synchronize()
            assert rec.cpu().numpy().tobytes() == ref.cpu().numpy().tobytes(), f"replay {r}"
            assert torch.equal(fv_g, fv_e), f"replay {r}"
        log(f"[tick graph] precision {prec}: 3 replays equal eager ticks")
    finally:
        g.close()
