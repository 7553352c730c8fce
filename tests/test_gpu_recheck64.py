"""GPU checks of the FP32 tick with the FP64 re-roll of its rounding band
(precision FP32_RECHECK64): first violations equal to the FP64 oracle's
outside the FP64 band, decisions that agree with the oracle's, the many-loop
form equal to single-loop ticks, and the FP32 margin error measured against
the bands the re-roll relies on."""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import mpmi_oracle as o
from paper_1906_02318_amd import mpmi
from tests import workloads as W
from tests.parity import agreed, recheck64_eps, replay_job, tally

pytestmark = pytest.mark.gpu

R64 = mpmi.PREC_FP32_RECHECK64


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return mpmi.Context(0)


NOISE_BB = [0.0, 2e-3, 0.0, 5e-3]  # FP32 values; cart velocity and pole rate


EPS32 = {"bb": [1e-4, 4e-4], "bb_noise": [1e-4, 4e-4], "rc": [1e-3, 1e-3], "rc3": [1e-3, 1e-3]}


def _case(name):
    """(oracle system, K, library system, grid, H, states, user inputs)."""
    if name in ("bb", "bb_noise"):
        K = W.bb_model()[0]
        so = W.bb_oracle_system()
        sg = mpmi.balance_bot_system(noise=NOISE_BB if name == "bb_noise" else None)
        if name == "bb_noise":
            so = o.System("balance_bot", 4, 1, box=so.box, u_lo=so.u_lo, u_hi=so.u_hi,
                          noise=list(W.f32(NOISE_BB)))
        T = 150
        return so, K, sg, [1024], 20, synth.balance_bot_states(T, seed=1), \
            synth.uniform_user(T, [-5.0], [5.0], seed=2)
    if name == "rc":
        K = W.rc_model()[0]
        T = 24
        return W.rc_oracle_system(W.rc_track()), K, mpmi.race_car_system(W.track_dict(W.rc_track())), [128, 128], \
            60, synth.race_car_states(T, W.rc_track(), seed=1), synth.uniform_user(T, synth.RC_U_LO, synth.RC_U_HI,
                                                                                   seed=2)
    K = W.rc3_model()[0]
    T = 24
    return W.rc3_oracle_system(W.rc_track()), K, W.rc3_gpu_system(mpmi, W.rc_track()), [22, 23, 20], 25, \
        synth.race_car_states(T, W.rc_track(), seed=1), synth.uniform_user(T, synth.RC3_U_LO, synth.RC3_U_HI, seed=2)


@pytest.mark.parametrize("name", ["bb", "bb_noise", "rc", "rc3"])
def test_recheck64_ticks_against_the_fp64_oracle(ctx, oracle_pool, name):
    """FP32_RECHECK64 ticks (cart-pole N = 1,024, H = 20, with and without
    process noise; race car 128 x 128, H = 60; the three-input car's custom
    basis, 10,120 points, H = 25) against the oracle: every record is the
    selection rule over the kernel's own verdicts; first violations equal the
    oracle's outside the FP32 band, and outside 1e-9 on ticks where nothing is
    safe (every band candidate re-rolled in FP64); every decision agrees with
    the oracle's.  The ticks are deterministic."""
    so, K, sg, grid, H, xs, uhs = _case(name)
    model = mpmi.mpmi_model_pack(ctx, sg, dev(K, torch.float64))
    N = int(np.prod(grid))
    jobs, rechecked = [], []
    for t in range(len(xs)):
        x, u = W.f32(xs[t]), W.f32(uhs[t])
        desc = mpmi.tick_desc(N, H, gen=mpmi.GEN_GRID, grid=grid, precision=R64, seed=11, tick=t)
        fv = torch.empty(N + 1, dtype=torch.int16, device="cuda")
        rec = mpmi.mpmi_tick(ctx, model, desc, dev(x, torch.float32), dev(u, torch.float32), first_violation=fv)
        if t < 3:
            fv2 = torch.empty(N + 1, dtype=torch.int16, device="cuda")
            rec2 = mpmi.mpmi_tick(ctx, model, desc, dev(x, torch.float32), dev(u, torch.float32), first_violation=fv2)
            assert rec.cpu().numpy().tobytes() == rec2.cpu().numpy().tobytes() and torch.equal(fv, fv2)
        sel = mpmi.decode_selection(rec)
        rechecked.append(sel["n_recheck"])
        noise_key = (11, t, 0) if name == "bb_noise" else None
        jobs.append((so, K, x, u, ("grid", grid), H, EPS32[name], noise_key,
                     [(sel, fv.cpu().numpy(), f"{name} tick {t}", recheck64_eps(so, sel, EPS32[name]))]))
    res = [r for rs in oracle_pool.map(replay_job, jobs) for r in rs]
    kinds = tally(res)
    log(f"[recheck64] {name}: {kinds}; re-rolled per tick mean {np.mean(rechecked):.1f} max {max(rechecked)}")
    assert agreed(kinds) == len(res)
    assert sum(rechecked) > 0


def test_recheck64_limits(ctx):
    """Ticks beyond the list's capacity and several lanes per candidate are
    refused; the autotuner keeps one lane per candidate."""
    K = W.bb_model()[0]
    model = mpmi.mpmi_model_pack(ctx, mpmi.balance_bot_system(), dev(K, torch.float64))
    x, u = dev(W.f32([0.0, 0.0, 0.1, 0.0]), torch.float32), dev(W.f32([1.0]), torch.float32)
    with pytest.raises(mpmi.MpmiError) as e:
        mpmi.mpmi_tick(ctx, model, mpmi.tick_desc((1 << 22), 10, gen=mpmi.GEN_GRID, grid=[1 << 22], precision=R64),
                       x, u)
    assert e.value.status == mpmi.EUNSUPPORTED
    with pytest.raises(mpmi.MpmiError):
        mpmi.mpmi_tick(ctx, model, mpmi.tick_desc(1024, 10, gen=mpmi.GEN_GRID, grid=[1024], precision=R64,
                                                  lanes_per_cand=4), x, u)
    shape = mpmi.mpmi_tick_autotune(ctx, model, mpmi.tick_desc(4096, 20, gen=mpmi.GEN_GRID, grid=[4096],
                                                               precision=R64), x, u, reps=3)
    assert shape["lanes_per_cand"] == 1


def test_multi_recheck64_equals_single_ticks(ctx):
    """Eight mixed loops in one many-loop launch with the FP64 re-roll: the
    records equal single-loop FP32_RECHECK64 ticks of the same loops, eagerly
    and over three graph replays (eager work between them), and the tick
    counters advance once per tick."""
    Kb, Kr = W.bb_model()[0], W.rc_model()[0]
    mb = mpmi.mpmi_model_pack(ctx, mpmi.balance_bot_system(), dev(Kb, torch.float64))
    mr = mpmi.mpmi_model_pack(ctx, mpmi.race_car_system(W.track_dict(W.rc_track())), dev(Kr, torch.float64))
    rng = np.random.default_rng(7)
    kinds = ["rc", "bb", "rc", "bb", "rc", "rc", "bb", "bb"]
    Ns = [5000, 300, 16384, 20000, 777, 2500, 64, 1024]
    Hs = [60, 20, 45, 50, 33, 25, 60, 41]
    xb, xr = synth.balance_bot_states(8, seed=19), synth.race_car_states(8, W.rc_track(), seed=19)
    loops, meta = [], []
    for i, (k, N, H) in enumerate(zip(kinds, Ns, Hs)):
        if k == "bb":
            x, u = W.f32(xb[i]), W.f32(rng.uniform(-5, 5, size=1))
        else:
            x, u = W.f32(xr[i]), W.f32(rng.uniform(synth.RC_U_LO, synth.RC_U_HI))
        loops.append(dict(model=mb if k == "bb" else mr, x_t=dev(x, torch.float32), u_user=dev(u, torch.float32),
                          out=torch.zeros(mpmi.SELECTION_BYTES, dtype=torch.uint8, device="cuda"),
                          first_violation=torch.zeros(N + 1, dtype=torch.int16, device="cuda"),
                          n_cand=N, horizon=H, gen=mpmi.GEN_UNIFORM, seed=200 + i, tick=10 * i))
        meta.append(dict(model=mb if k == "bb" else mr, N=N, H=H, seed=200 + i, tick0=10 * i))
    multi = mpmi.Multi(ctx, loops, block=256, precision=R64)
    assert multi.config()["precision"] == R64

    def singles(offset):
        recs, fvs = [], []
        for i, (l, mt) in enumerate(zip(loops, meta)):
            d = mpmi.tick_desc(mt["N"], mt["H"], gen=mpmi.GEN_UNIFORM, seed=mt["seed"], tick=mt["tick0"] + offset,
                               loop=i, precision=R64)
            fv = torch.empty(mt["N"] + 1, dtype=torch.int16, device="cuda")
            recs.append(mpmi.mpmi_tick(ctx, mt["model"], d, l["x_t"], l["u_user"],
                                       first_violation=fv).cpu().numpy().tobytes())
            fvs.append(fv)
        return recs, fvs

    try:
        n_re = 0
        for offset in range(2):
            multi.tick()
            torch.cuda.synchronize()
            got = [l["out"].cpu().numpy().tobytes() for l in loops]
            got_fv = [l["first_violation"].clone() for l in loops]
            want, want_fv = singles(offset)
            assert got == want, f"eager tick {offset}"
            assert all(torch.equal(a, b) for a, b in zip(got_fv, want_fv))
            n_re += sum(mpmi.decode_selection(l["out"])["n_recheck"] for l in loops)
        multi.capture_graph()
        for r in range(3):
            multi.launch_graph()
            torch.cuda.synchronize()
            got = [l["out"].cpu().numpy().tobytes() for l in loops]
            junk = torch.randn(1 << 20, device="cuda").sum()
            torch.cuda.synchronize()
            assert got == singles(2 + r)[0], f"replay {r}"
            del junk
        assert multi.ticks() == [mt["tick0"] + 5 for mt in meta]
        log(f"[multi recheck64] 2 eager ticks and 3 replays equal single ticks; re-rolled {n_re} in the eager ticks")
        assert n_re > 0
    finally:
        multi.close()


@pytest.mark.parametrize("name", ["bb", "rc", "rc3"])
def test_fp32_margin_error_within_the_recheck_bands(ctx, name):
    """The FP32 bands must cover the FP32 tick's margin error.  Over full-
    horizon FP32 rollouts (rollout_batch: the tick's step) and the kernel's
    own FP32 least margins (safe_mask), against the oracle's FP64 rollouts of
    the same candidates: the largest error of a margin, over every step up to
    the oracle's first violation, is below half the band of its constraint,
    and the error of the kernel's least margin (some constraint's) below half
    the widest band."""
    so, K, sg, grid, H, xs, uhs = _case(name)
    model = mpmi.mpmi_model_pack(ctx, sg, dev(K, torch.float64))
    eps = np.array([sg.eps32_box[b] for b in range(sg.n_box)] + ([sg.eps32_track] if sg.has_track else []))
    N = int(np.prod(grid))
    worst_state = np.zeros(eps.size)
    worst_least = 0.0
    ticks = 40 if name == "bb" else 12
    for t in range(ticks):
        x, u = W.f32(xs[t]), W.f32(uhs[t])
        desc = mpmi.tick_desc(N, H, gen=mpmi.GEN_GRID, grid=grid)
        cand = mpmi.mpmi_generate_candidates(ctx, model, desc, dev(u, torch.float32))
        traj = mpmi.rollout_batch(ctx, model, dev(x, torch.float32), cand, H)
        fv, mm = mpmi.safe_mask(ctx, model, traj, with_margin=True)
        c64 = np.transpose(cand.cpu().numpy().astype(np.float64), (2, 0, 1))
        t64, fv_o = o.rollout(so, K, x, c64, H, early_exit=False)
        g = traj.cpu().numpy().astype(np.float64)[:, :, : N + 1].transpose(0, 2, 1)
        M_o = o.margins(so, t64.reshape(-1, so.n)).reshape(H, N + 1, -1)
        M_g = o.margins(so, g.reshape(-1, so.n)).reshape(H, N + 1, -1)
        upto = np.minimum(fv_o, H)
        keep = np.arange(1, H + 1)[:, None] <= upto[None, :]
        d = np.where(keep[:, :, None], np.abs(M_g - M_o), 0.0)
        worst_state = np.maximum(worst_state, np.nanmax(d, axis=(0, 1)))
        # the kernel's least margin (FP32 evaluation of the constraints) where
        # both sides stop at the same step
        fvg = fv.cpu().numpy().astype(np.int64)
        same = fvg == fv_o
        least_o = np.min(np.where(keep[:, :, None], M_o, np.inf), axis=(0, 2))
        dl = np.abs(mm.cpu().numpy().astype(np.float64) - least_o)[same & np.isfinite(least_o)]
        worst_least = max(worst_least, float(dl.max()) if dl.size else 0.0)
    log(f"[margin error] {name}: per-constraint FP32 state error in the margins {worst_state} "
        f"(bands {eps}); kernel least-margin error {worst_least:.3e}")
    assert np.all(worst_state <= 0.5 * eps)
    assert worst_least <= 0.5 * eps.max()


def test_reroll_sincos_accuracy(ctx):
    """The FP64 re-roll's sin/cos of the heading (mpmi_sincos64): within 2
    ulp of NumPy's over ordinary headings, arguments next to multiples of
    pi/2 (where the reduction cancels), tiny and signed-zero arguments, and
    the library path (|x| >= 2^20, infinities, NaN)."""
    rng = np.random.default_rng(31)
    k = rng.integers(-60, 61, size=20000).astype(np.float64)
    delta = rng.choice([-1.0, 1.0], size=k.size) * 10.0 ** rng.uniform(-14, -2, size=k.size)
    finite = np.concatenate([
        rng.uniform(-30.0, 30.0, size=200000),
        k * (np.pi / 2) + delta,
        np.array([0.0, -0.0, 1e-300, -1e-300, 1e-20, -1e-8, np.pi / 4, -np.pi / 4, 3 * np.pi / 4,
                  2.0 ** 20 - 1.0, 2.0 ** 20, -(2.0 ** 20), 1e6, -1e10, 1e300]),
    ])
    special = np.array([np.nan, np.inf, -np.inf])
    x = np.concatenate([finite, special])
    xd = dev(x, torch.float64)
    sn = torch.empty_like(xd)
    cs = torch.empty_like(xd)
    mpmi.mpmi_sincos64(ctx, xd, sn, cs)
    torch.cuda.synchronize()
    s, c = sn.cpu().numpy(), cs.cpu().numpy()
    nf = finite.size
    rs, rc = np.sin(finite), np.cos(finite)
    es = np.abs(s[:nf] - rs) / np.spacing(np.abs(rs))
    ec = np.abs(c[:nf] - rc) / np.spacing(np.abs(rc))
    log(f"[sincos64] {nf} arguments: max error sin {es.max():.2f} ulp, cos {ec.max():.2f} ulp; "
        f"mean {es.mean():.3f} / {ec.mean():.3f} ulp")
    assert es.max() <= 2.0 and ec.max() <= 2.0
    assert s[nf - 15] == 0.0 and c[nf - 15] == 1.0  # x = 0 exactly
    assert np.all(np.isnan(s[nf:])) and np.all(np.isnan(c[nf:]))
    with pytest.raises(mpmi.MpmiError):
        ctx.check(ctx.lib.mpmi_sincos64(ctx.handle, None, None, None, 4, None))
