"""GPU checks of the many-loop tick (one persistent launch for many control
loops), its HIP-graph replay and its autotuner."""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import mpmi_oracle as o
from paper_1906_02318_amd import mpmi
from tests import workloads as W
from tests.parity import agreed, check_tick, recheck64_eps, replay_job, tally

pytestmark = pytest.mark.gpu

EPS = {"bb": [1e-4, 4e-4], "rc": [1e-3, 1e-3]}


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


@pytest.fixture(scope="module")
def setup():
    assert torch.cuda.is_available()
    ctx = mpmi.Context(0)
    Kb, Kr = W.bb_model()[0], W.rc_model()[0]
    mb = mpmi.mpmi_model_pack(ctx, mpmi.balance_bot_system(), dev(Kb, torch.float64))
    mr = mpmi.mpmi_model_pack(ctx, mpmi.race_car_system(W.track_dict(W.rc_track())), dev(Kr, torch.float64))
    rng = np.random.default_rng(5)
    kinds = ["bb", "rc", "bb", "rc", "rc", "bb", "rc", "bb"]
    Ns = [300, 5000, 20000, 777, 12000, 64, 2500, 1024]
    Hs = [20, 60, 45, 33, 25, 60, 41, 50]
    xb = synth.balance_bot_states(8, seed=17)
    xr = synth.race_car_states(8, W.rc_track(), seed=17)
    loops, meta = [], []
    for i, (k, N, H) in enumerate(zip(kinds, Ns, Hs)):
        if k == "bb":
            x, u = W.f32(xb[i]), W.f32(rng.uniform(-5, 5, size=1))
        else:
            x, u = W.f32(xr[i]), W.f32(rng.uniform(synth.RC_U_LO, synth.RC_U_HI))
        loops.append(dict(model=mb if k == "bb" else mr, x_t=dev(x, torch.float32), u_user=dev(u, torch.float32),
                          out=torch.zeros(mpmi.SELECTION_BYTES, dtype=torch.uint8, device="cuda"),
                          first_violation=torch.zeros(N + 1, dtype=torch.int16, device="cuda"),
                          n_cand=N, horizon=H, gen=mpmi.GEN_UNIFORM, seed=100 + i, tick=1000 * i))
        meta.append(dict(kind=k, x=x, u=u, N=N, H=H, seed=100 + i, tick0=1000 * i))
    multi = mpmi.Multi(ctx, loops, block=256)
    systems = {"bb": (W.bb_oracle_system(), Kb, mb), "rc": (W.rc_oracle_system(W.rc_track()), Kr, mr)}
    return ctx, multi, loops, meta, systems


def single_tick_records(ctx, loops, meta, systems, tick_offset):
    """The same ticks run one loop at a time through mpmi_tick."""
    recs = []
    for i, (l, mt) in enumerate(zip(loops, meta)):
        model = systems[mt["kind"]][2]
        d = mpmi.tick_desc(mt["N"], mt["H"], gen=mpmi.GEN_UNIFORM, seed=mt["seed"], tick=mt["tick0"] + tick_offset,
                           loop=i)
        recs.append(mpmi.mpmi_tick(ctx, model, d, l["x_t"], l["u_user"]).cpu().numpy().tobytes())
    return recs


def multi_records(loops):
    return [l["out"].cpu().numpy().tobytes() for l in loops]


def test_multi_tick_matches_oracle_and_single_ticks(setup):
    ctx, multi, loops, meta, systems = setup
    log(f"[multi] config {multi.config()}")
    multi.tick()
    torch.cuda.synchronize()
    got = multi_records(loops)
    for i, (l, mt) in enumerate(zip(loops, meta)):
        so, K, _ = systems[mt["kind"]]
        cand = o.with_user(o.uniform_candidates(so, mt["N"], 1, mt["seed"], mt["tick0"], i), mt["u"], 1)
        sel = mpmi.decode_selection(l["out"])
        res = check_tick(so, K, mt["x"], mt["u"], cand, mt["H"], sel, l["first_violation"].cpu().numpy(),
                         EPS[mt["kind"]], label=f"multi loop {i} ({mt['kind']} N={mt['N']} H={mt['H']})")
        log(f"[multi] loop {i}: {res['kind']} idx={sel['idx']} status={sel['status']} n_safe={sel['n_safe']}")
    assert got == single_tick_records(ctx, loops, meta, systems, 0)
    # the device advanced every tick counter: the next tick uses tick0 + 1
    multi.tick()
    torch.cuda.synchronize()
    assert multi_records(loops) == single_tick_records(ctx, loops, meta, systems, 1)


def test_multi_graph_replay(setup):
    ctx, multi, loops, meta, systems = setup
    # two ticks ran in the previous test (offsets 0, 1): replays continue at 2
    multi.capture_graph()
    for r in range(3):
        multi.launch_graph()
        torch.cuda.synchronize()
        got = multi_records(loops)
        # eager work between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        assert got == single_tick_records(ctx, loops, meta, systems, 2 + r), f"replay {r}"
        del junk
    log("[multi] 3 graph replays identical to eager single ticks")


def test_multi_autotune_and_block_sizes_deterministic(setup):
    ctx, multi, loops, meta, systems = setup
    offset = 5  # ticks so far: 2 eager + 3 replays
    for block in (64, 128, 512, 1024):
        multi.set_config(block)
        multi.tick()
        torch.cuda.synchronize()
        assert multi_records(loops) == single_tick_records(ctx, loops, meta, systems, offset), f"block {block}"
        offset += 1
    best = multi.autotune(reps=5)
    log(f"[multi] autotuned {best}, plan {multi.config()}")
    assert best["block"] in (64, 128, 256, 512, 1024) and best["ms"] > 0
    assert best["grid"] == multi.config()["n_work"] >= len(loops)
    ticks = multi.ticks()
    offs = [t - mt["tick0"] for t, mt in zip(ticks, meta)]
    assert len(set(offs)) == 1 and offs[0] > offset
    multi.tick()
    torch.cuda.synchronize()
    assert multi_records(loops) == single_tick_records(ctx, loops, meta, systems, offs[0])


def test_multi_model_snapshot_taken_at_replan(setup):
    """The plan reads its own copy of each packed model: a model re-packed in
    place is used from the next re-plan on, not before."""
    ctx, multi, loops, meta, systems = setup
    so, Kr, mr = systems["rc"]
    ticks = multi.ticks()
    off = ticks[0] - meta[0]["tick0"]
    K2 = Kr.copy()
    K2[0, :] *= 0.5  # another constant-feature row: different predictions
    try:
        mpmi.mpmi_model_pack(ctx, mpmi.race_car_system(W.track_dict(W.rc_track())), dev(K2, torch.float64), into=mr)
        torch.cuda.synchronize()
        multi.tick()
        torch.cuda.synchronize()
        before = multi_records(loops)
        mpmi.mpmi_model_pack(ctx, mpmi.race_car_system(W.track_dict(W.rc_track())), dev(Kr, torch.float64), into=mr)
        torch.cuda.synchronize()
        assert before == single_tick_records(ctx, loops, meta, systems, off), "re-pack seen before re-plan"
        mpmi.mpmi_model_pack(ctx, mpmi.race_car_system(W.track_dict(W.rc_track())), dev(K2, torch.float64), into=mr)
        torch.cuda.synchronize()
        multi.set_config(multi.config()["block"])
        multi.tick()
        torch.cuda.synchronize()
        after = multi_records(loops)
        assert after == single_tick_records(ctx, loops, meta, systems, off + 1), "re-plan did not take the new model"
        rc_loops = [i for i, mt in enumerate(meta) if mt["kind"] == "rc"]
        mpmi.mpmi_model_pack(ctx, mpmi.race_car_system(W.track_dict(W.rc_track())), dev(Kr, torch.float64), into=mr)
        torch.cuda.synchronize()
        old = single_tick_records(ctx, loops, meta, systems, off + 1)
        assert any(after[i] != old[i] for i in rc_loops), "K2 changed no race-car selection"
    finally:
        mpmi.mpmi_model_pack(ctx, mpmi.race_car_system(W.track_dict(W.rc_track())), dev(Kr, torch.float64), into=mr)
        torch.cuda.synchronize()
        multi.set_config(multi.config()["block"])


def test_serving_workload_decisions_against_oracle(oracle_pool):
    """The bench's serving workload -- 64 closed loops (32 cart-poles, 32 race
    cars; N_l log-uniform in [1,024, 65,536], H_l in 20..60, AR(1) users), one
    graph replay per tick, FP32 ticks with the FP64 re-roll of each loop's
    FP32 band (FP32_RECHECK64) -- for 1,001 ticks; at every 500th tick all 64
    loops are replayed by the oracle on their visited (x_t, u_h, candidates):
    every record is the selection rule over its loop's first violations, those
    equal the oracle's outside the band of recheck64_eps, and at least 99.9%
    of the decisions agree with the oracle's."""
    ctx = mpmi.Context(0)
    track = W.rc_track()
    Kb, Kr = W.bb_model()[0], W.rc_model()[0]
    mb = mpmi.mpmi_model_pack(ctx, mpmi.balance_bot_system(), dev(Kb, torch.float64))
    mr = mpmi.mpmi_model_pack(ctx, mpmi.race_car_system(W.track_dict(track)), dev(Kr, torch.float64))
    systems = {"bb": (W.bb_oracle_system(), Kb, 4, 1), "rc": (W.rc_oracle_system(track), Kr, 6, 2)}
    scen = synth.ManyLoops(track, 64, seed=5)
    n = scen.n_loops
    x_dev = torch.zeros((n, 8), dtype=torch.float32, device="cuda")
    u_dev = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    out_dev = torch.zeros((n, mpmi.SELECTION_BYTES), dtype=torch.uint8, device="cuda")
    fvs = [torch.zeros(int(N) + 1, dtype=torch.int16, device="cuda") for N in scen.N]
    loops = [dict(model=mb if k == "bb" else mr, x_t=x_dev[i], u_user=u_dev[i], out=out_dev[i],
                  first_violation=fvs[i], n_cand=int(scen.N[i]), horizon=int(scen.H[i]), gen=mpmi.GEN_UNIFORM,
                  seed=scen.seeds[i], tick=0) for i, k in enumerate(scen.kinds)]
    multi = mpmi.Multi(ctx, loops, precision=mpmi.PREC_FP32_RECHECK64)
    multi.capture_graph()
    jobs = []
    for t in range(1001):
        x_dev.copy_(torch.from_numpy(scen.x))
        u_dev.copy_(torch.from_numpy(scen.u))
        multi.launch_graph()
        torch.cuda.synchronize()
        rec = out_dev.cpu().numpy()
        if t % 500 == 0:
            sels = mpmi.decode_selection(out_dev)
            for i, k in enumerate(scen.kinds):
                so, K, nx, nu = systems[k]
                x, u = W.f32(scen.x[i, :nx]), W.f32(scen.u[i, :nu])
                jobs.append((so, K, x, u, ("uniform", int(scen.N[i]), 1, scen.seeds[i], t, i), int(scen.H[i]),
                             recheck64_eps(so, sels[i], EPS[k]), None,
                             [(sels[i], fvs[i].cpu().numpy(), f"tick {t} loop {i} ({k})")]))
            log(f"[serving] tick {t}: records of {n} loops taken")
        scen.advance(rec.view(np.float32).reshape(n, -1)[:, 4:8], t)
    assert multi.ticks() == [1001] * n
    multi.close()
    res = [r for rs in oracle_pool.map(replay_job, jobs) for r in rs]
    kinds = tally(res)
    log(f"[serving] {len(res)} loop-ticks replayed: {kinds}; plant restarts {scen.resets}")
    assert agreed(kinds) >= 0.999 * len(res)
