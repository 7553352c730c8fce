"""Throughput benchmark of the MPMI-SC control tick on one MI355X.

A step is one control tick of the whole hot path -- candidate generation,
Koopman prediction with early exit, safety checks and the minimal-intervention
selection -- run as one fused kernel launch over the tick's candidate batch.
Inputs (model, tick states, user inputs) are resident in HBM before timing.

Prints one JSON line (see the keys below); `value` is candidate trajectories
per second, every candidate counted once whatever its early exit.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "candidate trajectories/sec + p99 tick latency, plain vs learned proposal"
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

# Algorithmic FP32 work of one unit (one candidate advanced one step and
# checked), flops with an FMA counted as 2.
#   race car: 51 feature products + 64x6 contraction (768) + ~41 for the
#     track and v_y checks (rho^2, the centreline's harmonics, two margins
#     and compares) = 860
#   balance bot: 15 feature products + 21x4 contraction (168) + two box checks (4)
FLOPS_PER_UNIT = {"race_car": 860, "balance_bot": 187}
# What the folded step executes per unit (input terms folded once per segment):
#   race car: 511, from the FP32 FMA/MUL/ADD instruction counters of the
#     1M-candidate tick per executed unit (27 feature products, 210 step FMAs,
#     the safety check with its degree-5 track polynomial, and the per-segment
#     fold spread over the horizon);
#   balance bot: 10 feature products + 56 FMAs + ~6 safety flops (estimate).
EXECUTED_FLOPS_PER_UNIT = {"race_car": 511, "balance_bot": 128}

# HBM traffic of the tick kernel, from rocprofv3 FETCH_SIZE / WRITE_SIZE runs
# scaled by a copy-kernel calibration; the record names a digest of the
# kernel's sources and is used only while the sources still match it.
TRAFFIC_PROFILES = {
    ("race_car_1m", "fp32"): os.path.join(ROOT, "profiles", "tick_fp32_race_car_N1048576_H60.md"),
    ("race_car_1m", "fp32_recheck64"): os.path.join(ROOT, "profiles", "tick_fp32_recheck64_race_car_N1048576_H60.md"),
}
TICK_SOURCES = ["paper_1906_02318_amd/csrc/mpmi_tick.hip", "paper_1906_02318_amd/csrc/mpmi_device.hpp",
                "paper_1906_02318_amd/csrc/mpmi_tick_common.hpp", "paper_1906_02318_amd/csrc/mpmi_recheck64.hip",
                "include/mpmi.h"]


def tick_source_digest() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in TICK_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_record(workload: str, precision: str):
    """(bytes per tick, detail) from the workload's profile summary, or (None, reason)."""
    path = TRAFFIC_PROFILES.get((workload, precision))
    if not path or not os.path.exists(path):
        return None, "no counter profile for this workload"
    rec = None
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic-record:"):
                rec = json.loads(line.split(":", 1)[1])
    if rec is None:
        return None, "profile has no traffic record"
    if rec.get("sources_sha256") != tick_source_digest():
        return None, "kernel sources changed since the counters were taken"
    detail = {k: rec[k] for k in ("fetch_bytes", "write_bytes", "fetch_scale", "write_scale") if k in rec}
    detail["profile"] = os.path.relpath(path, ROOT)
    return rec["fetch_bytes"] + rec["write_bytes"], detail


WORKLOADS = {
    # Race car scaled to the >= 1M candidates-per-tick target: 1024 x 1024 grid.
    "race_car_1m": dict(system="race_car", grid=[1024, 1024], H=60, gen="grid", S=1),
    # Race car at its stated size: 128 x 128 grid.
    "race_car": dict(system="race_car", grid=[128, 128], H=60, gen="grid", S=1),
    # Balance bot at real-time size: 10,240 five-segment random sequences.
    "balance_bot_rt": dict(system="balance_bot", N=10240, H=50, gen="uniform", S=5),
    # Balance bot small: 1,024-point grid.
    "balance_bot": dict(system="balance_bot", grid=[1024], H=20, gen="grid", S=1),
}


def setup(wl: dict, n_ticks: int):
    """GPU-side setup through the product path: fit K on the GPU, pack it, and
    place n_ticks tick inputs in HBM."""
    import torch

    import synth
    from paper_1906_02318_amd import mpmi

    ctx = mpmi.Context(0)
    if wl["system"] == "race_car":
        track = synth.make_track(3)
        X, U, Y = synth.race_car_transitions(50000, seed=0, track=track)
        trd = dict(r0=track.r0, half=track.half_width, amp=list(track.amp), freq=list(track.freq),
                   phase=list(track.phase), infl=0.0)
        system = mpmi.race_car_system(trd)
        xs = synth.race_car_states(n_ticks, track, seed=1)
        uh = synth.uniform_user(n_ticks, synth.RC_U_LO, synth.RC_U_HI, seed=2)
    else:
        track = None
        X, U, Y = synth.balance_bot_transitions(5000, seed=0)
        system = mpmi.balance_bot_system()
        xs = synth.balance_bot_states(n_ticks, seed=1)
        uh = synth.uniform_user(n_ticks, [synth.BB_U_LO], [synth.BB_U_HI], seed=2)
    d = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    Xd, Ud, Yd = d(X), d(U), d(Y)
    K, cond = mpmi.koopman_fit(ctx, system, Xd, Ud, Yd)  # first call: code load
    # Refit time (the FP64 fit is synchronous: it returns the condition estimate).
    t0 = time.perf_counter()
    K, cond = mpmi.koopman_fit(ctx, system, Xd, Ud, Yd)
    fit_ms = (time.perf_counter() - t0) * 1e3
    model = mpmi.mpmi_model_pack(ctx, system, K)
    x_dev = torch.tensor(xs, dtype=torch.float32, device="cuda").contiguous()
    u_dev = torch.tensor(uh, dtype=torch.float32, device="cuda").contiguous()
    if wl["gen"] == "grid":
        N = int(np.prod(wl["grid"]))
        mk = lambda t: mpmi.tick_desc(N, wl["H"], gen=mpmi.GEN_GRID, grid=wl["grid"])
    else:
        N = wl["N"]
        mk = lambda t: mpmi.tick_desc(N, wl["H"], gen=mpmi.GEN_UNIFORM, n_seg=wl["S"], seed=4, tick=t)
    torch.cuda.synchronize()
    return dict(ctx=ctx, model=model, K=K, x=x_dev, u=u_dev, xs=xs, uh=uh, N=N, mk=mk, track=track,
                fit=(X, U, Y), cond=cond, fit_ms=fit_ms)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl: dict, st: dict, budget_s: float = 15.0, budget_1t_s: float = 5.0):
    """FP64 oracle timed on this host's cores on a bounded sample of the same
    workload: every k-th candidate of each tick's candidate set; then the same
    sample with one BLAS thread."""
    cores = len(os.sched_getaffinity(0))
    multi = _cpu_oracle_rate(wl, st, cores, budget_s)
    one = _cpu_oracle_rate(wl, st, 1, budget_1t_s)
    multi.update(cores=cores, kind="oracle", cpu_model=cpu_model(),
                 one_thread={"value": one["value"], "unit": one["unit"], "sample": one["sample"]})
    return multi


def _cpu_oracle_rate(wl: dict, st: dict, cores: int, budget_s: float):
    from threadpoolctl import threadpool_limits

    from oracle import mpmi_oracle as o

    X, U, Y = st["fit"]
    kind = wl["system"]
    K, _ = o.fit(kind, X, U, Y)
    if kind == "race_car":
        tr = st["track"]
        f32 = lambda v: float(np.float32(v))
        sysd = o.System("race_car", 6, 2, box=[(4, 2.0, 0.0)],
                        track=dict(r0=30.0, half=3.0, amp=[f32(a) for a in tr.amp], freq=list(tr.freq),
                                   phase=[f32(p) for p in tr.phase], infl=0.0),
                        u_lo=[-0.4, -3.0], u_hi=[0.4, 3.0])
    else:
        sysd = o.System("balance_bot", 4, 1, box=[(2, 0.5, 0.0), (0, 2.0, 0.0)], u_lo=[-5.0], u_hi=[5.0])
    N, H, S = st["N"], wl["H"], wl["S"]
    stride = max(1, N // 16384)
    sample = None
    n_eval, t_used, ticks = 0, 0.0, 0
    with threadpool_limits(limits=cores):
        for t in range(len(st["xs"])):
            if wl["gen"] == "grid":
                full = o.grid_candidates(sysd, wl["grid"]) if sample is None else None
                if sample is None:
                    sample = full[::stride]
                cand = o.with_user(sample, st["uh"][t].astype(np.float32), 1)
            else:
                cand = o.with_user(o.uniform_candidates(sysd, N, S, 4, t, 0)[::stride],
                                   st["uh"][t].astype(np.float32), S)
            x = st["xs"][t].astype(np.float32).astype(np.float64)
            u = st["uh"][t].astype(np.float32).astype(np.float64)
            t0 = time.perf_counter()
            o.tick(sysd, K, x, u, cand, H)
            t_used += time.perf_counter() - t0
            n_eval += cand.shape[0]
            ticks += 1
            if t_used > budget_s:
                break
    return dict(value=n_eval / t_used, unit="trajectories/s",
                sample=f"{ticks} ticks x {n_eval // ticks} candidates (every {stride}th of the {N}-candidate set "
                       f"plus u_h), H={H}, FP64 NumPy, {cores} BLAS thread(s), {t_used:.1f} s")


def run_multi(n_ticks: int = 2000, warmup: int = 50, seed: int = 5):
    """64 closed control loops (32 cart-pole, 32 race car; N_l log-uniform in
    [1,024, 65,536], H_l in 20..60) served by one graph-replayed launch per tick.
    Each tick: inputs host->device, replay, selections device->host, plants and
    AR(1) users advanced on the host with the applied inputs."""
    import torch

    import synth
    from paper_1906_02318_amd import mpmi

    ctx = mpmi.Context(0)
    track = synth.make_track(3)
    d = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    Xb, Ub, Yb = synth.balance_bot_transitions(5000, seed=0)
    sb = mpmi.balance_bot_system()
    mb = mpmi.mpmi_model_pack(ctx, sb, mpmi.koopman_fit(ctx, sb, d(Xb), d(Ub), d(Yb))[0])
    Xr, Ur, Yr = synth.race_car_transitions(50000, seed=0, track=track)
    trd = dict(r0=track.r0, half=track.half_width, amp=list(track.amp), freq=list(track.freq),
               phase=list(track.phase), infl=0.0)
    sr = mpmi.race_car_system(trd)
    mr = mpmi.mpmi_model_pack(ctx, sr, mpmi.koopman_fit(ctx, sr, d(Xr), d(Ur), d(Yr))[0])
    scen = synth.ManyLoops(track, 64, seed=seed)
    N, H = scen.N, scen.H
    x_dev = torch.zeros((64, 8), dtype=torch.float32, device="cuda")
    u_dev = torch.zeros((64, 4), dtype=torch.float32, device="cuda")
    out_dev = torch.zeros((64, mpmi.SELECTION_BYTES), dtype=torch.uint8, device="cuda")
    x_pin = torch.zeros((64, 8), dtype=torch.float32).pin_memory()
    u_pin = torch.zeros((64, 4), dtype=torch.float32).pin_memory()
    o_pin = torch.zeros((64, mpmi.SELECTION_BYTES), dtype=torch.uint8).pin_memory()
    loops = [dict(model=mb if k == "bb" else mr, x_t=x_dev[i], u_user=u_dev[i], out=out_dev[i], n_cand=int(N[i]),
                  horizon=int(H[i]), gen=mpmi.GEN_UNIFORM, seed=scen.seeds[i], tick=0)
             for i, k in enumerate(scen.kinds)]
    multi = mpmi.Multi(ctx, loops)
    stream = torch.cuda.current_stream()
    x_pin.copy_(torch.from_numpy(scen.x))
    u_pin.copy_(torch.from_numpy(scen.u))
    x_dev.copy_(x_pin)
    u_dev.copy_(u_pin)
    tuned = multi.autotune(reps=10)
    multi.capture_graph()
    dev_ms, e2e_ms, interventions, nosafe = [], [], 0, 0
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for t in range(warmup + n_ticks):
        t0 = time.perf_counter()
        x_pin.copy_(torch.from_numpy(scen.x))
        u_pin.copy_(torch.from_numpy(scen.u))
        x_dev.copy_(x_pin, non_blocking=True)
        u_dev.copy_(u_pin, non_blocking=True)
        ev0.record(stream)
        multi.launch_graph(stream)
        ev1.record(stream)
        o_pin.copy_(out_dev, non_blocking=True)
        stream.synchronize()
        t1 = time.perf_counter()
        rec = o_pin.numpy()
        raw = rec.view(np.int32).reshape(64, -1)
        flt = rec.view(np.float32).reshape(64, -1)
        if t >= warmup:
            dev_ms.append(ev0.elapsed_time(ev1))
            e2e_ms.append((t1 - t0) * 1e3)
            interventions += int(np.sum(raw[:, 0] != 0))
            nosafe += int(np.sum(raw[:, 1] != 0))
        # plants advance with the applied inputs; users move on
        scen.advance(flt[:, 4:8], t)
    multi.close()
    dev = np.array(dev_ms)
    e2e = np.array(e2e_ms)
    cands = float(np.sum(N + 1))
    return {
        "workload": "64 loops (32 cart-pole + 32 race car), N_l log-uniform [1024, 65536] "
                    f"(sum {int(cands)}), H_l in [20, 60], closed loop, one graph replay per tick",
        "ticks": n_ticks, "autotuned": tuned,
        "trajectories_per_s_device": cands / (dev.mean() * 1e-3),
        "trajectories_per_s_end_to_end": cands / (e2e.mean() * 1e-3),
        "p50_tick_ms": float(np.percentile(dev, 50)), "p99_tick_ms": float(np.percentile(dev, 99)),
        "p50_end_to_end_ms": float(np.percentile(e2e, 50)), "p99_end_to_end_ms": float(np.percentile(e2e, 99)),
        "interventions_per_tick": interventions / n_ticks, "no_safe_per_tick": nosafe / n_ticks,
        "plant_resets": scen.resets,
    }


def run_closed_loop_balance_bot(n_ticks: int = 1000, warmup: int = 20):
    """Cart-pole at real-time size: N = 10,240 five-segment sequences, H = 50,
    a 1,000-tick closed loop (plant advanced on the host with the applied input,
    user input an AR(1) walk, rho 0.95, sigma 1 N) against a 10 ms budget."""
    import torch

    import synth
    from paper_1906_02318_amd import mpmi

    st = setup(WORKLOADS["balance_bot_rt"], 1)
    ctx, model = st["ctx"], st["model"]
    stream = torch.cuda.current_stream()
    x = synth.balance_bot_states(1, seed=3)[0]
    user = synth.AR1User([-5.0], [5.0], rho=0.95, sigma=1.0, seed=2)
    x_pin = torch.zeros(4, dtype=torch.float32).pin_memory()
    u_pin = torch.zeros(1, dtype=torch.float32).pin_memory()
    o_pin = torch.zeros(mpmi.SELECTION_BYTES, dtype=torch.uint8).pin_memory()
    x_dev = torch.zeros(4, dtype=torch.float32, device="cuda")
    u_dev = torch.zeros(1, dtype=torch.float32, device="cuda")
    out = torch.zeros(mpmi.SELECTION_BYTES, dtype=torch.uint8, device="cuda")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    dev_ms, e2e_ms, falls, interventions = [], [], 0, 0
    # launch shape (block, lanes per candidate) from the tick autotuner, on the
    # first tick's inputs
    x_dev.copy_(torch.from_numpy(x.astype(np.float32)))
    shape = mpmi.mpmi_tick_autotune(ctx, model, mpmi.tick_desc(10240, 50, gen=mpmi.GEN_UNIFORM, n_seg=5, seed=4),
                                    x_dev, u_dev, reps=20)
    for t in range(warmup + n_ticks):
        u = user.next()
        t0 = time.perf_counter()
        x_pin.copy_(torch.from_numpy(x.astype(np.float32)))
        u_pin.copy_(torch.from_numpy(u.astype(np.float32)))
        x_dev.copy_(x_pin, non_blocking=True)
        u_dev.copy_(u_pin, non_blocking=True)
        desc = mpmi.tick_desc(10240, 50, gen=mpmi.GEN_UNIFORM, n_seg=5, seed=4, tick=t, block=shape["block"],
                              lanes_per_cand=shape["lanes_per_cand"])
        ev0.record(stream)
        mpmi.mpmi_tick(ctx, model, desc, x_dev, u_dev, out=out, stream=stream)
        ev1.record(stream)
        o_pin.copy_(out, non_blocking=True)
        stream.synchronize()
        t1 = time.perf_counter()
        rec = o_pin.numpy()
        u_r = float(rec.view(np.float32)[4])
        if t >= warmup:
            dev_ms.append(ev0.elapsed_time(ev1))
            e2e_ms.append((t1 - t0) * 1e3)
            interventions += int(rec.view(np.int32)[0] != 0)
        x = synth.cartpole_step(x, np.array([u_r]))[0]
        if abs(x[2]) > 0.5 or abs(x[0]) > 2.0:
            falls += 1
            x = synth.balance_bot_states(1, seed=100 + t)[0]
    dev, e2e = np.array(dev_ms), np.array(e2e_ms)
    return {"workload": "cart-pole closed loop, N=10240 sequences (S=5) + u_h, H=50, AR(1) user",
            "ticks": n_ticks, "trajectories_per_s_device": 10241 / (dev.mean() * 1e-3),
            "p50_tick_ms": float(np.percentile(dev, 50)), "p99_tick_ms": float(np.percentile(dev, 99)),
            "p50_end_to_end_ms": float(np.percentile(e2e, 50)), "p99_end_to_end_ms": float(np.percentile(e2e, 99)),
            "within_10ms_budget": float(np.mean(e2e < 10.0)), "interventions": interventions,
            "safety_violations": falls, "launch_shape": shape}


def run_trajectory_store(st: dict, reps: int = 10):
    """Trajectory mode (the predicted-state cloud stored, traj[H][n][N+1],
    candidate index fastest) against the decision-only tick, race car, H = 60,
    at the stated size (128 x 128 grid) and at 1,024 x 1,024.  Bytes written
    = executed units x n x 4 (a lane stores the states it computes, up to its
    first violation)."""
    import torch

    from paper_1906_02318_amd import mpmi

    ctx, model = st["ctx"], st["model"]
    stream = torch.cuda.current_stream()
    H, n = 60, 6
    res = {}
    for name, side in (("race_car_16k", 128), ("race_car_1m", 1024)):
        N = side * side
        desc = mpmi.tick_desc(N, H, gen=mpmi.GEN_GRID, grid=[side, side])
        x, u = st["x"][0], st["u"][0]
        fv = torch.empty(N + 1, dtype=torch.int16, device="cuda")
        mpmi.mpmi_tick(ctx, model, desc, x, u, first_violation=fv)
        units = int(torch.clamp(fv.to(torch.int64), max=H).sum().item())
        ld = mpmi.traj_ld(N + 1)
        base = torch.empty(H * n * ld, dtype=torch.float32, device="cuda")
        traj = base.view(H, n, ld)[:, :, : N + 1]  # rows padded to 256-byte boundaries
        out = torch.empty(mpmi.SELECTION_BYTES, dtype=torch.uint8, device="cuda")
        times = {}
        for mode, tr in (("decision", None), ("trajectory", traj)):
            for _ in range(3):
                mpmi.mpmi_tick(ctx, model, desc, x, u, out=out, traj=tr, stream=stream)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
            for a, b in ev:
                a.record(stream)
                mpmi.mpmi_tick(ctx, model, desc, x, u, out=out, traj=tr, stream=stream)
                b.record(stream)
            torch.cuda.synchronize()
            times[mode] = float(np.median([a.elapsed_time(b) for a, b in ev]))
        wbytes = units * n * 4
        rate = wbytes / (times["trajectory"] * 1e-3) / 1e9
        # the layout's own write ceiling (the store pattern alone, padded rows
        # as used, and unpadded rows N + 1 floats apart for comparison) and a
        # contiguous stream, measured live on the same buffer
        ceil = mpmi.mpmi_write_rates(ctx, base, N + 1, H * n, ld=ld)
        ceil_unpadded = mpmi.mpmi_write_rates(ctx, base, N + 1, H * n, ld=N + 1)
        rceil = mpmi.mpmi_read_rates(ctx, base, N + 1, H * n, ld=ld)
        res[name] = {"candidates": N + 1, "executed_units": units, "traj_row_floats": ld,
                     "traj_bytes_allocated": base.numel() * 4,
                     "ms_decision": times["decision"], "ms_trajectory": times["trajectory"],
                     "bytes_written": wbytes, "write_GB_s": rate, "hbm_frac": rate / 8000.0,
                     "pattern_ceiling_GB_s": ceil["pattern_GB_s"], "stream_ceiling_GB_s": ceil["stream_GB_s"],
                     "pattern_ceiling_unpadded_GB_s": ceil_unpadded["pattern_GB_s"],
                     "pattern_frac": rate / ceil["pattern_GB_s"],
                     "read_pattern_ceiling_GB_s": rceil["pattern_GB_s"],
                     "read_stream_ceiling_GB_s": rceil["stream_GB_s"]}
        if side == 1024:
            # The same tick through the separable calls: candidates, full
            # rollout (no early exit: the mask decides afterwards), safe mask,
            # selection -- against the fused launch.
            cand = mpmi.mpmi_generate_candidates(ctx, model, desc, u)
            sel_f = mpmi.decode_selection(mpmi.mpmi_tick(ctx, model, desc, x, u))
            ph = {"rollout_batch": [], "safe_mask": [], "select_min_intervention": []}
            for r in range(reps + 2):
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
                ev[0].record(stream)
                mpmi.rollout_batch(ctx, model, x, cand, H, traj=traj, stream=stream)
                ev[1].record(stream)
                fvs, _ = mpmi.safe_mask(ctx, model, traj, with_margin=False, stream=stream)
                ev[2].record(stream)
                rec = mpmi.select_min_intervention(ctx, model, cand, fvs, H, u, stream=stream)
                ev[3].record(stream)
                torch.cuda.synchronize()
                if r >= 2:
                    for k, name in enumerate(ph):
                        ph[name].append(ev[k].elapsed_time(ev[k + 1]))
            sel_s = mpmi.decode_selection(rec)
            res["separable_calls_1m"] = {k: float(np.median(v)) for k, v in ph.items()}
            res["separable_calls_1m"]["ms_total"] = float(sum(np.median(v) for v in ph.values()))
            res["separable_calls_1m"]["ms_fused_tick"] = times["decision"]
            res["separable_calls_1m"]["same_selection"] = bool(sel_s == sel_f)
            # safe_mask needs the states up to each first violation: the
            # executed units' bytes, against the read ceiling of its pattern
            mask_gbs = wbytes / (float(np.median(ph["safe_mask"])) * 1e-3) / 1e9
            res["separable_calls_1m"]["safe_mask_read_GB_s"] = mask_gbs
            res["separable_calls_1m"]["safe_mask_read_frac"] = mask_gbs / rceil["pattern_GB_s"]
            del cand
        del traj, base
        torch.cuda.empty_cache()
    return res


def timed_ticks(step, n_ticks: int, warmup: int, stream):
    """Per-tick device times (HIP events on `stream`) and the wall time of n_ticks calls of step(t)."""
    import torch

    for t in range(warmup):
        step(t)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_ticks)]
    t0 = time.perf_counter()
    for t in range(n_ticks):
        ev[t][0].record(stream)
        step(t)
        ev[t][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return np.array([a.elapsed_time(b) for a, b in ev]), wall


def run_precision(st: dict, precision: int, n_ticks: int = 100, warmup: int = 5):
    """The headline ticks in another arithmetic: plain FP32 (verdicts inside
    the FP32 rounding band decided in FP32), or FP32 with the FP64 re-roll of
    that band (every candidate whose FP32 margin comes within 2e-3 m of the
    track edge or 3e-4 m/s of the v_y bound is listed, and those that can
    still change the selection are predicted again in FP64)."""
    import torch

    from paper_1906_02318_amd import mpmi

    ctx, model, N = st["ctx"], st["model"], st["N"]
    stream = torch.cuda.current_stream()
    outs = torch.empty((64, mpmi.SELECTION_BYTES), dtype=torch.uint8, device="cuda")
    descs = [st["mk"](t) for t in range(64)]
    for d in descs:
        d.precision = precision

    def step(t):
        i = t % 64
        mpmi.mpmi_tick(ctx, model, descs[i], st["x"][i], st["u"][i], out=outs[i], stream=stream)

    ms, wall = timed_ticks(step, n_ticks, warmup, stream)
    out = {"trajectories_per_s": (N + 1) * n_ticks / wall, "ms_per_tick": wall * 1e3 / n_ticks,
           "p50_tick_ms": float(np.percentile(ms, 50)), "p99_tick_ms": float(np.percentile(ms, 99)),
           "mean_tick_ms": float(ms.mean())}
    if precision == mpmi.PREC_FP32_RECHECK64:
        re = [s_["n_recheck"] for s_ in mpmi.decode_selection(outs)[:min(n_ticks, 64)]]
        out.update({"listed_per_tick_mean": float(np.mean(re)), "listed_per_tick_max": int(np.max(re)),
                    "note": "FP32 tick listing its rounding band + filter + FP64 re-roll of the kept "
                            "candidates; decisions those of FP64 rollouts (tests: 1M tick identical to the "
                            "full oracle)"})
    else:
        out["note"] = ("plain FP32: the decision inside the FP32 rounding band is FP32's (tests: the 1M tick "
                       "picks a different candidate than the FP64 oracle; closed-loop agreement 99.5%)")
    return out


def run_lifted(st: dict, wl: dict, n_ticks: int = 100, warmup: int = 5):
    """The same ticks in the lifted whole-horizon form (Sec. IV-A's batch
    prediction as one matrix product): the full lifted operator fitted on the
    GPU, powers folded on the host, every candidate's horizon as
    [candidates x 12] x [12 x 4 H] products on v_mfma_f32_16x16x4f32 with the
    safety check on each output tile."""
    import torch

    from paper_1906_02318_amd import mpmi

    ctx, model, N, H = st["ctx"], st["model"], st["N"], wl["H"]
    stream = torch.cuda.current_stream()
    X, U, Y = st["fit"]
    d = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    KL, cond = mpmi.koopman_fit_lifted(ctx, model.system, d(X), d(U), d(Y))
    fit_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    lifted = mpmi.mpmi_lifted_pack(ctx, model, KL, H)
    pack_ms = (time.perf_counter() - t0) * 1e3
    outs = torch.empty((64, mpmi.SELECTION_BYTES), dtype=torch.uint8, device="cuda")
    descs = [st["mk"](t) for t in range(64)]
    fv = torch.empty(N + 1, dtype=torch.int16, device="cuda")
    units = []
    for i in range(64):
        mpmi.mpmi_tick_lifted(ctx, lifted, descs[i], st["x"][i], st["u"][i], out=outs[i], first_violation=fv,
                              stream=stream)
        units.append(int(torch.clamp(fv.to(torch.int64), max=H).sum().item()))

    def step(t):
        i = t % 64
        mpmi.mpmi_tick_lifted(ctx, lifted, descs[i], st["x"][i], st["u"][i], out=outs[i], stream=stream)

    ms, wall = timed_ticks(step, n_ticks, warmup, stream)
    units_tick = float(np.mean([units[t % 64] for t in range(n_ticks)]))
    # Matrix-core work: per 16 candidates x 4 steps, three 16x16x4 FP32 MFMAs
    # (2 * 16 * 16 * 12 flops), i.e. 96 flops per candidate-step, of which the
    # 9 input functions x 4 output slots are algorithmic (72).
    mfma_tflops = 96.0 * units_tick / (float(ms.mean()) * 1e-3) / 1e12
    return {"trajectories_per_s": (N + 1) * n_ticks / wall, "ms_per_tick": wall * 1e3 / n_ticks,
            "p50_tick_ms": float(np.percentile(ms, 50)), "p99_tick_ms": float(np.percentile(ms, 99)),
            "units_per_tick": units_tick, "lifted_fit_ms": fit_ms, "lifted_pack_ms": pack_ms, "cond": cond,
            "mfma_tflops_executed_lower_bound": mfma_tflops, "mfma_peak_fp32_tflops": PEAK_FP32_VECTOR_TFLOPS,
            "note": "lifted predictions differ from the re-lifting model's (tests: median position error vs the "
                    "plant 0.68 m lifted / 0.31 m re-lift at step 60); MFMA busy from rocprofv3 counters in "
                    "profiles/"}


MLP_FLOPS_PER_SAMPLE = 917504  # forward 2(8*256 + 2*256*256 + 256*80) + the same for dW + dX of layers 1..3
PEAK_BF16_MFMA_TFLOPS = 2500.0


def run_mlp_training(batch: int = 4096, steps: int = 50, warmup: int = 5):
    """One training step of the proposal network (forward, mixture loss,
    backward, Adam) on the library's kernels, synthetic rows: step time, and
    the BF16 matrix-core rate of its dense products."""
    import torch

    import synth
    from paper_1906_02318_amd import mpmi
    from paper_1906_02318_amd.proposal import ProposalNet

    ctx = mpmi.Context(0)
    rng = np.random.default_rng(21)
    X = rng.normal(size=(batch, 8)).astype(np.float32)
    T = rng.uniform(-0.9, 0.9, size=(batch, 2)).astype(np.float32)
    net = ProposalNet(ctx, synth.mlp_init(6), X.mean(axis=0), X.std(axis=0))
    Xd, Td = torch.tensor(X, device="cuda"), torch.tensor(T, device="cuda")
    work = mpmi.mlp_workspace(ctx, batch)
    grad = torch.empty(mpmi.MLP_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def step(t):
        mpmi.mlp_grad(ctx, net.w16, net.w32, net.mean, net.std, Xd, Td, work=work, grad=grad, loss=loss,
                      stream=stream)
        net.step += 1
        mpmi.mlp_adam(ctx, net.w32, net.w16, net.m, net.v, grad, net.step, 1e-3, stream=stream)

    ms, wall = timed_ticks(step, steps, warmup, stream)
    step_ms = float(np.median(ms))
    tflops = MLP_FLOPS_PER_SAMPLE * batch / (step_ms * 1e-3) / 1e12
    return {"batch": batch, "step_ms_p50": step_ms, "step_ms_wall": wall * 1e3 / steps,
            "tflops": tflops, "bf16_mfma_peak_tflops": PEAK_BF16_MFMA_TFLOPS,
            "mfma_frac": tflops / PEAK_BF16_MFMA_TFLOPS,
            "note": (f"11 dense products of at most {batch} x 256 x 256 plus loss, split-K reductions and "
                     "Adam; " + ("launch- and latency-bound" if batch <= 8192 else
                                 "HBM-bound (37-51 flops per byte moved)") + "; kernel times in profiles/")}


def run_plain_vs_learned(n_ticks: int = 500, warmup: int = 20):
    """Race car at its stated size: exhaustive 128 x 128 grid tick vs the learned
    2,048-proposal tick (exhaustive fallback), on the same tick inputs."""
    import torch

    import synth
    from paper_1906_02318_amd import mpmi
    from paper_1906_02318_amd.proposal import ASSET, LearnedTicker, ProposalNet

    st = setup(WORKLOADS["race_car"], 64)
    ctx, model = st["ctx"], st["model"]
    stream = torch.cuda.current_stream()
    # Launch shapes (block, lanes per candidate) of both forms from the tick
    # autotuner, on the first tick's inputs.
    plain = mpmi.tick_desc(128 * 128, 60, gen=mpmi.GEN_GRID, grid=[128, 128], loop=0)
    shapes = {"plain": mpmi.mpmi_tick_autotune(ctx, model, plain, st["x"][0], st["u"][0], reps=20)}
    out = {}
    runs = [("plain", None)]
    if os.path.exists(ASSET):
        ticker = LearnedTicker(ctx, model, ProposalNet.load(ctx, ASSET))
        ticker.tick(st["x"][0], st["u"][0], tick=0)  # fills ticker.cand with the first tick's proposals
        pdesc = mpmi.tick_desc(ticker.P, ticker.H, gen=mpmi.GEN_EXPLICIT, loop=ticker.loop)
        shapes["learned"] = mpmi.mpmi_tick_autotune(ctx, model, pdesc, st["x"][0], st["u"][0],
                                                    cand=ticker.cand.reshape(-1), reps=20)
        ticker.lanes, ticker.block = pdesc.lanes_per_cand, pdesc.block
        runs.append(("learned", ticker))
    for name, ticker in runs:
        outs = torch.empty((64, mpmi.SELECTION_BYTES), dtype=torch.uint8, device="cuda")

        def step(t):
            i = t % 64
            if ticker is None:
                mpmi.mpmi_tick(ctx, model, plain, st["x"][i], st["u"][i], out=outs[i], stream=stream)
            else:
                ticker.tick(st["x"][i], st["u"][i], tick=t, out=outs[i], stream=stream)

        for t in range(warmup):
            step(t)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_ticks)]
        n_eval = 0
        t0 = time.perf_counter()
        for t in range(n_ticks):
            ev[t][0].record(stream)
            step(t)
            ev[t][1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = np.array([a.elapsed_time(b) for a, b in ev])
        sels = mpmi.decode_selection(outs)
        ncand = float(np.mean([s["n_cand"] for s in sels]))
        out[name] = {"trajectories_per_s": ncand * n_ticks / wall, "candidates_per_tick": ncand,
                     "p50_tick_ms": float(np.percentile(ms, 50)), "p99_tick_ms": float(np.percentile(ms, 99)),
                     "ms_per_tick": wall * 1e3 / n_ticks, "launch_shape": shapes[name]}
        if ticker is not None:
            out[name]["fallback_rate"] = float(np.mean([s["n_cand"] != ticker.P + 1 for s in sels]))
    if "learned" not in out:
        out["learned"] = None
    else:
        # Decision quality of the learned ticks against exhaustive 128 x 128 ticks
        # (and of 2,048 uniform samples, the method without the network).
        from paper_1906_02318_amd.train_proposal import evaluate
        out["learned"]["quality"] = evaluate(ctx, model, ProposalNet.load(ctx, ASSET), st["track"], n_ticks=300,
                                             log=lambda m: None)
    return out


LEGS = ("bf16x3", "other_precision", "lifted", "trajectory", "learned", "mlp", "multi", "closed_loop")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="race_car_1m", choices=sorted(WORKLOADS))
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--precision", default="fp32_recheck64", choices=["fp32", "fp32_recheck64"],
                    help="arithmetic of the headline ticks (fp32_recheck64: FP32 with the FP64 re-roll of the "
                         "FP32 rounding band, the decisions of FP64 rollouts)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-extras", action="store_true", help="skip every leg after the headline ticks")
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="comma-separated legs to run after the headline ticks (of: " + ", ".join(LEGS) + ")")
    ap.add_argument("--multi-ticks", type=int, default=10000)
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="after timing, run one device-to-device copy of this many bytes (counter calibration)")
    args = ap.parse_args()
    legs = set() if args.no_extras or args.workload != "race_car_1m" else {x for x in args.legs.split(",") if x}
    if legs - set(LEGS):
        ap.error(f"unknown legs {sorted(legs - set(LEGS))}")
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the tick's candidates would shard "
              f"across GPUs with one 8-byte arg-min exchange per loop; multi-GPU runs are not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1906_02318_amd import mpmi

    wl = WORKLOADS[args.workload]
    n_inputs = 64
    st = setup(wl, n_inputs)
    ctx, model, N, H = st["ctx"], st["model"], st["N"], wl["H"]
    Nc = N + 1
    stream = torch.cuda.current_stream()
    outs = torch.empty((n_inputs, mpmi.SELECTION_BYTES), dtype=torch.uint8, device="cuda")
    prec = mpmi.PREC_FP32_RECHECK64 if args.precision == "fp32_recheck64" else mpmi.PREC_FP32
    descs = [st["mk"](t) for t in range(n_inputs)]
    for d in descs:
        d.block = args.block
        d.precision = prec

    def step(i):
        t = i % n_inputs
        mpmi.mpmi_tick(ctx, model, descs[t], st["x"][t], st["u"][t], out=outs[t], stream=stream)

    # Executed units (candidate-steps after early exit), from an untimed pass.
    fv = torch.empty(Nc, dtype=torch.int16, device="cuda")
    units = []
    for t in range(n_inputs):
        mpmi.mpmi_tick(ctx, model, descs[t], st["x"][t], st["u"][t], out=outs[t], first_violation=fv, stream=stream)
        units.append(int(torch.clamp(fv.to(torch.int64), max=H).sum().item()))
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        step(i)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dev_ms = np.array([a.elapsed_time(b) for a, b in ev])
    sels = mpmi.decode_selection(outs)
    n_safe_frac = float(np.mean([s["n_safe"] / N for s in sels]))
    zero_int = float(np.mean([s["idx"] == 0 for s in sels]))

    ms_per_step = wall * 1e3 / args.steps
    value = Nc * args.steps / wall
    units_per_tick = float(np.mean([units[i % n_inputs] for i in range(args.steps)]))
    avg_kernel_s = float(dev_ms.mean()) * 1e-3
    flops = FLOPS_PER_UNIT[wl["system"]] * units_per_tick
    achieved = flops / avg_kernel_s / 1e12
    traffic = traffic_record(args.workload, args.precision)
    fma_ceiling = mpmi.mpmi_fp32_fma_rate(ctx)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "trajectories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32+fp64" if prec == mpmi.PREC_FP32_RECHECK64 else "fp32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {wl['system']} tick, N={N} candidates + u_h, H={H}, "
                        f"{'grid ' + 'x'.join(map(str, wl['grid'])) if wl['gen'] == 'grid' else 'uniform S=' + str(wl['S'])}",
            "N": N, "H": H, "system": wl["system"], "precision": args.precision, "plain_or_learned": "plain",
        },
        "p50_tick_ms": float(np.percentile(dev_ms, 50)),
        "p99_tick_ms": float(np.percentile(dev_ms, 99)),
        "ticks_within_10ms": float(np.mean(dev_ms < 10.0)),
        "units_per_tick": units_per_tick,
        "units_per_s": units_per_tick * args.steps / wall,
        "safe_fraction": n_safe_frac,
        "koopman_fit": {"rows": int(st["fit"][0].shape[0]), "dim": int(st["K"].shape[0]), "ms": st["fit_ms"],
                        "cond": st["cond"]},
        "zero_intervention_fraction": zero_int,
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_VECTOR_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
            "traffic": traffic[0],
            "traffic_detail": traffic[1],
            "kernel": (f"tick_fp32_kernel<{wl['system']}, listing> + filter + FP64 re-roll (one tick, "
                       f"three launches)" if prec == mpmi.PREC_FP32_RECHECK64
                       else f"tick_fp32_kernel<{wl['system']}>"),
            "avg_kernel_ms": avg_kernel_s * 1e3,
            "flops_per_unit": FLOPS_PER_UNIT[wl["system"]],
            "executed_flops_per_unit": EXECUTED_FLOPS_PER_UNIT[wl["system"]],
            "executed_tflops": EXECUTED_FLOPS_PER_UNIT[wl["system"]] * units_per_tick / avg_kernel_s / 1e12,
            "fp32_fma_ceiling_tflops": fma_ceiling,
            "note": "algorithmic = plain psi^T K step of the FP32 pass over the whole tick's device time (with "
                    "fp32_recheck64 the filter and FP64 re-roll launches count as time, not flops); the kernel "
                    "folds input terms once per segment and executes fewer flops; packed FP32 is disabled, so "
                    "the reachable vector rate is the non-packed FMA ceiling measured live "
                    "(fp32_fma_ceiling_tflops; 78.6 theoretical)",
        },
    }
    if "bf16x3" in legs:
        # Same ticks with the shared-coefficient contraction on BF16 matrix cores
        # (hi/lo split) and the FP32 recheck of near-boundary candidates.
        bdescs = [st["mk"](t) for t in range(n_inputs)]
        for d in bdescs:
            d.precision = mpmi.PREC_BF16X3
        for i in range(5):
            mpmi.mpmi_tick(ctx, model, bdescs[i % n_inputs], st["x"][i % n_inputs], st["u"][i % n_inputs],
                           out=outs[i % n_inputs], stream=stream)
        torch.cuda.synchronize()
        nb = min(args.steps, 100)
        evb = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nb)]
        t0b = time.perf_counter()
        for i in range(nb):
            t = i % n_inputs
            evb[i][0].record(stream)
            mpmi.mpmi_tick(ctx, model, bdescs[t], st["x"][t], st["u"][t], out=outs[t], stream=stream)
            evb[i][1].record(stream)
        torch.cuda.synchronize()
        wb = time.perf_counter() - t0b
        msb = np.array([a.elapsed_time(b) for a, b in evb])
        sb = mpmi.decode_selection(outs)
        out["race_car_1m_bf16x3"] = {
            "trajectories_per_s": Nc * nb / wb, "p50_tick_ms": float(np.percentile(msb, 50)),
            "p99_tick_ms": float(np.percentile(msb, 99)),
            # the records the BF16 ticks wrote (inputs 0 .. min(nb, n_inputs) - 1)
            "rechecked_per_tick": float(np.mean([s_["n_recheck"] for s_ in sb[:min(nb, n_inputs)]])),
            "note": "27 shared-coefficient features on v_mfma_f32_16x16x32_bf16 (hi/lo split), FP32 recheck "
                    "of candidates within 0.02 of a constraint; two launches per tick"}
    if args.copy_bytes > 0:
        src = torch.empty(args.copy_bytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = args.copy_bytes
    if "other_precision" in legs:
        if prec == mpmi.PREC_FP32_RECHECK64:
            out["race_car_1m_fp32"] = run_precision(st, mpmi.PREC_FP32)
        else:
            out["race_car_1m_fp32_recheck64"] = run_precision(st, mpmi.PREC_FP32_RECHECK64)
    if "lifted" in legs:
        out["race_car_1m_lifted"] = run_lifted(st, wl)
    if "trajectory" in legs:
        out["trajectory_store"] = run_trajectory_store(st)
    if "learned" in legs:
        out["race_car_16k"] = run_plain_vs_learned()
    if "mlp" in legs:
        out["mlp_training"] = run_mlp_training()
        # the same step at a batch large enough that the products are not latency-bound
        out["mlp_training"]["batch_65536"] = run_mlp_training(batch=65536, steps=20)
    if "multi" in legs:
        out["many_loops"] = run_multi(n_ticks=args.multi_ticks)
    if "closed_loop" in legs:
        out["balance_bot_closed_loop"] = run_closed_loop_balance_bot()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, st, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
