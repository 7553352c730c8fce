"""Trains the race-car proposal network on labels produced by the exhaustive
tick, then evaluates it against the exhaustive sampler.

python -m paper_1906_02318_amd.train_proposal --labels 2000000 --epochs 40 --out PATH

Prints one JSON summary line (labels, losses, agreement and cost gaps).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from paper_1906_02318_amd import mpmi  # noqa: E402
from paper_1906_02318_amd.proposal import ProposalNet, LearnedTicker, generate_labels, normalise, train  # noqa: E402

HALF_CELL_DIAG_128 = np.sqrt(2.0) * (2.0 / 128) / 2.0  # normalised units


def race_car_model(ctx):
    track = synth.make_track(3)
    X, U, Y = synth.race_car_transitions(50000, seed=0, track=track)
    d = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    trd = dict(r0=track.r0, half=track.half_width, amp=list(track.amp), freq=list(track.freq),
               phase=list(track.phase), infl=0.0)
    system = mpmi.race_car_system(trd)
    K, _ = mpmi.koopman_fit(ctx, system, d(X), d(U), d(Y))
    return track, mpmi.mpmi_model_pack(ctx, system, K)


def evaluate(ctx, model, net, track, n_ticks=1000, seed=8, proposals=2048, log=print, precision=mpmi.PREC_FP32):
    """Learned ticks vs exhaustive 128 x 128 ticks vs 2,048 uniform samples on
    the same states.  Rates are over the ticks the exhaustive grid decides
    (some grid candidate safe); the fallback rate is over all ticks."""
    xs = synth.race_car_states(n_ticks, track, seed=seed)
    uh = synth.uniform_user(n_ticks, synth.RC_U_LO, synth.RC_U_HI, seed=seed + 100)
    ticker = LearnedTicker(ctx, model, net, proposals=proposals, precision=precision)
    exh = mpmi.tick_desc(128 * 128, 60, gen=mpmi.GEN_GRID, grid=[128, 128], loop=3)
    lo, hi = synth.RC_U_LO, synth.RC_U_HI
    res = dict(agree_learned=0, agree_uniform=0, fallback=0, ticks=n_ticks, gap_learned=[], gap_uniform=[],
               interventions=0, asgood_learned=0, asgood_uniform=0, decided=0)
    for t in range(n_ticks):
        xt = torch.tensor(xs[t], dtype=torch.float32, device="cuda")
        ut = torch.tensor(uh[t], dtype=torch.float32, device="cuda")
        sl = mpmi.decode_selection(ticker.tick(xt, ut, tick=t))
        se = mpmi.decode_selection(mpmi.mpmi_tick(ctx, model, exh, xt, ut))
        uni = mpmi.tick_desc(proposals, 60, gen=mpmi.GEN_UNIFORM, seed=seed, tick=t, loop=4)
        su = mpmi.decode_selection(mpmi.mpmi_tick(ctx, model, uni, xt, ut))
        res["fallback"] += int(sl["n_cand"] != proposals + 1)
        if se["status"] != mpmi.OK:
            continue
        res["decided"] += 1
        res["interventions"] += int(se["idx"] != 0)
        ue = normalise(se["u_r"][:2], lo, hi)
        for name, s in (("learned", sl), ("uniform", su)):
            same_zero = (s["idx"] == 0) == (se["idx"] == 0)
            close = np.linalg.norm(normalise(s["u_r"][:2], lo, hi) - ue) <= HALF_CELL_DIAG_128
            ok = s["status"] == mpmi.OK and same_zero and (se["idx"] == 0 or close)
            res[f"agree_{name}"] += int(ok)
            if s["status"] == mpmi.OK:
                res[f"gap_{name}"].append(s["cost"] - se["cost"])
                # as good as the exhaustive grid: a safe choice no costlier than the
                # grid's, up to the cost of half a grid cell's diagonal
                res[f"asgood_{name}"] += int(s["cost"] <= se["cost"] + HALF_CELL_DIAG_128 ** 2)
    n_ok = max(1, res["decided"])
    out = dict(ticks=n_ticks, decided=res["decided"], interventions=res["interventions"],
               fallback_rate=res["fallback"] / n_ticks,
               agreement_learned=res["agree_learned"] / n_ok, agreement_uniform=res["agree_uniform"] / n_ok,
               as_good_learned=res["asgood_learned"] / max(1, res["decided"]),
               as_good_uniform=res["asgood_uniform"] / max(1, res["decided"]),
               mean_cost_gap_learned=float(np.mean(res["gap_learned"])) if res["gap_learned"] else None,
               mean_cost_gap_uniform=float(np.mean(res["gap_uniform"])) if res["gap_uniform"] else None)
    log(json.dumps(out))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--labels", type=int, default=2_000_000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval-ticks", type=int, default=1000)
    ap.add_argument("--out", default="proposal_net.npz", help="where the trained network is saved (the served one is assets/proposal_net.npz)")
    ap.add_argument("--eval-only", default=None, help="evaluate a saved network instead of training")
    args = ap.parse_args()
    log = lambda m: print(m, flush=True)
    ctx = mpmi.Context(0)
    track, model = race_car_model(ctx)
    if args.eval_only:
        net = ProposalNet.load(ctx, args.eval_only)
        print(json.dumps(dict(eval=evaluate(ctx, model, net, track, n_ticks=args.eval_ticks, log=log))), flush=True)
        return
    states = synth.race_car_states(args.labels, track, seed=7)
    users = synth.uniform_user(args.labels, synth.RC_U_LO, synth.RC_U_HI, seed=17)
    t0 = time.perf_counter()
    u_star, status, _ = generate_labels(ctx, model, states, users, log=log)
    t_labels = time.perf_counter() - t0
    keep = status == mpmi.OK
    log(f"labels: {keep.sum()} of {args.labels} usable ({t_labels:.1f} s)")
    X = np.concatenate([states, users], axis=1)[keep]
    T = normalise(u_star[keep], synth.RC_U_LO, synth.RC_U_HI)
    net = ProposalNet(ctx, synth.mlp_init(6), X.mean(axis=0), X.std(axis=0))
    t1 = time.perf_counter()
    losses = train(ctx, net, X, T, args.epochs, batch=args.batch, lr=args.lr, log=log)
    t_train = time.perf_counter() - t1
    net.save(args.out)
    ev = evaluate(ctx, model, net, track, n_ticks=args.eval_ticks, log=log)
    print(json.dumps(dict(labels=int(args.labels), usable=int(keep.sum()), label_seconds=t_labels,
                          train_seconds=t_train, steps=net.step, losses=losses, eval=ev)), flush=True)


if __name__ == "__main__":
    main()
