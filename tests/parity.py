"""Comparison rules between the GPU library and the FP64 oracle.

* Rollout states: relative error |x_gpu - x_64| / max(|x_64|, floor_j) per
  component, floor_j the constraint bound or the data standard deviation;
  states the oracle predicts beyond 1e6 floors (diverged, unsafe on both
  sides) are excluded.
* Safety verdicts: first violations must be identical except for candidates
  whose oracle margin comes within eps_j of zero at some step up to the
  earlier of the two first violations (ambiguous by FP32 rounding).
* Selection, complete: the GPU's choice, status and safe count are those of
  the selection rule (Alg. 2 selection step; the fallback rule when nothing
  is safe) applied to the GPU's own first violations -- which the previous
  rule ties to the oracle's everywhere outside the eps band.  A different
  candidate of equal first violation and equal FP64 cost (to 1e-6
  relative; the GPU ranks FP32 costs) is accepted.
* Agreement with the oracle's decision (counted, not assumed): the same
  candidate ("identical"), or two candidates both oracle-safe or ambiguous
  whose FP64 costs agree to 1e-6 relative ("equal_cost").  Any other outcome
  ("eps_band") can only come from ambiguous verdicts, by the two rules above,
  and counts as a disagreement.

FP32_RECHECK64 ticks (FP32 tick, FP64 re-roll of the band's candidates that
could precede the best key outside the band -- all of them when nothing
outside the band is safe): a tick that found nothing safe re-rolled every
band candidate, so its first violations must equal the oracle's wherever its
margins are not within FP64 rounding of zero (EPS64, 1e-9); any other tick is
held to the FP32 band, and its decision must agree (the re-roll makes the
selection the FP64 one).

Long replays run the oracle in a pool of worker processes (spawn context;
the workers import only NumPy and the oracle, never the GPU library).
"""
from __future__ import annotations

import multiprocessing
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from oracle import mpmi_oracle as o


# Band for verdicts computed in FP64 on the GPU (margins of order one,
# rollouts of at most a few hundred steps).
EPS64 = 1e-9


def eps64(sys: o.System) -> list:
    """The FP64 band for every constraint of sys."""
    return [EPS64] * (len(sys.box) + (1 if sys.track is not None else 0))


def recheck64_eps(sys: o.System, sel: dict, eps32) -> list:
    """The band an FP32_RECHECK64 record is judged with (see the header)."""
    return eps64(sys) if sel["status"] != o.STATUS_OK else list(eps32)


def rollout_rel_err(x_gpu: np.ndarray, x_64: np.ndarray, floors: np.ndarray, comp_axis: int) -> float:
    shape = [1] * x_64.ndim
    shape[comp_axis] = -1
    fl = floors.reshape(shape)
    with np.errstate(invalid="ignore", over="ignore"):
        keep = np.isfinite(x_64) & (np.abs(x_64) < 1e6 * fl)
        err = np.abs(x_gpu.astype(np.float64) - x_64) / np.maximum(np.abs(x_64), fl)
    err = np.where(keep, err, 0.0)
    bad = keep & ~np.isfinite(err)
    assert not bad.any(), "GPU produced non-finite states where the oracle is finite"
    return float(err.max()) if err.size else 0.0


def ambiguous(sys: o.System, traj64: np.ndarray, fv_a: np.ndarray, fv_b: np.ndarray, eps) -> np.ndarray:
    """traj64 (H, Nc, n) full-horizon oracle states; True where some step
    s <= min(fv_a, fv_b, H) has a margin within eps of zero."""
    H, Nc, n = traj64.shape
    with np.errstate(invalid="ignore"):
        M = o.margins(sys, traj64.reshape(H * Nc, n)).reshape(H, Nc, -1)
        near = np.any(np.abs(M) < np.asarray(eps).reshape(1, 1, -1), axis=2)
    upto = np.minimum(np.minimum(fv_a, fv_b), H)
    steps = np.arange(1, H + 1)[:, None]
    return np.any(near & (steps <= upto[None, :]), axis=0)


def _same_choice(cost, fv, i, j) -> bool:
    return i == j or (fv[i] == fv[j] and abs(cost[i] - cost[j]) <= 1e-6 * max(abs(cost[j]), 1e-30))


def check_selection(sys: o.System, cand64: np.ndarray, H: int, u_h, sel: dict, fv_gpu: np.ndarray,
                    label: str = "") -> dict:
    """The GPU's record is the selection rule over its own first violations."""
    fv_gpu = np.asarray(fv_gpu, np.int64)
    own = o.select(sys, cand64, fv_gpu, H, u_h)
    cost = o.cost(sys, cand64, u_h)
    i_g = sel["idx"]
    assert 0 <= i_g < fv_gpu.size, f"{label}: index {i_g} out of range"
    assert _same_choice(cost, fv_gpu, i_g, own["idx"]), (
        f"{label}: GPU chose {i_g} (cost {cost[i_g]:.9g}, fv {fv_gpu[i_g]}) but its own verdicts select "
        f"{own['idx']} (cost {cost[own['idx']]:.9g}, fv {fv_gpu[own['idx']]})")
    assert sel["status"] == own["status"], f"{label}: status {sel['status']} vs {own['status']} over its verdicts"
    assert sel["n_safe"] == own["n_safe"], f"{label}: n_safe {sel['n_safe']} vs {own['n_safe']} over its verdicts"
    if "first_violation" in sel:
        assert sel["first_violation"] == fv_gpu[i_g], f"{label}: record's first violation"
    np.testing.assert_array_equal(np.asarray(sel["u_r"][: sys.m], np.float64), cand64[i_g, 0, :])
    return own


def judge(sys: o.System, cand64: np.ndarray, H: int, u_h, traj64: np.ndarray, fv_o: np.ndarray, sel: dict,
          fv_gpu: np.ndarray, eps, label: str = "") -> dict:
    """Checks one GPU tick against an oracle rollout (full horizon, traj64
    (H, Nc, n), first violations fv_o); returns counters for reporting."""
    fv_gpu = np.asarray(fv_gpu, np.int64)
    amb = ambiguous(sys, traj64, fv_o, fv_gpu, eps)
    mism = (fv_o != fv_gpu) & ~amb
    assert not mism.any(), (f"{label}: first-violation mismatch outside the eps band at candidates "
                            f"{np.nonzero(mism)[0][:10]} (oracle {fv_o[mism][:10]}, gpu {fv_gpu[mism][:10]})")
    check_selection(sys, cand64, H, u_h, sel, fv_gpu, label)
    return agreement(sys, cand64, H, u_h, fv_o, amb, sel)


def agreement(sys: o.System, cand64: np.ndarray, H: int, u_h, fv_o: np.ndarray, amb: np.ndarray, sel: dict) -> dict:
    """Agreement of the GPU's decision with the oracle's (see the module header)."""
    ref = o.select(sys, cand64, fv_o, H, u_h)
    cost = o.cost(sys, cand64, u_h)
    i_g, i_o = sel["idx"], ref["idx"]
    safe_o = fv_o == H + 1
    if i_g == i_o:
        kind = "identical"
    elif ((safe_o[i_g] or amb[i_g]) and (safe_o[i_o] or amb[i_o])
          and abs(cost[i_g] - cost[i_o]) <= 1e-6 * max(abs(cost[i_o]), 1e-30)):
        kind = "equal_cost"
    else:
        kind = "eps_band"
        assert amb.any(), "a disagreement with no ambiguous verdict"
    if not amb.any():
        assert sel["status"] == ref["status"] and sel["n_safe"] == ref["n_safe"]
    return dict(kind=kind, ambiguous=int(amb.sum()), status=ref["status"], idx=i_o, gpu_idx=i_g,
                n_safe=ref["n_safe"], zero_intervention=bool(i_o == 0),
                cost_gap=float(cost[i_g] - cost[i_o]))


def check_tick(sys: o.System, K, x_t, u_h, cand64: np.ndarray, H: int, sel: dict, fv_gpu: np.ndarray, eps,
               label: str = "", noise_key=None) -> dict:
    """Checks one GPU tick against the oracle; returns counters for reporting."""
    traj, fv_o = o.rollout(sys, K, x_t, cand64, H, early_exit=False, noise_key=noise_key)
    return judge(sys, cand64, H, u_h, traj, fv_o, sel, fv_gpu, eps, label)


def check_tick_lifted(sys: o.System, K_full, x_t, u_h, cand64: np.ndarray, H: int, sel: dict, fv_gpu: np.ndarray,
                      eps, label: str = "") -> dict:
    """check_tick for the lifted whole-horizon form (oracle: rollout_lifted)."""
    traj, fv_o = o.rollout_lifted(sys, K_full, x_t, cand64, H, early_exit=False)
    return judge(sys, cand64, H, u_h, traj, fv_o, sel, fv_gpu, eps, label)


def agreed(kinds: dict) -> int:
    return kinds.get("identical", 0) + kinds.get("equal_cost", 0)


def tally(results) -> dict:
    kinds = {}
    for r in results:
        kinds[r["kind"]] = kinds.get(r["kind"], 0) + 1
        kinds["zero_intervention"] = kinds.get("zero_intervention", 0) + int(r["zero_intervention"])
        kinds["no_safe"] = kinds.get("no_safe", 0) + int(r["status"] != o.STATUS_OK)
    return kinds


# ----------------------------------------------------------------------------
# Replays in worker processes
# ----------------------------------------------------------------------------
def _one_blas_thread():
    from threadpoolctl import threadpool_limits

    threadpool_limits(limits=1)


def replay_pool(workers: int = 0) -> ProcessPoolExecutor:
    """A pool of oracle workers (at most 8, never more than the usable cores)."""
    n = workers or max(1, min(8, len(os.sched_getaffinity(0))))
    return ProcessPoolExecutor(max_workers=n, mp_context=multiprocessing.get_context("spawn"),
                               initializer=_one_blas_thread)


def candidates(sys: o.System, spec, u_h) -> np.ndarray:
    """A tick's candidate set (N+1, S, m) from an array or a generator spec:
    ("grid", [G_0, ...]) or ("uniform", N, S, seed, tick, loop)."""
    if isinstance(spec, np.ndarray):
        return spec
    if spec[0] == "grid":
        return o.with_user(o.grid_candidates(sys, spec[1]), u_h, 1)
    _, N, S, seed, tick, loop = spec
    return o.with_user(o.uniform_candidates(sys, N, S, seed, tick, loop), u_h, S)


def replay_job(job) -> list:
    """One tick replayed by the oracle and judged against one or more GPU
    results: job = (sys, K, x_t, u_h, cand_spec, H, eps, noise_key,
    [(sel, fv_gpu, label[, eps of this result]), ...])."""
    sys, K, x_t, u_h, spec, H, eps, noise_key, results = job
    cand = candidates(sys, spec, u_h)
    traj, fv_o = o.rollout(sys, K, x_t, cand, H, early_exit=False, noise_key=noise_key)
    return [judge(sys, cand, H, u_h, traj, fv_o, r[0], r[1], r[3] if len(r) > 3 else eps, r[2]) for r in results]


def decision_job(job) -> list:
    """One tick's decisions (no first violations from the GPU) against the
    oracle over the same candidate set: job = (sys, K, x_t, u_h, cand_spec, H,
    [(sel, eps, label), ...]); each result's ambiguity mask is taken from the
    oracle's own verdicts."""
    sys, K, x_t, u_h, spec, H, results = job
    cand = candidates(sys, spec, u_h)
    traj, fv_o = o.rollout(sys, K, x_t, cand, H, early_exit=False)
    out = []
    for sel, eps, label in results:
        amb = ambiguous(sys, traj, fv_o, fv_o, eps)
        r = agreement(sys, cand, H, u_h, fv_o, amb, sel)
        r["label"] = label
        out.append(r)
    return out


def label_job(job) -> dict:
    """An exhaustive tick's decision checked by the oracle without rolling
    every candidate: job = (sys, K, x_t, u_h, cand_spec, H, idx, status).  A
    safe choice is right when the oracle finds it safe and finds unsafe every
    candidate of lower FP64 cost (candidates of equal cost to 1e-6 relative
    are accepted, as in the agreement rule); a NO_SAFE record needs the
    oracle's full selection."""
    sys, K, x_t, u_h, spec, H, idx, status = job
    cand = candidates(sys, spec, u_h)
    cost = o.cost(sys, cand, u_h)
    if status == o.STATUS_OK:
        cheaper = np.nonzero(cost < cost[idx] - 1e-6 * max(cost[idx], 1e-30))[0]
        sub = np.concatenate([[idx], cheaper]).astype(np.int64)
        _, fv = o.rollout(sys, K, x_t, cand[sub], H, early_exit=True)
        ok = bool(fv[0] == H + 1) and not np.any(fv[1:] == H + 1)
        return dict(ok=ok, rolled=int(sub.size), status=status, idx=int(idx), zero=bool(idx == 0))
    _, fv = o.rollout(sys, K, x_t, cand, H, early_exit=True)
    ref = o.select(sys, cand, fv, H, u_h)
    return dict(ok=bool(ref["status"] == o.STATUS_NO_SAFE and ref["idx"] == idx), rolled=int(cand.shape[0]),
                status=status, idx=int(idx), zero=False)


def oracle_chunk(job):
    """First violations and ambiguity of a slice of one tick's candidates:
    job = (sys, K, x_t, cand_slice, H, fv_gpu_slice, eps), or with a list of
    (fv_gpu_slice, eps) pairs in place of the last two (one ambiguity mask per
    pair: (fv_o, [amb, ...]))."""
    if len(job) == 6:
        sys, K, x_t, cand, H, pairs = job
    else:
        sys, K, x_t, cand, H, fv_gpu, eps = job
        pairs = None
    traj, fv_o = o.rollout(sys, K, x_t, cand, H, early_exit=False)
    if pairs is None:
        return fv_o, ambiguous(sys, traj, fv_o, np.asarray(fv_gpu, np.int64), eps)
    return fv_o, [ambiguous(sys, traj, fv_o, np.asarray(f, np.int64), e) for f, e in pairs]
