"""The GPU-versus-oracle comparison rules reject wrong selections.

A "GPU result" here is built from the oracle's own verdicts with one planted
change, so every case runs on the CPU: a wrong index, status or safe count
must fail the complete selection check even when ambiguous candidates exist.
"""
import numpy as np
import pytest

import synth
from oracle import mpmi_oracle as o
from tests import workloads as W
from tests.parity import check_tick

EPS_BB = [1e-4, 4e-4]


def _tick(seed, u_h, theta=0.5, N=400, x=None):
    K = W.bb_model()[0]
    so = W.bb_oracle_system(theta=theta)
    x = W.f32(synth.balance_bot_states(1, seed=seed)[0] if x is None else x)
    cand = o.with_user(o.grid_candidates(so, [N]), W.f32(u_h), 1)
    res = o.tick(so, K, x, W.f32(u_h), cand, 20)
    return so, K, x, W.f32(u_h), cand, res


def _record(res, cand, fv):
    i = res["idx"]
    return dict(idx=i, status=res["status"], n_safe=res["n_safe"], u_r=list(cand[i, 0, :]),
                first_violation=int(fv[i]))


def test_exact_copy_of_the_oracle_passes():
    so, K, x, u, cand, res = _tick(3, [4.9])
    out = check_tick(so, K, x, u, cand, 20, _record(res, cand, res["fv"]), res["fv"], EPS_BB)
    assert out["kind"] == "identical"


def test_wrong_safe_candidate_fails_even_with_a_wide_band():
    """A safe but dearer candidate is rejected, also when a band so wide that
    every candidate is ambiguous would have excused it before."""
    so, K, x, u, cand, res = _tick(3, [4.9])
    fv = res["fv"]
    safe = np.nonzero(fv == 21)[0]
    assert safe.size > 2
    c = o.cost(so, cand, u)
    wrong = int(safe[np.argmax(c[safe])])
    assert wrong != res["idx"]
    rec = _record(dict(res, idx=wrong), cand, fv)
    for eps in (EPS_BB, [10.0, 10.0]):
        with pytest.raises(AssertionError):
            check_tick(so, K, x, u, cand, 20, rec, fv, eps)


def test_wrong_fallback_choice_fails():
    """Nothing safe (a pole falling past a tight bound): the latest first
    violation must win."""
    so, K, x, u, cand, res = _tick(0, [0.3], theta=0.08, x=[0.0, 0.0, 0.05, 0.6])
    assert res["status"] == o.STATUS_NO_SAFE
    fv = res["fv"]
    wrong = int(np.argmin(fv))
    assert fv[wrong] < fv[res["idx"]]
    rec = _record(dict(res, idx=wrong), cand, fv)
    with pytest.raises(AssertionError):
        check_tick(so, K, x, u, cand, 20, rec, fv, [10.0, 10.0])


def test_wrong_count_or_status_fails():
    so, K, x, u, cand, res = _tick(3, [4.9])
    fv = res["fv"]
    for bad in (dict(n_safe=res["n_safe"] + 1), dict(status=o.STATUS_NO_SAFE)):
        rec = dict(_record(res, cand, fv), **bad)
        with pytest.raises(AssertionError):
            check_tick(so, K, x, u, cand, 20, rec, fv, [10.0, 10.0])


def test_flipped_verdict_outside_the_band_fails():
    so, K, x, u, cand, res = _tick(3, [4.9])
    fv = res["fv"].copy()
    j = int(np.nonzero(fv == 21)[0][-1])
    fv[j] = 5
    with pytest.raises(AssertionError):
        check_tick(so, K, x, u, cand, 20, _record(res, cand, fv), fv, EPS_BB)


def test_replays_run_in_worker_processes(oracle_pool):
    """The spawn-context pool replays ticks with the same verdicts as a direct call."""
    from tests.parity import replay_job

    so, K, x, u, cand, res = _tick(3, [4.9])
    job = (so, K, x, u, ("grid", [400]), 20, EPS_BB, None, [(_record(res, cand, res["fv"]), res["fv"], "pool")])
    out = list(oracle_pool.map(replay_job, [job, job]))
    assert [r[0]["kind"] for r in out] == ["identical", "identical"]
