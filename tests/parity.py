"""Comparison rules between the GPU library and the FP64 oracle.

* Rollout states: relative error |x_gpu - x_64| / max(|x_64|, floor_j) per
  component, floor_j the constraint bound or the data standard deviation;
  states the oracle predicts beyond 1e6 floors (diverged, unsafe on both
  sides) are excluded.
* Safety verdicts: first violations must be identical except for candidates
  whose oracle margin comes within eps_j of zero at some step up to the
  earlier of the two first violations (ambiguous by FP32 rounding).
* Selection: the same candidate, or two candidates that are both oracle-safe
  or ambiguous and whose FP64 costs agree to 1e-6 relative.
"""
from __future__ import annotations

import numpy as np

from oracle import mpmi_oracle as o


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


def check_tick(sys: o.System, K, x_t, u_h, cand64: np.ndarray, H: int, sel: dict, fv_gpu: np.ndarray, eps,
               label: str = "", noise_key=None) -> dict:
    """Checks one GPU tick against the oracle; returns counters for reporting."""
    traj, fv_o = o.rollout(sys, K, x_t, cand64, H, early_exit=False, noise_key=noise_key)
    fv_gpu = np.asarray(fv_gpu, np.int64)
    amb = ambiguous(sys, traj, fv_o, fv_gpu, eps)
    mism = (fv_o != fv_gpu) & ~amb
    assert not mism.any(), (f"{label}: first-violation mismatch outside the eps band at candidates "
                            f"{np.nonzero(mism)[0][:10]} (oracle {fv_o[mism][:10]}, gpu {fv_gpu[mism][:10]})")
    ref = o.select(sys, cand64, fv_o, H, u_h)
    cost = o.cost(sys, cand64, u_h)
    i_g, i_o = sel["idx"], ref["idx"]
    safe_o = fv_o == H + 1
    kind = "identical"
    if i_g != i_o:
        ok_g = safe_o[i_g] or amb[i_g]
        ok_o = safe_o[i_o] or amb[i_o]
        if ok_g and ok_o and abs(cost[i_g] - cost[i_o]) <= 1e-6 * max(abs(cost[i_o]), 1e-30):
            kind = "equal_cost"
        elif amb[i_g] and cost[i_g] <= cost[i_o]:
            kind = "eps_band"   # GPU kept an ambiguous candidate the oracle rejected
        elif amb[i_o] and ok_g and cost[i_g] >= cost[i_o]:
            kind = "eps_band"   # GPU rejected the oracle's ambiguous choice
        elif ref["status"] != o.STATUS_OK and sel["status"] != o.STATUS_OK and amb.any():
            kind = "eps_band"   # fallback ordering decided by ambiguous first violations
        else:
            raise AssertionError(
                f"{label}: selection {i_g} (cost {cost[i_g]:.9g}, fv {fv_o[i_g]}, amb {amb[i_g]}) vs oracle "
                f"{i_o} (cost {cost[i_o]:.9g}, fv {fv_o[i_o]}, amb {amb[i_o]}), status {sel['status']}/{ref['status']}")
    if not amb.any():
        assert sel["status"] == ref["status"], f"{label}: status {sel['status']} vs {ref['status']}"
        assert sel["n_safe"] == ref["n_safe"], f"{label}: n_safe {sel['n_safe']} vs {ref['n_safe']}"
    np.testing.assert_array_equal(np.asarray(sel["u_r"][: sys.m], np.float64), cand64[i_g, 0, :])
    return dict(kind=kind, ambiguous=int(amb.sum()), status=ref["status"], idx=i_o,
                n_safe=ref["n_safe"], zero_intervention=bool(i_o == 0))
