"""The allocation-free tick (mpmi_tick_noalloc: no context, its scratch in the
library's static device array) against mpmi_tick on the same inputs, through
the C ABI: two calls in a row per case, the second with a smaller input; the
records are bit-identical and so are the first violations."""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import mpmi_oracle as o
from paper_1906_02318_amd import mpmi
from tests import workloads as W

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


@pytest.fixture(scope="module")
def models():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ctx = mpmi.Context(0)
    mb = mpmi.mpmi_model_pack(ctx, mpmi.balance_bot_system(), dev(W.bb_model()[0], torch.float64))
    mr = mpmi.mpmi_model_pack(ctx, mpmi.race_car_system(W.track_dict(W.rc_track())), dev(W.rc_model()[0],
                                                                                         torch.float64))
    torch.cuda.synchronize()
    return ctx, mb, mr


def _intervening_inputs(kind):
    """Two (state, user input) pairs whose user input the oracle finds unsafe
    within 20 steps, so the ticks intervene (and re-roll near-band
    candidates)."""
    if kind == "bb":
        so, K = W.bb_oracle_system(), W.bb_model()[0]
        xs, us = synth.balance_bot_states(64, seed=31), synth.uniform_user(64, [-5.0], [5.0], seed=32)
    else:
        so, K = W.rc_oracle_system(W.rc_track()), W.rc_model()[0]
        xs = synth.race_car_states(64, W.rc_track(), seed=31)
        us = synth.uniform_user(64, synth.RC_U_LO, synth.RC_U_HI, seed=32)
    pick = []
    for x, u in zip(xs, us):
        x, u = W.f32(x), W.f32(u)
        _, fv = o.rollout(so, K, x, u.reshape(1, 1, -1), 20)
        if fv[0] <= 20:
            pick.append((x, u))
        if len(pick) == 2:
            break
    assert len(pick) == 2
    return [p[0] for p in pick], [p[1] for p in pick]


CASES = {
    # name: (system, precision, lanes, [(N, H, generator, grid), ...] -- larger first)
    "bb_fp32_seq": ("bb", mpmi.PREC_FP32, 0, [(10240, 50, "uniform", None), (1024, 20, "uniform", None)]),
    "bb_recheck64": ("bb", mpmi.PREC_FP32_RECHECK64, 0, [(8000, 40, "uniform", None), (500, 20, "uniform", None)]),
    "rc_recheck64": ("rc", mpmi.PREC_FP32_RECHECK64, 0, [(16384, 60, "grid", [128, 128]),
                                                         (4096, 30, "grid", [64, 64])]),
    "rc_fp32_4lanes": ("rc", mpmi.PREC_FP32, 4, [(16384, 60, "grid", [128, 128]), (2048, 60, "grid", [64, 32])]),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_noalloc_tick_equals_the_tick(models, name):
    ctx, mb, mr = models
    kind, prec, lanes, calls = CASES[name]
    model = mb if kind == "bb" else mr
    xs, us = _intervening_inputs(kind)
    for k, (N, H, gen, grid) in enumerate(calls):
        x, u = dev(W.f32(xs[k]), torch.float32), dev(W.f32(us[k]), torch.float32)
        loop = 63 if k == 0 else 5
        if gen == "grid":
            desc = mpmi.tick_desc(N, H, gen=mpmi.GEN_GRID, grid=grid, precision=prec, lanes_per_cand=lanes, loop=loop)
        else:
            desc = mpmi.tick_desc(N, H, gen=mpmi.GEN_UNIFORM, n_seg=5, seed=9, tick=k, precision=prec,
                                  lanes_per_cand=lanes, loop=loop)
        out = torch.zeros(mpmi.SELECTION_BYTES, dtype=torch.uint8, device="cuda")
        fv = torch.zeros(N + 1, dtype=torch.int16, device="cuda")
        mpmi.mpmi_tick_noalloc(model, desc, x, u, out, first_violation=fv)
        fv_ref = torch.zeros(N + 1, dtype=torch.int16, device="cuda")
        ref = mpmi.mpmi_tick(ctx, model, desc, x, u, first_violation=fv_ref)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy().tobytes(), ref.cpu().numpy().tobytes()
        sel = mpmi.decode_selection(out)
        log(f"[noalloc] {name} call {k}: N={N} H={H} idx={sel['idx']} status={sel['status']} "
            f"n_safe={sel['n_safe']} n_recheck={sel['n_recheck']}")
        assert a == b, f"{name} call {k}: records differ"
        assert sel["idx"] != 0 or sel["status"] != mpmi.OK  # the tick intervened
        assert torch.equal(fv, fv_ref), f"{name} call {k}: first violations differ"


def test_noalloc_limits(models):
    """Loops beyond the static slots, FP32_RECHECK64 ticks beyond the static
    list and BF16X3 ticks are refused with a message (and nothing runs)."""
    ctx, mb, mr = models
    x, u = dev(W.f32([0.0, 0.0, 0.1, 0.0]), torch.float32), dev(W.f32([1.0]), torch.float32)
    out = torch.zeros(mpmi.SELECTION_BYTES, dtype=torch.uint8, device="cuda")
    bad = [
        (mpmi.tick_desc(1024, 20, gen=mpmi.GEN_GRID, grid=[1024], loop=64), mpmi.EINVAL, "selection slots"),
        (mpmi.tick_desc(65536, 20, gen=mpmi.GEN_GRID, grid=[65536], precision=mpmi.PREC_FP32_RECHECK64),
         mpmi.EUNSUPPORTED, "65536"),
    ]
    for desc, code, text in bad:
        with pytest.raises(mpmi.MpmiError) as e:
            mpmi.mpmi_tick_noalloc(mb, desc, x, u, out)
        assert e.value.status == code and text in str(e.value), str(e.value)
    xr = dev(W.f32(synth.race_car_states(1, W.rc_track(), seed=3)[0]), torch.float32)
    ur = dev(W.f32([0.0, 0.0]), torch.float32)
    with pytest.raises(mpmi.MpmiError) as e:
        mpmi.mpmi_tick_noalloc(mr, mpmi.tick_desc(1024, 20, gen=mpmi.GEN_GRID, grid=[32, 32],
                                                  precision=mpmi.PREC_BF16X3), xr, ur, out)
    assert e.value.status == mpmi.EUNSUPPORTED
    # the largest FP32_RECHECK64 tick it takes runs and matches the tick
    desc = mpmi.tick_desc(65535, 20, gen=mpmi.GEN_GRID, grid=[65535], precision=mpmi.PREC_FP32_RECHECK64)
    mpmi.mpmi_tick_noalloc(mb, desc, x, u, out)
    ref = mpmi.mpmi_tick(ctx, mb, desc, x, u)
    torch.cuda.synchronize()
    assert out.cpu().numpy().tobytes() == ref.cpu().numpy().tobytes()
