"""Workload set-up shared by the tests: the same numbers, given once to the
oracle's own system description and once to the library's descriptor.

Nothing here computes any part of the method: it builds descriptors, draws
seeded inputs (via synth) and fits K with the oracle so both sides consume the
same FP64 model.
"""
from __future__ import annotations

import functools

import numpy as np

import synth
from oracle import mpmi_oracle as o

BB_THETA, BB_P = 0.5, 2.0
RC_VY = 2.0


def f32(v):
    return np.asarray(v, np.float64).astype(np.float32).astype(np.float64)


def track_dict(track: synth.Track, infl: float = 0.0) -> dict:
    """Track parameters rounded to FP32 (the library stores FP32)."""
    return dict(r0=float(f32(track.r0)), half=float(f32(track.half_width)), amp=list(f32(track.amp)),
                freq=[int(f) for f in track.freq], phase=list(f32(track.phase)), infl=float(f32(infl)))


def bb_oracle_system(infl=0.0, theta=BB_THETA, p=BB_P):
    return o.System("balance_bot", 4, 1, box=[(2, float(f32(theta)), float(f32(infl))),
                                               (0, float(f32(p)), float(f32(infl)))],
                    u_lo=[synth.BB_U_LO], u_hi=[synth.BB_U_HI])


def rc_oracle_system(track: synth.Track, infl=0.0):
    return o.System("race_car", 6, 2, box=[(4, float(f32(RC_VY)), float(f32(infl)))],
                    track=track_dict(track, infl), u_lo=synth.RC_U_LO, u_hi=synth.RC_U_HI)


@functools.lru_cache(maxsize=None)
def bb_model():
    """Oracle-fitted FP64 K of the cart-pole (5,000 transitions, seed 0) and the data."""
    X, U, Y = synth.balance_bot_transitions(5000, seed=0)
    K, info = o.fit("balance_bot", X, U, Y)
    return K, info, (X, U, Y)


@functools.lru_cache(maxsize=None)
def rc_track():
    return synth.make_track(3)


@functools.lru_cache(maxsize=None)
def rc_model():
    """Oracle-fitted FP64 K of the bicycle (50,000 transitions, seed 0) and the data."""
    X, U, Y = synth.race_car_transitions(50000, seed=0, track=rc_track())
    K, info = o.fit("race_car", X, U, Y)
    return K, info, (X, U, Y)


def bb_floors():
    """Relative-error floors per state component: the constraint bound for
    constrained components, else the data standard deviation."""
    X = bb_model()[2][0]
    s = X.std(axis=0)
    return np.array([BB_P, s[1], BB_THETA, s[3]])


def rc_floors():
    X = rc_model()[2][0]
    s = X.std(axis=0)
    return np.array([3.0, 3.0, s[2], s[3], RC_VY, s[5]])


@functools.lru_cache(maxsize=None)
def bb_lifted_model():
    """Oracle-fitted FP64 lifted operator (21 x 21) of the cart-pole data."""
    X, U, Y = bb_model()[2]
    return o.fit_lifted("balance_bot", X, U, Y)


@functools.lru_cache(maxsize=None)
def rc_lifted_model():
    """Oracle-fitted FP64 lifted operator (64 x 64) of the bicycle data."""
    X, U, Y = rc_model()[2]
    return o.fit_lifted("race_car", X, U, Y)


def rc3_basis():
    atoms, feats = synth.race_car3_basis()
    return o.Basis(atoms=tuple(atoms), feats=tuple(feats))


def rc3_oracle_system(track: synth.Track, infl=0.0):
    return o.System(rc3_basis(), 6, 3, box=[(4, float(f32(RC_VY)), float(f32(infl)))],
                    track=track_dict(track, infl), u_lo=synth.RC3_U_LO, u_hi=synth.RC3_U_HI)


def rc3_gpu_system(mpmi, track: synth.Track, infl=0.0):
    """The library's descriptor of the three-input car (custom basis)."""
    kinds = {"one": mpmi.ATOM_ONE, "var": mpmi.ATOM_VAR, "sin": mpmi.ATOM_SIN, "cos": mpmi.ATOM_COS}
    atoms, feats = synth.race_car3_basis()
    return mpmi.custom_system(6, 3, [(kinds[k], v) for k, v in atoms], feats, [(4, RC_VY, infl)],
                              synth.RC3_U_LO, synth.RC3_U_HI, track=track_dict(track, infl),
                              eps_box=[0.02], eps_track=0.02, eps32_box=[3e-4], eps32_track=2e-3)


@functools.lru_cache(maxsize=None)
def rc3_model():
    """Oracle-fitted FP64 K of the three-input car (50,000 transitions, seed 0)."""
    X, U, Y = synth.race_car3_transitions(50000, seed=0, track=rc_track())
    K, info = o.fit(rc3_basis(), X, U, Y)
    return K, info, (X, U, Y)
