"""Thin Python binding of libmpmi (include/mpmi.h), same names as the C ABI.

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides device memory (tensors) and streams; the
binding passes their raw pointers.  If libmpmi.so has not been built this
module raises on first use -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpmi.so")

# Constants mirrored from include/mpmi.h
ABI_VERSION = 7
MAX_STATE, MAX_INPUT, MAX_DIM, MAX_BOX = 8, 4, 64, 4
MAX_HORIZON, MAX_SEGMENTS, MAX_CAND, MAX_LOOPS = 255, 8, 33554431, 4096
OK, NO_SAFE, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, ESINGULAR = 0, 1, -1, -2, -3, -4, -5
BASIS_LINEAR, BASIS_BALANCE_BOT, BASIS_RACE_CAR, BASIS_CUSTOM = 0, 1, 2, 3
ATOM_ONE, ATOM_VAR, ATOM_SIN, ATOM_COS = 0, 1, 2, 3
MAX_ATOMS = 32
PREC_FP32, PREC_BF16X3, PREC_FP32_RECHECK64 = 0, 1, 2
GEN_EXPLICIT, GEN_GRID, GEN_UNIFORM = 0, 1, 2

_i32x4 = ctypes.c_int32 * 4
_f32x4 = ctypes.c_float * 4


class System(ctypes.Structure):
    _fields_ = [
        ("basis", ctypes.c_int32), ("n_state", ctypes.c_int32), ("n_input", ctypes.c_int32),
        ("n_box", ctypes.c_int32), ("box_index", _i32x4), ("box_bound", _f32x4), ("box_infl", _f32x4),
        ("eps_box", _f32x4), ("has_track", ctypes.c_int32), ("track_n", ctypes.c_int32),
        ("track_freq", _i32x4), ("track_amp", _f32x4), ("track_phase", _f32x4),
        ("track_r0", ctypes.c_float), ("track_half", ctypes.c_float), ("track_infl", ctypes.c_float),
        ("eps_track", ctypes.c_float), ("u_lo", _f32x4), ("u_hi", _f32x4),
        ("noise_sigma", ctypes.c_float * 8),
        ("n_atoms", ctypes.c_int32), ("dim", ctypes.c_int32),
        ("atom_kind", ctypes.c_int8 * 32), ("atom_var", ctypes.c_int8 * 32),
        ("feat_a", ctypes.c_int8 * 64), ("feat_b", ctypes.c_int8 * 64),
        ("eps32_box", _f32x4), ("eps32_track", ctypes.c_float), ("pad_eps", ctypes.c_int32),
    ]


class Selection(ctypes.Structure):
    _fields_ = [
        ("idx", ctypes.c_int32), ("status", ctypes.c_int32), ("n_safe", ctypes.c_int32),
        ("n_recheck", ctypes.c_int32), ("u_r", _f32x4), ("cost", ctypes.c_float),
        ("deviation", ctypes.c_float), ("first_violation", ctypes.c_int32), ("n_cand", ctypes.c_int32),
    ]


SELECTION_BYTES = ctypes.sizeof(Selection)  # 48


class TickDesc(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64), ("tick", ctypes.c_uint64), ("loop", ctypes.c_int32),
        ("gen", ctypes.c_int32), ("n_cand", ctypes.c_int32), ("grid", _i32x4),
        ("n_seg", ctypes.c_int32), ("horizon", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("block", ctypes.c_int32), ("lanes_per_cand", ctypes.c_int32),
    ]


class LoopDesc(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_void_p), ("x_t", ctypes.c_void_p), ("u_user", ctypes.c_void_p),
        ("cand", ctypes.c_void_p), ("out", ctypes.c_void_p), ("first_violation", ctypes.c_void_p),
        ("seed", ctypes.c_uint64), ("tick", ctypes.c_uint64), ("gen", ctypes.c_int32),
        ("n_cand", ctypes.c_int32), ("grid", _i32x4), ("n_seg", ctypes.c_int32), ("horizon", ctypes.c_int32),
    ]


class MultiConfig(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("grid", ctypes.c_int32), ("precision", ctypes.c_int32)]


MAX_LIBRARY = 160


class Library(ctypes.Structure):
    _fields_ = [
        ("n_state", ctypes.c_int32), ("n_input", ctypes.c_int32), ("n_atoms", ctypes.c_int32),
        ("n_feat", ctypes.c_int32), ("atom_kind", ctypes.c_int8 * 32), ("atom_var", ctypes.c_int8 * 32),
        ("feat_a", ctypes.c_uint8 * MAX_LIBRARY), ("feat_b", ctypes.c_uint8 * MAX_LIBRARY),
    ]


class MpmiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"mpmi status {status}: {msg}")
        self.status = status


_lib = None


def library() -> ctypes.CDLL:
    """Loads libmpmi.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1906_02318_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "mpmi_abi_version": (i32, []),
        "mpmi_create": (i32, [ctypes.POINTER(vp), i32]),
        "mpmi_destroy": (None, [vp]),
        "mpmi_last_error": (ctypes.c_char_p, [vp]),
        "mpmi_model_bytes": (ctypes.c_size_t, []),
        "mpmi_model_pack": (i32, [vp, ctypes.POINTER(System), vp, vp, vp]),
        "koopman_fit": (i32, [vp, ctypes.POINTER(System), vp, vp, vp, i64, f64, vp, ctypes.POINTER(f64), vp]),
        "rollout_batch": (i32, [vp, vp, i32, vp, vp, i32, i32, i32, vp, i64, vp]),
        "safe_mask": (i32, [vp, vp, vp, i64, i32, i32, vp, vp, vp, vp]),
        "mpmi_tick_graph": (i32, [vp, vp, ctypes.POINTER(TickDesc), vp, vp, vp, vp, vp, ctypes.POINTER(vp)]),
        "select_min_intervention": (i32, [vp, vp, vp, i32, i32, vp, i32, vp, i32, vp, vp]),
        "mpmi_tick": (i32, [vp, vp, ctypes.POINTER(TickDesc), vp, vp, vp, vp, vp, vp, i64, vp]),
        "mpmi_generate_candidates": (i32, [vp, vp, ctypes.POINTER(TickDesc), vp, vp, vp, vp]),
        "mpmi_fp32_fma_rate": (i32, [vp, ctypes.POINTER(f64)]),
        "mpmi_sincos64": (i32, [vp, vp, vp, vp, i32, vp]),
        "mpmi_write_rates": (i32, [vp, vp, i32, i64, i32, ctypes.POINTER(f64), ctypes.POINTER(f64)]),
        "mpmi_read_rates": (i32, [vp, vp, i32, i64, i32, ctypes.POINTER(f64), ctypes.POINTER(f64)]),
        "mpmi_multi_create": (i32, [vp, ctypes.POINTER(LoopDesc), i32, ctypes.POINTER(MultiConfig), ctypes.POINTER(vp)]),
        "mpmi_multi_destroy": (None, [vp]),
        "mpmi_multi_set_config": (i32, [vp, vp, ctypes.POINTER(MultiConfig)]),
        "mpmi_multi_get_config": (i32, [vp, ctypes.POINTER(MultiConfig), ctypes.POINTER(i32)]),
        "mpmi_multi_tick": (i32, [vp, vp, vp]),
        "mpmi_multi_get_ticks": (i32, [vp, vp, vp]),
        "mpmi_multi_autotune": (i32, [vp, vp, i32, ctypes.POINTER(MultiConfig), ctypes.POINTER(ctypes.c_float), vp]),
        "mpmi_multi_graph": (i32, [vp, vp, ctypes.POINTER(vp)]),
        "mpmi_graph_launch": (i32, [vp, vp, vp]),
        "mpmi_graph_destroy": (None, [vp]),
        "mlp_workspace_bytes": (ctypes.c_size_t, [i32]),
        "mlp_forward": (i32, [vp, vp, vp, vp, vp, vp, i32, vp, vp, ctypes.c_size_t, vp]),
        "mlp_grad": (i32, [vp, vp, vp, vp, vp, vp, vp, i32, vp, vp, vp, ctypes.c_size_t, vp]),
        "mlp_adam": (i32, [vp, vp, vp, vp, vp, vp, i32, ctypes.c_float, vp]),
        "mdn_sample": (i32, [vp, vp, vp, i32, ctypes.c_uint64, ctypes.c_uint64, i32, vp, vp]),
        "mpmi_proposal_tick": (i32, [vp, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(TickDesc),
                                     ctypes.POINTER(TickDesc), vp, vp, vp, vp, ctypes.c_size_t, vp]),
        "mpmi_gemm_bf16": (i32, [vp, vp, vp, i32, i32, i32, i32, i32, vp, vp]),
        "mpmi_tick_autotune": (i32, [vp, vp, ctypes.POINTER(TickDesc), vp, vp, vp, vp, i32,
                                     ctypes.POINTER(ctypes.c_float), vp]),
        "mpmi_basis_describe": (i32, [i32, i32, i32, ctypes.POINTER(System)]),
        "koopman_select_basis": (i32, [vp, ctypes.POINTER(Library), vp, vp, vp, i64, ctypes.POINTER(f64), i32, f64,
                                       i32, vp, vp, ctypes.POINTER(f64), vp]),
        "mpmi_tick_noalloc": (i32, [ctypes.POINTER(System), vp, ctypes.POINTER(TickDesc), vp, vp, vp, vp, vp, vp]),
        "mpmi_basis_match": (i32, [ctypes.POINTER(System)]),
        "koopman_fit_lifted": (i32, [vp, ctypes.POINTER(System), vp, vp, vp, i64, f64, vp, ctypes.POINTER(f64), vp]),
        "mpmi_lifted_bytes": (ctypes.c_size_t, [i32]),
        "mpmi_lifted_layout": (i32, [i32, i32, i32, vp, vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "mpmi_lifted_pack": (i32, [vp, vp, vp, i32, vp, vp]),
        "mpmi_tick_lifted": (i32, [vp, vp, ctypes.POINTER(TickDesc), vp, vp, vp, vp, vp, vp, i64, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.mpmi_abi_version() != ABI_VERSION:
        raise RuntimeError(f"libmpmi ABI {lib.mpmi_abi_version()} != binding ABI {ABI_VERSION}")
    _lib = lib
    return lib


# ---------------------------------------------------------------------------
# System descriptors (plain data)
# ---------------------------------------------------------------------------
def _sys(basis, n, m, box, u_lo, u_hi, track=None, eps_box=None, eps_track=0.0, noise=None, eps32_box=None,
         eps32_track=0.0):
    s = System()
    for j, v in enumerate(noise or []):
        s.noise_sigma[j] = float(v)
    s.basis, s.n_state, s.n_input = basis, n, m
    s.n_box = len(box)
    for b, (idx, bound, infl) in enumerate(box):
        s.box_index[b], s.box_bound[b], s.box_infl[b] = idx, bound, infl
        s.eps_box[b] = 0.0 if eps_box is None else eps_box[b]
        s.eps32_box[b] = 0.0 if eps32_box is None else eps32_box[b]
    for j in range(m):
        s.u_lo[j], s.u_hi[j] = float(u_lo[j]), float(u_hi[j])
    if track is not None:
        s.has_track = 1
        s.track_n = len(track["amp"])
        for k in range(s.track_n):
            s.track_freq[k] = int(track["freq"][k])
            s.track_amp[k] = float(track["amp"][k])
            s.track_phase[k] = float(track["phase"][k])
        s.track_r0, s.track_half, s.track_infl = track["r0"], track["half"], track.get("infl", 0.0)
        s.eps_track = eps_track
        s.eps32_track = eps32_track
    return s


def custom_system(n, m, atoms, feats, box, u_lo, u_hi, track=None, eps_box=None, eps_track=0.0, noise=None,
                  eps32_box=None, eps32_track=0.0):
    """A basis given as data: atoms [(ATOM_* or 'one'/'var'/'sin'/'cos', w index)],
    features [(atom a, atom b)] (psi_f = atom_a * atom_b, w = [x; u])."""
    s = _sys(BASIS_CUSTOM, n, m, box, u_lo, u_hi, track=track, eps_box=eps_box, eps_track=eps_track, noise=noise,
             eps32_box=eps32_box, eps32_track=eps32_track)
    if not 1 <= len(atoms) <= MAX_ATOMS or not 1 <= len(feats) <= MAX_DIM:
        raise ValueError("1..32 atoms and 1..64 features")
    s.n_atoms, s.dim = len(atoms), len(feats)
    for q, (kind, var) in enumerate(atoms):
        s.atom_kind[q], s.atom_var[q] = _ATOM_CODES.get(kind, kind), var
    for f, (a, b) in enumerate(feats):
        s.feat_a[f], s.feat_b[f] = a, b
    return s


def basis_describe(family: int, n: int, m: int, system: System) -> System:
    """system with its custom-basis fields set to the atoms and features of a fixed family."""
    st = library().mpmi_basis_describe(family, n, m, ctypes.byref(system))
    if st != OK:
        raise MpmiError(st, "mpmi_basis_describe failed")
    return system


def basis_match(system: System) -> int:
    """The fixed family a custom basis equals, or BASIS_CUSTOM."""
    return int(library().mpmi_basis_match(ctypes.byref(system)))


_ATOM_CODES = {"one": ATOM_ONE, "var": ATOM_VAR, "sin": ATOM_SIN, "cos": ATOM_COS}


def library_desc(n: int, m: int, atoms, feats) -> Library:
    """A basis-selection library: atoms [(ATOM_* or 'one'/'var'/'sin'/'cos', w index)],
    functions [(atom a, atom b)]."""
    lib = Library()
    if not 1 <= len(atoms) <= MAX_ATOMS or not 1 <= len(feats) <= MAX_LIBRARY:
        raise ValueError("1..32 atoms and 1..160 functions")
    lib.n_state, lib.n_input, lib.n_atoms, lib.n_feat = n, m, len(atoms), len(feats)
    for q, (kind, var) in enumerate(atoms):
        lib.atom_kind[q], lib.atom_var[q] = _ATOM_CODES.get(kind, kind), var
    for f, (a, b) in enumerate(feats):
        lib.feat_a[f], lib.feat_b[f] = a, b
    return lib


def linear_system(n, m, box, u_lo, u_hi):
    """psi = [x; u]; box = [(state index, bound, inflation), ...]."""
    return _sys(BASIS_LINEAR, n, m, box, u_lo, u_hi)


def balance_bot_system(theta_bound=0.5, p_bound=2.0, infl=0.0, u_lo=-5.0, u_hi=5.0, eps=(5e-5, 2e-4),
                       noise=None, eps32=(1e-4, 4e-4)):
    """Cart-pole: |theta| < theta_bound - infl, |p| < p_bound - infl, u in [u_lo, u_hi].
    eps: BF16X3 bands; eps32: FP32_RECHECK64 bands (theta, p)."""
    return _sys(BASIS_BALANCE_BOT, 4, 1, [(2, theta_bound, infl), (0, p_bound, infl)], [u_lo], [u_hi],
                eps_box=list(eps), noise=noise, eps32_box=list(eps32))


def race_car_system(track: dict, vy_bound=2.0, infl=0.0, u_lo=(-0.4, -3.0), u_hi=(0.4, 3.0),
                    eps_track=0.02, eps_vy=0.02, noise=None, eps32_track=2e-3, eps32_vy=3e-4):
    """Dynamic bicycle on a track (dict r0, half, amp, freq, phase, infl) with |v_y| < vy_bound - infl.
    eps_*: BF16X3 bands; eps32_*: FP32_RECHECK64 bands."""
    return _sys(BASIS_RACE_CAR, 6, 2, [(4, vy_bound, infl)], u_lo, u_hi, track=track,
                eps_box=[eps_vy], eps_track=eps_track, noise=noise, eps32_box=[eps32_vy], eps32_track=eps32_track)


# ---------------------------------------------------------------------------
# Context and calls
# ---------------------------------------------------------------------------
def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t, name, dtype, numel=None, device=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the context is on {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, needs {numel}")
    return t


# Trajectory buffers: rows of traj[H][n][.] start on 256-byte boundaries when
# the row stride is a multiple of 64 floats; with a stride of N + 1 floats
# each row starts 4 bytes further past such a boundary than the last, and
# the store runs at about half the rate.  The calls take the stride from the tensor, so a (H, n, Nc) view of a
# padded buffer is passed as is.
TRAJ_ROW_FLOATS = 64


def traj_ld(Nc: int) -> int:
    """Row stride (floats) of a padded trajectory buffer for Nc candidates."""
    return -(-Nc // TRAJ_ROW_FLOATS) * TRAJ_ROW_FLOATS


def new_traj(ctx: "Context", H: int, n: int, Nc: int):
    """A (H, n, Nc) float32 view of a (H, n, traj_ld(Nc)) device buffer."""
    return torch.empty((H, n, traj_ld(Nc)), dtype=torch.float32, device=ctx.device)[:, :, :Nc]


def _traj_stride(t, name, H, n, Nc, device):
    """Row stride of a trajectory tensor of shape (H, n, Nc): unit column
    stride, rows ld >= Nc floats apart, steps n * ld apart."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be torch.float32, got {t.dtype}")
    if not t.is_cuda or (device is not None and t.device != device):
        raise ValueError(f"{name} must be a device tensor on {device}")
    if tuple(t.shape) != (H, n, Nc):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, needs {(H, n, Nc)}")
    ld = t.stride(1) if n > 1 else (t.stride(0) if H > 1 else Nc)
    if (Nc > 1 and t.stride(2) != 1) or ld < Nc or (H > 1 and t.stride(0) != n * ld):
        raise ValueError(f"{name} needs unit column stride and rows ld >= Nc floats apart, steps n * ld apart; "
                         f"got strides {t.stride()}")
    return ld


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Context:
    """Owns an mpmi_ctx (selection slots + fit workspace) on one device."""

    def __init__(self, device: int = 0):
        self.lib = library()
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        h = ctypes.c_void_p()
        st = self.lib.mpmi_create(ctypes.byref(h), device)
        if st != OK:
            raise MpmiError(st, "mpmi_create failed")
        self.handle = h
        self._models = []

    def close(self):
        if getattr(self, "handle", None):
            self.lib.mpmi_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st: int):
        if st != OK:
            raise MpmiError(st, self.lib.mpmi_last_error(self.handle).decode())


@dataclass
class Model:
    """A packed model: the device blob plus the host descriptor it came from."""

    blob: torch.Tensor
    ptr: int
    system: System

    @property
    def n(self):
        return self.system.n_state

    @property
    def m(self):
        return self.system.n_input


def model_bytes() -> int:
    return int(library().mpmi_model_bytes())


def mpmi_model_pack(ctx: Context, system: System, K: torch.Tensor, stream=None, into: "Model" = None) -> Model:
    """Packs (system, K) into a new model, or in place into `into` (same blob)."""
    _need(K, "K", torch.float64, device=ctx.device)
    if into is None:
        blob = torch.empty(model_bytes() + 256, dtype=torch.uint8, device=ctx.device)
        ptr = (blob.data_ptr() + 255) // 256 * 256
    else:
        blob, ptr = into.blob, into.ptr
    ctx.check(ctx.lib.mpmi_model_pack(ctx.handle, ctypes.byref(system), _ptr(K), ctypes.c_void_p(ptr),
                                      _stream(stream)))
    return Model(blob=blob, ptr=ptr, system=system)


def koopman_fit(ctx: Context, system: System, X, U, Y, ridge: float = 0.0, stream=None):
    """Returns (K (D, n) float64 device tensor, condition estimate of the scaled lifted data)."""
    T, n = X.shape
    m = U.shape[1]
    for t, name in ((X, "X"), (U, "U"), (Y, "Y")):
        _need(t, name, torch.float64, device=ctx.device)
    if U.shape[0] != T or Y.shape != X.shape:
        raise ValueError("X, U, Y must have T rows; Y shaped like X")
    if n != system.n_state or m != system.n_input:
        raise ValueError("X/U widths do not match the system")
    D = basis_dim(system)
    K = torch.empty((D, n), dtype=torch.float64, device=ctx.device)
    cond = ctypes.c_double(0.0)
    ctx.check(ctx.lib.koopman_fit(ctx.handle, ctypes.byref(system), _ptr(X), _ptr(U), _ptr(Y), T, float(ridge),
                                  _ptr(K), ctypes.byref(cond), _stream(stream)))
    return K, cond.value


def basis_dim(system: System) -> int:
    if system.basis == BASIS_CUSTOM:
        return system.dim
    return {BASIS_LINEAR: system.n_state + system.n_input, BASIS_BALANCE_BOT: 21, BASIS_RACE_CAR: 64}[system.basis]


def koopman_select_basis(ctx: Context, lib: Library, X, U, Y, gammas, rho: float = 1.0, iters: int = 500,
                         stream=None):
    """Sparsity-promoting selection over the library for every penalty in
    gammas: returns (B (n_gamma, L, n) float64 device tensor, support
    (n_gamma, L) uint8 device tensor, residuals (n_gamma, 2) numpy)."""
    T, n = X.shape
    for t, name in ((X, "X"), (U, "U"), (Y, "Y")):
        _need(t, name, torch.float64, device=ctx.device)
    if U.shape[0] != T or Y.shape != X.shape or n != lib.n_state or U.shape[1] != lib.n_input:
        raise ValueError("X, U, Y must have T rows, n and m columns as the library states")
    g = (ctypes.c_double * len(gammas))(*[float(v) for v in gammas])
    B = torch.empty((len(gammas), lib.n_feat, n), dtype=torch.float64, device=ctx.device)
    sup = torch.empty((len(gammas), lib.n_feat), dtype=torch.uint8, device=ctx.device)
    res = (ctypes.c_double * (2 * len(gammas)))()
    ctx.check(ctx.lib.koopman_select_basis(ctx.handle, ctypes.byref(lib), _ptr(X.contiguous()),
                                           _ptr(U.contiguous()), _ptr(Y.contiguous()), T, g, len(gammas),
                                           float(rho), int(iters), _ptr(B), _ptr(sup), res, _stream(stream)))
    import numpy as _np
    return B, sup, _np.array(res[:]).reshape(len(gammas), 2)


def koopman_fit_lifted(ctx: Context, system: System, X, U, Y, ridge: float = 0.0, stream=None):
    """Lifted operator (D, D) float64 device tensor and the condition estimate."""
    T, n = X.shape
    for t, name in ((X, "X"), (U, "U"), (Y, "Y")):
        _need(t, name, torch.float64, device=ctx.device)
    if U.shape[0] != T or Y.shape != X.shape:
        raise ValueError("X, U, Y must have T rows; Y shaped like X")
    if n != system.n_state or U.shape[1] != system.n_input:
        raise ValueError("X/U widths do not match the system")
    D = basis_dim(system)
    K = torch.empty((D, D), dtype=torch.float64, device=ctx.device)
    cond = ctypes.c_double(0.0)
    ctx.check(ctx.lib.koopman_fit_lifted(ctx.handle, ctypes.byref(system), _ptr(X), _ptr(U), _ptr(Y), T,
                                         float(ridge), _ptr(K), ctypes.byref(cond), _stream(stream)))
    return K, cond.value


def mpmi_lifted_layout(basis: int, n: int, m: int):
    """(feat_g, feat_phi, n_phi, n_g) of a basis (host only)."""
    lib = library()
    D = {BASIS_LINEAR: n + m, BASIS_BALANCE_BOT: 21, BASIS_RACE_CAR: 64}[basis]
    fg, fp = (ctypes.c_int32 * D)(), (ctypes.c_int32 * D)()
    a, b = ctypes.c_int32(), ctypes.c_int32()
    st = lib.mpmi_lifted_layout(basis, n, m, fg, fp, ctypes.byref(a), ctypes.byref(b))
    if st != OK:
        raise MpmiError(st, "mpmi_lifted_layout failed")
    return list(fg), list(fp), a.value, b.value


@dataclass
class Lifted:
    """A packed lifted model (device blob) and the packed model it came from."""

    blob: torch.Tensor
    ptr: int
    model: Model
    h_max: int


def mpmi_lifted_pack(ctx: Context, model: Model, K_full, h_max: int, stream=None) -> Lifted:
    D = basis_dim(model.system)
    _need(K_full, "K_full", torch.float64, D * D, device=ctx.device)
    nbytes = int(ctx.lib.mpmi_lifted_bytes(h_max))
    if nbytes == 0:
        raise ValueError(f"h_max={h_max} out of range")
    blob = torch.empty(nbytes + 256, dtype=torch.uint8, device=ctx.device)
    ptr = (blob.data_ptr() + 255) // 256 * 256
    ctx.check(ctx.lib.mpmi_lifted_pack(ctx.handle, ctypes.c_void_p(model.ptr), _ptr(K_full), h_max,
                                       ctypes.c_void_p(ptr), _stream(stream)))
    return Lifted(blob=blob, ptr=ptr, model=model, h_max=h_max)


def mpmi_tick_lifted(ctx: Context, lifted: Lifted, desc: TickDesc, x_t, u_user, cand=None, out=None,
                     first_violation=None, traj=None, stream=None):
    """One tick with lifted predictions; returns the selection record (uint8 device tensor, 48 B)."""
    model = lifted.model
    _need(x_t, "x_t", torch.float32, model.n, device=ctx.device)
    _need(u_user, "u_user", torch.float32, model.m, device=ctx.device)
    Nc = desc.n_cand + 1
    if cand is not None:
        _need(cand, "cand", torch.float32, model.m * desc.n_cand, device=ctx.device)
    if first_violation is not None:
        _need(first_violation, "first_violation", torch.int16, Nc, device=ctx.device)
    ld = 0 if traj is None else _traj_stride(traj, "traj", desc.horizon, model.n, Nc, ctx.device)
    if out is None:
        out = torch.empty(SELECTION_BYTES, dtype=torch.uint8, device=ctx.device)
    _need(out, "out", torch.uint8, SELECTION_BYTES, device=ctx.device)
    ctx.check(ctx.lib.mpmi_tick_lifted(ctx.handle, ctypes.c_void_p(lifted.ptr), ctypes.byref(desc), _ptr(x_t),
                                       _ptr(u_user), _ptr(cand), _ptr(out), _ptr(first_violation), _ptr(traj), ld,
                                       _stream(stream)))
    return out


def rollout_batch(ctx: Context, model: Model, x0, cand, H: int, traj=None, precision=PREC_FP32, stream=None):
    """cand (S, m, Nc) float32 -> traj (H, n, Nc) float32 (full horizon); by
    default a view of a buffer with padded rows (new_traj)."""
    S, m, Nc = cand.shape
    _need(x0, "x0", torch.float32, model.n, device=ctx.device)
    _need(cand, "cand", torch.float32, device=ctx.device)
    if traj is None:
        traj = new_traj(ctx, H, model.n, Nc)
    ld = _traj_stride(traj, "traj", H, model.n, Nc, ctx.device)
    ctx.check(ctx.lib.rollout_batch(ctx.handle, ctypes.c_void_p(model.ptr), precision, _ptr(x0), _ptr(cand),
                                    Nc, S, H, _ptr(traj), ld, _stream(stream)))
    return traj


def safe_mask(ctx: Context, model: Model, traj, with_margin: bool = True, stream=None, with_near: bool = False):
    """traj (H, n, Nc), rows possibly padded -> (first_violation int16 (Nc,),
    min_margin float32 (Nc,) or None), and with_near: also the near-boundary
    bitmask int32 (ceil(Nc / 32),)."""
    H, n, Nc = traj.shape
    ld = _traj_stride(traj, "traj", H, n, Nc, ctx.device)
    fv = torch.empty(Nc, dtype=torch.int16, device=ctx.device)
    mm = torch.empty(Nc, dtype=torch.float32, device=ctx.device) if with_margin else None
    nb = torch.empty((Nc + 31) // 32, dtype=torch.int32, device=ctx.device) if with_near else None
    ctx.check(ctx.lib.safe_mask(ctx.handle, ctypes.c_void_p(model.ptr), _ptr(traj), ld, Nc, H, _ptr(fv), _ptr(nb),
                                _ptr(mm), _stream(stream)))
    return (fv, mm, nb) if with_near else (fv, mm)


def select_min_intervention(ctx: Context, model: Model, cand, first_violation, H: int, u_user, loop: int = 0,
                            out=None, stream=None):
    """cand (S, m, Nc), first_violation int16 (Nc,) -> selection record (uint8 device tensor of 48 B)."""
    S, m, Nc = cand.shape
    _need(cand, "cand", torch.float32, device=ctx.device)
    _need(first_violation, "first_violation", torch.int16, Nc, device=ctx.device)
    _need(u_user, "u_user", torch.float32, model.m, device=ctx.device)
    if out is None:
        out = torch.empty(SELECTION_BYTES, dtype=torch.uint8, device=ctx.device)
    _need(out, "out", torch.uint8, SELECTION_BYTES, device=ctx.device)
    ctx.check(ctx.lib.select_min_intervention(ctx.handle, ctypes.c_void_p(model.ptr), _ptr(cand), Nc, S,
                                              _ptr(first_violation), H, _ptr(u_user), loop, _ptr(out),
                                              _stream(stream)))
    return out


def tick_desc(n_cand, horizon, gen=GEN_GRID, grid=None, n_seg=1, seed=0, tick=0, loop=0,
              precision=PREC_FP32, block=0, lanes_per_cand=0) -> TickDesc:
    d = TickDesc()
    d.lanes_per_cand = lanes_per_cand
    d.seed, d.tick, d.loop, d.gen, d.n_cand = seed, tick, loop, gen, n_cand
    for j, g in enumerate(grid or []):
        d.grid[j] = g
    d.n_seg, d.horizon, d.precision, d.block = n_seg, horizon, precision, block
    return d


def mpmi_tick(ctx: Context, model: Model, desc: TickDesc, x_t, u_user, cand=None, out=None,
              first_violation=None, traj=None, stream=None):
    """One fused tick; returns the selection record (uint8 device tensor, 48 B)."""
    _need(x_t, "x_t", torch.float32, model.n, device=ctx.device)
    _need(u_user, "u_user", torch.float32, model.m, device=ctx.device)
    Nc = desc.n_cand + 1
    if cand is not None:
        _need(cand, "cand", torch.float32, desc.n_seg * model.m * desc.n_cand, device=ctx.device)
    if first_violation is not None:
        _need(first_violation, "first_violation", torch.int16, Nc, device=ctx.device)
    ld = 0 if traj is None else _traj_stride(traj, "traj", desc.horizon, model.n, Nc, ctx.device)
    if out is None:
        out = torch.empty(SELECTION_BYTES, dtype=torch.uint8, device=ctx.device)
    _need(out, "out", torch.uint8, SELECTION_BYTES, device=ctx.device)
    ctx.check(ctx.lib.mpmi_tick(ctx.handle, ctypes.c_void_p(model.ptr), ctypes.byref(desc), _ptr(x_t),
                                _ptr(u_user), _ptr(cand), _ptr(out), _ptr(first_violation), _ptr(traj), ld,
                                _stream(stream)))
    return out


def mpmi_tick_noalloc(model: Model, desc: TickDesc, x_t, u_user, out, cand=None, first_violation=None,
                      stream=None):
    """The allocation-free tick (no context; the library's static scratch on
    the current device): writes the record into `out` (uint8 device tensor,
    48 B) and returns it.  Argument checks only -- the binding allocates
    nothing either."""
    lib = library()
    dev = torch.device("cuda", torch.cuda.current_device())
    _need(x_t, "x_t", torch.float32, model.n, device=dev)
    _need(u_user, "u_user", torch.float32, model.m, device=dev)
    _need(out, "out", torch.uint8, SELECTION_BYTES, device=dev)
    if cand is not None:
        _need(cand, "cand", torch.float32, desc.n_seg * model.m * desc.n_cand, device=dev)
    if first_violation is not None:
        _need(first_violation, "first_violation", torch.int16, desc.n_cand + 1, device=dev)
    st = lib.mpmi_tick_noalloc(ctypes.byref(model.system), ctypes.c_void_p(model.ptr), ctypes.byref(desc), _ptr(x_t),
                               _ptr(u_user), _ptr(cand), _ptr(out), _ptr(first_violation), _stream(stream))
    if st != OK:
        raise MpmiError(st, lib.mpmi_last_error(None).decode())
    return out


class TickGraph:
    """One mpmi_tick captured as a HIP graph (mpmi_tick_graph); replays read
    the captured x_t / u_user / cand tensors and write out / first_violation."""

    def __init__(self, ctx: Context, model: Model, desc: TickDesc, x_t, u_user, cand=None, out=None,
                 first_violation=None):
        _need(x_t, "x_t", torch.float32, model.n, device=ctx.device)
        _need(u_user, "u_user", torch.float32, model.m, device=ctx.device)
        if cand is not None:
            _need(cand, "cand", torch.float32, desc.n_seg * model.m * desc.n_cand, device=ctx.device)
        if first_violation is not None:
            _need(first_violation, "first_violation", torch.int16, desc.n_cand + 1, device=ctx.device)
        self.out = torch.zeros(SELECTION_BYTES, dtype=torch.uint8, device=ctx.device) if out is None else out
        _need(self.out, "out", torch.uint8, SELECTION_BYTES, device=ctx.device)
        self.ctx, self._keep = ctx, (model, x_t, u_user, cand, first_violation)
        g = ctypes.c_void_p()
        ctx.check(ctx.lib.mpmi_tick_graph(ctx.handle, ctypes.c_void_p(model.ptr), ctypes.byref(desc), _ptr(x_t),
                                          _ptr(u_user), _ptr(cand), _ptr(self.out), _ptr(first_violation),
                                          ctypes.byref(g)))
        self.graph = g

    def launch(self, stream=None):
        self.ctx.check(self.ctx.lib.mpmi_graph_launch(self.ctx.handle, self.graph, _stream(stream)))
        return self.out

    def close(self):
        if getattr(self, "graph", None) is not None:
            self.ctx.lib.mpmi_graph_destroy(self.graph)
            self.graph = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mpmi_tick_autotune(ctx: Context, model: Model, desc: TickDesc, x_t, u_user, cand=None, reps: int = 20,
                       stream=None):
    """Times the launch shapes of a tick and sets desc.block / desc.lanes_per_cand to the fastest."""
    out = torch.empty(SELECTION_BYTES, dtype=torch.uint8, device=ctx.device)
    ms = ctypes.c_float()
    ctx.check(ctx.lib.mpmi_tick_autotune(ctx.handle, ctypes.c_void_p(model.ptr), ctypes.byref(desc), _ptr(x_t),
                                         _ptr(u_user), _ptr(cand), _ptr(out), reps, ctypes.byref(ms),
                                         _stream(stream)))
    return dict(block=desc.block, lanes_per_cand=desc.lanes_per_cand, ms=ms.value)


def mpmi_generate_candidates(ctx: Context, model: Model, desc: TickDesc, u_user, cand=None, stream=None):
    """The candidates a tick with `desc` evaluates, (S, m, N+1) float32 (column 0 = u_user)."""
    _need(u_user, "u_user", torch.float32, model.m, device=ctx.device)
    if cand is not None:
        _need(cand, "cand", torch.float32, desc.n_seg * model.m * desc.n_cand, device=ctx.device)
    out = torch.empty((desc.n_seg, model.m, desc.n_cand + 1), dtype=torch.float32, device=ctx.device)
    ctx.check(ctx.lib.mpmi_generate_candidates(ctx.handle, ctypes.c_void_p(model.ptr), ctypes.byref(desc),
                                               _ptr(u_user), _ptr(cand), _ptr(out), _stream(stream)))
    return out


def mpmi_write_rates(ctx: Context, buf, Nc: int, rows: int, ld: int = None) -> dict:
    """Write ceilings (GB/s) of the trajectory store's pattern (rows ld >= Nc
    floats apart; default Nc) and of a contiguous stream, on buf (rows * ld
    float32, overwritten; synchronous)."""
    ld = Nc if ld is None else ld
    _need(buf, "buf", torch.float32, rows * ld, device=ctx.device)
    p, q = ctypes.c_double(0.0), ctypes.c_double(0.0)
    ctx.check(ctx.lib.mpmi_write_rates(ctx.handle, _ptr(buf), Nc, ld, rows, ctypes.byref(p), ctypes.byref(q)))
    return dict(pattern_GB_s=p.value, stream_GB_s=q.value)


def mpmi_read_rates(ctx: Context, buf, Nc: int, rows: int, ld: int = None) -> dict:
    """Read ceilings (GB/s) of the safety check's load pattern over stored
    trajectories (rows ld >= Nc floats apart; default Nc) and of a contiguous
    stream, on buf (rows * ld float32, read only; synchronous)."""
    ld = Nc if ld is None else ld
    _need(buf, "buf", torch.float32, rows * ld, device=ctx.device)
    p, q = ctypes.c_double(0.0), ctypes.c_double(0.0)
    ctx.check(ctx.lib.mpmi_read_rates(ctx.handle, _ptr(buf), Nc, ld, rows, ctypes.byref(p), ctypes.byref(q)))
    return dict(pattern_GB_s=p.value, stream_GB_s=q.value)


def mpmi_fp32_fma_rate(ctx: Context) -> float:
    """Measured non-packed FP32 FMA issue rate of the device, TFLOP/s (synchronous)."""
    r = ctypes.c_double(0.0)
    ctx.check(ctx.lib.mpmi_fp32_fma_rate(ctx.handle, ctypes.byref(r)))
    return r.value


def mpmi_sincos64(ctx: Context, x, sn, cs, stream=None) -> None:
    """sn, cs = sin, cos of x (float64 device tensors of equal size) by the FP64 re-roll's function."""
    n = x.numel()
    for t, name in ((x, "x"), (sn, "sn"), (cs, "cs")):
        _need(t, name, torch.float64, n, device=ctx.device)
    ctx.check(ctx.lib.mpmi_sincos64(ctx.handle, _ptr(x), _ptr(sn), _ptr(cs), n, _stream(stream)))


def decode_selection(rec) -> dict:
    """Host view of one or more selection records (uint8 tensor of 48*k bytes)."""
    raw = bytes(rec.detach().cpu().numpy().tobytes())
    out = []
    for k in range(len(raw) // SELECTION_BYTES):
        s = Selection.from_buffer_copy(raw[k * SELECTION_BYTES:(k + 1) * SELECTION_BYTES])
        out.append(dict(idx=s.idx, status=s.status, n_safe=s.n_safe, n_recheck=s.n_recheck,
                        u_r=list(s.u_r), cost=s.cost, deviation=s.deviation,
                        first_violation=s.first_violation, n_cand=s.n_cand))
    return out[0] if len(out) == 1 else out


# ---------------------------------------------------------------------------
# Many loops in one launch per tick
# ---------------------------------------------------------------------------
class Multi:
    """A set of control loops served by one persistent launch per tick.

    `loops` is a list of dicts with keys model (Model), x_t, u_user (device
    tensors at fixed addresses, read every tick), out (uint8 tensor of 48 B),
    n_cand, horizon and optionally gen, grid, n_seg, seed, tick, cand,
    first_violation.  The tensors are kept alive by this object.
    """

    def __init__(self, ctx: Context, loops, block: int = 256, precision: int = PREC_FP32):
        self.ctx = ctx
        self._keep = []
        arr = (LoopDesc * len(loops))()
        for i, l in enumerate(loops):
            d = arr[i]
            model = l["model"]
            _need(l["x_t"], "x_t", torch.float32, model.n, device=ctx.device)
            _need(l["u_user"], "u_user", torch.float32, model.m, device=ctx.device)
            _need(l["out"], "out", torch.uint8, SELECTION_BYTES, device=ctx.device)
            d.model = model.ptr
            d.x_t = l["x_t"].data_ptr()
            d.u_user = l["u_user"].data_ptr()
            d.out = l["out"].data_ptr()
            d.cand = l["cand"].data_ptr() if l.get("cand") is not None else None
            fv = l.get("first_violation")
            if fv is not None:
                _need(fv, "first_violation", torch.int16, l["n_cand"] + 1, device=ctx.device)
            d.first_violation = fv.data_ptr() if fv is not None else None
            d.seed, d.tick = l.get("seed", 0), l.get("tick", 0)
            d.gen, d.n_cand = l.get("gen", GEN_UNIFORM), l["n_cand"]
            for j, g in enumerate(l.get("grid") or []):
                d.grid[j] = g
            d.n_seg, d.horizon = l.get("n_seg", 1), l["horizon"]
            self._keep.append(l)
        cfg = MultiConfig(block, 0, precision)
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.mpmi_multi_create(ctx.handle, arr, len(loops), ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self.graph = None

    def config(self):
        cfg, n = MultiConfig(), ctypes.c_int32()
        self.ctx.lib.mpmi_multi_get_config(self.handle, ctypes.byref(cfg), ctypes.byref(n))
        return dict(block=cfg.block, grid=cfg.grid, n_work=n.value, precision=cfg.precision)

    def _drop_graph(self):
        # A captured graph holds the launch shape of the plan it was taken from.
        if self.graph is not None:
            self.ctx.lib.mpmi_graph_destroy(self.graph)
            self.graph = None

    def set_config(self, block: int, precision=None):
        self._drop_graph()
        if precision is None:
            precision = self.config()["precision"]
        self.ctx.check(self.ctx.lib.mpmi_multi_set_config(self.ctx.handle, self.handle,
                                                         ctypes.byref(MultiConfig(block, 0, precision))))

    def tick(self, stream=None):
        self.ctx.check(self.ctx.lib.mpmi_multi_tick(self.ctx.handle, self.handle, _stream(stream)))

    def ticks(self):
        """Device tick counters of the loops (synchronous)."""
        arr = (ctypes.c_uint64 * len(self._keep))()
        self.ctx.check(self.ctx.lib.mpmi_multi_get_ticks(self.ctx.handle, self.handle, arr))
        return list(arr)

    def autotune(self, reps: int = 20, stream=None):
        self._drop_graph()
        best, ms = MultiConfig(), ctypes.c_float()
        self.ctx.check(self.ctx.lib.mpmi_multi_autotune(self.ctx.handle, self.handle, reps, ctypes.byref(best),
                                                        ctypes.byref(ms), _stream(stream)))
        return dict(block=best.block, grid=best.grid, ms=ms.value)

    def capture_graph(self):
        if self.graph is not None:
            self.ctx.lib.mpmi_graph_destroy(self.graph)
        g = ctypes.c_void_p()
        self.ctx.check(self.ctx.lib.mpmi_multi_graph(self.ctx.handle, self.handle, ctypes.byref(g)))
        self.graph = g
        return g

    def launch_graph(self, stream=None):
        self.ctx.check(self.ctx.lib.mpmi_graph_launch(self.ctx.handle, self.graph, _stream(stream)))

    def close(self):
        if getattr(self, "graph", None) is not None:
            self.ctx.lib.mpmi_graph_destroy(self.graph)
            self.graph = None
        if getattr(self, "handle", None):
            self.ctx.lib.mpmi_multi_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Proposal network
# ---------------------------------------------------------------------------
MLP_IN, MLP_HIDDEN, MLP_COMP, MLP_OUT, MLP_PARAMS = 8, 256, 16, 80, 154448


def mlp_workspace(ctx: Context, batch: int) -> torch.Tensor:
    n = int(ctx.lib.mlp_workspace_bytes(batch))
    if n == 0:
        raise ValueError(f"batch {batch} out of range")
    buf = torch.empty(n + 256, dtype=torch.uint8, device=ctx.device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + n]


def mlp_forward(ctx: Context, w16, w32, mean, std, X, work=None, stream=None):
    B = X.shape[0]
    _need(w16, "w16", torch.bfloat16, MLP_PARAMS, device=ctx.device)
    _need(w32, "w32", torch.float32, MLP_PARAMS, device=ctx.device)
    _need(X, "X", torch.float32, B * MLP_IN, device=ctx.device)
    work = mlp_workspace(ctx, B) if work is None else work
    Y = torch.empty((B, MLP_OUT), dtype=torch.float32, device=ctx.device)
    ctx.check(ctx.lib.mlp_forward(ctx.handle, _ptr(w16), _ptr(w32), _ptr(mean), _ptr(std), _ptr(X), B, _ptr(Y),
                                  _ptr(work), work.numel(), _stream(stream)))
    return Y


def mlp_grad(ctx: Context, w16, w32, mean, std, X, T, work=None, grad=None, loss=None, stream=None):
    B = X.shape[0]
    _need(X, "X", torch.float32, B * MLP_IN, device=ctx.device)
    _need(T, "T", torch.float32, B * 2, device=ctx.device)
    work = mlp_workspace(ctx, B) if work is None else work
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=ctx.device) if grad is None else grad
    loss = torch.empty(1, dtype=torch.float32, device=ctx.device) if loss is None else loss
    ctx.check(ctx.lib.mlp_grad(ctx.handle, _ptr(w16), _ptr(w32), _ptr(mean), _ptr(std), _ptr(X), _ptr(T), B,
                               _ptr(grad), _ptr(loss), _ptr(work), work.numel(), _stream(stream)))
    return grad, loss


def mlp_adam(ctx: Context, w32, w16, m, v, grad, step: int, lr: float = 1e-3, stream=None):
    ctx.check(ctx.lib.mlp_adam(ctx.handle, _ptr(w32), _ptr(w16), _ptr(m), _ptr(v), _ptr(grad), step, lr,
                               _stream(stream)))


def mdn_sample(ctx: Context, model: Model, head, P: int, seed: int = 0, tick: int = 0, loop: int = 0,
               cand=None, stream=None):
    """P proposals (1, 2, P) float32 from one head (80,)."""
    _need(head, "head", torch.float32, MLP_OUT, device=ctx.device)
    cand = torch.empty((1, 2, P), dtype=torch.float32, device=ctx.device) if cand is None else cand
    ctx.check(ctx.lib.mdn_sample(ctx.handle, ctypes.c_void_p(model.ptr), _ptr(head), P, seed, tick, loop,
                                 _ptr(cand), _stream(stream)))
    return cand


def mpmi_proposal_tick(ctx: Context, model: Model, net: dict, x_t, u_user, prop: TickDesc, fallback: TickDesc,
                       cand_work, work, out=None, head_out=None, stream=None):
    """Learned-proposal tick; net holds w16, w32, mean, std device tensors."""
    out = torch.empty(SELECTION_BYTES, dtype=torch.uint8, device=ctx.device) if out is None else out
    _need(cand_work, "cand_work", torch.float32, 2 * prop.n_cand, device=ctx.device)
    ctx.check(ctx.lib.mpmi_proposal_tick(
        ctx.handle, ctypes.c_void_p(model.ptr), _ptr(net["w16"]), _ptr(net["w32"]), _ptr(net["mean"]),
        _ptr(net["std"]), _ptr(x_t), _ptr(u_user), ctypes.byref(prop), ctypes.byref(fallback), _ptr(cand_work),
        _ptr(head_out), _ptr(out), _ptr(work), work.numel(), _stream(stream)))
    return out


def mpmi_gemm_bf16(ctx: Context, A, B, M: int, N: int, K: int, ta: int = 0, tb: int = 0, stream=None):
    _need(A, "A", torch.bfloat16, M * K, device=ctx.device)
    _need(B, "B", torch.bfloat16, K * N, device=ctx.device)
    C = torch.empty((M, N), dtype=torch.float32, device=ctx.device)
    ctx.check(ctx.lib.mpmi_gemm_bf16(ctx.handle, _ptr(A), _ptr(B), M, N, K, ta, tb, _ptr(C), _stream(stream)))
    return C
