"""ctypes binding of libtddftb.so: the C ABI of tddftb.h, one Python name per entry point.

Argument marshalling only: numpy arrays are passed as host pointers and
every step of the propagation runs in the library's HIP kernels. There is
no fallback: if the library is not built or cannot be loaded, importing
this module's functions raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
# TDDFTB_LIB selects another build of the same library (the host-sanitized one
# of the C ABI tests); the default is the in-tree build
LIB_PATH = os.environ.get("TDDFTB_LIB") or os.path.join(PKG, "libtddftb.so")

TD_OK, TD_EINVAL, TD_ENOMEM, TD_EHIP, TD_ENOTPOSDEF = 0, -1, -2, -3, -4
TD_ESCF, TD_EUNSTABLE, TD_ENOTSUP, TD_ESTATE = -5, -6, -7, -8
TD_FP64, TD_SPLIT_BF16 = 0, 1
TD_KT_GEMM_SH, TD_KT_GEMM_ARHO, TD_KT_UPDATE, TD_KT_OTHER = 0, 1, 2, 3
TD_DEVICE_PTRS = 1
TD_PLUS_U_NONE, TD_PLUS_U_FLL, TD_PLUS_U_PSIC = 0, 1, 2
TD_PLUS_U_MAX_SHELL = 7

EXPORTED = [
    "td_default_options", "td_create", "td_kick", "td_step", "td_get_charges",
    "td_get_dipole", "td_get_dipole_series", "td_get_energy", "td_get_rho", "td_set_rho",
    "td_get_info", "td_get_kernel_time", "td_reset_kernel_time", "td_get_forces",
    "td_last_error", "td_status_string", "td_destroy", "td_util_gemm",
    "td_batch_create", "td_batch_kick", "td_batch_step", "td_batch_get_dipole_series",
    "td_batch_get_charges", "td_batch_get_rho", "td_batch_get_info", "td_batch_last_error",
    "td_batch_destroy", "td_spectrum", "td_transient_absorption", "td_create_ehrenfest",
    "td_get_nuclei", "td_get_energy_series", "td_util_gemm_noalloc",
    "td_batch_create_ehrenfest", "td_batch_get_nuclei", "td_batch_get_energy_series",
]
TD_BATCH_NO_GRAPH, TD_BATCH_TILE_128, TD_BATCH_TILE_64 = 1, 2, 4
TD_BATCH_BUCKETS = 8

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


class TdSystem(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int32), ("n_orb", ctypes.c_int32),
                ("orb_offset", _ip), ("positions", _dp), ("S", _dp), ("H0", _dp),
                ("gamma", _dp), ("q0", _dp), ("n_elec", ctypes.c_int32), ("rho0", _dp),
                ("occ", _dp), ("flags", ctypes.c_uint32), ("plus_u", ctypes.c_int32),
                ("n_shells", ctypes.c_int32), ("shell_offset", _ip), ("shell_u", _dp)]


class TdOptions(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("n_slices", ctypes.c_int32),
                ("dt", ctypes.c_double), ("scc_tol", ctypes.c_double),
                ("scc_maxiter", ctypes.c_int32), ("mix_beta", ctypes.c_double),
                ("mix_history", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("hip_stream", ctypes.c_void_p), ("n_slices_dh", ctypes.c_int32)]


class TdInfo(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int32), ("n_orb", ctypes.c_int32), ("n_pad", ctypes.c_int32),
                ("inverse_iterations", ctypes.c_int32), ("inverse_residual", ctypes.c_double),
                ("scc_iterations", ctypes.c_int32), ("scc_residual", ctypes.c_double),
                ("purification_iterations", ctypes.c_int32),
                ("purification_error", ctypes.c_double),
                ("spectrum_lo", ctypes.c_double), ("spectrum_hi", ctypes.c_double),
                ("step", ctypes.c_int64), ("has_prev", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("inverse_updates", ctypes.c_int64),
                ("width_estimate", ctypes.c_double), ("stability", ctypes.c_double),
                ("inverse_restarts", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status_string(status)}: {message}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the library (once). Raises if it is missing: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    sig = {
        "td_default_options": (None, [ctypes.POINTER(TdOptions)]),
        "td_create": (ctypes.c_int32, [ctypes.POINTER(TdSystem), ctypes.POINTER(TdOptions),
                                       ctypes.POINTER(vp), ctypes.c_char_p, ctypes.c_int32]),
        "td_kick": (ctypes.c_int32, [vp, ctypes.c_double, _dp]),
        "td_step": (ctypes.c_int32, [vp, ctypes.c_int32, _dp]),
        "td_get_charges": (ctypes.c_int32, [vp, _dp]),
        "td_get_dipole": (ctypes.c_int32, [vp, _dp]),
        "td_get_dipole_series": (ctypes.c_int32, [vp, _dp, ctypes.c_int32, _ip]),
        "td_get_energy": (ctypes.c_int32, [vp, _dp, _dp]),
        "td_get_rho": (ctypes.c_int32, [vp, _dp, _dp, ctypes.POINTER(ctypes.c_int64), _ip]),
        "td_set_rho": (ctypes.c_int32, [vp, _dp, _dp, ctypes.c_int64]),
        "td_get_info": (ctypes.c_int32, [vp, ctypes.POINTER(TdInfo)]),
        "td_get_kernel_time": (ctypes.c_int32, [vp, ctypes.c_int32, _dp,
                                                ctypes.POINTER(ctypes.c_int64)]),
        "td_reset_kernel_time": (ctypes.c_int32, [vp]),
        "td_get_forces": (ctypes.c_int32, [vp, _dp]),
        "td_last_error": (ctypes.c_char_p, [vp]),
        "td_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
        "td_destroy": (None, [vp]),
        "td_util_gemm": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, _dp, _dp, _dp,
                                          ctypes.c_char_p, ctypes.c_int32]),
        "td_util_gemm_noalloc": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                  ctypes.c_int32, ctypes.c_int32, vp,
                                                  ctypes.c_int32, vp, ctypes.c_int32, vp,
                                                  ctypes.c_int32, vp, ctypes.c_char_p,
                                                  ctypes.c_int32]),
        "td_batch_create": (ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(TdSystem),
                                             ctypes.POINTER(TdOptions), ctypes.c_uint32,
                                             ctypes.POINTER(vp), ctypes.c_char_p,
                                             ctypes.c_int32]),
        "td_batch_kick": (ctypes.c_int32, [vp, _dp, _dp]),
        "td_batch_step": (ctypes.c_int32, [vp, ctypes.c_int32, _dp]),
        "td_batch_get_dipole_series": (ctypes.c_int32, [vp, ctypes.c_int32, _dp, ctypes.c_int32,
                                                        _ip]),
        "td_batch_get_charges": (ctypes.c_int32, [vp, ctypes.c_int32, _dp]),
        "td_batch_get_rho": (ctypes.c_int32, [vp, ctypes.c_int32, _dp, _dp,
                                              ctypes.POINTER(ctypes.c_int64), _ip]),
        "td_batch_get_info": (ctypes.c_int32, [vp, ctypes.POINTER(TdBatchInfo)]),
        "td_batch_last_error": (ctypes.c_char_p, [vp]),
        "td_batch_create_ehrenfest": (ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(TdSystem),
                                                       ctypes.POINTER(TdModel), _dp,
                                                       ctypes.POINTER(TdOptions),
                                                       ctypes.POINTER(vp), ctypes.c_char_p,
                                                       ctypes.c_int32]),
        "td_batch_get_nuclei": (ctypes.c_int32, [vp, ctypes.c_int32, _dp, _dp]),
        "td_batch_get_energy_series": (ctypes.c_int32, [vp, ctypes.c_int32, _dp, _dp,
                                                        ctypes.c_int32, _ip]),
        "td_batch_destroy": (None, [vp]),
        "td_create_ehrenfest": (ctypes.c_int32, [ctypes.POINTER(TdSystem), ctypes.POINTER(TdModel),
                                                 _dp, ctypes.POINTER(TdOptions),
                                                 ctypes.POINTER(vp), ctypes.c_char_p,
                                                 ctypes.c_int32]),
        "td_get_nuclei": (ctypes.c_int32, [vp, _dp, _dp]),
        "td_get_energy_series": (ctypes.c_int32, [vp, _dp, _dp, ctypes.c_int32, _ip]),
        "td_spectrum": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, _dp, _dp, _dp,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_int32, _dp,
                                         _dp, _dp, _dp, ctypes.c_char_p, ctypes.c_int32]),
        "td_transient_absorption": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32,
                                                     ctypes.c_int32, _dp, _dp, _dp,
                                                     ctypes.c_double, ctypes.c_double,
                                                     ctypes.c_int32, _dp, ctypes.c_int32,
                                                     ctypes.c_double, ctypes.c_double, _dp,
                                                     ctypes.c_char_p, ctypes.c_int32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray], dtype=np.float64):
    if a is None:
        return None
    assert a.dtype == dtype and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_ip if dtype == np.int32 else _dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def status_string(status: int) -> str:
    return load().td_status_string(status).decode()


def td_default_options() -> TdOptions:
    o = TdOptions()
    load().td_default_options(ctypes.byref(o))
    return o


class TdModel(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("species", _ip), ("species_norb", _ip),
                ("sk_s", _dp), ("sk_h", _dp), ("decay", ctypes.c_double), ("scale_s", _dp),
                ("scale_h", _dp), ("onsite", _dp), ("hubbard_u", ctypes.c_double),
                ("mass", _dp), ("rep_a", _dp), ("rep_decay", ctypes.c_double)]


class TdBatchInfo(ctypes.Structure):
    _fields_ = [("n_members", ctypes.c_int32), ("step", ctypes.c_int64),
                ("has_prev", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("bucket_members", ctypes.c_int32 * TD_BATCH_BUCKETS),
                ("bucket_tile", ctypes.c_int32 * TD_BATCH_BUCKETS),
                ("bucket_ms", (ctypes.c_double * 2) * TD_BATCH_BUCKETS)]

    def as_dict(self):
        return {"n_members": self.n_members, "step": self.step, "has_prev": bool(self.has_prev),
                "graph": bool(self.graph), "bucket_members": list(self.bucket_members),
                "bucket_tile": list(self.bucket_tile),
                "bucket_ms": [list(x) for x in self.bucket_ms]}


class _Keep:
    """Host arrays kept alive while a td_system refers to them."""


def _create(s: TdSystem, options: Optional[TdOptions]):
    opt = options if options is not None else td_default_options()
    ctx = ctypes.c_void_p()
    err = ctypes.create_string_buffer(1024)
    st = load().td_create(ctypes.byref(s), ctypes.byref(opt), ctypes.byref(ctx), err, 1024)
    if st != TD_OK:
        raise TdError(st, err.value.decode())
    return ctx


def td_create_from_tensors(orb_offset, positions, S, H0, gamma, q0, n_elec: int = 0,
                           rho0=None, occ=None, options: Optional[TdOptions] = None):
    """td_create with TD_DEVICE_PTRS: the arrays are contiguous GPU tensors
    (int32 orb_offset, float64 arrays, complex128 rho0). Unless options name a
    stream, the library reads them on, and then uses, the current stream."""
    import torch
    arrs = {"orb_offset": (orb_offset, torch.int32), "positions": (positions, torch.float64),
            "S": (S, torch.float64), "H0": (H0, torch.float64), "gamma": (gamma, torch.float64),
            "q0": (q0, torch.float64), "rho0": (rho0, torch.complex128),
            "occ": (occ, torch.float64)}
    ptrs = {}
    for name, (t, dt) in arrs.items():
        if t is None:
            ptrs[name] = None
            continue
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dt and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {dt} GPU tensor")
        ptrs[name] = ctypes.cast(ctypes.c_void_p(t.data_ptr()),
                                 _ip if dt == torch.int32 else _dp)
    opt = options if options is not None else td_default_options()
    if not opt.hip_stream:
        opt.hip_stream = torch.cuda.current_stream().cuda_stream
    s = TdSystem(n_atoms=int(q0.numel()), n_orb=int(S.shape[0]), n_elec=int(n_elec),
                 flags=TD_DEVICE_PTRS, **ptrs)
    return _create(s, opt)


def _plus_u_mode(mode) -> int:
    """'fll' / 'psic', or an integer passed through for the library to check."""
    if isinstance(mode, (int, np.integer)):
        return int(mode)
    names = {"fll": TD_PLUS_U_FLL, "psic": TD_PLUS_U_PSIC}
    if mode not in names:
        raise ValueError(f"unknown plus_u mode {mode!r}")
    return names[mode]


def _host_system(system, rho0=None, occ=None, plus_u=None):
    """TdSystem over host copies of `system`'s arrays (kept alive in the result's _keep).
    ``plus_u``: None, or an object with ``mode`` ('fll' / 'psic' or TD_PLUS_U_*),
    ``shell_offset`` and ``shell_u`` (the on-site corrections)."""
    keep = _Keep()
    keep.off = np.ascontiguousarray(system.orb_offset, dtype=np.int32)
    keep.pos = _f64(system.positions)
    keep.S = _f64(system.S)
    keep.H0 = _f64(system.H0)
    keep.gamma = _f64(system.gamma)
    keep.q0 = _f64(system.q0)
    keep.rho0 = None if rho0 is None else np.ascontiguousarray(rho0, dtype=np.complex128)
    keep.occ = None if occ is None else _f64(occ)
    s = TdSystem(n_atoms=len(keep.q0), n_orb=int(keep.off[-1]), orb_offset=_ptr(keep.off, np.int32),
                 positions=_ptr(keep.pos), S=_ptr(keep.S), H0=_ptr(keep.H0),
                 gamma=_ptr(keep.gamma), q0=_ptr(keep.q0),
                 n_elec=int(system.n_elec) if occ is None else 0,
                 rho0=None if keep.rho0 is None else keep.rho0.ctypes.data_as(_dp),
                 occ=_ptr(keep.occ), flags=0)
    if plus_u is not None:
        keep.shell_off = np.ascontiguousarray(plus_u.shell_offset, dtype=np.int32)
        keep.shell_u = _f64(plus_u.shell_u)
        s.plus_u = _plus_u_mode(plus_u.mode)
        s.n_shells = len(keep.shell_u)
        s.shell_offset = _ptr(keep.shell_off, np.int32)
        s.shell_u = _ptr(keep.shell_u)
    s._keep = keep
    return s


def td_create(system, options: Optional[TdOptions] = None, rho0: Optional[np.ndarray] = None,
              occ: Optional[np.ndarray] = None, plus_u=None):
    """td_create: returns an opaque context handle (c_void_p)."""
    return _create(_host_system(system, rho0, occ, plus_u), options)


def _model_struct(model: dict, keep):
    """TdModel over host arrays held by ``keep``."""
    keep.species = np.ascontiguousarray(model["species"], dtype=np.int32)
    keep.norb = np.ascontiguousarray(model["species_norb"], dtype=np.int32)
    keep.sk_s = _f64(model["sk_s"])
    keep.sk_h = _f64(model["sk_h"])
    keep.scale_s = _f64(model["scale_s"])
    keep.scale_h = _f64(model["scale_h"])
    keep.onsite = _f64(model["onsite"])
    keep.mass = _f64(model["mass"])
    rep = model.get("rep_a")
    keep.rep_a = None if rep is None else _f64(rep)
    return TdModel(n_species=len(keep.norb), species=_ptr(keep.species, np.int32),
                   species_norb=_ptr(keep.norb, np.int32), sk_s=_ptr(keep.sk_s),
                   sk_h=_ptr(keep.sk_h), decay=float(model["decay"]), scale_s=_ptr(keep.scale_s),
                   scale_h=_ptr(keep.scale_h), onsite=_ptr(keep.onsite),
                   hubbard_u=float(model["hubbard_u"]), mass=_ptr(keep.mass),
                   rep_a=None if rep is None else _ptr(keep.rep_a),
                   rep_decay=float(model.get("rep_decay", 0.0)))


def td_create_ehrenfest(system, model: dict, velocities=None, options: Optional[TdOptions] = None,
                        rho0: Optional[np.ndarray] = None, plus_u=None):
    """td_create_ehrenfest over host arrays; ``model`` as workloads.two_centre_model."""
    hs = _host_system(system, rho0, None, plus_u)
    keep = _Keep()
    m = _model_struct(model, keep)
    keep.vel = None if velocities is None else _f64(velocities)
    opt = options if options is not None else td_default_options()
    ctx = ctypes.c_void_p()
    err = ctypes.create_string_buffer(1024)
    st = load().td_create_ehrenfest(ctypes.byref(hs), ctypes.byref(m), _ptr(keep.vel),
                                    ctypes.byref(opt), ctypes.byref(ctx), err, 1024)
    if st != TD_OK:
        raise TdError(st, err.value.decode())
    return ctx


def td_get_nuclei(ctx, n_atoms: int):
    pos = np.empty((n_atoms, 3))
    vel = np.empty((n_atoms, 3))
    _check(ctx, load().td_get_nuclei(ctx, _ptr(pos), _ptr(vel)))
    return pos, vel


def td_get_energy_series(ctx, cap: int):
    ee = np.empty(max(cap, 1))
    ek = np.empty(max(cap, 1))
    n = ctypes.c_int32()
    _check(ctx, load().td_get_energy_series(ctx, _ptr(ee), _ptr(ek), int(cap), ctypes.byref(n)))
    k = min(cap, n.value)
    return ee[:k], ek[:k]


def td_batch_create_ehrenfest(system, model: dict, n: int, velocities=None,
                              options: Optional[TdOptions] = None,
                              rho0: Optional[np.ndarray] = None):
    """td_batch_create_ehrenfest: n members of one system; velocities None or
    [n, n_atoms, 3]."""
    hs = _host_system(system, rho0, None, None)
    keep = _Keep()
    m = _model_struct(model, keep)
    if velocities is not None:
        keep.vel = _f64(velocities).reshape(-1)
        if keep.vel.size != n * 3 * len(system.q0):
            raise ValueError("velocities must have shape [n, n_atoms, 3]")
    else:
        keep.vel = None
    opt = options if options is not None else td_default_options()
    b = ctypes.c_void_p()
    err = ctypes.create_string_buffer(1024)
    st = load().td_batch_create_ehrenfest(int(n), ctypes.byref(hs), ctypes.byref(m),
                                          _ptr(keep.vel), ctypes.byref(opt), ctypes.byref(b),
                                          err, 1024)
    if st != TD_OK:
        raise TdError(st, err.value.decode())
    return b


def td_batch_get_nuclei(b, member: int, n_atoms: int):
    pos = np.empty((n_atoms, 3))
    vel = np.empty((n_atoms, 3))
    _bcheck(b, load().td_batch_get_nuclei(b, int(member), _ptr(pos), _ptr(vel)))
    return pos, vel


def td_batch_get_energy_series(b, member: int, cap: int):
    ee = np.empty(max(cap, 1))
    ek = np.empty(max(cap, 1))
    n = ctypes.c_int32()
    _bcheck(b, load().td_batch_get_energy_series(b, int(member), _ptr(ee), _ptr(ek), int(cap),
                                                 ctypes.byref(n)))
    k = min(cap, n.value)
    return ee[:k], ek[:k]


def _bcheck(b, st):
    if st != TD_OK:
        raise TdError(st, load().td_batch_last_error(b).decode())


def td_batch_create(systems, options: Optional[TdOptions] = None, rho0s=None, flags: int = 0,
                    plus_us=None):
    """td_batch_create over host arrays; rho0s, plus_us: None or lists (entries may be None)."""
    n = len(systems)
    rho0s = rho0s if rho0s is not None else [None] * n
    plus_us = plus_us if plus_us is not None else [None] * n
    hs = [_host_system(s, r, None, u) for s, r, u in zip(systems, rho0s, plus_us)]
    arr = (TdSystem * n)(*hs)
    opt = options if options is not None else td_default_options()
    b = ctypes.c_void_p()
    err = ctypes.create_string_buffer(1024)
    st = load().td_batch_create(n, arr, ctypes.byref(opt), int(flags), ctypes.byref(b), err, 1024)
    if st != TD_OK:
        raise TdError(st, err.value.decode())
    return b


def td_batch_kick(b, e0, directions) -> None:
    e = _f64(e0).reshape(-1)
    d = _f64(directions).reshape(-1)
    if d.size != 3 * e.size:
        raise ValueError("directions must have shape [n, 3]")
    _bcheck(b, load().td_batch_kick(b, _ptr(e), _ptr(d)))


def td_batch_step(b, n: int, field: Optional[np.ndarray] = None) -> None:
    f = None if field is None else _f64(field).reshape(-1)
    if f is not None and f.size != 3 * n:
        raise ValueError("field must have shape [n, 3]")
    _bcheck(b, load().td_batch_step(b, int(n), _ptr(f)))


def td_batch_get_dipole_series(b, member: int, cap: int) -> np.ndarray:
    out = np.empty((max(cap, 1), 3))
    n = ctypes.c_int32()
    _bcheck(b, load().td_batch_get_dipole_series(b, int(member), _ptr(out), int(cap),
                                                 ctypes.byref(n)))
    return out[:min(cap, n.value)]


def td_batch_get_charges(b, member: int, n_atoms: int) -> np.ndarray:
    out = np.empty(n_atoms)
    _bcheck(b, load().td_batch_get_charges(b, int(member), _ptr(out)))
    return out


def td_batch_get_rho(b, member: int, n_orb: int, with_prev: bool = False):
    rho = np.empty((n_orb, n_orb), dtype=np.complex128)
    prev = np.empty((n_orb, n_orb), dtype=np.complex128) if with_prev else None
    step = ctypes.c_int64()
    has_prev = ctypes.c_int32()
    _bcheck(b, load().td_batch_get_rho(b, int(member), rho.ctypes.data_as(_dp),
                                       None if prev is None else prev.ctypes.data_as(_dp),
                                       ctypes.byref(step), ctypes.byref(has_prev)))
    return rho, prev, step.value, bool(has_prev.value)


def td_batch_get_info(b) -> dict:
    info = TdBatchInfo()
    _bcheck(b, load().td_batch_get_info(b, ctypes.byref(info)))
    return info.as_dict()


def td_batch_destroy(b) -> None:
    if b:
        load().td_batch_destroy(b)


def _check(ctx, st):
    if st != TD_OK:
        raise TdError(st, load().td_last_error(ctx).decode())


def td_kick(ctx, e0: float, direction) -> None:
    d = _f64(direction)
    _check(ctx, load().td_kick(ctx, float(e0), _ptr(d)))


def td_step(ctx, n: int, field: Optional[np.ndarray] = None) -> None:
    f = None if field is None else _f64(field).reshape(-1)
    if f is not None and f.size != 3 * n:
        raise ValueError("field must have shape [n, 3]")
    _check(ctx, load().td_step(ctx, int(n), _ptr(f)))


def td_get_charges(ctx, n_atoms: int) -> np.ndarray:
    out = np.empty(n_atoms)
    _check(ctx, load().td_get_charges(ctx, _ptr(out)))
    return out


def td_get_dipole(ctx) -> np.ndarray:
    out = np.empty(3)
    _check(ctx, load().td_get_dipole(ctx, _ptr(out)))
    return out


def td_get_dipole_series(ctx, cap: int) -> np.ndarray:
    out = np.empty((max(cap, 1), 3))
    n = ctypes.c_int32()
    _check(ctx, load().td_get_dipole_series(ctx, _ptr(out), int(cap), ctypes.byref(n)))
    return out[:min(cap, n.value)]


def td_get_energy(ctx, field=None) -> float:
    f = None if field is None else _f64(field)
    e = np.empty(1)
    _check(ctx, load().td_get_energy(ctx, _ptr(f), _ptr(e)))
    return float(e[0])


def td_get_rho(ctx, n_orb: int, with_prev: bool = False):
    rho = np.empty((n_orb, n_orb), dtype=np.complex128)
    prev = np.empty((n_orb, n_orb), dtype=np.complex128) if with_prev else None
    step = ctypes.c_int64()
    has_prev = ctypes.c_int32()
    _check(ctx, load().td_get_rho(ctx, rho.ctypes.data_as(_dp),
                                  None if prev is None else prev.ctypes.data_as(_dp),
                                  ctypes.byref(step), ctypes.byref(has_prev)))
    return rho, prev, step.value, bool(has_prev.value)


def td_set_rho(ctx, rho: np.ndarray, rho_prev: Optional[np.ndarray], step: int) -> None:
    r = np.ascontiguousarray(rho, dtype=np.complex128)
    p = None if rho_prev is None else np.ascontiguousarray(rho_prev, dtype=np.complex128)
    _check(ctx, load().td_set_rho(ctx, r.ctypes.data_as(_dp),
                                  None if p is None else p.ctypes.data_as(_dp), int(step)))


def td_get_info(ctx) -> dict:
    info = TdInfo()
    _check(ctx, load().td_get_info(ctx, ctypes.byref(info)))
    return info.as_dict()


def td_get_kernel_time(ctx, kind: int):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(ctx, load().td_get_kernel_time(ctx, int(kind), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def td_reset_kernel_time(ctx) -> None:
    _check(ctx, load().td_reset_kernel_time(ctx))


def td_get_forces(ctx, n_atoms: int) -> np.ndarray:
    out = np.empty((n_atoms, 3))
    _check(ctx, load().td_get_forces(ctx, _ptr(out)))
    return out


def td_last_error(ctx) -> str:
    return load().td_last_error(ctx).decode()


def td_destroy(ctx) -> None:
    if ctx:
        load().td_destroy(ctx)


def td_util_gemm(A: np.ndarray, B: np.ndarray, precision: int = TD_FP64,
                 n_slices: int = 4) -> np.ndarray:
    A = _f64(A)
    B = _f64(B)
    m, k = A.shape
    k2, n = B.shape
    assert k == k2
    C = np.empty((m, n))
    err = ctypes.create_string_buffer(1024)
    st = load().td_util_gemm(int(precision), int(n_slices), m, n, k, _ptr(A), _ptr(B), _ptr(C),
                             err, 1024)
    if st != TD_OK:
        raise TdError(st, err.value.decode())
    return C


def td_util_gemm_noalloc(m: int, n: int, k: int, A_ptr: int, lda: int, B_ptr: int, ldb: int,
                         C_ptr: int, ldc: int, precision: int = TD_FP64, n_slices: int = 4,
                         stream: int = 0) -> None:
    """C = A B on device pointers (integers, e.g. tensor.data_ptr()) on the
    given stream handle, with no allocation; the caller synchronises."""
    err = ctypes.create_string_buffer(1024)
    st = load().td_util_gemm_noalloc(int(precision), int(n_slices), int(m), int(n), int(k),
                                     ctypes.c_void_p(A_ptr), int(lda), ctypes.c_void_p(B_ptr),
                                     int(ldb), ctypes.c_void_p(C_ptr), int(ldc),
                                     ctypes.c_void_p(stream or None), err, 1024)
    if st != TD_OK:
        raise TdError(st, err.value.decode())


class Propagator:
    """Convenience wrapper owning one context (one trajectory)."""

    def __init__(self, system, dt=0.2, precision=TD_FP64, n_slices=4, rho0=None, occ=None,
                 profile=False,
                 scc_tol=1e-12, scc_maxiter=300, plus_u=None, n_slices_dh=0):
        opt = td_default_options()
        opt.dt = dt
        opt.precision = precision
        opt.n_slices = n_slices
        opt.n_slices_dh = n_slices_dh
        opt.profile = 1 if profile else 0
        opt.scc_tol = scc_tol
        opt.scc_maxiter = scc_maxiter
        self.n_atoms = len(system.q0)
        self.n_orb = int(system.orb_offset[-1])
        self.ctx = td_create(system, opt, rho0=rho0, occ=occ, plus_u=plus_u)

    def kick(self, e0, direction):
        td_kick(self.ctx, e0, direction)

    def step(self, n, field=None):
        td_step(self.ctx, n, field)
        return td_get_dipole_series(self.ctx, n)

    def dipole(self):
        return td_get_dipole(self.ctx)

    def charges(self):
        return td_get_charges(self.ctx, self.n_atoms)

    def energy(self, field=None):
        return td_get_energy(self.ctx, field)

    def rho(self, with_prev=False):
        return td_get_rho(self.ctx, self.n_orb, with_prev)

    def set_rho(self, rho, rho_prev=None, step=0):
        td_set_rho(self.ctx, rho, rho_prev, step)

    def info(self):
        return td_get_info(self.ctx)

    def kernel_time(self, kind):
        return td_get_kernel_time(self.ctx, kind)

    def reset_kernel_time(self):
        td_reset_kernel_time(self.ctx)

    def close(self):
        if self.ctx:
            td_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def td_spectrum(mu, e0, dt, omega, ref=None, tau=0.0):
    """td_spectrum: mu [n_series, n_t] (or [n_t]), e0 scalar or [n_series];
    returns (alpha [n_series, n_omega] complex, sigma [n_series, n_omega])."""
    m = np.atleast_2d(_f64(mu))
    r = None if ref is None else np.atleast_2d(_f64(ref))
    if r is not None and r.shape != m.shape:
        raise ValueError("ref must have the shape of mu")
    J, T = m.shape
    e = _f64(np.broadcast_to(np.asarray(e0, dtype=np.float64), (J,)))
    w = _f64(omega).reshape(-1)
    are, aim, sig = (np.empty((J, w.size)) for _ in range(3))
    err = ctypes.create_string_buffer(1024)
    st = load().td_spectrum(J, T, _ptr(m), _ptr(r), _ptr(e), float(dt), float(tau), w.size,
                            _ptr(w), _ptr(are), _ptr(aim), _ptr(sig), err, 1024)
    if st != TD_OK:
        raise TdError(st, err.value.decode())
    return are + 1j * aim, sig


def td_transient_absorption(mu, ref, e0, dt, omega, tau=0.0, ref_delay=-1, delay_step=0.0,
                            filter_width=0.0):
    """td_transient_absorption: mu, ref [n_delay, n_avg, n_t]; e0 scalar or
    [n_delay, n_avg]; returns [n_delay, n_omega]."""
    m = _f64(mu)
    r = _f64(ref)
    if m.ndim != 3 or r.shape != m.shape:
        raise ValueError("mu and ref must be [n_delay, n_avg, n_t]")
    D, A, T = m.shape
    e = _f64(np.broadcast_to(np.asarray(e0, dtype=np.float64), (D, A)))
    w = _f64(omega).reshape(-1)
    out = np.empty((D, w.size))
    err = ctypes.create_string_buffer(1024)
    st = load().td_transient_absorption(D, A, T, _ptr(m), _ptr(r), _ptr(e), float(dt),
                                        float(tau), w.size, _ptr(w), int(ref_delay),
                                        float(delay_step), float(filter_width), _ptr(out), err,
                                        1024)
    if st != TD_OK:
        raise TdError(st, err.value.decode())
    return out


class Batch:
    """Convenience wrapper owning one batch of trajectories."""

    def __init__(self, systems, dt=0.2, rho0s=None, flags=0, scc_tol=1e-12, scc_maxiter=300):
        opt = td_default_options()
        opt.dt = dt
        opt.scc_tol = scc_tol
        opt.scc_maxiter = scc_maxiter
        self.n_atoms = [len(s.q0) for s in systems]
        self.n_orb = [int(s.orb_offset[-1]) for s in systems]
        self.b = td_batch_create(systems, opt, rho0s, flags)

    def kick(self, e0, directions):
        td_batch_kick(self.b, e0, directions)

    def step(self, n, field=None):
        td_batch_step(self.b, n, field)

    def dipoles(self, member, n):
        return td_batch_get_dipole_series(self.b, member, n)

    def charges(self, member):
        return td_batch_get_charges(self.b, member, self.n_atoms[member])

    def rho(self, member, with_prev=False):
        return td_batch_get_rho(self.b, member, self.n_orb[member], with_prev)

    def info(self):
        return td_batch_get_info(self.b)

    def close(self):
        if self.b:
            td_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class EhrenfestBatch(Batch):
    """Convenience wrapper owning a batch of moving-nuclei trajectories of one system."""

    def __init__(self, system, model, n, velocities=None, dt=0.2, rho0=None, scc_tol=1e-12,
                 scc_maxiter=300, precision=TD_FP64, n_slices=4):
        opt = td_default_options()
        opt.dt = dt
        opt.scc_tol = scc_tol
        opt.scc_maxiter = scc_maxiter
        opt.precision = precision
        opt.n_slices = n_slices
        self.n_atoms = [len(system.q0)] * n
        self.n_orb = [int(system.orb_offset[-1])] * n
        self.b = td_batch_create_ehrenfest(system, model, n, velocities, opt, rho0)

    def nuclei(self, member):
        return td_batch_get_nuclei(self.b, member, self.n_atoms[member])

    def energy_series(self, member, n):
        return td_batch_get_energy_series(self.b, member, n)


class Ehrenfest(Propagator):
    """One trajectory with moving nuclei (td_create_ehrenfest)."""

    def __init__(self, system, model, velocities=None, dt=0.2, rho0=None, scc_tol=1e-12,
                 scc_maxiter=300, precision=TD_FP64, n_slices=4):
        opt = td_default_options()
        opt.dt = dt
        opt.scc_tol = scc_tol
        opt.scc_maxiter = scc_maxiter
        opt.precision = precision
        opt.n_slices = n_slices
        self.n_atoms = len(system.q0)
        self.n_orb = int(system.orb_offset[-1])
        self.ctx = td_create_ehrenfest(system, model, velocities, opt, rho0=rho0)

    def forces(self):
        return td_get_forces(self.ctx, self.n_atoms)

    def nuclei(self):
        return td_get_nuclei(self.ctx, self.n_atoms)

    def energy_series(self, n):
        return td_get_energy_series(self.ctx, n)

