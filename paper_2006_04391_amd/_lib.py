"""ctypes loader and C struct mirrors for libautomat.so.

Argument marshalling only: every step of the computation runs in the HIP
library. If the library is missing or cannot be loaded, every call raises;
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libautomat.so")

MAX_PHASES = 16
NPAR = 7
GRAD_KEYS = ("E", "nu", "H", "sigma_y", "sigma0", "eps0", "n")

OK, EINVAL, EHIP, ENOMEM, EBUDGET = 0, -1, -2, -3, -4
SIGMA_CRITERION = 1
HAND_PARTIALS = 2


class Phase(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("E", ctypes.c_double), ("nu", ctypes.c_double), ("H", ctypes.c_double),
                ("sigma_y", ctypes.c_double), ("sigma0", ctypes.c_double),
                ("eps0", ctypes.c_double), ("n", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("n_phases", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("phase", Phase * MAX_PHASES)]


class MsOptions(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("fixed_iter", ctypes.c_int32), ("lambda0", ctypes.c_double),
                ("mu0", ctypes.c_double), ("newton_tol", ctypes.c_double),
                ("newton_max_iter", ctypes.c_int32), ("ref_update", ctypes.c_int32),
                ("warm_start", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("phase", ctypes.POINTER(ctypes.c_uint8)),
                ("params", Params), ("h", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("E_final", ctypes.c_double * 6), ("noise_std", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("a_init", ctypes.POINTER(ctypes.c_double)),
                ("sigma_host", ctypes.POINTER(ctypes.c_double)),
                ("a_host", ctypes.POINTER(ctypes.c_double)), ("t_arrival", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("steps_done", ctypes.c_int32), ("n", ctypes.c_int64),
                ("nonconverged", ctypes.c_int64), ("t_arrival", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("clock_s", ctypes.c_double), ("pending", ctypes.c_int64),
                ("active", ctypes.c_int64), ("used_bytes", ctypes.c_int64),
                ("launches", ctypes.c_int64), ("updates", ctypes.c_int64),
                ("busy_s", ctypes.c_double)]


class AutomatError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed: {msg} ({code})")
        self.code = code


# Exported symbols and their signatures; the tests check that the library
# exports each name the header declares.
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_dbl = ctypes.c_double
SIGNATURES = {
    "automat_evaluate": (_i32, [_i64, _vp, _vp, _vp, _vp, _dbl, _dbl, _i32, _vp, _vp, _vp, _vp]),
    "automat_evaluate_ex": (_i32, [_i64, _vp, _vp, _vp, _vp, _dbl, _dbl, _i32, _vp, _vp, _vp,
                                   _vp, _vp, ctypes.c_uint32, _vp]),
    "automat_evaluate_backward": (_i32, [_i64, _vp, _vp, _vp, _vp, _vp, _dbl, _vp, _vp, _vp, _vp,
                                         _vp, _vp]),
    "automat_ms_create": (_i32, [_i32, _i32, _i32, _vp, _vp, _vp]),
    "automat_ms_step": (_i32, [_vp, _vp, _vp, _dbl, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "automat_ms_step_noalloc": (_i32, [_vp, _vp, _vp, _dbl, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "automat_ms_newton_failures": (_i32, [_vp, _vp]),
    "automat_ms_step_mixed": (_i32, [_vp, _vp, _vp, _vp, ctypes.c_uint32, _dbl, _vp, _vp, _vp,
                                      _vp, _vp, _vp, _vp, _vp]),
    "automat_ms_set_macro": (_i32, [_vp, _vp]),
    "automat_ms_reference": (_i32, [_vp, _vp, _vp]),
    "automat_ms_adjoint_step": (_i32, [_vp, _vp, _dbl, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                        _vp, _vp, _vp, _vp]),
    "automat_ms_destroy": (_i32, [_vp]),
    "automat_server_create": (_i32, [ctypes.c_size_t, _i64, _i32, _vp]),
    "automat_server_submit": (_i32, [_vp, _vp, _vp]),
    "automat_server_poll": (_i32, [_vp, _vp, _i32, _vp]),
    "automat_server_stats": (_i32, [_vp, _vp]),
    "automat_server_destroy": (_i32, [_vp]),
    "automat_evaluate_rk23": (_i32, [_i64, _vp, _vp, _vp, _vp, _vp, _dbl, _dbl, _dbl, _i32, _vp,
                                      _vp, _vp, _vp, _vp]),
    "automat_evaluate_rk12": (_i32, [_i64, _vp, _vp, _vp, _vp, _vp, _dbl, _dbl, _dbl, _i32, _vp,
                                      _vp, _vp, _vp, _vp]),
    "automat_evaluate_rk23_ex": (_i32, [_i64, _vp, _vp, _vp, _vp, _vp, _dbl, _dbl, _dbl, _i32,
                                         _vp, _vp, _vp, _vp, _vp, _vp]),
    "automat_evaluate_rk12_ex": (_i32, [_i64, _vp, _vp, _vp, _vp, _vp, _dbl, _dbl, _dbl, _i32,
                                         _vp, _vp, _vp, _vp, _vp, _vp]),
    "automat_evaluate_f32": (_i32, [_i64, _vp, _vp, _vp, _vp, _dbl, _dbl, _i32, _vp, _vp, _vp,
                                     _vp, _vp, _vp]),
    "automat_evaluate_conventional": (_i32, [_i64, _vp, _vp, _vp, _vp, _dbl, _dbl, _i32, _vp, _vp,
                                              _vp, _vp, _vp]),
    "automat_evaluate_conventional_ex": (_i32, [_i64, _vp, _vp, _vp, _vp, _dbl, _dbl, _i32, _vp,
                                                 _vp, _vp, _vp, _vp, _vp]),
    "automat_strerror": (ctypes.c_char_p, [_i32]),
    "automat_version": (ctypes.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the library once; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"libautomat.so not found at {path}: build it with "
            "`python -m paper_2006_04391_amd.build` (there is no CPU fallback)")
    # The library works on PyTorch's device memory and streams, so it must
    # bind to the HIP runtime PyTorch loads; opened first, it would pull in
    # another copy of the runtime, which PyTorch would then share.
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        if not hasattr(L, name):
            continue
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(fn: str, code: int):
    if code != OK:
        msg = load().automat_strerror(code).decode()
        raise AutomatError(fn, code, msg)


def make_params(phases) -> Params:
    """Pack a list of phase dicts (keys kind, E, nu, H, sigma_y, sigma0,
    eps0, n) into the C struct."""
    if len(phases) < 1 or len(phases) > MAX_PHASES:
        raise ValueError(f"between 1 and {MAX_PHASES} phases required")
    p = Params()
    p.n_phases = len(phases)
    for k, ph in enumerate(phases):
        q = p.phase[k]
        q.kind = int(ph["kind"])
        for key in ("E", "nu", "H", "sigma_y", "sigma0", "eps0", "n"):
            setattr(q, key, float(ph[key]))
    return p
