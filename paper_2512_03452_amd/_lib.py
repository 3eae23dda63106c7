"""ctypes declarations of the C ABI in ``include/sipf.h`` (argument marshalling only).

The library ``libsipf.so`` is built in-tree by ``paper_2512_03452_amd/build.py``.
There is no fallback: if the library is missing, loading raises.
"""

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsipf.so")

SIPF_OK = 0
SIPF_EINVAL = -1
SIPF_ENOMEM = -2
SIPF_EDEVICE = -3
SIPF_ENUMERIC = -4
SIPF_ESTATE = -5
SIPF_EIO = -6
CODE_NAMES = {SIPF_EINVAL: "SIPF_EINVAL", SIPF_ENOMEM: "SIPF_ENOMEM", SIPF_EDEVICE: "SIPF_EDEVICE",
              SIPF_ENUMERIC: "SIPF_ENUMERIC", SIPF_ESTATE: "SIPF_ESTATE", SIPF_EIO: "SIPF_EIO"}

SIPF_STRANG = 0
SIPF_EM = 1
SIPF_FP32 = 0
SIPF_FP64 = 1
SIPF_PROP_IMPLICIT = 0
SIPF_PROP_EXP = 1
SIPF_METHOD_PIC = 0
SIPF_METHOD_DIRECT = 1
SIPF_PASS_DEFAULT = 0
SIPF_PASS_SORTED = 1
SIPF_PASS_TWO_PHASE = 2
SIPF_FIELD_RHO = 0
SIPF_FIELD_ALPHA = 1
SIPF_FIELD_GRAD = 2
PHASES = ("sort", "particles", "fwd_planes", "xpencils", "inv_planes")


class SipfParams(ctypes.Structure):
    """Mirror of ``sipf_params``."""
    _fields_ = [
        ("L", ctypes.c_double), ("chi", ctypes.c_double), ("mu", ctypes.c_double),
        ("eps", ctypes.c_double), ("k", ctypes.c_double), ("M0", ctypes.c_double),
        ("dt", ctypes.c_double), ("H0", ctypes.c_double),
        ("H", ctypes.c_int32), ("p2g_order", ctypes.c_int32), ("g2p_order", ctypes.c_int32),
        ("scheme", ctypes.c_int32), ("precision", ctypes.c_int32), ("tile", ctypes.c_int32),
        ("resort_every", ctypes.c_int32), ("chunk", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("instance", ctypes.c_uint32), ("dim", ctypes.c_uint32),
        ("propagator", ctypes.c_int32), ("method", ctypes.c_int32), ("positivity", ctypes.c_int32),
        ("particle_pass", ctypes.c_int32),
    ]


class SipfDiag(ctypes.Structure):
    """Mirror of ``sipf_diag``."""
    _fields_ = [
        ("step", ctypes.c_int64), ("mass", ctypes.c_double), ("rho_max", ctypes.c_double),
        ("hf_share", ctypes.c_double), ("c_integral", ctypes.c_double), ("r_num", ctypes.c_double),
        ("m2", ctypes.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class SipfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{CODE_NAMES.get(code, code)}: {msg}")
        self.code = code


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_dp = ctypes.POINTER(ctypes.c_double)
_pp = ctypes.POINTER(SipfParams)

# name -> argtypes (all return int unless listed in _RESTYPES)
SIGNATURES = {
    "sipf_params_default": [_pp],
    "sipf_init": [_pp, _i64, _vp, ctypes.c_int, _vp, ctypes.c_int, _vp, ctypes.POINTER(_vp)],
    "sipf_step": [_vp],
    "sipf_run": [_vp, _i64],
    "sipf_prepare_run": [_vp, _i64],
    "sipf_sync": [_vp],
    "sipf_get_step": [_vp, ctypes.POINTER(_i64)],
    "sipf_get_positions": [_vp, _vp, ctypes.c_int],
    "sipf_get_field": [_vp, ctypes.c_int, _vp, ctypes.c_int],
    "sipf_diagnostics": [_vp, ctypes.POINTER(SipfDiag)],
    "sipf_batch_diagnostics": [_vp, ctypes.POINTER(SipfDiag)],
    "sipf_adjoint": [_vp, _i64, _i32, _vp, _dp, _dp, _dp, _vp],
    "sipf_positivity_stats": [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i32)],
    "sipf_profile": [_vp, ctypes.c_int],
    "sipf_profile_read": [_vp, _dp, ctypes.POINTER(_i64)],
    "sipf_save": [_vp, ctypes.c_char_p],
    "sipf_load": [ctypes.c_char_p, _vp, ctypes.POINTER(_vp)],
    "sipf_destroy": [_vp],
    "sipf_last_error": [],
    "sipf_use_graphs": [_vp, ctypes.c_int],
    "sipf_get_params": [_vp, _pp, ctypes.POINTER(_i64)],
    "sipf_autotune": [_pp, _i64, _vp, ctypes.c_int, _i32, _vp, _pp, _dp],
    "sipf_batch_init": [_i32, _pp, ctypes.POINTER(_i64), ctypes.POINTER(_vp), ctypes.c_int, _vp,
                        ctypes.POINTER(_vp)],
    "sipf_batch_run": [_vp, _i64],
    "sipf_batch_prepare_run": [_vp, _i64],
    "sipf_batch_use_graphs": [_vp, ctypes.c_int],
    "sipf_batch_sync": [_vp],
    "sipf_batch_get_step": [_vp, _i32, ctypes.POINTER(_i64)],
    "sipf_batch_get_positions": [_vp, _i32, _vp, ctypes.c_int],
    "sipf_batch_get_field": [_vp, _i32, ctypes.c_int, _vp, ctypes.c_int],
    "sipf_batch_profile": [_vp, ctypes.c_int],
    "sipf_batch_profile_read": [_vp, _dp, ctypes.POINTER(_i64)],
    "sipf_batch_destroy": [_vp],
    "sipf_dbg_philox": [_u64, _i64, _vp, _vp, _vp, ctypes.c_int, _vp],
    "sipf_dbg_cells": [_pp, _i64, _vp, _vp, _vp],
    "sipf_dbg_deposit": [_pp, _i64, _vp, _vp, _vp],
    "sipf_deposit_noalloc": [_pp, _i64, _vp, _vp, _vp],
    "sipf_release_cached_memory": [],
}
_RESTYPES = {"sipf_last_error": ctypes.c_char_p}

_lib = None


def load():
    """Load libsipf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2512_03452_amd/build.py "
                          "(or __graft_entry__.build()); there is no fallback implementation")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = _RESTYPES.get(name, ctypes.c_int)
    _lib = lib
    return lib


def check(rc):
    if rc != SIPF_OK:
        msg = load().sipf_last_error().decode(errors="replace")
        raise SipfError(rc, msg)
    return rc


def default_params(**overrides):
    p = SipfParams()
    check(load().sipf_params_default(ctypes.byref(p)))
    for k, v in overrides.items():
        if k == "scheme" and isinstance(v, str):
            v = {"strang": SIPF_STRANG, "em": SIPF_EM}[v]
        if k == "precision" and isinstance(v, str):
            v = {"fp32": SIPF_FP32, "fp64": SIPF_FP64}[v]
        if k == "propagator" and isinstance(v, str):
            v = {"implicit": SIPF_PROP_IMPLICIT, "exp": SIPF_PROP_EXP}[v]
        if k == "method" and isinstance(v, str):
            v = {"pic": SIPF_METHOD_PIC, "direct": SIPF_METHOD_DIRECT}[v]
        if k == "particle_pass" and isinstance(v, str):
            v = {"default": SIPF_PASS_DEFAULT, "sorted": SIPF_PASS_SORTED, "two_phase": SIPF_PASS_TWO_PHASE}[v]
        if not hasattr(p, k):
            raise KeyError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p
