"""ctypes binding of librad.so (the C ABI declared in include/rad.h).

Argument marshalling only.  The library must have been built
(``python -m paper_2511_04277_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import pathlib

_PKG = pathlib.Path(__file__).resolve().parent
LIB_PATH = pathlib.Path(os.environ.get("RAD_LIBRARY", _PKG / "librad.so"))

RAD_OK = 0
RAD_WNOTCONVERGED = 1
RAD_EINVAL = -1
RAD_ENONFINITE = -2
RAD_EZEROROW = -3
RAD_ESINGULAR = -4
RAD_EHIP = -5
RAD_EWORKSPACE = -6

RAD_KAPPA_FRACVAR = 0
RAD_KAPPA_HALF = 1
RAD_PREC_FP64 = 0
RAD_PREC_FP32_IR = 1
RAD_PREC_FP64_I8 = 2
RAD_ENFORCE_NOALLOC_BYTES = 36 << 20
RAD_LSQ_NNR = 1
RAD_LSQ_SPVA = 2


class RadStats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("ir_steps", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("device_status", ctypes.c_int32),
        ("closure_defect", ctypes.c_double),
        ("recip_err", ctypes.c_double),
        ("ir_correction", ctypes.c_double),
        ("ir_residual", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class RadKernelProfile(ctypes.Structure):
    _fields_ = [
        ("launches", ctypes.c_int64),
        ("total_ms", ctypes.c_double),
        ("flops", ctypes.c_double),
        ("bytes", ctypes.c_double),
    ]


class RadInstance(ctypes.Structure):
    """One model of a batch (struct rad_instance); pointers are device addresses."""
    _fields_ = [
        ("F", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("ldf", ctypes.c_int64),
        ("area", ctypes.c_void_p),
        ("n_rays", ctypes.c_void_p),
        ("bands", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("eps", ctypes.c_void_p * 2),
        ("rho", ctypes.c_void_p * 2),
        ("B", ctypes.c_void_p * 2),
        ("ldb", ctypes.c_int64 * 2),
    ]


class RadTuning(ctypes.Structure):
    _fields_ = [
        ("small_tile_below_f64", ctypes.c_int32),
        ("small_tile_below_f32", ctypes.c_int32),
        ("lookahead", ctypes.c_int32),
        ("side_chunk_tiles", ctypes.c_int32),
    ]


PROFILE_KINDS = ["gemm_f64", "gemm_f32", "enforce_sweep", "diag_inverse", "aggregate", "gemm_f64_t",
                 "gemm_f32_t", "gemm_i8x", "i8x_split", "ahf"]


class RadError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed with status {code}: {msg}")
        self.code = code


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_D = ctypes.c_double
_SZ = ctypes.c_size_t
_STATS = ctypes.POINTER(RadStats)

# name -> (restype, argtypes); mirrors include/rad.h
SIGNATURES = {
    "rad_status_string": (ctypes.c_char_p, [_I32]),
    "rad_last_error": (ctypes.c_char_p, []),
    "rad_version": (_I32, []),
    "rad_enforce_workspace_bytes": (_SZ, [_I64]),
    "rad_enforce_vf": (_I32, [_P, _I64, _I64, _P, _P, _I32, _D, _I32, _P, _SZ, _STATS, _P]),
    "rad_enforce_vf_noalloc": (_I32, [_P, _I64, _I64, _P, _P, _I32, _D, _I32, _STATS, _P]),
    "rad_gebhart_factor_bytes": (_SZ, [_I64, _I32]),
    "rad_gebhart_workspace_bytes": (_SZ, [_I64, _I32]),
    "rad_gebhart_ref": (_I32, [_P, _I64, _I64, _P, _P, _P, _I64, _I32, _D, _I32, _P, _SZ, _P, _SZ, _STATS, _P]),
    "rad_ref_check_workspace_bytes": (_SZ, [_I64]),
    "rad_ref_check": (_I32, [_P, _I64, _I64, _P, _P, _P, _P, _SZ, _P]),
    "rad_adjoint_workspace_bytes": (_SZ, [_I64, _I32]),
    "rad_gebhart_ref_adjoint": (_I32, [_P, _SZ, _I32, _P, _I64, _I64, _P, _P, _I64, _P, _I64, _P, _P, _P,
                                      _I64, _D, _I32, _P, _SZ, _STATS, _P]),
    "rad_aggregate_workspace_bytes": (_SZ, [_I64, _I64]),
    "rad_enforce_lsq_workspace_bytes": (_SZ, [_I64, _I32]),
    "rad_enforce_lsq": (_I32, [_P, _I64, _I64, _P, _P, _I64, _I32, _I32, _I32, _P, _SZ, _P, _SZ, _STATS, _P]),
    "rad_view_fractions_workspace_bytes": (_SZ, [_I64, _I64]),
    "rad_view_fractions": (_I32, [_P, _I64, _I64, _P, _I64, _P, _I64, _P, _SZ, _STATS, _P]),
    "rad_node_emissivity_workspace_bytes": (_SZ, [_I64, _I64]),
    "rad_node_emissivity": (_I32, [_P, _I64, _I64, _P, _P, _P, _I64, _P, _I64, _P, _SZ, _STATS, _P]),
    "rad_steady_temperature_workspace_bytes": (_SZ, [_I64, _I32]),
    "rad_steady_temperature": (_I32, [_P, _I64, _I64, _P, _P, _I64, _I64, _P, _D, _D, _P, _I64, _I32, _P, _SZ,
                                      _P, _SZ, _STATS, _P]),
    "rad_absorbed_flux_workspace_bytes": (_SZ, [_I64, _I64]),
    "rad_absorbed_flux": (_I32, [_P, _I64, _I64, _P, _P, _P, _P, _I64, _I64, _P, _I64, _P, _SZ, _P]),
    "rad_aggregate_nodes": (_I32, [_P, _I64, _I64, _P, _P, _I64, _P, _I64, _P, _P, _SZ, _STATS, _P]),
    "rad_batch_plan_create": (_I32, [ctypes.POINTER(RadInstance), _I32, _I32, _I32, ctypes.POINTER(_P),
                                     ctypes.POINTER(_SZ)]),
    "rad_batch_prepare": (_I32, [_P, _P, _SZ, _P]),
    "rad_batch_run": (_I32, [_P, _P, _D, _I32, _I32, _P]),
    "rad_batch_stats": (_I32, [_P, _P, _STATS, _P]),
    "rad_batch_plan_destroy": (None, [_P]),
    "rad_tuning_get": (_I32, [ctypes.POINTER(RadTuning)]),
    "rad_tuning_set": (_I32, [ctypes.POINTER(RadTuning)]),
    "rad_profile_enable": (_I32, [_I32]),
    "rad_profile_kinds": (_I32, [ctypes.c_uint32]),
    "rad_profile_read": (_I32, [ctypes.POINTER(RadKernelProfile), _I32]),
}

_lib = None
TUNING_PATH = _PKG / "tuning.json"


def apply_tuning(chosen: dict) -> None:
    """Set the library's runtime knobs (rad_tuning_set) from a dict with keys
    small_tile_below_f64, small_tile_below_f32, lookahead and optionally
    side_chunk_tiles (0 when absent)."""
    t = RadTuning(int(chosen["small_tile_below_f64"]), int(chosen["small_tile_below_f32"]),
                  int(chosen["lookahead"]), int(chosen.get("side_chunk_tiles", 0)))
    check(lib().rad_tuning_set(ctypes.byref(t)), "rad_tuning_set")


def tuning() -> dict:
    t = RadTuning()
    check(lib().rad_tuning_get(ctypes.byref(t)), "rad_tuning_get")
    return {name: getattr(t, name) for name, _ in t._fields_}


def lib() -> ctypes.CDLL:
    """Load librad.so once; raise if it is missing (no fallback path exists).
    The autotuner's table (tuning.json beside this file), if present, is
    applied on load."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise ImportError(f"{LIB_PATH} not found: build it with `python -m paper_2511_04277_amd.build`")
        l = ctypes.CDLL(str(LIB_PATH))
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(l, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = l
        if TUNING_PATH.exists() and os.environ.get("RAD_NO_TUNING") != "1":
            import json
            apply_tuning(json.loads(TUNING_PATH.read_text())["chosen"])
    return _lib


def check(code: int, where: str) -> int:
    if code < 0:
        msg = lib().rad_last_error().decode() or lib().rad_status_string(code).decode()
        raise RadError(code, where, msg)
    return code
