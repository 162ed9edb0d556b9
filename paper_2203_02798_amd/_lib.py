"""ctypes loader for libpsk.so (the C ABI declared in include/psk.h).

Argument marshalling only: no arithmetic of the method happens in Python.
Importing this module does not load the library; ``lib()`` does, and raises
if the in-tree build is missing (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsk.so")

PSK_OK = 0
STATUS_NAMES = {
    0: "PSK_OK", -1: "PSK_EINVAL", -2: "PSK_EDTYPE", -3: "PSK_ENOMEM",
    -4: "PSK_EDEVICE", -5: "PSK_ENOCONV", -6: "PSK_ERANK", -7: "PSK_EUNSUPPORTED",
    -8: "PSK_ENONFINITE", 1: "PSK_PENDING",
}
PSK_PENDING = 1
PSK_REQ_LSQ, PSK_REQ_LEVERAGE = 0, 1
PSK_DENSE, PSK_CSR = 0, 1
PSK_MAT_CHECKED = 1
PSK_F64, PSK_F32 = 0, 1
PSK_PROBE_BLOCKS = 4096
PSK_NOALLOC_SCRATCH_BYTES = 64 << 20
PSK_PREC_F64, PSK_PREC_BF16, PSK_PREC_FP8 = 0, 1, 2
(PSK_OP_SKETCH_CS, PSK_OP_SKETCH_GCS, PSK_OP_GRAM, PSK_OP_ROWNORMS, PSK_OP_QR,
 PSK_OP_LSQ, PSK_OP_SKETCH_G, PSK_OP_LEVERAGE_GRAM, PSK_OP_LSQ_GRAM,
 PSK_OP_LSQ_SKETCH, PSK_OP_LEVERAGE_SKETCH, PSK_OP_CSS, PSK_OP_LEVERAGE_CSS,
 PSK_OP_DELTA, PSK_OP_CHECK, PSK_OP_SKETCH_OSNAP) = range(16)
PSK_EINVAL, PSK_ERANK, PSK_ENONFINITE = -1, -6, -8

EXPORTED = ["psk_version", "psk_last_error", "psk_workspace_size", "cs_hash",
            "sketch_cs", "sketch_gcs", "sketch_g", "gram", "rownorms_sq", "sketch_qr",
            "lsq_solve", "leverage_sketch", "css_select", "leverage_css", "leverage_gram",
            "lsq_gram", "lsq_sketch_solve", "sketch_delta", "sketch_qr_noalloc", "psk_check", "osnap_hash", "sketch_osnap",
            "psk_probe_copy", "psk_probe_mfma_f64", "psk_probe_mfma_lowp",
            "psk_probe_valu_f32",
            "psk_timing_enable", "psk_timing_only", "psk_timing_reset",
            "psk_timing_collect", "psk_timing_names", "psk_server_create",
            "psk_server_submit", "psk_server_wait", "psk_server_poll",
            "psk_server_stats", "psk_server_destroy"]


class PskMat(ctypes.Structure):
    _fields_ = [
        ("format", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("n", ctypes.c_int64),
        ("d", ctypes.c_int64),
        ("ld", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("values", ctypes.c_void_p),
        ("indptr", ctypes.c_void_p),
        ("indices", ctypes.c_void_p),
        ("flags", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


class PskLsqOpts(ctypes.Structure):
    _fields_ = [
        ("Rinv", ctypes.c_void_p),
        ("m", ctypes.c_int64),
        ("r", ctypes.c_int64),
        ("seed", ctypes.c_uint64),
        ("prec", ctypes.c_int32),
        ("max_iter", ctypes.c_int32),
        ("refine", ctypes.c_int32),
        ("check_every", ctypes.c_int32),
        ("atol", ctypes.c_double),
        ("btol", ctypes.c_double),
        ("escalate_cond", ctypes.c_double),
        ("want_delta", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class PskLsqInfo(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("resid", ctypes.c_double),
        ("ne_resid", ctypes.c_double),
        ("prec_used", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("delta_est", ctypes.c_double),
    ]


class PskServerOpts(ctypes.Structure):
    _fields_ = [
        ("pool", ctypes.c_void_p),
        ("pool_bytes", ctypes.c_size_t),
        ("slots", ctypes.c_int32),
    ]


class PskRequest(ctypes.Structure):
    _fields_ = [
        ("op", ctypes.c_int32),
        ("A", PskMat),
        ("b", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("opts", PskLsqOpts),
    ]


class PskResult(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("iters", ctypes.c_int32),
        ("resid", ctypes.c_double),
        ("ne_resid", ctypes.c_double),
        ("t_submit", ctypes.c_double),
        ("t_start", ctypes.c_double),
        ("t_end", ctypes.c_double),
        ("prec_used", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("delta_est", ctypes.c_double),
    ]


class PskServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64),
        ("completed", ctypes.c_int64),
        ("queued", ctypes.c_int64),
        ("inflight", ctypes.c_int32),
        ("inflight_peak", ctypes.c_int32),
        ("pool_bytes", ctypes.c_size_t),
        ("pool_used", ctypes.c_size_t),
        ("pool_peak", ctypes.c_size_t),
    ]


class PskError(RuntimeError):
    def __init__(self, status, where, message):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")


_LIB = None

_vp, _i64, _u64, _i32, _dbl = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64,
                               ctypes.c_int32, ctypes.c_double)
_PM = ctypes.POINTER(PskMat)

_SIGS = {
    "psk_version": ([], ctypes.c_char_p),
    "psk_last_error": ([], ctypes.c_char_p),
    "psk_workspace_size": ([ctypes.c_int, _PM, _i64, _i64, _i64, ctypes.c_int,
                            ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "cs_hash": ([_i64, _i64, _i64, _u64, _vp, _vp, _vp], ctypes.c_int),
    "sketch_cs": ([_PM, _i64, _u64, _vp, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    "sketch_gcs": ([_PM, _i64, _i64, _u64, ctypes.c_int, _vp, _vp, ctypes.c_size_t, _vp],
                   ctypes.c_int),
    "sketch_g": ([_PM, _i64, _u64, ctypes.c_int, _vp, _vp, ctypes.c_size_t, _vp],
                 ctypes.c_int),
    "gram": ([_dbl, _PM, _dbl, _vp, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    "rownorms_sq": ([_dbl, _PM, _vp, _i64, _dbl, _vp, _vp, ctypes.c_size_t, _vp],
                    ctypes.c_int),
    "sketch_qr": ([_vp, _i64, _i64, _vp, _vp, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    "sketch_qr_noalloc": ([_vp, _i64, _i64, _vp, _vp, _vp], ctypes.c_int),
    "lsq_solve": ([_PM, _vp, _vp, ctypes.POINTER(PskLsqOpts), ctypes.POINTER(PskLsqInfo),
                   _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    "leverage_sketch": ([_PM, _i64, _i64, _i64, _u64, ctypes.c_int, _vp, _vp, ctypes.c_size_t,
                         _vp], ctypes.c_int),
    "css_select": ([_PM, _i64, _i64, _i64, _u64, ctypes.c_int, _vp, _vp, ctypes.c_size_t, _vp],
                   ctypes.c_int),
    "leverage_css": ([_PM, _i64, _i64, _i64, _u64, ctypes.c_int, _vp, _vp, _vp, ctypes.c_size_t,
                      _vp], ctypes.c_int),
    "leverage_gram": ([_PM, _vp, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    "lsq_gram": ([_PM, _vp, _vp, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    "lsq_sketch_solve": ([_PM, _vp, _vp, _i64, _i64, _u64, ctypes.c_int, _vp, ctypes.c_size_t,
                          _vp], ctypes.c_int),
    "sketch_delta": ([_vp, _vp, _i64, _i64, _vp, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    "psk_check": ([_PM, ctypes.c_int, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    "osnap_hash": ([_i64, _i64, _i64, _i64, _u64, _vp, _vp, _vp], ctypes.c_int),
    "sketch_osnap": ([_PM, _i64, _i64, _i64, _u64, ctypes.c_int, _vp, _vp, ctypes.c_size_t,
                      _vp], ctypes.c_int),
    "psk_probe_copy": ([_vp, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    "psk_probe_mfma_f64": ([_i64, _vp, _vp], ctypes.c_int),
    "psk_probe_mfma_lowp": ([ctypes.c_int, _i64, _vp, _vp], ctypes.c_int),
    "psk_probe_valu_f32": ([_i64, _vp, _vp], ctypes.c_int),
    "psk_timing_enable": ([ctypes.c_int], ctypes.c_int),
    "psk_timing_only": ([ctypes.c_char_p], ctypes.c_int),
    "psk_timing_reset": ([], ctypes.c_int),
    "psk_timing_collect": ([ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                            ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "psk_timing_names": ([], ctypes.c_char_p),
    "psk_server_create": ([ctypes.POINTER(PskServerOpts), ctypes.POINTER(ctypes.c_void_p)],
                          ctypes.c_int),
    "psk_server_submit": ([_vp, ctypes.POINTER(PskRequest), ctypes.POINTER(ctypes.c_int64)],
                          ctypes.c_int),
    "psk_server_wait": ([_vp, _i64, ctypes.POINTER(PskResult)], ctypes.c_int),
    "psk_server_poll": ([_vp, _i64, ctypes.POINTER(PskResult)], ctypes.c_int),
    "psk_server_stats": ([_vp, ctypes.POINTER(PskServerStats)], ctypes.c_int),
    "psk_server_destroy": ([_vp], ctypes.c_int),
}


def lib():
    """The loaded libpsk.so (loaded once).  Raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"libpsk.so not found at {LIB_PATH}; build it with "
                "`python -m paper_2203_02798_amd.build` (there is no fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _LIB = L
    return _LIB


def check(status, where):
    if status != PSK_OK:
        msg = lib().psk_last_error().decode(errors="replace")
        raise PskError(status, where, msg)
