"""ctypes loader for libmimocg.so (the C ABI declared in include/mimo_cg.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation anywhere in the package.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmimocg.so")

MIMO_C32, MIMO_C16, MIMO_CBF16 = 0, 1, 2
MIMO_SINR_APPROX, MIMO_SINR_EXACT = 0, 1
MIMO_SCALAR_F32, MIMO_SCALAR_F64 = 0, 1
MIMO_OP_GRAM_MF, MIMO_OP_DETECT, MIMO_OP_PRECODE, MIMO_OP_SLOT = 0, 1, 2, 3
MIMO_OK, MIMO_EINVAL, MIMO_EUNSUPPORTED, MIMO_EWORKSPACE, MIMO_EHIP = 0, -1, -2, -3, -4
MIMO_MAX_USERS = 64
MIMO_MAX_USERS_COMMON = 32
MIMO_MAX_ANTENNAS = 4096
MIMO_MAX_SPAN_BYTES = 1 << 31


class MimoShape(ctypes.Structure):
    _fields_ = [("B", ctypes.c_int32), ("U", ctypes.c_int32), ("S", ctypes.c_int32),
                ("K", ctypes.c_int32), ("n_sc", ctypes.c_int64)]


MIMO_MAX_BATCH = 32


class MimoFrame(ctypes.Structure):
    _fields_ = [("n_sc", ctypes.c_int64), ("B", ctypes.c_int32), ("U", ctypes.c_int32),
                ("S", ctypes.c_int32), ("K", ctypes.c_int32), ("H", ctypes.c_void_p),
                ("Y", ctypes.c_void_p), ("out", ctypes.c_void_p), ("out2", ctypes.c_void_p),
                ("n0", ctypes.c_float), ("es", ctypes.c_float), ("beta", ctypes.c_float),
                ("normalize", ctypes.c_int32), ("gram", ctypes.c_void_p)]


class MimoServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_int64), ("n_slots", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("lookahead", ctypes.c_int32),
                ("paused", ctypes.c_int32), ("keep_outputs", ctypes.c_int32)]


class MimoUplinkReq(ctypes.Structure):
    _fields_ = [("ch_id", ctypes.c_int64), ("Y", ctypes.c_void_p), ("S", ctypes.c_int32),
                ("qam_bits", ctypes.c_int32), ("K", ctypes.c_int32), ("sinr_mode", ctypes.c_int32),
                ("scalar_prec", ctypes.c_int32), ("want_xhat", ctypes.c_int32),
                ("n0", ctypes.c_float), ("es", ctypes.c_float)]


class MimoDownlinkReq(ctypes.Structure):
    _fields_ = [("ch_id", ctypes.c_int64), ("T", ctypes.c_void_p), ("S", ctypes.c_int32),
                ("K", ctypes.c_int32), ("normalize", ctypes.c_int32),
                ("scalar_prec", ctypes.c_int32), ("beta", ctypes.c_float)]


class MimoCompletion(ctypes.Structure):
    _fields_ = [("req_id", ctypes.c_int64), ("status", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("out", ctypes.c_void_p), ("out2", ctypes.c_void_p),
                ("n_sc", ctypes.c_int64), ("B", ctypes.c_int32), ("U", ctypes.c_int32),
                ("S", ctypes.c_int32), ("qam_bits", ctypes.c_int32), ("solves", ctypes.c_int64),
                ("llr_bits", ctypes.c_int64)]


class MimoServerStats(ctypes.Structure):
    _fields_ = [("frames", ctypes.c_int64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("frames_per_s", ctypes.c_double), ("solves_per_s", ctypes.c_double),
                ("llr_gbit_s", ctypes.c_double), ("peak_bytes", ctypes.c_int64),
                ("budget_waits", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("mean_batch", ctypes.c_double)]


MIMO_SERVE_MAX_SLOTS = 16


class MimoError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status


_lib = None
_vp = ctypes.c_void_p
_f = ctypes.c_float
_i = ctypes.c_int
_sz = ctypes.c_size_t
_shape_p = ctypes.POINTER(MimoShape)

_SIGNATURES = {
    "mimo_gram_mf": (_i, [_shape_p, _vp, _vp, _i, _f, _vp, _vp, _vp]),
    "mimo_detect_cg": (_i, [_shape_p, _vp, _vp, _i, _f, _f, _i, _i, _i, _vp, _vp, _vp, _vp,
                            _vp, _sz, _vp]),
    "mimo_precode_cg": (_i, [_shape_p, _vp, _vp, _i, _f, _i, _i, _vp, _vp, _vp, _sz, _vp]),
    "mimo_detect_precode_cg": (_i, [_shape_p, _shape_p, _vp, _vp, _vp, _i, _f, _f, _i, _f, _i,
                                    _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "mimo_detect_cg_gram": (_i, [_shape_p, _vp, _vp, _vp, _i, _f, _f, _i, _i, _vp, _vp, _vp,
                                 _vp, _vp]),
    "mimo_precode_cg_gram": (_i, [_shape_p, _vp, _vp, _vp, _i, _f, _i, _i, _vp, _vp, _vp]),
    "mimo_convert": (_i, [_vp, _vp, _i, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _vp]),
    "mimo_workspace_bytes": (_sz, [_shape_p, _i, _i]),
    "mimo_status_string": (ctypes.c_char_p, [_i]),
    "mimo_last_error": (ctypes.c_char_p, []),
    "mimo_version": (ctypes.c_char_p, []),
    "mimo_detect_cg_batch": (_i, [ctypes.c_void_p, _i, _i, _i, _i, _vp]),
    "mimo_precode_cg_batch": (_i, [ctypes.c_void_p, _i, _i, _i, _vp]),
    "mimo_detect_cholesky": (_i, [_shape_p, _vp, _vp, _i, _f, _f, _i, _vp, _vp, _vp, _vp, _vp]),
    "mimo_detect_neumann": (_i, [_shape_p, _vp, _vp, _i, _f, _f, _i, _vp, _vp, _vp, _vp, _vp]),
    "mimo_precode_cholesky": (_i, [_shape_p, _vp, _vp, _i, _f, _i, _vp, _vp, _vp]),
    "mimo_precode_neumann": (_i, [_shape_p, _vp, _vp, _i, _f, _i, _vp, _vp, _vp]),
    "mimo_detect_cgls": (_i, [_shape_p, _vp, _vp, _i, _f, _f, _i, _i, _vp, _vp, _vp, _vp, _vp]),
    "mimo_precode_cgls": (_i, [_shape_p, _vp, _vp, _i, _f, _i, _i, _vp, _vp, _vp]),
    "mimo_tune_set": (_i, [_i, _i, _i, _i, _i]),
    "mimo_tune_get": (_i, [_i, _i, _i, ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "mimo_tune_variant_count": (_i, [_i]),
    "mimo_tune_variant_name": (ctypes.c_char_p, [_i, _i]),
    # native serving runtime (include/mimo_serve.h)
    "mimo_server_create": (_i, [ctypes.POINTER(MimoServerConfig), _i, ctypes.POINTER(_vp)]),
    "mimo_server_destroy": (_i, [_vp]),
    "mimo_server_register_channel": (_i, [_vp, ctypes.c_int64, _vp, _i, ctypes.c_int64,
                                          ctypes.c_int32, ctypes.c_int32]),
    "mimo_server_register_channel_gram": (_i, [_vp, ctypes.c_int64, _vp, _vp, _i, ctypes.c_int64,
                                               ctypes.c_int32, ctypes.c_int32]),
    "mimo_server_unregister_channel": (_i, [_vp, ctypes.c_int64]),
    "mimo_server_submit_uplink": (_i, [_vp, ctypes.POINTER(MimoUplinkReq), _vp,
                                       ctypes.POINTER(ctypes.c_int64)]),
    "mimo_server_submit_downlink": (_i, [_vp, ctypes.POINTER(MimoDownlinkReq), _vp,
                                         ctypes.POINTER(ctypes.c_int64)]),
    "mimo_server_poll": (_i, [_vp, ctypes.POINTER(MimoCompletion), _i, ctypes.c_int64]),
    "mimo_server_release": (_i, [_vp, ctypes.c_int64]),
    "mimo_server_dlpack": (_i, [_vp, ctypes.c_int64, _i, ctypes.POINTER(_vp)]),
    "mimo_server_pause": (_i, [_vp]),
    "mimo_server_resume": (_i, [_vp]),
    "mimo_server_drain": (_i, [_vp, ctypes.c_int64]),
    "mimo_server_stats_get": (_i, [_vp, ctypes.c_int64, _i, ctypes.POINTER(MimoServerStats)]),
    "mimo_server_memory": (_i, [_vp, ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(ctypes.c_int64)]),
}


def lib() -> ctypes.CDLL:
    """The loaded library (built by paper_1404_0424_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1404_0424_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != MIMO_OK:
        L = lib()
        msg = (L.mimo_last_error() or b"").decode() or L.mimo_status_string(status).decode()
        raise MimoError(status, msg)


def shape(B: int, U: int, S: int, K: int, n_sc: int) -> MimoShape:
    return MimoShape(int(B), int(U), int(S), int(K), int(n_sc))
