"""ctypes view of ``include/sas_bp.h``: structures and the exported functions.

The library is loaded from this package directory (built in-tree by
``paper_2101_05888_amd.build``) on first use. There is no fallback: any call
into the library when it has not been built raises ``ImportError``.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsas_bp.so")

SAS_BP_OK, SAS_BP_EINVAL, SAS_BP_EUNSUPPORTED, SAS_BP_ENOMEM, SAS_BP_EDEVICE, SAS_BP_ENAV, SAS_BP_ECONVERGE = range(7)
ECHO_C64, ECHO_F16X2, ECHO_BF16X2 = 0, 1, 2
INTERP_LINEAR, INTERP_SINC8 = 0, 1
TUNE_DEFAULT, TUNE_CACHED, TUNE_SEARCH = 0, 1, 2

EXPORTED = (
    "sas_bp_plan", "sas_bp_workspace_size", "sas_bp_image", "sas_bp_adjoint", "sas_bp_reproject",
    "sas_bp_useful_updates", "sas_bp_sharpness", "sas_bp_sharpness_static", "sas_bp_drc", "sas_bp_tvg", "sas_bp_envelope", "sas_bp_whiten",
    "sas_bp_range_compress", "sas_bp_dpc_tde", "sas_bp_dpc_footprints", "sas_bp_dpc_residual", "sas_bp_dpc_fine_delay",
    "sas_bp_dpc_solve", "sas_bp_plan_status", "sas_bp_plan_info",
    "sas_bp_autotune", "sas_bp_gate_class", "sas_bp_set_kernel_timing", "sas_bp_kernel_time", "sas_bp_destroy", "sas_bp_error_string",
    "sas_bp_last_error_detail", "sas_bp_abi_version",
)


class SwathDesc(C.Structure):
    _fields_ = [
        ("n_ping", C.c_int32), ("n_elem", C.c_int32), ("n_sample", C.c_int32), ("echo_dtype", C.c_int32),
        ("n", C.c_int64 * 3), ("origin", C.c_double * 3), ("spacing", C.c_double * 3),
        ("f_c", C.c_double), ("f_s", C.c_double), ("t0", C.c_double),
        ("gate_half_angle", C.c_double), ("c_min", C.c_double), ("interp", C.c_int32),
        ("motion", C.c_int32), ("refract", C.c_int32), ("track_n", C.c_int32), ("c_sediment", C.c_double),
        ("z_interface", C.c_double), ("track_dt", C.c_double),
    ]


class Options(C.Structure):
    _fields_ = [
        ("device", C.c_int32), ("tile_x", C.c_int32), ("tile_y", C.c_int32), ("tile_z", C.c_int32),
        ("pings_per_chunk", C.c_int32), ("threads", C.c_int32), ("use_graph", C.c_int32),
        ("elems_per_chunk", C.c_int32), ("workspace_limit", C.c_size_t), ("tune_mode", C.c_int32),
        ("no_cull", C.c_int32), ("tune_cache", C.c_char_p),
    ]


class DpcDesc(C.Structure):
    _fields_ = [
        ("n_ping", C.c_int32), ("n_window", C.c_int32), ("n_pairs", C.c_int32), ("n_elem", C.c_int32),
        ("robust", C.c_int32), ("max_iter", C.c_int32), ("c", C.c_double), ("sigma", C.c_double),
        ("lambda_smooth", C.c_double), ("lambda_dvl", C.c_double), ("p0", C.c_double * 3),
        ("lever_tx", C.c_double * 3),
    ]


class SwathIO(C.Structure):
    _fields_ = [
        ("echo", C.c_void_p), ("echo_scale", C.c_void_p), ("tx_pos", C.c_void_p),
        ("rx_pos", C.c_void_p), ("c", C.c_void_p), ("image", C.c_void_p), ("rx_vel", C.c_void_p),
        ("rx_track", C.c_void_p),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"HIP library {LIB_PATH} is missing; build it with `python -m paper_2101_05888_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    lib.sas_bp_plan.argtypes = [C.POINTER(SwathDesc), C.c_int, C.POINTER(Options), C.POINTER(P)]
    lib.sas_bp_workspace_size.argtypes = [C.POINTER(SwathDesc), C.c_int, C.POINTER(Options), C.POINTER(C.c_size_t)]
    lib.sas_bp_image.argtypes = [P, C.POINTER(SwathIO), C.c_int, P]
    lib.sas_bp_adjoint.argtypes = [P, C.POINTER(SwathIO), C.POINTER(P), C.POINTER(P), C.POINTER(P),
                                   C.POINTER(P), C.c_int, P]
    lib.sas_bp_reproject.argtypes = [P, C.POINTER(SwathIO), C.POINTER(P), C.POINTER(P), C.c_int, P]
    lib.sas_bp_drc.argtypes = [P, P, C.c_int64, C.c_double, P, P, P]
    lib.sas_bp_tvg.argtypes = [P, C.c_int, P, C.c_double, P, P]
    lib.sas_bp_envelope.argtypes = [P, C.c_int, P, P, P]
    lib.sas_bp_whiten.argtypes = [P, C.c_int, P, C.c_double, P]
    lib.sas_bp_range_compress.argtypes = [P, C.c_int, P, P, C.c_int32, C.c_int, P]
    lib.sas_bp_dpc_tde.argtypes = [P, C.c_int, P, P, C.c_int, C.c_int32, C.c_int32, C.c_int32, P, P]
    DP = C.POINTER(DpcDesc)
    lib.sas_bp_dpc_footprints.argtypes = [DP, P, P, P, P, P, C.c_double, C.c_double, P]
    lib.sas_bp_dpc_residual.argtypes = [DP, P, P, P, P, P, P, P, P, P, P]
    lib.sas_bp_dpc_solve.argtypes = [DP, P, P, P, P, P, P, P, P, P, P, P, C.c_int]
    lib.sas_bp_dpc_fine_delay.argtypes = [P, P, C.c_int64, C.c_double, P, P]
    lib.sas_bp_useful_updates.argtypes = [P, C.POINTER(SwathIO), C.c_int, P, C.POINTER(C.c_int64)]
    lib.sas_bp_sharpness.argtypes = [P, P, C.c_int64, P, P, P]
    lib.sas_bp_sharpness_static.argtypes = [P, C.c_int64, P, P, P]
    lib.sas_bp_plan_status.argtypes = [P]
    lib.sas_bp_plan_info.argtypes = [P, C.POINTER(C.c_int64)]
    lib.sas_bp_autotune.argtypes = [C.POINTER(SwathDesc), C.c_int, C.POINTER(SwathIO), C.POINTER(Options), C.c_int,
                                    P, C.POINTER(Options), C.POINTER(C.c_double)]
    D3 = C.POINTER(C.c_double)
    lib.sas_bp_gate_class.argtypes = [D3, D3, D3, C.c_double, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.sas_bp_set_kernel_timing.argtypes = [P, C.c_int]
    lib.sas_bp_kernel_time.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.sas_bp_destroy.argtypes = [P]
    lib.sas_bp_destroy.restype = None
    lib.sas_bp_error_string.argtypes = [C.c_int]
    lib.sas_bp_error_string.restype = C.c_char_p
    lib.sas_bp_last_error_detail.argtypes = []
    lib.sas_bp_last_error_detail.restype = C.c_char_p
    lib.sas_bp_abi_version.argtypes = []
    for name in EXPORTED:
        fn = getattr(lib, name)
        if name not in ("sas_bp_destroy", "sas_bp_error_string", "sas_bp_last_error_detail"):
            fn.restype = C.c_int
    return lib


_LIB = None


def lib():
    """The loaded HIP library (loaded on first call)."""
    global _LIB
    if _LIB is None:
        _LIB = _load()
    return _LIB


class SasBpError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib().sas_bp_error_string(status).decode()
        detail = lib().sas_bp_last_error_detail().decode()
        super().__init__(f"{where}: {msg} ({detail})" if detail else f"{where}: {msg}")


def check(status: int, where: str) -> None:
    if status != SAS_BP_OK:
        raise SasBpError(status, where)
