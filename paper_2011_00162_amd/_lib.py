"""ctypes declarations of the libodp.so C ABI (include/odp.h).

Loading fails loudly when the library has not been built: there is no other
implementation to fall back to.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libodp.so")

ODP_OK, ODP_EINVAL, ODP_EGEOM, ODP_EHIP, ODP_ENOMEM, ODP_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
ODP_FFT_F32, ODP_DFT_SPLIT_BF16, ODP_HYBRID_MFMA = 0, 1, 2
ODP_STOP_NONE, ODP_STOP_RF, ODP_STOP_RE = 0, 1, 2
ODP_BALANCE_R, ODP_BALANCE_ETA = 1, 2

# every symbol include/odp.h declares
EXPORTS = [
    "odp_plan_create", "odp_plan_destroy", "odp_plan_get_info", "odp_state_get_layout",
    "odp_plan_get_rects", "odp_plan_get_pairs", "odp_plan_get_cover", "odp_plan_bind",
    "odp_plan_illum_max", "odp_plan_set_params", "odp_forward", "odp_adjoint", "odp_prox_stagm",
    "odp_state_init", "odp_admm_iterate", "odp_frame_sweep", "odp_probe_update", "odp_blind_initial_probe",
    "odp_blind_initial_probe_static",
    "odp_pixel_update", "odp_merge", "odp_amp_loss", "odp_last_error", "odp_version",
    "odp_batch_plan_create", "odp_batch_get_entry", "odp_batch_set_penalties", "odp_plan_get_tuning",
    "odp_plan_set_tuning", "odp_plan_set_streaming", "odp_plan_set_pixel_pairs", "odp_plan_autotune", "odp_graph_create", "odp_graph_launch", "odp_graph_destroy",
    "odp_plan_set_sweep_events", "odp_plan_set_stopping", "odp_state_get_stop_status", "odp_plan_set_balancing",
    "odp_plan_workspace_bytes", "odp_state_bytes", "odp_plan_get_eta",
]


class OdpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"odp error {code}: {msg}")
        self.code = code


class Problem(C.Structure):
    _fields_ = [
        ("H", C.c_int32), ("W", C.c_int32), ("p", C.c_int32), ("J", C.c_int32),
        ("offsets", C.POINTER(C.c_int32)), ("D", C.c_int32), ("frame_sub", C.POINTER(C.c_int32)),
        ("eps", C.c_double), ("eta", C.c_double), ("r", C.c_double), ("mu", C.c_double),
        ("gamma", C.c_double), ("transform", C.c_int32), ("blind", C.c_int32),
        ("probe_fmask", C.POINTER(C.c_uint8)),
    ]


class PlanInfo(C.Structure):
    _fields_ = [
        ("H", C.c_int32), ("W", C.c_int32), ("p", C.c_int32), ("J", C.c_int32), ("D", C.c_int32),
        ("n_pairs", C.c_int32), ("max_cover", C.c_int32), ("n_cells", C.c_int32), ("n_tiles", C.c_int32),
        ("p_sub", C.c_int64), ("n_lam", C.c_int64), ("workspace_bytes", C.c_size_t),
        ("state_bytes", C.c_size_t),
    ]


class StateLayout(C.Structure):
    _fields_ = [(n, C.c_size_t) for n in ("u_sub", "gamma", "lam", "w", "w_sub", "delta", "stop", "bytes")]


class StopStatus(C.Structure):
    _fields_ = [("iters", C.c_int32), ("stopped", C.c_int32), ("rf", C.c_double), ("re", C.c_double),
                ("g", C.c_double)]


class BatchEntry(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("row0", "col0", "H", "W", "J0", "J", "D0", "D")] + [
        ("r", C.c_double), ("illum_max", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("transform", "xcd_slice", "tiling", "tile_rows", "tile_cols")] + [
        ("ms_per_iter", C.c_double), ("n_tried", C.c_int32), ("pixel_pairs", C.c_int32)]


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2011_00162_amd.build`")
    L = C.CDLL(LIB_PATH, mode=os.RTLD_NOW | os.RTLD_LOCAL)
    vp, i32, i64, dbl, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_float
    sig = {
        "odp_plan_create": (C.c_int, [C.POINTER(Problem), C.POINTER(vp)]),
        "odp_plan_destroy": (None, [vp]),
        "odp_plan_get_info": (C.c_int, [vp, C.POINTER(PlanInfo)]),
        "odp_state_get_layout": (C.c_int, [vp, C.POINTER(StateLayout)]),
        "odp_plan_get_rects": (C.c_int, [vp, vp, vp]),
        "odp_plan_get_pairs": (C.c_int, [vp, vp, vp]),
        "odp_plan_get_cover": (C.c_int, [vp, vp]),
        "odp_plan_bind": (C.c_int, [vp, vp, vp, vp, vp]),
        "odp_plan_illum_max": (C.c_int, [vp, C.POINTER(dbl)]),
        "odp_plan_set_params": (C.c_int, [vp, dbl, dbl, dbl, dbl, dbl, vp]),
        "odp_forward": (C.c_int, [vp, vp, vp, vp, vp]),
        "odp_adjoint": (C.c_int, [vp, vp, vp, vp, vp]),
        "odp_prox_stagm": (C.c_int, [vp, vp, i64, f32, f32, vp, vp]),
        "odp_state_init": (C.c_int, [vp, vp, vp, vp]),
        "odp_admm_iterate": (C.c_int, [vp, vp, i32, vp, vp]),
        "odp_frame_sweep": (C.c_int, [vp, vp, vp, vp]),
        "odp_plan_set_sweep_events": (C.c_int, [vp, C.POINTER(vp), C.POINTER(vp), i32, i32]),
        "odp_probe_update": (C.c_int, [vp, vp, vp]),
        "odp_blind_initial_probe": (C.c_int, [vp, vp, vp]),
        "odp_blind_initial_probe_static": (C.c_int, [vp, i32, i32, vp, vp]),
        "odp_pixel_update": (C.c_int, [vp, vp, vp, vp]),
        "odp_merge": (C.c_int, [vp, vp, vp, vp]),
        "odp_amp_loss": (C.c_int, [vp, vp, vp, vp, vp, vp, vp]),
        "odp_batch_plan_create": (C.c_int, [C.POINTER(Problem), i32, C.POINTER(vp)]),
        "odp_batch_get_entry": (C.c_int, [vp, i32, C.POINTER(BatchEntry)]),
        "odp_batch_set_penalties": (C.c_int, [vp, vp, vp]),
        "odp_plan_get_tuning": (C.c_int, [vp, C.POINTER(Tuning)]),
        "odp_plan_set_tuning": (C.c_int, [vp, i32, i32, i32, vp]),
        "odp_plan_set_streaming": (C.c_int, [vp, i32]),
        "odp_plan_set_pixel_pairs": (C.c_int, [vp, i32]),
        "odp_plan_set_stopping": (C.c_int, [vp, i32, C.c_double, i32, i32]),
        "odp_plan_set_balancing": (C.c_int, [vp, C.c_double, C.c_double, i32, i32, i32]),
        "odp_plan_get_eta": (C.c_double, [vp]),
        "odp_plan_workspace_bytes": (C.c_size_t, [vp]),
        "odp_state_bytes": (C.c_size_t, [vp]),
        "odp_state_get_stop_status": (C.c_int, [vp, vp, vp, vp]),
        "odp_plan_autotune": (C.c_int, [vp, vp, i32, vp, C.POINTER(Tuning)]),
        "odp_graph_create": (C.c_int, [vp, vp, i32, i32, C.POINTER(vp)]),
        "odp_graph_launch": (C.c_int, [vp, vp]),
        "odp_graph_destroy": (None, [vp]),
        "odp_last_error": (C.c_char_p, []),
        "odp_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(code: int) -> None:
    if code != ODP_OK:
        raise OdpError(code, lib().odp_last_error().decode())
