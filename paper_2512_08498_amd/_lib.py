"""ctypes declarations of the C ABI in include/gsr.h (argument marshalling only).

Loading fails loudly if libgsr.so has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsr.so")

GSR_OK = 0
GSR_ERR_INVALID_ARG = -1
GSR_ERR_CAPACITY = -2
GSR_ERR_HIP = -3
GSR_ERR_UNSUPPORTED = -4
GSR_ERR_NOT_PLANNED = -5

N_STAGES = 9
STAGE_NAMES = ("preprocess", "binning", "sort", "raster_fwd", "loss", "raster_bwd", "reduce", "pre_bwd", "adam")

STATUS_NAMES = {0: "OK", -1: "INVALID_ARG", -2: "CAPACITY", -3: "HIP", -4: "UNSUPPORTED", -5: "NOT_PLANNED"}

P = C.c_void_p


class Gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("mean", P), ("log_scale", P), ("quat", P),
                ("opacity_logit", P), ("sh", P)]


class Camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class PlanOptions(C.Structure):
    _fields_ = [("tile_size", C.c_int32), ("capacity_records", C.c_int64), ("capacity_pairs", C.c_int64),
                ("bg", C.c_float * 3)]


class Tuning(C.Structure):
    _fields_ = [("tile_size", C.c_int32), ("long_list", C.c_uint32), ("persistent", C.c_int32),
                ("step_ms", C.c_float)]


class FwdOut(C.Structure):
    _fields_ = [("image", P), ("t_final", P), ("last_pos", P), ("n_contrib", P)]


class Grads(C.Structure):
    _fields_ = [("mean", P), ("log_scale", P), ("quat", P), ("opacity_logit", P), ("sh", P), ("camera", P)]


class InsertConfig(C.Structure):
    _fields_ = [("sigma", C.c_float), ("tau_a", C.c_float)]


class InsertOut(C.Structure):
    _fields_ = [("pix", P), ("scale", P), ("mean", P), ("count", P), ("capacity", C.c_int64)]


class MergeConfig(C.Structure):
    _fields_ = [("tau_d", C.c_float), ("kappa", C.c_float)]


class MergeOut(C.Structure):
    _fields_ = [("keep", P), ("colour", P), ("keep_new", P), ("colour_new", P), ("mean", P), ("mean_new", P)]


class Moments(C.Structure):
    _fields_ = [("mean", P), ("log_scale", P), ("quat", P), ("opacity_logit", P), ("sh", P)]


class AdamConfig(C.Structure):
    _fields_ = [("lr", C.c_float * 6), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


_SIGS = {
    "gsr_create": [C.POINTER(P)],
    "gsr_destroy": [P],
    "gsr_plan": [P, C.POINTER(Camera), C.c_int32, C.c_int64, C.c_int32, C.POINTER(PlanOptions),
                 C.POINTER(C.c_size_t), C.POINTER(C.c_int64)],
    "gsr_render_forward": [P, C.POINTER(Gaussians), P, C.c_int32, P, C.c_size_t, C.POINTER(FwdOut), P],
    "gsr_l1_loss": [P, P, P, C.c_int64, P, P, P],
    "gsr_render_forward_l1": [P, C.POINTER(Gaussians), P, C.c_int32, P, C.c_size_t, C.POINTER(FwdOut), P, P, P, P],
    "gsr_render_forward_noalloc": [P, C.POINTER(Gaussians), P, C.c_int32, C.POINTER(FwdOut), P],
    "gsr_render_backward": [P, C.POINTER(Gaussians), P, C.c_int32, P, C.c_size_t, C.POINTER(FwdOut), P,
                            C.POINTER(Grads), C.c_int32, P],
    "gsr_adam_step": [P, C.POINTER(Grads), C.POINTER(Grads), C.POINTER(Moments), C.POINTER(Moments),
                      C.POINTER(AdamConfig), P, C.c_int64, C.c_int32, P],
    "gsr_render_backward_adam": [P, C.POINTER(Gaussians), P, C.c_int32, P, C.c_size_t, C.POINTER(FwdOut), P,
                                 C.POINTER(Grads), C.POINTER(Moments), C.POINTER(Moments),
                                 C.POINTER(AdamConfig), P, C.POINTER(Grads), P],
    "gsr_debug_binning": [P, P, P, P, P, P],
    "gsr_count_evaluations": [P, P, C.POINTER(FwdOut), P, P],
    "gsr_copy_bytes": [P, P, C.c_size_t, P],
    "gsr_check": [P, P, P],
    "gsr_required_capacity": [P, P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64), P],
    "gsr_set_tuning": [P, C.POINTER(Tuning)],
    "gsr_get_tuning": [P, C.POINTER(Tuning)],
    "gsr_autotune": [P, C.POINTER(Gaussians), C.POINTER(Camera), C.c_int32, C.POINTER(PlanOptions), C.c_int32,
                     C.c_char_p, C.POINTER(Tuning), P],
    "gsr_profile": [P, C.c_int32],
    "gsr_profile_read": [P, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32],
    "gsr_last_error": [P],
    "gsr_rig_plan": [P, P, P, C.c_int32, C.c_int32, C.c_int32],
    "gsr_freq_plan": [P, P, P, C.c_int32, C.POINTER(C.c_size_t)],
    "gsr_insert_workspace": [P, C.POINTER(C.c_size_t)],
    "gsr_merge_workspace": [P, C.c_int64, C.POINTER(C.c_size_t)],
    "gsr_merge": [P, C.POINTER(Gaussians), C.c_int32, P, P, P, C.POINTER(InsertOut), C.POINTER(MergeConfig),
                  C.POINTER(MergeOut), P, C.c_size_t, P],
    "gsr_log_insert": [P, P, P, P, P, C.POINTER(InsertConfig), P, P, C.POINTER(InsertOut), P, C.c_size_t, P],
    "gsr_freq_significance": [P, P, P, C.c_size_t, P, P],
    "gsr_downsample": [P, P, C.c_int32, C.c_int32, C.c_int32, P, P],
    "gsr_freq_schedule": [P, P, P, P, C.c_int32, C.c_float, P, P, C.c_int32, P, P, P, P],
    "gsr_rig_compose": [P, P, P, P, P],
    "gsr_rig_gradients": [P, P, P, P, P, P, P, P, P],
}

EXPORTED = tuple(_SIGS)

_lib = None


def load():
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2512_08498_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = None if name == "gsr_destroy" else (C.c_char_p if name == "gsr_last_error" else C.c_int)
        _lib = lib
    return _lib


class GsrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"gsr status {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(ctx, status):
    if status != GSR_OK:
        msg = load().gsr_last_error(ctx)
        raise GsrError(status, msg.decode() if msg else "")
