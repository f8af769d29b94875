"""ctypes declarations of the C ABI in include/kete_mi.h.

Argument marshalling only: every numerical step runs in the HIP kernels
of libkete_mi.so.  Loading fails loudly when the library has not been
built; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libkete_mi.so")

KETE_OK, KETE_EINVAL, KETE_ERANGE, KETE_ECAPACITY, KETE_EDEVICE, KETE_EWORKSPACE = 0, -1, -2, -3, -4, -5
ADJ_FWD, ADJ_BWD = 0, 1
ST_OK, ST_NONFINITE, ST_STEP_UNDERFLOW, ST_MAX_STEPS, ST_KEPLER_NOCONV = 0, 1, 2, 3, 4
MAX_BODIES, MAX_DEGREE, MAX_SUB, MAX_OBJ = 16, 15, 128, 1 << 25
MAG_NOALLOC_MAX_FRAMES = 1 << 21

ERROR_NAMES = {KETE_EINVAL: "EINVAL", KETE_ERANGE: "ERANGE", KETE_ECAPACITY: "ECAPACITY",
               KETE_EDEVICE: "EDEVICE", KETE_EWORKSPACE: "EWORKSPACE"}


class KeteError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"kete error {ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class EphemT(C.Structure):
    _fields_ = [("n_body", C.c_int32), ("n_seg", C.c_int32), ("degree", C.c_int32), ("reserved", C.c_int32),
                ("t_start", C.c_double), ("seg_days", C.c_double), ("coef", C.c_void_p),
                ("gm", C.POINTER(C.c_double)), ("flags", C.POINTER(C.c_uint32)),
                ("j2", C.POINTER(C.c_double))]


class OptsT(C.Structure):
    _fields_ = [("eps", C.c_double), ("h_init", C.c_double), ("h_min", C.c_double), ("h_max", C.c_double),
                ("c_light", C.c_double), ("batch_span", C.c_double), ("cell_chord", C.c_double),
                ("lt_tol", C.c_double), ("max_steps", C.c_int32), ("max_iter", C.c_int32),
                ("n_buckets", C.c_int32), ("block", C.c_int32), ("rebucket_epochs", C.c_int32),
                ("window_segs", C.c_int32), ("lt_iter", C.c_int32), ("fov_block", C.c_int32),
                ("adj_seg_steps", C.c_int32), ("persist_waves", C.c_int32),
                ("lanes_per_body", C.c_int32), ("zero_start", C.c_int32),
                ("land_epochs", C.c_int32), ("kepler_iter", C.c_int32)]


class FramesT(C.Structure):
    _fields_ = [("n_frames", C.c_int64), ("n_sub", C.c_int32), ("reserved", C.c_int32), ("t", C.c_void_p),
                ("obs", C.c_void_p), ("normals", C.c_void_p)]


class JobT(C.Structure):
    _fields_ = [("obj_off", C.c_int64), ("epoch_off", C.c_int64), ("xout_off", C.c_int64), ("n_obj", C.c_int32),
                ("n_epoch", C.c_int32), ("t0", C.c_double)]


class BatchT(C.Structure):
    _fields_ = [("n_jobs", C.c_int32), ("reserved", C.c_int32), ("n_bodies", C.c_int64), ("n_epochs", C.c_int64),
                ("n_batch", C.c_int64), ("jobs_host", C.c_void_p), ("jobs", C.c_void_p), ("x0", C.c_void_p),
                ("epochs", C.c_void_p), ("epochs_host", C.c_void_p), ("batch_job_host", C.c_void_p), ("batch_epoch_host", C.c_void_p),
                ("batch_off_host", C.c_void_p), ("t_ref", C.c_void_p), ("batch_off", C.c_void_p),
                ("frame_order", C.c_void_p), ("frames", FramesT)]


TUNE_PROGRESS = C.CFUNCTYPE(None, C.POINTER(OptsT), C.c_double, C.c_void_p)

# name -> (restype, argtypes)
SIGNATURES = {
    "kete_default_opts": (None, [C.POINTER(OptsT)]),
    "kete_last_error": (C.c_char_p, []),
    "kete_version": (C.c_char_p, []),
    "kete_make_batches": (C.c_int, [C.c_void_p, C.c_int64, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.POINTER(C.c_int64)]),
    "kete_propagate_workspace_size": (C.c_size_t, [C.c_int64, C.c_int64, C.POINTER(OptsT)]),
    "kete_propagate_nbody": (C.c_int, [C.POINTER(EphemT), C.c_void_p, C.c_double, C.c_int64, C.c_void_p,
                                       C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(OptsT),
                                       C.c_void_p, C.c_size_t, C.c_void_p]),
    "kete_fov_workspace_size": (C.c_size_t, [C.c_int64, C.c_int64, C.c_int64, C.c_int32, C.c_int64,
                                             C.POINTER(OptsT)]),
    "kete_fov_check": (C.c_int, [C.POINTER(EphemT), C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.POINTER(FramesT), C.POINTER(OptsT), C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_int64), C.c_void_p,
                                 C.c_size_t, C.c_void_p]),
    "kete_fov_last_stats": (None, [C.c_void_p]),
    "kete_magnitudes_workspace_size": (C.c_size_t, [C.c_int64]),
    "kete_pair_magnitudes": (C.c_int, [C.POINTER(EphemT), C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.POINTER(FramesT), C.c_void_p, C.c_void_p, C.c_int64,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(OptsT),
                                       C.c_void_p, C.c_size_t, C.c_void_p]),
    "kete_pair_magnitudes_noalloc": (C.c_int, [C.POINTER(EphemT), C.c_void_p, C.c_int64, C.c_int64, C.c_void_p,
                                               C.c_void_p, C.c_void_p, C.POINTER(FramesT), C.c_void_p, C.c_void_p,
                                               C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                               C.POINTER(OptsT), C.c_void_p]),
    "kete_lighttime_directions": (C.c_int, [C.POINTER(EphemT), C.c_void_p, C.c_double, C.c_int64, C.c_void_p,
                                            C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.POINTER(OptsT),
                                            C.c_void_p]),
    "kete_ephem_eval": (C.c_int, [C.POINTER(EphemT), C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "kete_adjoint_workspace_size": (C.c_size_t, [C.c_int64, C.c_int32, C.c_double, C.c_double, C.c_double, C.POINTER(OptsT)]),
    "kete_propagate_adjoint": (C.c_int, [C.POINTER(EphemT), C.c_int32, C.c_void_p, C.c_double, C.c_double,
                                         C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                         C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(OptsT), C.c_void_p,
                                         C.c_size_t, C.c_void_p]),
    "kete_batch_workspace_size": (C.c_size_t, [C.POINTER(EphemT), C.POINTER(BatchT), C.c_int64, C.POINTER(OptsT)]),
    "kete_batch_plan": (C.c_int, [C.POINTER(EphemT), C.POINTER(BatchT), C.c_int64, C.POINTER(OptsT), C.c_void_p,
                                  C.c_size_t, C.c_void_p]),
    "kete_batch_run": (C.c_int, [C.POINTER(EphemT), C.POINTER(BatchT), C.c_int64, C.POINTER(OptsT), C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "kete_batch_pairs": (C.c_int, [C.POINTER(BatchT), C.c_int64, C.POINTER(OptsT), C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.POINTER(C.c_int64), C.c_void_p, C.c_size_t, C.c_void_p]),
    "kete_batch_graph_create": (C.c_int, [C.POINTER(EphemT), C.POINTER(BatchT), C.c_int64, C.POINTER(OptsT),
                                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p,
                                          C.POINTER(C.c_void_p)]),
    "kete_batch_graph_launch": (C.c_int, [C.c_void_p, C.c_void_p]),
    "kete_batch_graph_destroy": (C.c_int, [C.c_void_p]),
    "kete_batch_autotune": (C.c_int, [C.POINTER(EphemT), C.POINTER(BatchT), C.c_int64, C.POINTER(OptsT), C.c_int32,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, TUNE_PROGRESS,
                                      C.c_void_p, C.POINTER(OptsT), C.POINTER(C.c_double)]),
    "kete_timing_enable": (None, [C.c_int]),
    "kete_timing_read": (C.c_int, [C.c_void_p, C.c_void_p]),
    "kete_timing_read_all": (C.c_int, [C.c_void_p, C.c_void_p]),
    "kete_fov_last_counts": (None, [C.c_void_p]),
}

_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2509_04666_amd.build` "
                               "(there is no fallback path)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != KETE_OK:
        raise KeteError(rc, lib().kete_last_error().decode())


def exported_symbols():
    return list(SIGNATURES)
