"""ctypes declarations of the C ABI in include/heom.h (argument marshalling only)."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libheom.so")

HEOM_OK = 0
HEOM_PENDING = 1
STATUS_NAMES = {0: "HEOM_OK", 1: "HEOM_PENDING", -1: "HEOM_E_INVAL", -2: "HEOM_E_RANGE",
                -3: "HEOM_E_NOMEM", -4: "HEOM_E_DEVICE", -5: "HEOM_E_NUMERIC",
                -6: "HEOM_E_UNSTABLE", -7: "HEOM_E_NOTFOUND", -8: "HEOM_E_CANCELLED"}
FP64 = 0
FP32_MIXED = 1
FP32_HERM = 2  # Hermitian-packed real FP32 ADOs (Hermitian runs, matrix-core path)
OBS_POPULATION = 0
OBS_DIPOLE = 1


class HeomBath(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("n_matsubara", ctypes.c_int32),
                ("lambda_cm", ctypes.c_double), ("tau_fs", ctypes.c_double)]


class HeomProblem(ctypes.Structure):
    _fields_ = [("n_states", ctypes.c_int32), ("n_baths", ctypes.c_int32),
                ("h_re_cm", ctypes.POINTER(ctypes.c_double)),
                ("h_im_cm", ctypes.POINTER(ctypes.c_double)),
                ("baths", ctypes.POINTER(HeomBath)), ("temperature_K", ctypes.c_double),
                ("depth", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class HeomInfo(ctypes.Structure):
    _fields_ = [("n_ado", ctypes.c_int64), ("n_plus_edges", ctypes.c_int64),
                ("n_states", ctypes.c_int32), ("n_modes", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("elem_bytes", ctypes.c_int32),
                ("tables_bytes", ctypes.c_size_t), ("sigma0_bytes", ctypes.c_size_t),
                ("rest_bytes", ctypes.c_size_t), ("work_bytes", ctypes.c_size_t),
                ("bulk_kernel", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class HeomState(ctypes.Structure):
    _fields_ = [("sigma0", ctypes.c_void_p), ("rest", ctypes.c_void_p)]


class HeomObservable(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("ground", ctypes.c_int32),
                ("mu", ctypes.POINTER(ctypes.c_double))]


class HeomRequest(ctypes.Structure):
    _fields_ = [("problem", HeomProblem), ("n_runs", ctypes.c_int32),
                ("record_every", ctypes.c_int32), ("n_steps", ctypes.c_int64),
                ("dt_fs", ctypes.c_double), ("rho0", ctypes.POINTER(ctypes.c_double)),
                ("obs", HeomObservable), ("hermitian", ctypes.c_int32), ("form", ctypes.c_int32)]


class HeomResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_records", ctypes.c_int64),
                ("record_doubles", ctypes.c_int32),
                ("records", ctypes.POINTER(ctypes.c_double)),
                ("t_submit_s", ctypes.c_double), ("t_admit_s", ctypes.c_double),
                ("t_finish_s", ctypes.c_double),
                ("form", ctypes.c_int32)]


P = ctypes.POINTER
vp = ctypes.c_void_p
i32, i64, u64, f64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t

# name -> (restype, argtypes); every entry point declared in include/heom.h
SIGNATURES = {
    "heom_last_error": (ctypes.c_char_p, []),
    "heom_status_string": (ctypes.c_char_p, [i32]),
    "heom_plan": (i32, [P(HeomProblem), P(HeomInfo)]),
    "heom_record_doubles": (i32, [i32, i32]),
    "heom_record_count": (i64, [i64, i32]),
    "heom_propagate_work_bytes": (sz, [P(HeomInfo), i64, i32, i32]),
    "heom_build_hierarchy": (i32, [P(HeomProblem), vp, sz, vp, P(vp)]),
    "heom_copy_tables": (i32, [vp, vp, vp, vp, vp, vp]),
    "heom_coefficients": (i32, [vp, vp, vp, vp, vp]),
    "heom_problem_coefficients": (i32, [vp, vp, vp, vp, vp]),
    "heom_emission_start": (i32, [vp, HeomState, vp, HeomState, vp, vp]),
    "heom_block_work_bytes": (sz, [vp, i64, i32]),
    "heom_cd_vectors": (i32, [vp, vp, i32, vp]),
    "heom_propagate_block": (i32, [vp, vp, vp, sz, f64, i64, i32, vp, vp, vp]),
    "heom_rhs": (i32, [vp, HeomState, HeomState, i32, vp]),
    "heom_propagate": (i32, [vp, HeomState, vp, sz, f64, i64, i32, P(HeomObservable), i32, vp,
                             vp]),
    "heom_propagate_noalloc": (i32, [vp, HeomState, f64, i64, i32, P(HeomObservable), i32, vp,
                                     vp]),
    "heom_get_state": (i32, [vp, HeomState, vp, vp, vp]),
    "heom_set_state": (i32, [vp, HeomState, vp, vp, vp]),
    "heom_destroy": (i32, [vp]),
    "heom_spectrum": (i32, [vp, i32, i64, f64, vp, i64, vp]),
    "heom_timing_enable": (i32, [i32]),
    "heom_set_launch_shape": (i32, [i32, i32]),
    "heom_timing_read": (i32, [P(f64), P(i64), P(f64), i32]),
    "heom_server_create": (i32, [vp, sz, i32, vp, P(vp)]),
    "heom_submit": (i32, [vp, P(HeomRequest), P(u64)]),
    "heom_poll": (i32, [vp, u64, P(HeomResult)]),
    "heom_wait": (i32, [vp, u64, f64, P(HeomResult)]),
    "heom_cancel": (i32, [vp, u64]),
    "heom_release": (i32, [vp, u64]),
    "heom_server_destroy": (i32, [vp]),
    "heom_server_set_log": (i32, [vp, ctypes.c_char_p]),
}

_lib = None


def load():
    """Load libheom.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libheom.so is not built: run __graft_entry__.build() or "
                               "python paper_1803_03498_amd/build.py")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class HeomError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


def check(status):
    if status not in (HEOM_OK, HEOM_PENDING):
        msg = load().heom_last_error().decode(errors="replace")
        raise HeomError(status, msg)
    return status
