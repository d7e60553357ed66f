"""ctypes binding of libparspin.so (include/parspin.h).

Argument marshalling only: every step of the simulation runs in the HIP
library.  There is no CPU fallback; when the library cannot be loaded the
import of this module fails.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libparspin.so")

PS_OK = 0
STATUS_NAMES = {0: "PS_OK", 1: "PS_E_INVALID_ARG", 2: "PS_E_NO_MEMORY", 3: "PS_E_DEVICE",
                4: "PS_E_TOO_LARGE", 5: "PS_E_NOT_READY", 6: "PS_E_CANCELLED", 7: "PS_E_NO_DEVICE"}
PS_EV_SPOIL = 1
PS_EV_SNAPSHOT = 2
PS_EV_TRAJECTORY = 4
PS_CFG_KERNEL_TIMING = 1
PS_CFG_NO_SHAPE_CACHE = 2
PS_CFG_NO_READOUT_SPLIT = 4
PS_CFG_AUTOTUNE = 8
PS_CFG_SERVE_DIRECT = 16
PS_CFG_NO_MATRIX_READOUT = 32
PS_TUNE_FORCE = 1
PS_TUNE_MAX_CANDIDATES = 12


class PsError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")


class ps_config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("spins_per_lane", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("max_partial_bytes", ctypes.c_int64), ("max_footprint_bytes", ctypes.c_int64),
                ("max_slice_steps", ctypes.c_int64)]


_fp = ctypes.POINTER(ctypes.c_float)
_dp = ctypes.POINTER(ctypes.c_double)


class ps_object(ctypes.Structure):
    _fields_ = [("n_spins", ctypes.c_int64), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("z", ctypes.c_void_p), ("m0", ctypes.c_void_p), ("t1", ctypes.c_void_p),
                ("t2", ctypes.c_void_p), ("dw", ctypes.c_void_p)]


class ps_event(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("m", ctypes.c_double * 3), ("rf_alpha", ctypes.c_double),
                ("rf_phase", ctypes.c_double), ("rf_shape", ctypes.c_int32), ("n_adc", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("trajectory", ctypes.c_uint32)]


class ps_rf_shape(ctypes.Structure):
    _fields_ = [("n_sub", ctypes.c_int32), ("reserved", ctypes.c_int32), ("tau", ctypes.c_double),
                ("m_sub", ctypes.c_double * 3), ("alpha", ctypes.c_void_p), ("phase", ctypes.c_void_p)]


class ps_trajectory(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("k", ctypes.c_void_p), ("t", ctypes.c_void_p)]


class ps_sequence(ctypes.Structure):
    _fields_ = [("n_events", ctypes.c_int64), ("events", ctypes.c_void_p), ("n_shapes", ctypes.c_int32),
                ("n_trajectories", ctypes.c_int32), ("shapes", ctypes.c_void_p), ("trajectories", ctypes.c_void_p)]


class ps_receive(ctypes.Structure):
    _fields_ = [("n_coils", ctypes.c_int32), ("reserved", ctypes.c_int32), ("s_x", ctypes.c_void_p),
                ("s_y", ctypes.c_void_p)]


assert ctypes.sizeof(ps_receive) == 24
assert ctypes.sizeof(ps_event) == 64
assert ctypes.sizeof(ps_trajectory) == 24
assert ctypes.sizeof(ps_sequence) == 40
assert ctypes.sizeof(ps_rf_shape) == 56
assert ctypes.sizeof(ps_config) == 40

class ps_request_info(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("status", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double), ("n_slices", ctypes.c_int64),
                ("footprint_bytes", ctypes.c_int64), ("n_spins", ctypes.c_int64),
                ("n_steps_per_spin", ctypes.c_int64), ("t_kernel", ctypes.c_double)]


class ps_server_stats_t(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("queued", ctypes.c_int64), ("running", ctypes.c_int64),
                ("footprint_in_use", ctypes.c_int64), ("now", ctypes.c_double)]


class ps_tune_result(ctypes.Structure):
    _fields_ = [("spins_per_lane", ctypes.c_int32), ("replicas", ctypes.c_int32), ("from_table", ctypes.c_int32),
                ("n_candidates", ctypes.c_int32), ("best_ms", ctypes.c_double), ("rule_ms", ctypes.c_double),
                ("probe_events", ctypes.c_int64),
                ("cand_spins_per_lane", ctypes.c_int32 * PS_TUNE_MAX_CANDIDATES),
                ("cand_replicas", ctypes.c_int32 * PS_TUNE_MAX_CANDIDATES),
                ("cand_ms", ctypes.c_double * PS_TUNE_MAX_CANDIDATES)]


assert ctypes.sizeof(ps_tune_result) == 232


class ps_test_backend(ctypes.Structure):
    _fields_ = [("iteration_seconds", ctypes.c_double), ("fail_iteration", ctypes.c_int64)]


class ps_kt_object(ctypes.Structure):
    _fields_ = [("n_tissues", ctypes.c_int32), ("reserved", ctypes.c_int32), ("t1", ctypes.c_void_p),
                ("t2", ctypes.c_void_p), ("dw", ctypes.c_void_p), ("tissue_begin", ctypes.c_void_p),
                ("n_spins", ctypes.c_int64), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("z", ctypes.c_void_p), ("m0", ctypes.c_void_p), ("voxel", ctypes.c_double * 3)]


assert ctypes.sizeof(ps_kt_object) == 104

REQ_STATES = {0: "queued", 1: "running", 2: "done", 3: "failed", 4: "cancelled"}
REPLICA_MODES = {0: "none", 1: "rule", 2: "twice the rule"}

# name -> (restype, argtypes)
SIGNATURES = {
    "ps_config_default": (ctypes.c_int, [ctypes.POINTER(ps_config)]),
    "ps_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ps_config)]),
    "ps_destroy": (None, [ctypes.c_void_p]),
    "ps_last_error": (ctypes.c_char_p, []),
    "ps_count": (ctypes.c_int, [ctypes.POINTER(ps_sequence), ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(ctypes.c_int64)]),
    "ps_kernel_times": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int64,
                                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]),
    "ps_simulate_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ps_object),
                                         ctypes.POINTER(ps_sequence), ctypes.POINTER(ctypes.c_void_p),
                                         ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]),
    "ps_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ps_object), ctypes.POINTER(ps_sequence),
                                 ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64)]),
    "ps_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32)]),
    "ps_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double]),
    "ps_cancel": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "ps_request_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ps_request_info)]),
    "ps_release": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "ps_server_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ps_server_stats_t)]),
    "ps_valu_peak": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "ps_tile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_int64)]),
    "ps_simulate": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ps_object), ctypes.POINTER(ps_sequence),
                                   ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "ps_simulate_rx": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ps_object), ctypes.POINTER(ps_sequence),
                                      ctypes.POINTER(ps_receive), ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_void_p]),
    "ps_count_snapshots": (ctypes.c_int, [ctypes.POINTER(ps_sequence), ctypes.POINTER(ctypes.c_int64)]),
    "ps_plan_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ps_object), ctypes.POINTER(ps_sequence),
                                      ctypes.POINTER(ps_receive), ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_void_p)]),
    "ps_plan_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "ps_kt_extent": (ctypes.c_int, [ctypes.POINTER(ps_sequence), ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "ps_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "ps_plan_destroy": (None, [ctypes.c_void_p]),
    "ps_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ps_object), ctypes.POINTER(ps_sequence),
                               ctypes.POINTER(ps_receive), ctypes.c_uint32, ctypes.POINTER(ps_tune_result)]),
    "ps_readout_path": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ps_sequence), ctypes.c_int32,
                                       ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]),
    "ps_tile_for": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ps_sequence), ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32)]),
    "ps_tune_save": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p]),
    "ps_tune_load": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32)]),
    "ps_tune_clear": (ctypes.c_int, [ctypes.c_void_p]),
    "ps_kt_simulate": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ps_kt_object), ctypes.POINTER(ps_sequence),
                                      ctypes.POINTER(ctypes.c_double), ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_void_p]),
    "ps_create_scheduler_test": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ps_config),
                                                ctypes.POINTER(ps_test_backend)]),
    "ps_simulate_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ps_object), ctypes.POINTER(ps_sequence),
                                           ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "ps_simulate_ex": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ps_object), ctypes.POINTER(ps_sequence),
                                      ctypes.POINTER(ps_receive), ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
}


def _load():
    # PyTorch ships its own HIP runtime with the same soname as ROCm's
    # (libamdhip64.so.7).  Loading torch first lets this library bind to that
    # already-loaded runtime; otherwise the process would hold two HIP/HSA
    # runtimes and torch would find no GPU.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def last_error() -> str:
    msg = lib.ps_last_error()
    return msg.decode() if msg else ""


def check(status: int):
    if status != PS_OK:
        raise PsError(status, last_error())
