"""ctypes declarations of the C ABI in include/bltc.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("BLTC_LIBRARY") or os.path.join(_PKG, "libbltc.so")

BLTC_OK = 0
BLTC_EINVAL = -1
BLTC_ENOMEM = -2
BLTC_EHIP = -3
BLTC_EUNSUPPORTED = -4
BLTC_EINTERNAL = -5

COULOMB = 0
YUKAWA = 1
REGULARIZED = 2
FP64 = 0
FP32_MIXED = 1
PARTICLE_CLUSTER = 0
CLUSTER_PARTICLE = 1
CLUSTER_CLUSTER = 2
HERMITE = 3

# every exported symbol of include/bltc.h
EXPORTS = (
    "bltc_params_default", "bltc_potential", "bltc_plan_create", "bltc_plan_create_host",
    "bltc_plan_execute", "bltc_plan_modified_charges", "bltc_plan_stats", "bltc_plan_view_get",
    "bltc_plan_set_timing", "bltc_plan_phase_times", "bltc_plan_destroy", "bltc_direct",
    "bltc_batch_create", "bltc_batch_execute", "bltc_batch_set_graph", "bltc_batch_info_get",
    "bltc_batch_destroy", "bltc_batch_potential", "bltc_autotune", "bltc_status_string",
    "bltc_last_error", "bltc_version", "bltc_direct_noalloc",
)


class Params(ctypes.Structure):
    _fields_ = [
        ("kernel", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("kappa", ctypes.c_double),
        ("theta", ctypes.c_double),
        ("degree", ctypes.c_int32),
        ("leaf_size", ctypes.c_int32),
        ("batch_size", ctypes.c_int32),
        ("threads_per_target", ctypes.c_int32),
        ("method", ctypes.c_int32),
        ("delta", ctypes.c_double),
        ("no_symmetry", ctypes.c_int32),
        ("workspace_limit", ctypes.c_int64),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("clusters", ctypes.c_int64),
        ("leaves", ctypes.c_int64),
        ("batches", ctypes.c_int64),
        ("approx_pairs", ctypes.c_int64),
        ("direct_pairs", ctypes.c_int64),
        ("approx_clusters", ctypes.c_int64),
        ("far_evals", ctypes.c_int64),
        ("near_evals", ctypes.c_int64),
        ("upward_terms", ctypes.c_int64),
        ("depth", ctypes.c_int32),
        ("degree", ctypes.c_int32),
        ("leaf_size", ctypes.c_int32),
        ("batch_size", ctypes.c_int32),
        ("setup_seconds", ctypes.c_double),
        ("mutual_pair_evals", ctypes.c_int64),
        ("threads_per_target", ctypes.c_int32),
        ("workspace_bytes", ctypes.c_int64),
        ("mutual_pairs", ctypes.c_int64),
        ("pair_workspace_bytes", ctypes.c_int64),
        ("pair_rounds", ctypes.c_int32),
    ]


_P64 = ctypes.POINTER(ctypes.c_int64)
_P32 = ctypes.POINTER(ctypes.c_int32)
_PD = ctypes.POINTER(ctypes.c_double)


class PlanView(ctypes.Structure):
    _fields_ = [
        ("nt", ctypes.c_int64), ("ns", ctypes.c_int64), ("n_clusters", ctypes.c_int64),
        ("n_batches", ctypes.c_int64), ("n_items", ctypes.c_int64),
        ("source_order", _P64), ("target_order", _P64),
        ("cluster_begin", _P64), ("cluster_count", _P64),
        ("cluster_lo", _PD), ("cluster_hi", _PD),
        ("cluster_first_child", _P32), ("cluster_nchild", _P32), ("cluster_level", _P32),
        ("batch_begin", _P64), ("batch_count", _P64),
        ("batch_lo", _PD), ("batch_hi", _PD),
        ("item_batch", _P32), ("item_cluster", _P32), ("item_kind", _P32),
    ]


class BatchInfo(ctypes.Structure):
    _fields_ = [
        ("systems", ctypes.c_int32),
        ("units", ctypes.c_int32),
        ("upward_units", ctypes.c_int32),
        ("workgroups", ctypes.c_int32),
        ("graph_captures", ctypes.c_int64),
        ("launches", ctypes.c_int64),
    ]


_lib = None


def load():
    """Loads libbltc.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            "libbltc.so is missing: build the HIP library first "
            "(python -m paper_2003_01836_amd.build); there is no fallback path")
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, vp, d = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_double
    PP = ctypes.POINTER(Params)
    lib.bltc_params_default.argtypes = [PP]
    lib.bltc_params_default.restype = None
    lib.bltc_potential.argtypes = [PP, i64, vp, vp, vp, i64, vp, vp, vp, vp, i32, i64, vp, i64, vp]
    lib.bltc_plan_create.argtypes = [ctypes.POINTER(vp), PP, i64, vp, vp, vp, i64, vp, vp, vp, i32, vp]
    lib.bltc_plan_create_host.argtypes = [ctypes.POINTER(vp), PP, i64, vp, vp, vp, i64, vp, vp, vp, i32]
    lib.bltc_plan_execute.argtypes = [vp, vp, i32, i64, vp, i64, vp]
    lib.bltc_plan_modified_charges.argtypes = [vp, i64, i32, vp, vp]
    lib.bltc_plan_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.bltc_plan_view_get.argtypes = [vp, ctypes.POINTER(PlanView)]
    lib.bltc_plan_set_timing.argtypes = [vp, i32]
    lib.bltc_plan_phase_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.bltc_plan_destroy.argtypes = [vp]
    lib.bltc_plan_destroy.restype = None
    lib.bltc_direct.argtypes = [PP, i64, vp, vp, vp, i64, vp, vp, vp, vp, i32, i64, vp, i64, vp]
    lib.bltc_direct_noalloc.argtypes = lib.bltc_direct.argtypes
    lib.bltc_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), i32, vp]
    lib.bltc_batch_execute.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(i32),
                                       ctypes.POINTER(i64), ctypes.POINTER(vp), ctypes.POINTER(i64), vp]
    lib.bltc_batch_set_graph.argtypes = [vp, i32]
    lib.bltc_batch_info_get.argtypes = [vp, ctypes.POINTER(BatchInfo)]
    lib.bltc_batch_destroy.argtypes = [vp]
    lib.bltc_batch_destroy.restype = None
    lib.bltc_batch_potential.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp), ctypes.POINTER(i32),
                                         ctypes.POINTER(i64), ctypes.POINTER(vp), ctypes.POINTER(i64), vp]
    lib.bltc_autotune.argtypes = [PP, i64, vp, vp, vp, i64, vp, vp, vp, i32, ctypes.POINTER(i32), i32,
                                  i32, PP, ctypes.POINTER(d), vp]
    lib.bltc_status_string.argtypes = [ctypes.c_int]
    lib.bltc_status_string.restype = ctypes.c_char_p
    lib.bltc_last_error.argtypes = []
    lib.bltc_last_error.restype = ctypes.c_char_p
    lib.bltc_version.restype = ctypes.c_char_p
    for name in ("bltc_potential", "bltc_plan_create", "bltc_plan_create_host", "bltc_plan_execute",
                 "bltc_plan_modified_charges", "bltc_plan_stats", "bltc_plan_view_get", "bltc_direct",
                 "bltc_plan_set_timing", "bltc_plan_phase_times", "bltc_batch_create",
                 "bltc_batch_execute", "bltc_batch_set_graph", "bltc_batch_info_get",
                 "bltc_batch_potential", "bltc_autotune", "bltc_direct_noalloc"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


class BLTCError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"{message} (status {code})")
        self.code = code


class InvalidArgument(BLTCError, ValueError):
    pass


def check(rc):
    if rc == BLTC_OK:
        return
    lib = load()
    msg = lib.bltc_last_error().decode(errors="replace")
    if rc == BLTC_EINVAL:
        raise InvalidArgument(rc, msg)
    raise BLTCError(rc, msg)
