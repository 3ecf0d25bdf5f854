"""ctypes binding of libupir (include/upir.h): argument marshalling only.

Every function keeps its C name. Status codes other than UPIR_OK raise
``UpirError`` carrying the status and ``upir_last_error`` text. Structures
mirror the C layouts field for field. Nothing here computes: loops,
reductions and tasks run in the library's HIP kernels. If the library is
missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libupir.so")

# ------------------------------------------------------------------ constants
UPIR_OK, UPIR_EINVAL, UPIR_ENOTMAPPED, UPIR_EOVERLAP, UPIR_ENOMEM = 0, -1, -2, -3, -4
UPIR_EHIP, UPIR_EUNSUPPORTED, UPIR_EDEPEND, UPIR_ESTATE = -5, -6, -7, -8
UPIR_DEVICE_NONE = -1
UPIR_MAP_TO, UPIR_MAP_FROM, UPIR_MAP_TOFROM, UPIR_MAP_ALLOC = 1, 2, 3, 4
UPIR_ACCESS_RO, UPIR_ACCESS_WO, UPIR_ACCESS_RW = 1, 2, 3
UPIR_TO_DEVICE, UPIR_FROM_DEVICE = 1, 2
UPIR_TARGET_GPU, UPIR_TARGET_CPU, UPIR_TARGET_CLUSTER = 1, 2, 3
(UPIR_SCHED_STATIC, UPIR_SCHED_STATIC_CHUNK, UPIR_SCHED_DYNAMIC, UPIR_SCHED_GUIDED,
 UPIR_SCHED_RUNTIME, UPIR_SCHED_AUTO) = range(6)
UPIR_DIST_TEAMS_UNITS, UPIR_DIST_TEAMS, UPIR_DIST_UNITS = 0, 1, 2
UPIR_RED_NONE, UPIR_RED_SUM, UPIR_RED_MAX, UPIR_RED_MIN = 0, 1, 2, 3
(UPIR_BODY_AXPY, UPIR_BODY_SUM, UPIR_BODY_JACOBI5, UPIR_BODY_MATMUL_F32, UPIR_BODY_MATMUL_BF16,
 UPIR_BODY_MATMUL_SPLIT3, UPIR_BODY_MATVEC, UPIR_BODY_OWNER, UPIR_BODY_COVER, UPIR_BODY_FILTER7) = range(1, 11)
UPIR_DT_F32, UPIR_DT_F64, UPIR_DT_I32, UPIR_DT_I64 = 1, 2, 3, 4
UPIR_DEP_IN, UPIR_DEP_OUT, UPIR_DEP_INOUT = 1, 2, 3
UPIR_TASKWAIT_PLAIN, UPIR_TASKWAIT_BATCHED = 0, 1
UPIR_MLP_PARAMS = 6337
UPIR_ENGINE_CANDIDATES = 27
(UPIR_ENGINE_FROM_DEFAULT, UPIR_ENGINE_FROM_TUNER, UPIR_ENGINE_FROM_MODEL, UPIR_ENGINE_FROM_CALLER) = range(4)
VARIANTS = {0: "generic", 1: "stream4", 2: "jacobi_tile", 3: "matvec_wave", 4: "matmul_mfma", 5: "dynamic",
            6: "filter7_tile"}

# ---------------------------------------------------------------- structures
class upir_spmd(C.Structure):
    _fields_ = [("num_teams", C.c_int32), ("num_units", C.c_int32), ("target", C.c_int32)]


class upir_dim(C.Structure):
    _fields_ = [("lb", C.c_int64), ("ub", C.c_int64), ("step", C.c_int64)]


class upir_loop(C.Structure):
    _fields_ = [("collapse", C.c_int32), ("pad_", C.c_int32), ("dim", upir_dim * 3)]


class upir_sched(C.Structure):
    _fields_ = [("policy", C.c_int32), ("distribute", C.c_int32), ("chunk", C.c_int64),
                ("tile", C.c_int32 * 3), ("pad_", C.c_int32)]


class upir_reduction(C.Structure):
    _fields_ = [("op", C.c_int32), ("result_on_host", C.c_int32), ("init", C.c_double),
                ("result", C.c_void_p), ("async_", C.c_int32), ("pad_", C.c_int32)]


class upir_axpy_args(C.Structure):
    _fields_ = [("a", C.c_float), ("pad_", C.c_int32), ("x", C.c_void_p), ("y", C.c_void_p)]


class upir_sum_args(C.Structure):
    _fields_ = [("x", C.c_void_p), ("dtype", C.c_int32), ("pad_", C.c_int32)]


class upir_jacobi5_args(C.Structure):
    _fields_ = [("src", C.c_void_p), ("dst", C.c_void_p), ("ld", C.c_int64)]


class upir_matmul_args(C.Structure):
    _fields_ = [("A", C.c_void_p), ("B", C.c_void_p), ("C", C.c_void_p), ("K", C.c_int64),
                ("lda", C.c_int64), ("ldb", C.c_int64), ("ldc", C.c_int64),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t)]


class upir_matvec_args(C.Structure):
    _fields_ = [("A", C.c_void_p), ("x", C.c_void_p), ("y", C.c_void_p), ("cols", C.c_int64),
                ("lda", C.c_int64)]


class upir_owner_args(C.Structure):
    _fields_ = [("out", C.c_void_p)]


class upir_cover_args(C.Structure):
    _fields_ = [("count", C.c_void_p)]


class upir_filter7_args(C.Structure):
    _fields_ = [("src", C.c_void_p), ("dst", C.c_void_p), ("w", C.c_void_p), ("ld", C.c_int64)]


class upir_body(C.Structure):
    _fields_ = [("kind", C.c_int32), ("args_are_device_ptrs", C.c_int32), ("args", C.c_void_p),
                ("args_size", C.c_size_t)]


class upir_depend(C.Structure):
    _fields_ = [("addr", C.c_void_p), ("type", C.c_int32), ("pad_", C.c_int32)]


class upir_task_trace(C.Structure):
    _fields_ = [("tokens", C.c_void_p), ("start_stamp", C.c_void_p), ("done_stamp", C.c_void_p)]


class upir_engine_sched(C.Structure):
    _fields_ = [("tile_axpy", C.c_int64), ("tile_sum", C.c_int64), ("rows_matvec", C.c_int64)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
P = C.POINTER
_ctx_p = C.c_void_p

# name -> (restype, argtypes); restype None means upir_status
_SIGS = {
    "upir_init": (None, [C.c_int, C.c_void_p, P(C.c_void_p)]),
    "upir_finalize": (None, [_ctx_p]),
    "upir_strerror": (C.c_char_p, [C.c_int32]),
    "upir_last_error": (C.c_char_p, [_ctx_p]),
    "upir_sync": (None, [_ctx_p]),
    "upir_version": (C.c_char_p, []),
    "upir_set_allocator": (None, [_ctx_p, ALLOC_FN, FREE_FN, C.c_void_p]),
    "upir_data_map": (None, [_ctx_p, C.c_void_p, C.c_size_t, C.c_int32, C.c_int32, P(C.c_void_p)]),
    "upir_data_unmap": (None, [_ctx_p, C.c_void_p, C.c_int32]),
    "upir_data_update": (None, [_ctx_p, C.c_void_p, C.c_size_t, C.c_int32]),
    "upir_data_lookup": (None, [_ctx_p, C.c_void_p, P(C.c_void_p)]),
    "upir_loop_parallel": (None, [_ctx_p, P(upir_loop), P(upir_sched), P(upir_body), P(upir_reduction),
                                  P(C.c_void_p)]),
    "upir_loop_free": (None, [_ctx_p, C.c_void_p]),
    "upir_loop_set_result": (None, [_ctx_p, C.c_void_p, C.c_void_p]),
    "upir_loop_set_args": (None, [_ctx_p, C.c_void_p, C.c_void_p, C.c_size_t]),
    "upir_spmd_launch": (None, [_ctx_p, P(upir_spmd), P(C.c_void_p), C.c_int32]),
    "upir_reduce_wait": (None, [_ctx_p, C.c_void_p]),
    "upir_reduce": (None, [_ctx_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int64, P(upir_spmd), P(upir_sched),
                           P(upir_reduction)]),
    "upir_reduce_noalloc": (None, [_ctx_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int64, P(upir_spmd),
                                   P(upir_sched), P(upir_reduction)]),
    "upir_loop_resolve": (None, [_ctx_p, P(upir_spmd), C.c_void_p, P(upir_spmd), P(upir_sched), P(C.c_int32)]),
    "upir_matmul_workspace_bytes": (C.c_size_t, [C.c_int32, C.c_int64, C.c_int64, C.c_int64]),
    "upir_graph_begin": (None, [_ctx_p]),
    "upir_graph_end": (None, [_ctx_p, P(C.c_void_p)]),
    "upir_graph_launch": (None, [_ctx_p, C.c_void_p]),
    "upir_graph_destroy": (None, [_ctx_p, C.c_void_p]),
    "upir_task": (None, [_ctx_p, P(upir_spmd), C.c_void_p, P(upir_depend), C.c_int32, P(C.c_int64)]),
    "upir_taskloop": (None, [_ctx_p, P(upir_spmd), C.c_void_p, C.c_int64, C.c_int64, P(upir_depend), C.c_int32,
                             P(C.c_int64), P(C.c_int64)]),
    "upir_task_update": (None, [_ctx_p, C.c_void_p, C.c_size_t, C.c_int32, P(upir_depend), C.c_int32,
                                P(C.c_int64)]),
    "upir_task_preds": (None, [_ctx_p, C.c_int64, P(C.c_int64), C.c_int32, P(C.c_int32)]),
    "upir_set_task_trace": (None, [_ctx_p, P(upir_task_trace)]),
    "upir_taskwait": (None, [_ctx_p, C.c_int32]),
    "upir_taskwait_graph": (None, [_ctx_p, C.c_int32, P(C.c_void_p)]),
    "upir_tune": (None, [_ctx_p, P(upir_spmd), C.c_void_p, C.c_int32, P(upir_sched), P(upir_spmd),
                         P(C.c_double)]),
    "upir_candidates": (None, [_ctx_p, C.c_void_p, P(C.c_int32)]),
    "upir_candidate_features": (None, [_ctx_p, C.c_void_p, C.c_int32, P(C.c_float), P(upir_spmd),
                                       P(upir_sched)]),
    "upir_tune_db_save": (None, [_ctx_p, C.c_char_p]),
    "upir_tune_db_load": (None, [_ctx_p, C.c_char_p]),
    "upir_tune_db_size": (None, [_ctx_p, P(C.c_int64)]),
    "upir_tune_db_row": (None, [_ctx_p, C.c_int64, P(C.c_float), P(C.c_float), P(C.c_int64)]),
    "upir_engine_sched_set": (None, [_ctx_p, P(upir_engine_sched)]),
    "upir_engine_sched_resolve": (None, [_ctx_p, P(upir_engine_sched), P(C.c_int32)]),
    "upir_engine_candidate": (None, [_ctx_p, C.c_int32, P(upir_engine_sched), P(C.c_float)]),
    "upir_tune_batched": (None, [_ctx_p, C.c_int32, P(upir_engine_sched), P(C.c_double)]),
    "upir_model_init": (None, [_ctx_p, C.c_uint64]),
    "upir_model_set_params": (None, [_ctx_p, P(C.c_float)]),
    "upir_model_get_params": (None, [_ctx_p, P(C.c_float)]),
    "upir_model_forward": (None, [_ctx_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "upir_model_step": (None, [_ctx_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_float, C.c_int32, C.c_void_p,
                               P(C.c_float)]),
    "upir_model_train": (None, [_ctx_p, C.c_int32, C.c_int32, C.c_float, C.c_int32, P(C.c_float),
                                P(C.c_float)]),
    "upir_model_enable": (None, [_ctx_p, C.c_int32]),
    "upir_model_save": (None, [_ctx_p, C.c_char_p]),
    "upir_model_load": (None, [_ctx_p, C.c_char_p]),
}

_lib = None


class UpirError(RuntimeError):
    def __init__(self, status: int, fn: str, msg: str):
        super().__init__(f"{fn}: status {status} ({_STATUS.get(status, '?')}): {msg}")
        self.status = status


_STATUS = {0: "UPIR_OK", -1: "UPIR_EINVAL", -2: "UPIR_ENOTMAPPED", -3: "UPIR_EOVERLAP", -4: "UPIR_ENOMEM",
           -5: "UPIR_EHIP", -6: "UPIR_EUNSUPPORTED", -7: "UPIR_EDEPEND", -8: "UPIR_ESTATE"}


def lib():
    """Load libupir.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2209_10643_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res if res is not None else C.c_int32
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _wrap(name):
    res = _SIGS[name][0]

    def call(*args):
        f = getattr(lib(), name)
        r = f(*args)
        if res is None and r != UPIR_OK:
            ctx = args[0] if args and name not in ("upir_init", "upir_strerror") else None
            msg = lib().upir_last_error(ctx).decode() if ctx else lib().upir_strerror(r).decode()
            raise UpirError(r, name, msg)
        return r
    call.__name__ = name
    return call


for _n in _SIGS:
    globals()[_n] = _wrap(_n)


def raw(name):
    """The ctypes function itself (returns the status instead of raising)."""
    return getattr(lib(), name)
