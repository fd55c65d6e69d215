"""ctypes mirror of include/rsm.h and the loader of librsm.so.

Argument marshalling only: every computation runs in librsm's HIP kernels.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

MAX_RANK = 8
PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librsm.so")

# rsm_status
OK, E_INVALID, E_RANK, E_SHAPE, E_OVERFLOW, E_OVERLAP, E_UNSUPPORTED, E_HIP, E_NOMEM = range(9)
# rsm_dtype
F32, BF16, F64, I64 = 0, 1, 2, 3
# rsm_task_kind
TASK_COPY, TASK_SUM, TASK_WSUM, TASK_DOT = 0, 1, 2, 3
# flags
CHECK_SINGLE_ASSIGN = 0x1
ACCUMULATE = 0x2
NO_FUSE = 0x4
FORCE_GENERIC = 0x8
PLAN_ADJOINT = 0x20
CHECK_INDICES = 0x10
NO_GRAPH = 0x40
REDUCE_IN_KERNEL = 0x80

I64x8 = ctypes.c_int64 * MAX_RANK
I64x8x8 = (ctypes.c_int64 * MAX_RANK) * MAX_RANK


class Space(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int32), ("reserved", ctypes.c_int32), ("shape", I64x8)]


class Tiler(ctypes.Structure):
    _fields_ = [
        ("array_rank", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("array_shape", I64x8),
        ("pattern_rank", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("pattern_shape", I64x8),
        ("origin", I64x8),
        ("paving", I64x8x8),
        ("fitting", I64x8x8),
    ]


class Task(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("compute", ctypes.c_int32), ("coeffs", ctypes.c_void_p)]


class Stage(ctypes.Structure):
    _fields_ = [("rep", Space), ("in_", Tiler), ("out", Tiler), ("task", Task)]


class Problem(ctypes.Structure):
    _fields_ = [("rep", Space), ("in_", Tiler), ("out", Tiler), ("task", Task),
                ("d_in", ctypes.c_void_p), ("d_out", ctypes.c_void_p)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("n_problems", ctypes.c_int64), ("n_persistent", ctypes.c_int64),
                ("n_tiles", ctypes.c_int64), ("grid", ctypes.c_int64),
                ("tuned_classes", ctypes.c_int64), ("cached_classes", ctypes.c_int64)]


class CgInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("residual_norm", ctypes.c_double),
                ("rhs_norm", ctypes.c_double), ("converged", ctypes.c_int32),
                ("breakdown", ctypes.c_int32)]


class PortPlacement(ctypes.Structure):
    _fields_ = [("port", ctypes.c_int32), ("is_output", ctypes.c_int32), ("space", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("bytes_per_workgroup", ctypes.c_int64)]


MEM_SPACES = {0: "global", 1: "constant", 2: "local", 3: "private"}
MEM_CODES = {"any": -1, "global": 0, "constant": 1, "local": 2, "private": 3}

EXPORTS = [
    "rsm_validate", "rsm_plan", "rsm_indices", "rsm_run", "rsm_run_chain", "rsm_run_adjoint",
    "rsm_run_chain_adjoint", "rsm_batch_create", "rsm_batch_run", "rsm_batch_run_plain",
    "rsm_batch_query",
    "rsm_batch_tile", "rsm_batch_destroy", "rsm_status_string", "rsm_last_error",
    "rsm_abi_version", "rsm_run_csr", "rsm_cg_solve", "rsm_time_next_kernel", "rsm_run_chain_train",
    "rsm_plan_ports", "rsm_run_chain_train_noalloc", "rsm_plan_placed", "rsm_run_placed",
    "rsm_plan_cache_hits", "rsm_prepare", "rsm_prepared_name", "rsm_run_prepared", "rsm_prepared_destroy",
]

_lib = None


def load(path: str = LIB_PATH):
    """Load librsm.so and declare its signatures (raises if it is not built)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("librsm.so is not built (%s); run python -m paper_1105_4424_amd.build" % path)
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    st = ctypes.c_int
    u32 = ctypes.c_uint32
    i32 = ctypes.c_int32
    lib.rsm_validate.argtypes = [P(Space), P(Tiler), i32, P(Tiler), P(Task), u32]
    lib.rsm_plan.argtypes = [P(Space), P(Tiler), i32, P(Tiler), P(Task), u32, ctypes.c_char_p, i32]
    lib.rsm_plan_ports.argtypes = [P(Space), P(Tiler), i32, P(Tiler), P(Task), u32, P(PortPlacement), i32,
                                   P(i32)]
    lib.rsm_plan_placed.argtypes = [P(Space), P(Tiler), i32, P(Tiler), P(Task), u32, P(i32), i32,
                                    ctypes.c_char_p, i32, P(PortPlacement), i32, P(i32)]
    lib.rsm_run_placed.argtypes = [P(Space), P(Tiler), P(vp), i32, P(Tiler), vp, P(Task), P(i32), i32, u32, vp]
    lib.rsm_prepare.argtypes = [P(Space), P(Tiler), i32, P(Tiler), P(Task), u32, P(vp)]
    lib.rsm_prepared_name.argtypes = [vp, ctypes.c_char_p, i32]
    lib.rsm_run_prepared.argtypes = [vp, P(vp), vp, vp, vp]
    lib.rsm_prepared_destroy.argtypes = [vp]
    lib.rsm_prepared_destroy.restype = None
    lib.rsm_plan_cache_hits.argtypes = []
    lib.rsm_plan_cache_hits.restype = ctypes.c_uint64
    lib.rsm_indices.argtypes = [P(Space), P(Tiler), vp, vp]
    lib.rsm_run.argtypes = [P(Space), P(Tiler), P(vp), i32, P(Tiler), vp, P(Task), u32, vp]
    lib.rsm_run_chain.argtypes = [P(Stage), i32, vp, P(vp), vp, u32, vp]
    lib.rsm_run_adjoint.argtypes = [P(Space), P(Tiler), vp, P(Tiler), vp, P(Task), vp, vp, u32, vp]
    lib.rsm_run_chain_adjoint.argtypes = [P(Stage), i32, vp, P(vp), vp, vp, P(vp), u32, vp]
    lib.rsm_run_csr.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, vp, vp, vp, vp, vp,
                                i32, u32, vp]
    lib.rsm_run_chain_train.argtypes = [P(Stage), i32, vp, vp, vp, vp, P(vp), u32, vp]
    lib.rsm_run_chain_train_noalloc.argtypes = [P(Stage), i32, vp, vp, vp, vp, P(vp), u32, vp]
    lib.rsm_cg_solve.argtypes = [ctypes.c_int64, ctypes.c_int64, vp, vp, vp, vp, vp, ctypes.c_double,
                                 ctypes.c_int64, i32, u32, vp, vp, vp, P(CgInfo), vp]
    lib.rsm_batch_create.argtypes = [P(Problem), i32, ctypes.c_char_p, u32, vp, P(vp)]
    lib.rsm_batch_run.argtypes = [vp, vp]
    lib.rsm_batch_run_plain.argtypes = [vp, vp]
    lib.rsm_batch_query.argtypes = [vp, P(BatchInfo)]
    lib.rsm_batch_tile.argtypes = [vp, i32, P(i32), P(i32)]
    lib.rsm_batch_destroy.argtypes = [vp]
    for name in ("rsm_validate", "rsm_plan", "rsm_plan_ports", "rsm_indices", "rsm_run", "rsm_run_chain",
                 "rsm_run_adjoint", "rsm_run_chain_adjoint", "rsm_batch_create", "rsm_batch_run",
                 "rsm_run_csr", "rsm_cg_solve", "rsm_run_chain_train", "rsm_run_chain_train_noalloc",
                 "rsm_plan_placed", "rsm_run_placed", "rsm_prepare", "rsm_prepared_name", "rsm_run_prepared",
                 "rsm_batch_run_plain", "rsm_batch_query", "rsm_batch_tile", "rsm_batch_destroy"):
        getattr(lib, name).restype = st
    lib.rsm_time_next_kernel.argtypes = [vp, vp]
    lib.rsm_time_next_kernel.restype = st
    lib.rsm_status_string.argtypes = [st]
    lib.rsm_status_string.restype = ctypes.c_char_p
    lib.rsm_last_error.argtypes = []
    lib.rsm_last_error.restype = ctypes.c_char_p
    lib.rsm_abi_version.argtypes = []
    lib.rsm_abi_version.restype = i32
    if path == LIB_PATH:
        _lib = lib
    return lib
