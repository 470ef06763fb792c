"""ctypes declarations of the C ABI in include/pie.h (argument marshalling only).

The library is the in-tree libpie.so built by ``paper_1806_04164_amd.build``.
If torch is importable it is imported first, so that libpie binds to the same
HIP runtime instance that owns torch's device memory and streams.
"""
from __future__ import annotations

import ctypes
import os

try:  # share torch's HIP runtime (same soname) when torch is present
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpie.so")

PIE_OK = 0
PIE_ERR_ARG = -1
PIE_ERR_MESH = -2
PIE_ERR_NONFINITE = -3
PIE_ERR_PRECISION = -4
PIE_ERR_OOM = -5
PIE_ERR_HIP = -6
PIE_ERR_UNSUPPORTED = -7
PIE_WARN_NOT_CONVERGED = 1
PIE_FP32 = 32
PIE_OPT_MATRIX_SHIFTS = 1
PIE_FP64 = 64
PIE_NEAR_SERIAL = 0
PIE_NEAR_FORK_START = 1
PIE_NEAR_FORK_AFTER_AGGREGATE = 2

TQ = dict(NBOX=1, COORDS=2, PARENT=3, PERM=4, BOXPTR=5, NEAR_PTR=6, NEAR_IDX=7,
          IL_PTR=8, IL_SRC=9, IL_OFF=10)
OI = dict(N=1, Q=2, TAU=3, NEAR_BLOCKS=4, NEAR_ENTRIES=5, NEAR_BYTES=6, NBOX_FINEST=7,
          IL_PAIRS=8, INCIDENCES=9, DEVICE_BYTES=10, NEAR_ENTRIES_RWG=11, NEAR_ENTRIES_TRI=12)

# every function declared in include/pie.h
EXPORTS = [
    "pie_last_error", "pie_version", "pie_mesh_create", "pie_mesh_destroy", "pie_mesh_icosphere",
    "pie_mesh_geometry", "pie_mesh_sizes",
    "pie_mesh_edges", "pie_tree_build", "pie_tree_destroy", "pie_tree_query",
    "pie_options_default", "pie_operator_create", "pie_operator_destroy", "pie_operator_info",
    "pie_operator_level", "pie_matvec", "pie_matvec_near", "pie_matvec_far",
    "pie_rhs_planewave", "pie_solve_opts_default", "pie_solve", "pie_precond_apply", "pie_charge", "pie_farfield",
    "pie_profile_enable", "pie_profile_read", "pie_farfield_adjoint",
    "pie_schedule_get", "pie_schedule_set", "pie_autotune",
    "pie_graph_create", "pie_graph_launch", "pie_graph_destroy", "pie_graph_create_batch",
    "pie_solve_noalloc", "pie_batch_create", "pie_batch_matvec", "pie_batch_destroy",
]
STAGES = ["permute", "near", "aggregate", "shift_up", "translate", "receive", "shift_down"]


class pie_options(ctypes.Structure):
    _fields_ = [("version", ctypes.c_int32), ("near_prec", ctypes.c_int32),
                ("far_prec", ctypes.c_int32), ("tau", ctypes.c_int32), ("x", ctypes.c_double),
                ("n_theta", ctypes.c_int32), ("n_phi", ctypes.c_int32),
                ("max_rhs", ctypes.c_int32), ("flags", ctypes.c_int32)]


class pie_schedule(ctypes.Structure):
    _fields_ = [("version", ctypes.c_int32), ("near_fork", ctypes.c_int32),
                ("il_fork", ctypes.c_int32), ("max_chunk", ctypes.c_int32)]


class pie_solve_opts(ctypes.Structure):
    _fields_ = [("version", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("maxit", ctypes.c_int32), ("refine", ctypes.c_int32), ("tol", ctypes.c_double),
                ("inner_tol", ctypes.c_double), ("use_x0", ctypes.c_int32),
                ("adjoint", ctypes.c_int32), ("precond", ctypes.c_int32)]


class pie_solve_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("refinements", ctypes.c_int32),
                ("rel_residual", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run python -m paper_1806_04164_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    pI64, pI32, pD = ctypes.POINTER(I64), ctypes.POINTER(I32), ctypes.POINTER(D)
    sig = {
        "pie_last_error": (ctypes.c_size_t, [ctypes.c_char_p, ctypes.c_size_t]),
        "pie_version": (I32, []),
        "pie_mesh_create": (I32, [P, I64, P, I64, ctypes.POINTER(P)]),
        "pie_mesh_destroy": (None, [P]),
        "pie_mesh_icosphere": (I32, [I32, D, D, ctypes.c_uint64, ctypes.POINTER(P)]),
        "pie_mesh_geometry": (I32, [P, pI64, pI64, P, P]),
        "pie_mesh_sizes": (I32, [P, pI64, pI64]),
        "pie_mesh_edges": (I32, [P, P, P, P]),
        "pie_tree_build": (I32, [P, I32, ctypes.POINTER(P)]),
        "pie_tree_destroy": (None, [P]),
        "pie_tree_query": (I32, [P, I32, I32, pI64, P]),
        "pie_options_default": (None, [ctypes.POINTER(pie_options)]),
        "pie_operator_create": (I32, [P, P, D, ctypes.POINTER(pie_options), P, ctypes.POINTER(P)]),
        "pie_operator_destroy": (None, [P]),
        "pie_operator_info": (I32, [P, I32, pI64]),
        "pie_operator_level": (I32, [P, I32, pD, pD, pD]),
        "pie_matvec": (I32, [P, P, P, I64, I32, P]),
        "pie_matvec_near": (I32, [P, P, P, I64, P]),
        "pie_matvec_far": (I32, [P, P, P, I64, P]),
        "pie_rhs_planewave": (I32, [P, I64, P, P, P, I32, P, P]),
        "pie_solve_opts_default": (None, [ctypes.POINTER(pie_solve_opts)]),
        "pie_solve": (I32, [P, P, P, P, I64, ctypes.POINTER(pie_solve_opts),
                            ctypes.POINTER(pie_solve_info), P]),
        "pie_solve_noalloc": (I32, [P, P, P, P, I64, ctypes.POINTER(pie_solve_opts),
                                    ctypes.POINTER(pie_solve_info), P]),
        "pie_precond_apply": (I32, [P, P, P, I64, P]),
        "pie_charge": (I32, [P, I64, P, P, P, I32, P, P, P, ctypes.POINTER(pie_solve_opts),
                             ctypes.POINTER(pie_solve_info), P]),
        "pie_farfield": (I32, [P, P, I64, P, I64, P, P]),
        "pie_profile_enable": (I32, [P, I32]),
        "pie_profile_read": (I32, [P, P, P]),
        "pie_farfield_adjoint": (I32, [P, P, I64, P, I64, P, P]),
        "pie_schedule_get": (I32, [P, ctypes.POINTER(pie_schedule)]),
        "pie_schedule_set": (I32, [P, ctypes.POINTER(pie_schedule)]),
        "pie_autotune": (I32, [P, P, P, I64, I32, P, ctypes.POINTER(pie_schedule), pD]),
        "pie_graph_create": (I32, [P, P, P, I64, I32, ctypes.POINTER(P)]),
        "pie_graph_launch": (I32, [P, P]),
        "pie_graph_destroy": (None, [P]),
        "pie_batch_create": (I32, [ctypes.POINTER(P), I32, ctypes.POINTER(P)]),
        "pie_batch_matvec": (I32, [P, ctypes.POINTER(P), ctypes.POINTER(P), pI64, I32, P]),
        "pie_batch_destroy": (None, [P]),
        "pie_graph_create_batch": (I32, [ctypes.POINTER(P), I32, ctypes.POINTER(P), ctypes.POINTER(P),
                                         pI64, I32, ctypes.POINTER(P)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


class PieError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"pie status {status}: {msg}")
        self.status = status


def last_error() -> str:
    buf = ctypes.create_string_buffer(1024)
    lib().pie_last_error(buf, 1024)
    return buf.value.decode()


def check(status):
    if status < 0:
        raise PieError(status, last_error())
    return status
