"""ctypes declarations of the C ABI in include/hopf.h (libhopf.so, built in-tree).

Loading fails loudly if the library has not been built: there is no fallback
implementation of any step of the solver in Python.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhopf.so")

HOPF_OK, HOPF_EINVAL, HOPF_ENOTSPD, HOPF_ENOMEM, HOPF_EDEVICE = 0, -1, -2, -3, -4
HKIND = {"wl1": 0, "l2": 1, "l2_wl1": 2, "wl2": 3, "al2": 4, "linf": 5, "linctrl": 6}
JKIND = {"quad": 0, "l1sq": 1, "linfsq": 2}
PRECISION = {"f64": 0, "f32": 1, "bf16_refined": 2}

# every symbol include/hopf.h declares
EXPORTS = [
    "hopf_problem_create", "hopf_problem_create_batch", "hopf_problem_destroy", "hopf_eval",
    "hopf_closest_point", "hopf_eval_ragged", "hopf_backward", "hopf_problem_get_inverse",
    "hopf_problem_info", "hopf_last_error", "hopf_version", "hopf_control", "hopf_max_over_hamiltonians",
    "hopf_backward_noalloc", "hopf_problem_iterations", "hopf_closest_point_ragged",
    "hopf_ragged_plan_create", "hopf_ragged_plan_launch", "hopf_ragged_plan_destroy",
    "hopf_set_deterministic", "hopf_get_deterministic",
]


class HopfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("hopf status %d: %s" % (status, msg))
        self.status = status


class ProblemDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("A", ctypes.c_void_p), ("A_is_diagonal", ctypes.c_int32),
        ("K", ctypes.c_int32), ("centres", ctypes.c_void_p), ("level_set", ctypes.c_int32),
        ("hkind", ctypes.c_int), ("w", ctypes.c_void_p), ("lam", ctypes.c_double),
        ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("precision", ctypes.c_int),
        ("HA", ctypes.c_void_p), ("jkind", ctypes.c_int32), ("drift", ctypes.c_void_p),
    ]


_lib = None


def load():
    """Load libhopf.so and declare the signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhopf.so is not built (run `python -m paper_1605_01799_amd.build` or "
                          "`__graft_entry__.build()`); there is no fallback path")
    lib = ctypes.CDLL(LIB_PATH)
    V, I32, I64, D, P = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    pdesc = ctypes.POINTER(ProblemDesc)
    sig = {
        "hopf_problem_create": [pdesc, V, ctypes.POINTER(P)],
        "hopf_problem_create_batch": [I32, pdesc, V, ctypes.POINTER(P)],
        "hopf_problem_destroy": [P],
        "hopf_eval": [P, I64, V, V, V, V, V, V, V, V],
        "hopf_closest_point": [P, I64, V, D, V, V, V, V, V, V],
        "hopf_eval_ragged": [I32, ctypes.POINTER(P), ctypes.POINTER(I64), V, V, V, V, V, V, V, V],
        "hopf_closest_point_ragged": [I32, ctypes.POINTER(P), ctypes.POINTER(I64), V, D, V, V, V, V, V, V],
        "hopf_ragged_plan_create": [I32, ctypes.POINTER(P), ctypes.POINTER(I64), V, V, V, V, V, V, V,
                                    ctypes.POINTER(P)],
        "hopf_ragged_plan_launch": [P, V],
        "hopf_ragged_plan_destroy": [P],
        "hopf_backward": [P, I64, V, V, V, V, V, V, V, V, V],
        "hopf_backward_noalloc": [P, I64, V, V, V, V, V, V, V, V, V],
        "hopf_control": [P, I64, V, V, V, V, V, V, V],
        "hopf_max_over_hamiltonians": [I32, I64, I32, I32, ctypes.POINTER(V), ctypes.POINTER(V),
                                       ctypes.POINTER(V), V, V, V, V, V],
        "hopf_problem_get_inverse": [P, V],
        "hopf_problem_iterations": [P, ctypes.POINTER(I64), I32],
        "hopf_problem_info": [P, V, V, V, V],
        "hopf_set_deterministic": [I32],
        "hopf_get_deterministic": [],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.hopf_last_error.restype = ctypes.c_char_p
    lib.hopf_last_error.argtypes = []
    lib.hopf_version.restype = ctypes.c_char_p
    lib.hopf_version.argtypes = []
    _lib = lib
    return lib


def check(status):
    if status != HOPF_OK:
        raise HopfError(status, load().hopf_last_error().decode())
