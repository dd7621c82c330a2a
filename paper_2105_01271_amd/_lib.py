"""ctypes loader for libdsketch.so (the HIP/C-ABI library of this package).

torch is imported first so that the library's libamdhip64 dependency binds to
the HIP runtime torch already loaded (one runtime per process; torch streams
and device pointers are then valid inside the library).  There is no fallback:
if the shared library is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch  # noqa: F401  (must precede the CDLL load, see module docstring)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdsketch.so")

EXPORTED = (
    "dsk_opts_default", "dsk_create", "dsk_destroy", "dsk_set_stream", "dsk_restrict",
    "dsk_project", "dsk_sketch_svd", "dsk_sketch_id", "dsk_power_iter", "dsk_status_string",
    "dsk_timing_enable", "dsk_timing_read", "dsk_conv_restrict_bwd", "dsk_learned_loss_grad",
    "dsk_adam_step", "dsk_sketch_svd_batched", "dsk_autotune", "dsk_sketch_svd_id", "dsk_sketch_svd_sp",
    "dsk_spc_id_err", "dsk_spc_id",
)
DSK_BATCH_GRAPH = 1

DSK_F64, DSK_F32, DSK_BF16, DSK_F16 = 0, 1, 2, 3
DSK_R_INDEX, DSK_R_NN, DSK_R_GLOBAL, DSK_R_LEARNED = 0, 1, 2, 3
DSK_MODE_DEFAULT, DSK_MODE_SPLIT3, DSK_MODE_F32, DSK_MODE_SPLIT6 = 0, 1, 2, 3
FLAG_NAMES = {1: "fallback", 2: "rank_deficient", 4: "nonfinite", 8: "bad_index", 16: "sync_timeout"}


class Restriction(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("s", ctypes.c_int64),
        ("index", ctypes.c_void_p),
        ("ny", ctypes.c_int32), ("nx", ctypes.c_int32),
        ("sy", ctypes.c_int32), ("sx", ctypes.c_int32),
        ("channels", ctypes.c_int32),
        ("w1", ctypes.c_void_p),
        ("w2", ctypes.c_void_p),
    ]


class Problem(ctypes.Structure):
    _fields_ = [
        ("A", ctypes.c_void_p),
        ("dtype", ctypes.c_int32),
        ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("lda", ctypes.c_int64),
        ("k", ctypes.c_int32), ("q", ctypes.c_int32),
        ("R", Restriction),
        ("U", ctypes.c_void_p),
        ("S", ctypes.c_void_p),
        ("V", ctypes.c_void_p),
    ]


class Opts(ctypes.Structure):
    _fields_ = [
        ("p", ctypes.c_int32),
        ("S", ctypes.c_void_p),
        ("ell", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("id_projected", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("refine", ctypes.c_int32),
        ("id_per_step", ctypes.c_int32),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("ell", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("normA_fro2", ctypes.c_double),
        ("normB_fro2", ctypes.c_double),
        ("sigma_tail", ctypes.c_double),
        ("core_sweeps", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


_lib = None
_lock = threading.Lock()


def load():
    """Load and type the library once; raise if it is not built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2105_01271_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        P = ctypes.POINTER
        lib.dsk_opts_default.argtypes = [P(Opts)]
        lib.dsk_opts_default.restype = None
        lib.dsk_create.argtypes = [P(vp), ctypes.c_int, vp]
        lib.dsk_destroy.argtypes = [vp]
        lib.dsk_set_stream.argtypes = [vp, vp]
        lib.dsk_restrict.argtypes = [vp, vp, i32, i64, i64, i64, P(Restriction), vp]
        lib.dsk_project.argtypes = [vp, vp, i32, i64, i64, i64, vp, i32, vp, i32]
        lib.dsk_project_noalloc.argtypes = [vp, vp, i32, i64, i64, i64, vp, i32, vp, i32]
        lib.dsk_sketch_svd.argtypes = [vp, vp, i32, i64, i64, i64, i32, P(Restriction), i32, P(Opts),
                                       vp, vp, vp, P(Info)]
        lib.dsk_sketch_id.argtypes = [vp, vp, i32, i64, i64, i64, i32, P(Restriction), i32, P(Opts),
                                      vp, vp, vp, P(Info)]
        lib.dsk_sketch_svd_sp.argtypes = [vp, vp, i32, i64, i64, i64, i32, P(Restriction), P(Opts),
                                          vp, vp, vp, P(Info)]
        lib.dsk_spc_id_err.argtypes = [vp, vp, i32, i64, i64, i64, P(Restriction), i32, vp, i32, vp, vp]
        lib.dsk_spc_id.argtypes = [vp, vp, i32, i64, i64, i64, i32, i32, P(Restriction), i32, P(Opts),
                                   vp, vp, vp, vp, vp, P(Info)]
        lib.dsk_power_iter.argtypes = [vp, vp, i32, i64, i64, i64, vp, i32, i32, dbl, i32, vp]
        lib.dsk_status_string.argtypes = [ctypes.c_int]
        lib.dsk_status_string.restype = ctypes.c_char_p
        lib.dsk_timing_enable.argtypes = [vp, ctypes.c_int]
        lib.dsk_timing_read.argtypes = [vp, P(ctypes.c_int), P(ctypes.c_double)]
        lib.dsk_conv_restrict_bwd.argtypes = [vp, vp, i32, i64, i64, i64, P(Restriction), vp, vp, vp]
        lib.dsk_learned_loss_grad.argtypes = [vp, vp, i32, i64, i64, i64, P(Restriction), i32, i32, P(dbl),
                                              vp, vp]
        f32 = ctypes.c_float
        lib.dsk_adam_step.argtypes = [vp, vp, vp, vp, vp, i64, f32, f32, f32, f32, i32]
        lib.dsk_sketch_svd_batched.argtypes = [vp, i32, P(Problem), P(Opts), i32, P(i32)]
        lib.dsk_autotune.argtypes = [vp, vp, i32, i64, i64, i64, i32, i32, P(i32), P(f32)]
        lib.dsk_sketch_svd_id.argtypes = [vp, vp, i32, i64, i64, i64, i32, P(Restriction), i32, i32, P(Opts),
                                          vp, vp, vp, vp, vp, vp, P(Info), P(Info)]
        for name in ("dsk_create", "dsk_destroy", "dsk_set_stream", "dsk_restrict", "dsk_project",
                     "dsk_sketch_svd", "dsk_sketch_id", "dsk_power_iter", "dsk_timing_enable",
                     "dsk_timing_read", "dsk_conv_restrict_bwd", "dsk_learned_loss_grad", "dsk_adam_step",
                     "dsk_sketch_svd_batched", "dsk_autotune", "dsk_sketch_svd_id", "dsk_sketch_svd_sp", "dsk_spc_id_err",
                     "dsk_spc_id"):
            getattr(lib, name).restype = ctypes.c_int
        _lib = lib
        return lib


class DskError(RuntimeError):
    def __init__(self, fn: str, status: int):
        msg = load().dsk_status_string(status).decode()
        super().__init__(f"{fn} returned {status}: {msg}")
        self.status = status


def check(fn: str, status: int):
    if status != 0:
        raise DskError(fn, status)
