"""ctypes loader for libfamst.so (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfamst.so")

FAMST_OK = 0
FAMST_EINVAL = -1
FAMST_ECAPACITY = -2
FAMST_EDISCONNECTED = -3
FAMST_EHIP = -4
FAMST_ENOTIMPL = -5
FAMST_ENONFINITE = -6
FAMST_EWORKSPACE = -7
FAMST_ETIMEOUT = -8
FAMST_WNOTCONVERGED = 1

FAMST_FP32 = 0
FAMST_BF16 = 1
FAMST_FP8_E4M3 = 2
FAMST_EXACT = 0x100
FAMST_NNDESCENT = 0x200

FAMST_BORUVKA = 0
FAMST_KRUSKAL = 1
FAMST_DENSE_PRIM = 2

FAMST_NSTATS = 8
FAMST_NOALLOC_SCRATCH_BYTES = 64 << 20
FAMST_REFINE_MAX_ROUNDS = 4096

EXPORTS = [
    "famst_strerror", "famst_version", "famst_knn_graph", "famst_connect", "famst_refine",
    "famst_mst", "famst_mst_backward", "famst_mst_backward_noalloc", "famst_mst_dense_fused", "famst_profile_enable", "famst_profile_reset",
    "famst_profile_read",
]

_lib = None

P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
U64 = ctypes.c_uint64
PI64 = ctypes.POINTER(ctypes.c_int64)
PI32 = ctypes.POINTER(ctypes.c_int32)
PSZ = ctypes.POINTER(ctypes.c_size_t)
PD = ctypes.POINTER(ctypes.c_double)


class FamstError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


def load():
    """Load the in-tree library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2507_14261_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    lib.famst_strerror.restype = ctypes.c_char_p
    lib.famst_strerror.argtypes = [ctypes.c_int]
    lib.famst_version.restype = ctypes.c_int
    lib.famst_version.argtypes = []
    lib.famst_knn_graph.restype = ctypes.c_int
    lib.famst_knn_graph.argtypes = [P, I64, I32, PI64, I32, I32, I32, I32, P, P, PI64, P, PSZ, P]
    lib.famst_connect.restype = ctypes.c_int
    lib.famst_connect.argtypes = [P, I64, I32, PI64, I32, P, I32, I32, U64, P, P, PI64, P, P, P, PI32,
                                  P, P, P, P, P, I64, PI64, P, PSZ, P]
    lib.famst_refine.restype = ctypes.c_int
    lib.famst_refine.argtypes = [P, I64, I32, P, P, P, P, P, P, P, P, I64, I32, PI32, PI64, P, PSZ, P]
    lib.famst_mst.restype = ctypes.c_int
    lib.famst_mst.argtypes = [P, I64, I32, PI64, I32, P, P, I32, P, P, P, I64, I32, P, P, P, P, P, PSZ, P]
    lib.famst_mst_backward.restype = ctypes.c_int
    lib.famst_mst_backward.argtypes = [P, I64, I32, PI64, I32, P, P, P, P, P, PSZ, P]
    lib.famst_mst_backward_noalloc.restype = ctypes.c_int
    lib.famst_mst_backward_noalloc.argtypes = [P, I64, I32, PI64, I32, P, P, P, P, PSZ, P]
    lib.famst_mst_dense_fused.restype = ctypes.c_int
    lib.famst_mst_dense_fused.argtypes = [P, I64, I32, PI64, I32, P, P, P, P, P, P, PSZ, P]
    lib.famst_profile_enable.restype = ctypes.c_int
    lib.famst_profile_enable.argtypes = [ctypes.c_int]
    lib.famst_profile_reset.restype = ctypes.c_int
    lib.famst_profile_reset.argtypes = []
    lib.famst_profile_read.restype = ctypes.c_int
    lib.famst_profile_read.argtypes = [ctypes.c_char_p, PI64, PD]
    _lib = lib
    return lib


def strerror(code: int) -> str:
    try:
        return load().famst_strerror(code).decode()
    except Exception:  # library missing: describe the code only
        return f"status {code}"


def check(code: int, where: str, allow=()):
    if code < 0 and code not in allow:
        raise FamstError(code, where)
    return code
