"""Binding of libfamst_peaks.so (declared in include/famst_peaks.h): measured
matrix-core throughput and HBM bandwidth of the current device, for the
rooflines next to the datasheet peaks.  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

import torch

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfamst_peaks.so")
EXPORTS = ["famst_peak_hbm", "famst_peak_mfma"]
_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(PATH):
            raise RuntimeError(f"{PATH} is missing: build it with `python -m paper_2507_14261_amd.build`")
        lib = ctypes.CDLL(PATH)
        P, D = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
        lib.famst_peak_mfma.restype = ctypes.c_int
        lib.famst_peak_mfma.argtypes = [ctypes.c_int32, ctypes.c_int32, P, D, P]
        lib.famst_peak_hbm.restype = ctypes.c_int
        lib.famst_peak_hbm.argtypes = [P, P, ctypes.c_size_t, ctypes.c_int32, P, D, D, P]
        _lib = lib
    return _lib


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def mfma_tflops(precision: str, iters: int) -> float:
    lib = load()
    code = {"fp32": 0, "bf16": 1, "fp8": 2}[precision]
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")
    out = ctypes.c_double(0.0)
    rc = lib.famst_peak_mfma(code, iters, ctypes.c_void_p(sink.data_ptr()), ctypes.byref(out), _stream())
    if rc != 0:
        raise RuntimeError(f"famst_peak_mfma({precision}) returned {rc}")
    return out.value


def hbm_gbps(nbytes: int, reps: int):
    """(copy GB/s counting bytes read + written, read-only GB/s)."""
    lib = load()
    src = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")
    c, r = ctypes.c_double(0.0), ctypes.c_double(0.0)
    rc = lib.famst_peak_hbm(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nbytes, reps,
                            ctypes.c_void_p(sink.data_ptr()), ctypes.byref(c), ctypes.byref(r), _stream())
    if rc != 0:
        raise RuntimeError(f"famst_peak_hbm returned {rc}")
    return c.value, r.value
