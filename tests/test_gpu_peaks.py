"""The measured-ceiling helpers bench.py reports beside the datasheet peaks
run and give plausible figures (positive, below 1.2x the datasheet)."""
import pytest
import torch

from paper_2507_14261_amd import peaks as P

pytestmark = pytest.mark.gpu

DATASHEET = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_mfma_ceiling(prec):
    t = P.mfma_tflops(prec, 2000)
    print(prec, "TFLOP/s", t, flush=True)
    assert 0.05 * DATASHEET[prec] < t < 1.2 * DATASHEET[prec]


def test_hbm_ceiling():
    c, r = P.hbm_gbps(1 << 28, 3)
    print("copy GB/s", c, "read GB/s", r, flush=True)
    assert 100.0 < c < 9600.0 and 100.0 < r < 9600.0


def test_rejects_bad_arguments():
    lib = P.load()
    import ctypes
    out = ctypes.c_double(0.0)
    sink = torch.zeros(1, device="cuda")
    assert lib.famst_peak_mfma(3, 10, ctypes.c_void_p(sink.data_ptr()), ctypes.byref(out), None) == -1
    assert lib.famst_peak_mfma(1, 0, ctypes.c_void_p(sink.data_ptr()), ctypes.byref(out), None) == -1
