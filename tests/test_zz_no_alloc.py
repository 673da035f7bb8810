"""The allocation-free gradient entry point against famst_mst_backward: the
same kernels on the library's fixed scratch array must give the same bits,
call after call, with the scratch keeping the previous call's contents."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2507_14261_amd as F
from paper_2507_14261_amd import _lib as L

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _random_forest(sizes, d, seed):
    """Clouds of the given sizes with a random spanning tree in each (edge
    v -> a random earlier vertex of its cloud), as famst_mst lays them out."""
    rng = np.random.default_rng(seed)
    offs = np.zeros(len(sizes) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(sizes)
    X = rng.standard_normal((int(offs[-1]), d)).astype(np.float32)
    tu, tv = [], []
    for b, m in enumerate(sizes):
        o = int(offs[b])
        for v in range(1, int(m)):
            p = int(rng.integers(0, v))
            tu.append(o + min(p, v)), tv.append(o + max(p, v))
    X[int(offs[1]) - 1] = X[int(offs[1]) - 2]           # one zero-length edge candidate
    t = lambda a: torch.tensor(a, dtype=torch.int32, device=DEV)
    return torch.from_numpy(X).to(DEV), t(tu), t(tv), offs


@pytest.mark.parametrize("d", [64, 37])
def test_noalloc_equals_workspace_entry_point_two_calls(d):
    # two calls in a row, the second smaller: the scratch keeps the first
    # call's (larger) contents, which the second must not depend on
    for sizes, seed in (([40000, 513, 2, 9000], 1), ([3000, 17], 2)):
        print(f"case noalloc d={d} sizes={sizes}", flush=True)
        X, tu, tv, offs = _random_forest(sizes, d, seed)
        gW = torch.linspace(0.5, 2.0, len(sizes), device=DEV, dtype=torch.float32)
        ref = F.mst_backward(X, tu, tv, gW, offs=offs)
        got, need = F.mst_backward_noalloc(X, tu, tv, gW, offs=offs)
        torch.cuda.synchronize()
        assert 0 < need <= L.FAMST_NOALLOC_SCRATCH_BYTES
        assert torch.equal(got, ref)


def test_noalloc_single_cloud_and_preallocated_output():
    X, tu, tv, _ = _random_forest([20000], 96, 3)
    gW = torch.ones(1, device=DEV)
    ref = F.mst_backward(X, tu, tv, gW)
    out = torch.full_like(X, float("nan"))
    got, _ = F.mst_backward_noalloc(X, tu, tv, gW, grad=out)
    torch.cuda.synchronize()
    assert got.data_ptr() == out.data_ptr() and torch.equal(out, ref)


def test_noalloc_rejects_beyond_its_scratch():
    # a call that needs more than the fixed array returns ECAPACITY with the
    # size it needs, and queues nothing (the output keeps its contents)
    n = 2_000_000
    X = torch.zeros((n, 1), device=DEV)
    tu = torch.zeros(n - 1, dtype=torch.int32, device=DEV)
    tv = torch.arange(1, n, dtype=torch.int32, device=DEV)
    gW = torch.ones(1, device=DEV)
    grad = torch.full_like(X, 7.0)
    need = ctypes.c_size_t(0)
    lib = L.load()
    code = lib.famst_mst_backward_noalloc(ctypes.c_void_p(X.data_ptr()), n, 1, None, 1,
                                          ctypes.c_void_p(tu.data_ptr()), ctypes.c_void_p(tv.data_ptr()),
                                          ctypes.c_void_p(gW.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                                          ctypes.byref(need), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert code == L.FAMST_ECAPACITY
    assert need.value > L.FAMST_NOALLOC_SCRATCH_BYTES
    assert bool(torch.all(grad == 7.0))
