"""Every entry point stays inside the workspace it asked for: the binding's
workspace allocation is wrapped so that a guard band of known bytes follows
the reported size, and the band is checked after each call.  A write past
the reported size would land in whatever the caller placed next."""
import ctypes

import numpy as np
import pytest
import torch

import datagen
import paper_2507_14261_amd as F
from paper_2507_14261_amd import _lib as L
from paper_2507_14261_amd import api as A

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GUARD = 1 << 16
PATTERN = 0xA5


@pytest.fixture
def guarded(monkeypatch):
    calls = []

    def _workspace(fn, *args):
        sz = ctypes.c_size_t(0)
        L.check(fn(*args, None, ctypes.byref(sz), A._stream()), fn.__name__ + " (size query)")
        m = max(int(sz.value), 256)
        buf = torch.empty(m + GUARD, dtype=torch.uint8, device=DEV)
        buf[m:].fill_(PATTERN)
        code = fn(*args, A._ptr(buf), ctypes.byref(sz), A._stream())
        torch.cuda.synchronize()
        bad = int((buf[m:] != PATTERN).sum().item())
        calls.append((fn.__name__, m, bad))
        return code, buf[:m]

    monkeypatch.setattr(A, "_workspace", _workspace)
    return calls


def _check(calls):
    assert calls
    for name, m, bad in calls:
        assert bad == 0, f"{name} wrote {bad} bytes past its {m}-byte workspace"


@pytest.mark.parametrize("n,d,prec", [(100, 4, "fp32"), (100, 4, "bf16"), (100, 4, "fp8"),
                                      (3000, 200, "bf16"), (3000, 100, "fp32"), (2000, 300, "fp8"),
                                      (33000, 64, "bf16"), (33000, 64, "fp32"), (33000, 200, "bf16"),
                                      (33000, 100, "fp8"), (33000, 960, "bf16")])
def test_knn_graph_stays_in_workspace(guarded, n, d, prec):
    print(f"case n={n} d={d} {prec}", flush=True)
    X = torch.from_numpy(datagen.blobs(n=n, d=d, n_clusters=8, seed=n + d)).to(DEV)
    for exact in (False, True):
        F.knn_graph(X, 5, precision=prec, exact=exact)
    _check(guarded)


def test_many_component_pipeline_stays_in_workspace(guarded):
    # k = 1: hundreds of components, over 32768 lambda-edges (group-per-edge
    # refinement with change flags and compaction, 64-slot lambda sampling)
    X = torch.from_numpy(datagen.blobs(n=3000, d=32, n_clusters=10, seed=9)).to(DEV)
    out = F.famst(X, 1, 5, seed=0, precision="fp32")
    print("components", out.graph.n_comp, "edges", len(out.E), flush=True)
    assert len(out.E) >= 32768
    _check(guarded)


def test_pipeline_entry_points_stay_in_workspace(guarded):
    X = torch.from_numpy(datagen.blobs(n=3000, d=32, n_clusters=10, seed=5)).to(DEV)
    F.famst(X, 10, 5, seed=0, precision="bf16")
    Xg = X[:800].clone().requires_grad_(True)
    F.MSTWeight.apply(Xg, 8, 3, 0).sum().backward()
    Xc, offs = datagen.clouds(n_clouds=5, lo=40, hi=200, d=16, seed=2)
    Xc = torch.from_numpy(Xc).to(DEV)
    F.mst(Xc, algo="prim", offs=offs)
    F.mst_dense_fused(Xc, offs=offs)
    names = {c[0] for c in guarded}
    print("entry points checked", sorted(names), flush=True)
    assert {"famst_knn_graph", "famst_connect", "famst_refine", "famst_mst", "famst_mst_backward",
            "famst_mst_dense_fused"} <= names
    _check(guarded)
