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


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def test_undersized_or_misaligned_workspace_is_rejected():
    # EWORKSPACE before any work is queued: outputs keep their contents
    lib = L.load()
    X = torch.from_numpy(datagen.blobs(n=600, d=16, seed=2)).to(DEV)
    n, d, k = 600, 16, 5
    nbr = torch.full((n, k), -7, dtype=torch.int32, device=DEV)
    dist = torch.full((n, k), -7.0, device=DEV)
    sz = ctypes.c_size_t(0)
    s = A._stream()
    assert lib.famst_knn_graph(_p(X), n, d, None, 1, k, L.FAMST_FP32, 0, _p(nbr), _p(dist), None, None,
                               ctypes.byref(sz), s) == L.FAMST_OK
    need = sz.value
    ws = torch.empty(need + 512, dtype=torch.uint8, device=DEV)
    small = ctypes.c_size_t(need - 256)
    assert lib.famst_knn_graph(_p(X), n, d, None, 1, k, L.FAMST_FP32, 0, _p(nbr), _p(dist), None, _p(ws),
                               ctypes.byref(small), s) == L.FAMST_EWORKSPACE
    full = ctypes.c_size_t(need + 256)
    off = ctypes.c_void_p(ws.data_ptr() + 16)   # not 256-byte aligned
    assert lib.famst_knn_graph(_p(X), n, d, None, 1, k, L.FAMST_FP32, 0, _p(nbr), _p(dist), None, off,
                               ctypes.byref(full), s) == L.FAMST_EWORKSPACE
    torch.cuda.synchronize()
    assert bool(torch.all(nbr == -7)) and bool(torch.all(dist == -7.0))


def test_connect_capacity_reports_required_size_and_keeps_labels():
    # e_cap below lambda * t (t - 1) / 2: ECAPACITY, the required count in
    # n_edges, graph and components complete, E untouched
    lib = L.load()
    X = datagen.blobs(n=3000, d=32, n_clusters=10, seed=0)
    Xd = torch.from_numpy(X).to(DEV)
    k, lam = 2, 4
    nbr, _ = F.knn_graph(Xd, k, precision="fp32", exact=True)
    G_ref, E_ref = F.connect(Xd, nbr, lam, 3)
    t = G_ref.n_comp[0]
    need_edges = lam * t * (t - 1) // 2
    assert t > 2 and len(E_ref) == need_edges
    n = len(X)
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device=DEV)
    col = torch.empty(2 * n * k, dtype=torch.int32, device=DEV)
    comp = torch.full((n,), -1, dtype=torch.int32, device=DEV)
    members = torch.empty(n, dtype=torch.int32, device=DEV)
    comp_ptr = torch.empty(n + 1, dtype=torch.int64, device=DEV)
    cap = need_edges - 1
    eu = torch.full((cap,), -9, dtype=torch.int32, device=DEV)
    ev, ea, eb = (torch.full((cap,), -9, dtype=torch.int32, device=DEV) for _ in range(3))
    ew = torch.full((cap,), -9.0, device=DEV)
    n_col, n_edges = ctypes.c_int64(0), ctypes.c_int64(0)
    n_comp = (ctypes.c_int32 * 1)()
    args = [_p(Xd), n, 32, None, 1, _p(nbr), k, lam, ctypes.c_uint64(3), _p(row_ptr), _p(col), ctypes.byref(n_col),
            _p(comp), _p(members), _p(comp_ptr), n_comp, _p(eu), _p(ev), _p(ew), _p(ea), _p(eb), cap,
            ctypes.byref(n_edges)]
    sz = ctypes.c_size_t(0)
    assert lib.famst_connect(*args, None, ctypes.byref(sz), A._stream()) == L.FAMST_OK
    ws = torch.empty(max(sz.value, 256), dtype=torch.uint8, device=DEV)
    code = lib.famst_connect(*args, _p(ws), ctypes.byref(sz), A._stream())
    torch.cuda.synchronize()
    assert code == L.FAMST_ECAPACITY
    assert n_edges.value == need_edges and n_comp[0] == t
    assert torch.equal(comp, G_ref.comp) and n_col.value == G_ref.col.numel()
    assert torch.equal(row_ptr, G_ref.row_ptr) and torch.equal(col[:n_col.value], G_ref.col)
    assert bool(torch.all(eu == -9)) and bool(torch.all(ew == -9.0))


def test_dense_fused_smaller_workspace_runs_cloud_groups():
    """d <= 64: the size query covers every cloud's pair matrix; a workspace
    that holds only the largest matrix (plus the fixed part) runs the clouds
    in consecutive groups with the same results, and one byte less is
    rejected."""
    lib = L.load()
    X, offs = datagen.clouds(n_clouds=9, lo=100, hi=700, d=64, seed=12)
    n, d, B = X.shape[0], X.shape[1], len(offs) - 1
    Xd = torch.from_numpy(X).to(DEV)
    ref = F.mst_dense_fused(Xd, offs=offs)
    torch.cuda.synchronize()
    sizes = np.diff(offs)
    o = np.ascontiguousarray(offs, dtype=np.int64)
    op = o.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    outs = [torch.empty(n - B, dtype=torch.int32, device=DEV), torch.empty(n - B, dtype=torch.int32, device=DEV),
            torch.empty(n - B, device=DEV), torch.empty(B, device=DEV), torch.empty_like(Xd)]
    s = A._stream()
    sz = ctypes.c_size_t(0)
    assert lib.famst_mst_dense_fused(_p(Xd), n, d, op, B, *[_p(t) for t in outs], None, ctypes.byref(sz), s) == 0
    full = sz.value
    mat = int((sizes.astype(np.int64) ** 2).sum()) * 4
    fixed = full - ((mat + 255) // 256) * 256
    small = fixed + int(sizes.max()) ** 2 * 4
    print("workspace full", full, "smallest accepted", small, flush=True)
    assert small < full // 2
    ws = torch.empty(full, dtype=torch.uint8, device=DEV)
    short = ctypes.c_size_t(small - 1)
    assert lib.famst_mst_dense_fused(_p(Xd), n, d, op, B, *[_p(t) for t in outs], _p(ws), ctypes.byref(short),
                                     s) == L.FAMST_EWORKSPACE
    for w in (small, small + 3 * 700 * 700):
        for t in outs:
            t.fill_(-5)
        ws_sz = ctypes.c_size_t(w)
        assert lib.famst_mst_dense_fused(_p(Xd), n, d, op, B, *[_p(t) for t in outs], _p(ws), ctypes.byref(ws_sz),
                                         s) == 0
        torch.cuda.synchronize()
        for a, b in zip(outs, ref):
            assert torch.equal(a, b)
