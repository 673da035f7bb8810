"""Parity at the measured workloads' full sizes, in the configuration
bench.py times: sampled rows are checked one by one against the oracle's
exact float64 kNN over all points, and the tree against properties that
hold at any size."""
import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_2507_14261_amd as F

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _sample_rows(n, m, seed):
    return np.sort(np.random.default_rng(seed).choice(n, size=m, replace=False))


def test_gamma_int_1m_d128_sampled_knn_and_tree():
    print("case gamma-int n=1e6 d=128 k=20 lambda=10", flush=True)
    X = datagen.gamma_int(n=1_000_000, d=128, seed=0)
    Xd = torch.from_numpy(X).to(DEV)
    k, lam = 20, 10
    out_b = F.famst(Xd, k, lam, seed=0, precision="bf16", exact=False, with_stats=True)
    out_f = F.famst(Xd, k, lam, seed=0, precision="fp32", exact=True)
    torch.cuda.synchronize()
    rows = _sample_rows(len(X), 48, 3)
    ref_n, ref_s = oracle.knn_exact(X, k, rows=rows, block=16)
    for out in (out_b, out_f):
        nb = out.nbr[torch.from_numpy(rows).to(DEV)].cpu().numpy()
        ds = out.dist[torch.from_numpy(rows).to(DEV)].cpu().numpy()
        for i in range(len(rows)):
            assert set(nb[i].tolist()) == set(ref_n[i].tolist()), rows[i]
        # integer data: squared distances are exact integers in float32
        np.testing.assert_array_equal(np.sort(ds.astype(np.float64) ** 2, axis=1).round(), np.sort(ref_s, axis=1))
    # integer data: bf16 screening is exact, so both paths give the same bits
    assert torch.equal(out_b.nbr, out_f.nbr) and torch.equal(out_b.dist, out_f.dist)
    assert torch.equal(out_b.tu, out_f.tu) and torch.equal(out_b.W, out_f.W)
    assert out_b.knn_stats["uncertified"] == 0
    # spanning tree: n - 1 edges, (min, max) ordered, weight = sum of its edges
    n = len(X)
    tu, tv, tw = out_b.tu.cpu().numpy(), out_b.tv.cpu().numpy(), out_b.tw.cpu().numpy()
    assert len(tu) == n - 1 and np.all(tu < tv)
    assert np.all(np.diff(tu.astype(np.int64) * n + tv) > 0)
    assert abs(float(out_b.W[0]) - float(np.sum(tw.astype(np.float64)))) <= 1e-6 * float(out_b.W[0])
    parent = np.arange(n)

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x
    for a, b in zip(tu.tolist(), tv.tolist()):
        ra, rb = find(a), find(b)
        assert ra != rb
        parent[max(ra, rb)] = min(ra, rb)
    # every refined inter-component edge joins the components it was drawn for
    comp = out_b.graph.comp.cpu().numpy()
    E = out_b.E
    assert np.array_equal(comp[E.u.cpu().numpy()], E.a.cpu().numpy())
    assert np.array_equal(comp[E.v.cpu().numpy()], E.b.cpu().numpy())


def test_vmf_100k_subsample_knn_recall_and_weight():
    # the 4M x 96 workload is checked on its stated 100k subsample
    print("case vmf d=96 subsample 100k of 4M, k=16 lambda=8", flush=True)
    n_full = 4_000_000
    idx = datagen.subsample(n_full, 100_000, seed=1)
    X = datagen.vmf(n=n_full, d=96, seed=0)[idx]
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to(DEV)
    out = F.famst(Xd, 16, 8, seed=0, precision="bf16", exact=False, with_stats=True)
    ex = F.famst(Xd, 16, 8, seed=0, precision="fp32", exact=True)
    torch.cuda.synchronize()
    rows = _sample_rows(len(X), 64, 4)
    ref_n, _ = oracle.knn_exact(X, 16, rows=rows, block=64)
    rec = oracle.recall_at_k(out.nbr[torch.from_numpy(rows).to(DEV)].cpu().numpy(), ref_n)
    rec_f = oracle.recall_at_k(ex.nbr[torch.from_numpy(rows).to(DEV)].cpu().numpy(), ref_n)
    print("bf16 recall", rec, "stats", out.knn_stats, "W", float(out.W[0]), float(ex.W[0]))
    assert rec_f == 1.0
    assert rec >= 0.99
    assert abs(float(out.W[0]) - float(ex.W[0])) / float(ex.W[0]) <= 1e-3


def test_lowrank_500k_d960_sampled_knn_all_precisions():
    print("case lowrank n=5e5 d=960 k=20 lambda=10", flush=True)
    X = datagen.lowrank(n=500_000, d=960, seed=0)
    Xd = torch.from_numpy(X).to(DEV)
    k = 20
    res = {}
    for prec, exact in (("bf16", False), ("fp8", False), ("fp32", True)):
        out = F.knn_graph(Xd, k, precision=prec, exact=exact, with_stats=True)
        torch.cuda.synchronize()
        res[prec] = (out[0].cpu().numpy(), out[1].cpu().numpy(), out[2])
        print(prec, "stats", out[2], flush=True)
    rows = _sample_rows(len(X), 32, 5)
    ref_n, ref_s = oracle.knn_exact(X, k, rows=rows, block=16)
    nb, ds, _ = res["fp32"]
    for i, r in enumerate(rows):
        assert set(nb[r].tolist()) == set(ref_n[i].tolist()), r
    np.testing.assert_allclose(np.sort(ds[rows], axis=1), np.sqrt(np.sort(ref_s, axis=1)), rtol=1e-5)
    for prec in ("bf16", "fp8"):
        rec = oracle.recall_at_k(res[prec][0][rows], ref_n)
        print(prec, "recall", rec, flush=True)
        assert rec >= 0.99
