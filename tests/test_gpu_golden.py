"""Whole-pipeline parity at the measured workloads: the tree weight W,
component count t, lambda-edge count and refinement deltas of the GPU
pipeline against the oracle's FAMST on the same input, as stored in
tests/golden/oracle_weights.json by tests/golden/make_oracle_weights.py
(which calls only the oracle).  The float32 exact path must give the
oracle's t, |E| and delta sequence and W within 1e-5 relative; the bf16 and
fp8 screened paths with float32 re-rank W within 1e-3 relative, the relative
error of Eq. (1) being reported against the oracle."""
import json
import os

import numpy as np
import pytest
import torch

import datagen
import paper_2507_14261_amd as F

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_weights.json")
_DATA = json.load(open(GOLDEN)) if os.path.exists(GOLDEN) else {}


def _golden(name):
    if name not in _DATA:
        pytest.skip(f"{name}: no stored oracle result")
    return _DATA[name]


def _input(name):
    if name == "blobs-10k-d32":
        return datagen.blobs(n=10_000, d=32, seed=0)
    if name == "gamma-int-1m-d128":
        return datagen.gamma_int(n=1_000_000, d=128, seed=0)
    if name == "vmf-4m-d96-sub100k":
        idx = datagen.subsample(4_000_000, 100_000, seed=1)
        return np.ascontiguousarray(datagen.vmf(n=4_000_000, d=96, seed=0)[idx])
    if name == "lowrank-500k-d960-sub50k":
        idx = datagen.subsample(500_000, 50_000, seed=1)
        return np.ascontiguousarray(datagen.lowrank(n=500_000, d=960, seed=0)[idx])
    raise KeyError(name)


def _rel(a, b):
    return (a - b) / b


# (workload, [(precision, exact mode, bound on |W - W_oracle| / W_oracle)])
CASES = [
    ("blobs-10k-d32", [("fp32", True, 1e-5), ("bf16", False, 1e-3), ("fp8", False, 1e-3)]),
    ("vmf-4m-d96-sub100k", [("fp32", True, 1e-5), ("bf16", False, 1e-3), ("fp8", False, 1e-3)]),
    ("lowrank-500k-d960-sub50k", [("fp32", True, 1e-5), ("bf16", False, 1e-3), ("fp8", False, 1e-3)]),
    ("gamma-int-1m-d128", [("fp32", True, 1e-5), ("bf16", False, 1e-5), ("fp8", False, 1e-3)]),
]


@pytest.mark.parametrize("name,runs", CASES, ids=[c[0] for c in CASES])
def test_pipeline_weight_against_oracle(name, runs):
    g = _golden(name)
    print(f"case {name} n={g['n']} d={g['d']} k={g['k']} lambda={g['lam']}", flush=True)
    X = _input(name)
    assert X.shape == (g["n"], g["d"])
    Xd = torch.from_numpy(X).to(DEV)
    for prec, exact, bound in runs:
        out = F.famst(Xd, g["k"], g["lam"], seed=g["seed"], max_rounds=g["max_rounds"], precision=prec,
                      exact=exact, with_stats=True)
        torch.cuda.synchronize()
        W = float(out.W[0])
        rel = _rel(W, g["W"])
        extra = f" vs exact tree {_rel(W, g['W_exact']):.3e}" if "W_exact" in g else ""
        print(f"  {prec}{' exact' if exact else ''}: W={W!r} oracle={g['W']!r} rel={rel:.3e}{extra} "
              f"t={out.graph.n_comp[0]} |E|={len(out.E)} deltas={out.deltas} stats={out.knn_stats}", flush=True)
        assert abs(rel) <= bound, (prec, rel)
        if exact:
            assert out.graph.n_comp[0] == g["t"]
            assert len(out.E) == g["n_edges"]
            assert out.deltas == g["deltas"] and out.rounds == g["rounds"]
        assert out.tu.numel() == g["n"] - 1


def _clouds():
    g = _golden("clouds-256-d64")
    X, offs = datagen.clouds(n_clouds=256, d=64, seed=0)
    assert len(X) == g["n"]
    return g, X, offs


def test_clouds_k16_per_cloud_weight_against_oracle():
    # the batched k = 16 path: every cloud's W, t, |E| and deltas against the
    # oracle run on that cloud alone (its cloud index in the edge counters)
    g, X, offs = _clouds()
    print(f"case clouds-256-d64 k={g['k']} lambda={g['lam']}", flush=True)
    Xd = torch.from_numpy(X).to(DEV)
    out = F.famst(Xd, g["k"], g["lam"], seed=g["seed"], max_rounds=g["max_rounds"], precision="fp32",
                  exact=True, offs=offs)
    torch.cuda.synchronize()
    W = out.W.cpu().numpy().astype(np.float64)
    rel = np.abs(W - np.array(g["W"])) / np.array(g["W"])
    print(f"  max rel {rel.max():.3e}; vs exact trees mean {np.mean((W - g['W_exact']) / g['W_exact']):.3e}",
          flush=True)
    assert rel.max() <= 1e-5
    assert out.graph.n_comp == g["t"]
    assert len(out.E) == sum(g["n_edges"])
    # rounds run on the whole batch: as many as the slowest cloud, and each
    # round changes as many edges as the clouds' own rounds summed
    R = max(g["rounds"])
    want = [sum(dl[r] if r < len(dl) else 0 for dl in g["deltas"]) for r in range(R)]
    assert out.deltas == want


def test_clouds_dense_fused_exact_weights_against_oracle():
    # the persistent exact path on all 256 clouds (sizes 512..8192, d = 64):
    # every cloud's W against the oracle's float64 Prim
    g, X, offs = _clouds()
    print("case clouds-256-d64 dense fused", flush=True)
    Xd = torch.from_numpy(X).to(DEV)
    tu, tv, tw, W, G = F.mst_dense_fused(Xd, offs=offs)
    torch.cuda.synchronize()
    W = W.cpu().numpy().astype(np.float64)
    rel = np.abs(W - np.array(g["W_exact"])) / np.array(g["W_exact"])
    print(f"  max rel {rel.max():.3e}", flush=True)
    assert rel.max() <= 1e-5


def test_dense_fused_tree_and_gradient_at_cloud_shape():
    # clouds of the batched workload's shape (d = 64, 512 to 8192 points):
    # the persistent launch's tree, weight and gradient against the oracle's
    # float64 Prim tree and its closed-form gradient
    import oracle
    sizes = np.array([8192, 512, 2048, 5001])
    X, offs = datagen.clouds(d=64, sizes=sizes, seed=7)
    print(f"case dense fused sizes={sizes.tolist()} d=64", flush=True)
    Xd = torch.from_numpy(X).to(DEV)
    tu, tv, tw, W, G = F.mst_dense_fused(Xd, offs=offs)
    torch.cuda.synchronize()
    tu, tv, W, G = tu.cpu().numpy(), tv.cpu().numpy(), W.cpu().numpy(), G.cpu().numpy()
    e0 = 0
    for b, m in enumerate(sizes.tolist()):
        sl = slice(int(offs[b]), int(offs[b + 1]))
        ru, rv, rw, RW = oracle.prim_exact(X[sl])
        gu, gv = tu[e0:e0 + m - 1] - offs[b], tv[e0:e0 + m - 1] - offs[b]
        e0 += m - 1
        got = set(zip(np.minimum(gu, gv).tolist(), np.maximum(gu, gv).tolist()))
        ref = set(zip(np.minimum(ru, rv).tolist(), np.maximum(ru, rv).tolist()))
        assert got == ref, b
        assert abs(float(W[b]) - RW) / RW <= 1e-5
        g_ref = oracle.mst_weight_grad(X[sl], ru, rv)
        err = float(np.abs(G[sl] - g_ref).max())
        print(f"  cloud {b} n={m}: W rel {(float(W[b]) - RW) / RW:.2e}, grad max abs err {err:.2e}", flush=True)
        assert err <= 1e-4
