"""Degenerate inputs of the whole pipeline (Alg. 1) on the device: two and
three points, points on a line, identical points, k = n - 1, and batches
holding clouds of two and three points.  Each case is checked against the
oracle's FAMST and against a closed form of the exact tree."""
import math

import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_2507_14261_amd as F

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _spanning(tu, tv, n):
    ds = oracle.DisjointSet(n)
    return len(tu) == n - 1 and all(ds.union(int(a), int(b)) for a, b in zip(tu, tv))


SEEDS = {"two": 0, "three": 3, "line": 7, "identical": 0, "complete": 2}


def _case(name):
    rng = np.random.default_rng(SEEDS[name])
    if name == "two":
        return np.array([[0.5, -1.0, 2.0], [1.5, 1.0, 0.0]], dtype=np.float32), 1, 3, 3.0
    if name == "three":
        X = rng.standard_normal((3, 2)).astype(np.float32)
        dd = [float(np.linalg.norm(X[a].astype(np.float64) - X[b])) for a, b in ((0, 1), (0, 2), (1, 2))]
        return X, 1, 2, sum(dd) - max(dd)
    if name == "line":
        X = rng.standard_normal((700, 1)).astype(np.float32)
        return X, 2, 4, float(X.max()) - float(X.min())
    if name == "identical":
        return np.full((300, 8), 0.75, dtype=np.float32), 5, 3, 0.0
    if name == "complete":
        X = datagen.blobs(n=60, d=5, n_clusters=3, seed=2)
        return X, 59, 3, oracle.prim_exact(X)[3]
    raise ValueError(name)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("name", ["two", "three", "line", "identical", "complete"])
def test_famst_degenerate_single_cloud(name, prec):
    X, k, lam, exact_W = _case(name)
    n = len(X)
    print(f"case {name} n={n} d={X.shape[1]} k={k} lam={lam} prec={prec}", flush=True)
    ref = oracle.famst(X, k, lam, seed=1)
    out = F.famst(_dev(X), k, lam, seed=1, precision=prec, exact=(prec == "fp32"))
    W = float(out.W[0].item())
    print("W", W, "oracle", ref.W, "exact tree", exact_W, flush=True)
    assert _spanning(out.tu.cpu().numpy(), out.tv.cpu().numpy(), n)
    if name == "identical":
        # every distance is a sum of exact zeros
        assert W == 0.0 and ref.W == 0.0
        return
    tol = 1e-5 if prec == "fp32" or n - 1 <= 32 else 1e-3
    assert abs(W - ref.W) <= tol * ref.W
    # the exact tree's weight bounds FAMST's from below; where the kNN graph
    # holds the exact tree (two points, k = 1 on a triangle, k = n - 1) they agree
    assert W >= exact_W * (1 - 1e-5)
    if name in ("two", "three", "complete"):
        assert math.isclose(W, exact_W, rel_tol=1e-5)
    if prec == "fp32":
        assert out.deltas == ref.deltas


def test_famst_batched_tiny_clouds():
    # clouds of 2 and 3 points beside larger ones (k = 1: every larger cloud
    # splits into many components and takes lambda-edges and refinement)
    X, offs = datagen.clouds(n_clouds=5, sizes=[2, 3, 64, 2, 257], d=16, seed=3)
    print("case tiny clouds", np.diff(offs).tolist(), flush=True)
    refs = oracle.famst_batched(X, offs, 1, 3, seed=2)
    out = F.famst(_dev(X), 1, 3, seed=2, precision="fp32", exact=True, offs=offs)
    W = out.W.cpu().numpy()
    tu, tv = out.tu.cpu().numpy(), out.tv.cpu().numpy()
    assert len(tu) == len(X) - 5
    for b, ref in enumerate(refs):
        lo, hi = int(offs[b]), int(offs[b + 1])
        inb = (tu >= lo) & (tu < hi)
        assert np.all((tv[inb] >= lo) & (tv[inb] < hi))
        assert _spanning(tu[inb] - lo, tv[inb] - lo, hi - lo)
        assert abs(float(W[b]) - ref.W) <= 1e-5 * ref.W, (b, float(W[b]), ref.W)
    X64 = X.astype(np.float64)
    assert math.isclose(float(W[0]), float(np.linalg.norm(X64[0] - X64[1])), rel_tol=1e-5)
    assert math.isclose(float(W[3]), float(np.linalg.norm(X64[69] - X64[70])), rel_tol=1e-5)


def test_dense_tree_and_gradient_tiny_clouds():
    # the persistent dense path on clouds of 2, 3 and 17 points: weights,
    # gradients, and the two-point closed form (a unit vector per point)
    X, offs = datagen.clouds(n_clouds=3, sizes=[2, 3, 17], d=5, seed=4)
    print("case dense tiny clouds", np.diff(offs).tolist(), flush=True)
    Xd = _dev(X).requires_grad_(True)
    W = F.MSTWeight.apply(Xd, 1, 1, 0, 10, "fp32", offs, True)
    W.sum().backward()
    g = Xd.grad.cpu().numpy()
    Wh = W.detach().cpu().numpy()
    for b in range(3):
        sl = slice(int(offs[b]), int(offs[b + 1]))
        tu, tv, _, Wr = oracle.prim_exact(X[sl])
        assert math.isclose(float(Wh[b]), Wr, rel_tol=1e-5)
        np.testing.assert_allclose(g[sl], oracle.mst_weight_grad(X[sl], tu, tv), atol=1e-5)
    e = X[0].astype(np.float64) - X[1]
    unit = e / np.linalg.norm(e)
    np.testing.assert_allclose(g[0], unit, atol=1e-6)
    np.testing.assert_allclose(g[1], -unit, atol=1e-6)
