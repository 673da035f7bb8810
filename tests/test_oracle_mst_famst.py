"""Pins for the oracle's tree extraction, the whole FAMST driver and the
tree-weight gradient (CPU only)."""
import itertools
import math

import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import minimum_spanning_tree
from scipy.spatial.distance import cdist

import datagen
import oracle


def _random_graph(n, m, seed, int_weights=False):
    rng = np.random.default_rng(seed)
    eu = list(range(1, n))
    ev = [int(rng.integers(0, i)) for i in range(1, n)]       # a random spanning tree
    eu += rng.integers(0, n, size=m).tolist()
    ev += rng.integers(0, n, size=m).tolist()
    if int_weights:
        w = rng.integers(1, 4, size=len(eu)).astype(np.float64)
    else:
        w = rng.uniform(0.1, 10.0, size=len(eu))
    return np.array(eu), np.array(ev), w


def _scipy_mst_weight(n, lo, hi, w):
    A = sp.coo_matrix((w, (lo, hi)), shape=(n, n)).tocsr()
    return float(minimum_spanning_tree(A).sum())


@pytest.mark.parametrize("seed", range(4))
def test_kruskal_weight_matches_scipy_and_networkx(seed):
    n = 60
    eu, ev, w = _random_graph(n, 200, seed)
    tu, tv, tw, W, spanning = oracle.kruskal(n, eu, ev, w)
    assert spanning and len(tu) == n - 1
    lo, hi, ww = oracle.canonical_edges(eu, ev, w)
    assert math.isclose(W, _scipy_mst_weight(n, lo, hi, ww), rel_tol=1e-12)
    Gx = nx.Graph()
    Gx.add_weighted_edges_from(zip(lo.tolist(), hi.tolist(), ww.tolist()))
    Tx = nx.minimum_spanning_tree(Gx)
    assert math.isclose(W, Tx.size(weight="weight"), rel_tol=1e-12)


def _is_spanning_tree(n, edges):
    ds = oracle.DisjointSet(n)
    return all(ds.union(a, b) for a, b in edges)


@pytest.mark.parametrize("seed", range(6))
def test_kruskal_bruteforce_with_ties(seed):
    # enumerate every spanning tree of a small multigraph-free graph; under the
    # strict order (w, min, max) the minimum tree is the one whose sorted key
    # sequence is lexicographically smallest
    n = 6
    eu, ev, w = _random_graph(n, 8, seed, int_weights=True)
    lo, hi, ww = oracle.canonical_edges(eu, ev, w)
    keys = [(ww[i], lo[i], hi[i]) for i in range(len(lo))]
    best = None
    for sub in itertools.combinations(range(len(keys)), n - 1):
        if _is_spanning_tree(n, [(lo[i], hi[i]) for i in sub]):
            cand = sorted(keys[i] for i in sub)
            if best is None or cand < best:
                best = cand
    tu, tv, tw, W, spanning = oracle.kruskal(n, eu, ev, w)
    got = sorted(zip(tw.tolist(), tu.tolist(), tv.tolist()))
    assert got == [(float(a), int(b), int(c)) for a, b, c in best]


@pytest.mark.parametrize("seed", range(3))
def test_cycle_and_cut_properties(seed):
    n = 30
    eu, ev, w = _random_graph(n, 80, seed)
    tu, tv, tw, W, _ = oracle.kruskal(n, eu, ev, w)
    lo, hi, ww = oracle.canonical_edges(eu, ev, w)
    T = nx.Graph()
    T.add_weighted_edges_from(zip(tu.tolist(), tv.tolist(), tw.tolist()))
    tree = set(zip(tu.tolist(), tv.tolist()))
    for a, b, x in zip(lo.tolist(), hi.tolist(), ww.tolist()):
        if (a, b) in tree:
            # cut property: the tree edge is the lightest across its cut
            T2 = T.copy()
            T2.remove_edge(a, b)
            side = nx.node_connected_component(T2, a)
            for c, dd, y in zip(lo.tolist(), hi.tolist(), ww.tolist()):
                if (c in side) != (dd in side):
                    assert x <= y
        else:
            # cycle property: a non-tree edge is no lighter than the path max
            path = nx.shortest_path(T, a, b)
            pmax = max(T[p][q]["weight"] for p, q in zip(path, path[1:]))
            assert x >= pmax


def test_kruskal_disconnected_reports_forest():
    tu, tv, tw, W, spanning = oracle.kruskal(4, [0, 2], [1, 3], [1.0, 2.0])
    assert not spanning and len(tu) == 2 and W == 3.0


@pytest.mark.parametrize("seed", [0, 1])
def test_prim_matches_scipy_dense(seed):
    X = datagen.blobs(n=400, d=7, n_clusters=3, seed=seed)
    tu, tv, tw, W = oracle.prim_exact(X)
    D = cdist(X.astype(np.float64), X.astype(np.float64))
    assert len(tu) == len(X) - 1
    assert math.isclose(W, float(minimum_spanning_tree(D).sum()), rel_tol=1e-12)


def test_famst_k_full_is_exact_mst():
    X = datagen.blobs(n=120, d=5, n_clusters=3, seed=2)
    r = oracle.famst(X, k=119, lam=5, seed=0)
    assert len(r.comps) == 1 and len(r.E) == 0 and r.spanning
    assert math.isclose(r.W, oracle.prim_exact(X)[3], rel_tol=1e-12)


def test_famst_single_component_is_knn_graph_mst():
    X = datagen.blobs(n=500, d=6, n_clusters=1, seed=4)
    r = oracle.famst(X, k=8, lam=5, seed=0)
    assert len(r.comps) == 1
    n = len(X)
    wmap = {}
    for i in range(n):
        for j, s in zip(r.nbr[i].tolist(), r.sq[i].tolist()):
            wmap[(min(i, j), max(i, j))] = math.sqrt(s)
    keys = list(wmap)
    A = sp.coo_matrix(([wmap[q] for q in keys], ([q[0] for q in keys], [q[1] for q in keys])),
                      shape=(n, n)).tocsr()
    assert math.isclose(r.W, float(minimum_spanning_tree(A).sum()), rel_tol=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_famst_multi_component_properties(seed):
    X = datagen.blobs(n=1500, d=8, n_clusters=6, seed=seed)
    r = oracle.famst(X, k=3, lam=3, seed=seed, max_rounds=50)
    t = len(r.comps)
    assert t >= 2
    assert r.spanning and len(r.tu) == len(X) - 1
    assert r.deltas[-1] == 0
    assert len(r.E) == 3 * t * (t - 1) // 2
    W_exact = oracle.prim_exact(X)[3]
    err = oracle.relative_error(r.W, W_exact)
    assert err >= -1e-12          # an approximate spanning tree is never lighter
    assert err < 0.05


def test_famst_blobs_paper_defaults_small():
    X = datagen.blobs(n=2000, d=32, n_clusters=10, seed=0)
    r = oracle.famst(X, k=10, lam=5, seed=0)
    assert r.spanning
    assert len(r.comps) == 10
    W_exact = oracle.prim_exact(X)[3]
    assert 0 <= oracle.relative_error(r.W, W_exact) < 0.02


def test_batched_equals_per_cloud():
    X, offs = datagen.clouds(n_clouds=3, lo=40, hi=60, d=4, seed=1)
    out = oracle.famst_batched(X, offs, k=4, lam=2, seed=7)
    for b, r in enumerate(out):
        r2 = oracle.famst(X[offs[b]:offs[b + 1]], 4, 2, 7, cloud=b)
        assert r.W == r2.W


# ------------------------------------------------------------- gradient
def test_grad_two_points_unit_vector():
    X = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0]])
    g = oracle.mst_weight_grad(X, [0], [1])
    np.testing.assert_allclose(g, [[-0.6, -0.8, 0.0], [0.6, 0.8, 0.0]])


def test_grad_collinear_interior_zero():
    X = np.array([[0.0, 0.0], [1.0, 0.0], [2.0, 0.0], [3.0, 0.0]])
    tu, tv, tw, W = oracle.prim_exact(X)
    g = oracle.mst_weight_grad(X, tu, tv)
    np.testing.assert_allclose(g, [[-1, 0], [0, 0], [0, 0], [1, 0]], atol=1e-15)


def test_grad_zero_length_edge():
    X = np.array([[1.0, 1.0], [1.0, 1.0]])
    assert np.all(oracle.mst_weight_grad(X, [0], [1]) == 0)


def test_grad_matches_finite_differences_exact_mst():
    X, offs = datagen.clouds(n_clouds=1, sizes=[64], d=8, seed=1)
    tu, tv, _, _ = oracle.prim_exact(X)
    g = oracle.mst_weight_grad(X, tu, tv)
    rng = np.random.default_rng(0)
    coords = [(int(rng.integers(0, 64)), int(rng.integers(0, 8))) for _ in range(40)]
    fd = oracle.fd_grad(lambda Y: oracle.prim_exact(Y)[3], X, coords, h=1e-6)
    np.testing.assert_allclose(fd, [g[i, j] for i, j in coords], atol=1e-6)


def test_grad_matches_finite_differences_famst():
    X, offs = datagen.clouds(n_clouds=1, sizes=[64], d=6, seed=3)
    r = oracle.famst(X, k=5, lam=3, seed=0)
    g = oracle.mst_weight_grad(X, r.tu, r.tv)
    rng = np.random.default_rng(1)
    coords = [(int(rng.integers(0, 64)), int(rng.integers(0, 6))) for _ in range(20)]
    fd = oracle.fd_grad(lambda Y: oracle.famst(Y, k=5, lam=3, seed=0).W, X, coords, h=1e-6)
    np.testing.assert_allclose(fd, [g[i, j] for i, j in coords], atol=1e-6)


def test_recall():
    a = np.array([[1, 2], [0, 2]])
    b = np.array([[2, 1], [0, 3]])
    assert oracle.recall_at_k(a, b) == 0.75


def test_famst_degenerate_inputs_closed_forms():
    # two points: the tree is the one edge
    X2 = np.array([[0.5, -1.0, 2.0], [1.5, 1.0, 0.0]])
    r = oracle.famst(X2, 1, 3)
    assert math.isclose(r.W, 3.0, rel_tol=1e-15) and len(r.tu) == 1
    # three points, k = 1: the 1-NN graph of a triangle is its MST, whose
    # weight is the perimeter minus the longest side
    rng = np.random.default_rng(5)
    for _ in range(20):
        X3 = rng.standard_normal((3, 2))
        dd = [np.linalg.norm(X3[a] - X3[b]) for a, b in ((0, 1), (0, 2), (1, 2))]
        assert math.isclose(oracle.famst(X3, 1, 2).W, sum(dd) - max(dd), rel_tol=1e-12)
    # points on a line: the exact tree joins neighbours in sorted order, so
    # its weight is max - min; FAMST's tree weighs no less
    x = np.random.default_rng(6).standard_normal((400, 1))
    span = float(x.max() - x.min())
    assert math.isclose(oracle.prim_exact(x)[3], span, rel_tol=1e-12)
    r = oracle.famst(x, 2, 4, seed=1)
    assert r.W >= span * (1 - 1e-12) and r.spanning and len(r.tu) == 399
    # identical points: every distance is zero
    r = oracle.famst(np.ones((50, 4)), 3, 2)
    assert r.W == 0.0 and len(r.tu) == 49 and r.spanning


def test_canonical_edges_first_occurrence_and_order():
    # (min, max) keys, self-loops dropped, the first occurrence's weight kept,
    # output in ascending (min, max) order
    lo, hi, w = oracle.canonical_edges([3, 1, 2, 0, 2, 3, 4], [1, 3, 0, 2, 2, 0, 1], [5.0, 7.0, 1.0, 2.0, 9.0, 4.0, 3.0])
    assert lo.tolist() == [0, 0, 1, 1] and hi.tolist() == [2, 3, 3, 4]
    assert w.tolist() == [1.0, 4.0, 5.0, 3.0]
