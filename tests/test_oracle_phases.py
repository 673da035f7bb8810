"""Pins for the oracle's Phase 2 and Phase 3 (Alg. 2-4), CPU only."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import datagen
import oracle


def _partition(labels):
    groups = {}
    for v, c in enumerate(labels):
        groups.setdefault(int(c), []).append(v)
    return sorted(tuple(g) for g in groups.values())


@pytest.mark.parametrize("k", [1, 2, 4])
def test_components_match_scipy(k):
    X = datagen.blobs(n=800, d=8, n_clusters=6, seed=k)
    nbr, _ = oracle.knn_exact(X, k)
    G = oracle.undirected_graph(nbr)
    comp, comps = oracle.components(G)
    n = len(X)
    rows = np.repeat(np.arange(n), k)
    A = sp.coo_matrix((np.ones(n * k), (rows, nbr.reshape(-1))), shape=(n, n))
    t, lab = connected_components(A, directed=True, connection="weak")
    assert len(comps) == t
    assert _partition(comp) == _partition(lab)
    # canonical numbering: by ascending minimum vertex, members ascending
    mins = [int(c[0]) for c in comps]
    assert mins == sorted(mins)
    for c in comps:
        assert np.all(np.diff(c) > 0)
    assert comp[0] == 0


def test_undirected_graph_symmetric_sorted():
    nbr = np.array([[1, 2], [0, 2], [0, 1], [0, 1]])
    G = oracle.undirected_graph(nbr)
    assert [g.tolist() for g in G] == [[1, 2, 3], [0, 2, 3], [0, 1], [0, 1]]


def test_undirected_graph_drops_self_loops():
    G = oracle.undirected_graph(np.array([[0], [0]]))
    assert [g.tolist() for g in G] == [[1], [0]]


def _two_line_clusters():
    # two clusters on a line: A = {0..4} at x=0..4, B = {5..9} at x=10..14
    X = np.zeros((10, 2), dtype=np.float32)
    X[:5, 0] = np.arange(5)
    X[5:, 0] = 10 + np.arange(5)
    return X


def test_random_edges_invariants():
    X = datagen.blobs(n=600, d=6, n_clusters=5, seed=4)
    nbr, _ = oracle.knn_exact(X, 2)
    G = oracle.undirected_graph(nbr)
    comp, comps = oracle.components(G)
    t = len(comps)
    assert t >= 3
    lam = 3
    E = oracle.random_edges(X, comps, lam, seed=11)
    assert len(E) == lam * t * (t - 1) // 2
    X64 = oracle.as64(X)
    key = oracle.seed_key(11)
    e = 0
    for a in range(t - 1):
        for b in range(a + 1, t):
            kept = E.s[e:e + lam]
            assert np.all(E.a[e:e + lam] == a) and np.all(E.b[e:e + lam] == b)
            assert np.all(comp[E.u[e:e + lam]] == a) and np.all(comp[E.v[e:e + lam]] == b)
            assert np.all(np.diff(kept) >= 0)
            # regenerate all lambda^2 samples directly from the generator
            allv = []
            for smp in range(lam * lam):
                r = oracle.philox4x32_10((a, b, smp, 0), key)
                u = comps[a][oracle.uniform_index(r[0], len(comps[a]))]
                v = comps[b][oracle.uniform_index(r[1], len(comps[b]))]
                d = X64[u] - X64[v]
                allv.append(float(d @ d))
            allv = np.sort(allv)
            np.testing.assert_allclose(kept, allv[:lam], rtol=1e-13)
            assert kept.max() <= allv[lam] * (1 + 1e-13) if lam < len(allv) else True
            e += lam
    assert e == len(E)


def test_random_edges_single_component_empty():
    X = datagen.blobs(n=50, d=3, n_clusters=1, seed=0)
    E = oracle.random_edges(X, [np.arange(50)], 5, seed=0)
    assert len(E) == 0


def test_random_edges_stable_ties():
    # every sample has the same length: selection must keep sample order
    X = np.array([[0.0], [0.0], [1.0], [1.0]], dtype=np.float32)
    comps = [np.array([0, 1]), np.array([2, 3])]
    E = oracle.random_edges(X, comps, 2, seed=5)
    key = oracle.seed_key(5)
    expect = []
    for smp in range(2):
        r = oracle.philox4x32_10((0, 1, smp, 0), key)
        expect.append((comps[0][oracle.uniform_index(r[0], 2)], comps[1][oracle.uniform_index(r[1], 2)]))
    assert list(zip(E.u.tolist(), E.v.tolist())) == [tuple(map(int, p)) for p in expect]


def test_refine_line_example_known_outcome():
    X = _two_line_clusters()
    nbr, _ = oracle.knn_exact(X, 1)
    G = oracle.undirected_graph(nbr)
    comp, comps = oracle.components(G)
    assert len(comps) == 2
    # start from the worst pair (0, 9); the closest pair is (4, 5)
    E = oracle.EdgeSet(np.array([0]), np.array([9]), np.array([196.0]), np.array([0]), np.array([1]))
    rounds = 0
    while True:
        E, delta = oracle.refine_edges(X, G, comp, E)
        rounds += 1
        if delta == 0:
            break
    assert (int(E.u[0]), int(E.v[0])) == (4, 5) and E.s[0] == 36.0
    # each round moves u one step right (neighbour of u) and v one step left
    assert rounds == 5


def test_refine_uses_updated_u_star_and_original_u():
    # G[u] = {u1}, G[v] = {v1}; u1 is closer to v, v1 is closer to u1 than v
    X = np.array([[0.0, 0.0], [2.0, 0.0], [10.0, 0.0], [4.0, 0.0]], dtype=np.float32)
    # ids: u=0, u1=1 (component 0), v=2, v1=3 (component 1)
    G = [np.array([1]), np.array([0]), np.array([3]), np.array([2])]
    comp = np.array([0, 0, 1, 1])
    E = oracle.EdgeSet(np.array([0]), np.array([2]), np.array([100.0]), np.array([0]), np.array([1]))
    R, delta = oracle.refine_edges(X, G, comp, E)
    assert delta == 1
    assert (int(R.u[0]), int(R.v[0]), float(R.s[0])) == (1, 3, 4.0)


def test_refine_strict_less_keeps_incumbent_on_tie():
    X = np.array([[0.0], [2.0], [1.0]], dtype=np.float32)   # u=0 and u'=1 both at s=1 from v=2
    G = [np.array([1]), np.array([0]), np.array([], dtype=np.int64)]
    comp = np.array([0, 0, 1])
    E = oracle.EdgeSet(np.array([0]), np.array([2]), np.array([1.0]), np.array([0]), np.array([1]))
    R, delta = oracle.refine_edges(X, G, comp, E)
    assert delta == 0 and int(R.u[0]) == 0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_refine_vectorised_equals_literal(seed):
    X = datagen.blobs(n=500, d=5, n_clusters=4, seed=seed)
    nbr, _ = oracle.knn_exact(X, 2)
    G = oracle.undirected_graph(nbr)
    comp, comps = oracle.components(G)
    E = oracle.random_edges(X, comps, 3, seed=seed)
    for _ in range(4):
        A, da = oracle.refine_edges(X, G, comp, E)
        B, db = oracle.refine_edges_literal(X, G, comp, E)
        assert da == db
        assert np.array_equal(A.u, B.u) and np.array_equal(A.v, B.v) and np.array_equal(A.s, B.s)
        E = A


def test_refine_invariants_and_local_optimality():
    X = datagen.blobs(n=700, d=6, n_clusters=5, seed=9)
    nbr, _ = oracle.knn_exact(X, 2)
    G = oracle.undirected_graph(nbr)
    comp, comps = oracle.components(G)
    E = oracle.random_edges(X, comps, 4, seed=3)
    X64 = oracle.as64(X)
    for _ in range(100):
        R, delta = oracle.refine_edges(X, G, comp, E)
        assert np.all(comp[R.u] == R.a) and np.all(comp[R.v] == R.b)
        assert np.all(R.s <= E.s)
        E = R
        if delta == 0:
            break
    assert delta == 0
    for e in range(len(E)):
        u, v, s = int(E.u[e]), int(E.v[e]), float(E.s[e])
        for up in G[u]:
            if comp[up] == E.a[e] and up != v:
                assert oracle.sqdist(X64, int(up), v) >= s
        for vp in G[v]:
            if comp[vp] == E.b[e] and vp != u:
                assert oracle.sqdist(X64, u, int(vp)) >= s


@pytest.mark.parametrize("fn", [oracle.refine_edges, oracle.refine_edges_literal])
def test_refine_tie_among_neighbours_takes_smaller_id(fn):
    # u=0 at x=0; its neighbours 1 and 2 sit at the same distance from v=3
    X = np.array([[0.0, 0.0], [5.0, 1.0], [5.0, -1.0], [10.0, 0.0]], dtype=np.float32)
    G = [np.array([1, 2]), np.array([0]), np.array([0]), np.array([], dtype=np.int64)]
    comp = np.array([0, 0, 0, 1])
    E = oracle.EdgeSet(np.array([0]), np.array([3]), np.array([100.0]), np.array([0]), np.array([1]))
    R, delta = fn(X, G, comp, E)
    assert delta == 1 and int(R.u[0]) == 1 and float(R.s[0]) == 26.0


@pytest.mark.parametrize("fn", [oracle.refine_edges, oracle.refine_edges_literal])
def test_refine_equal_to_incumbent_not_taken(fn):
    X = np.array([[0.0], [2.0], [1.0]], dtype=np.float32)
    G = [np.array([1]), np.array([0]), np.array([], dtype=np.int64)]
    comp = np.array([0, 0, 1])
    E = oracle.EdgeSet(np.array([0]), np.array([2]), np.array([1.0]), np.array([0]), np.array([1]))
    R, delta = fn(X, G, comp, E)
    assert delta == 0 and int(R.u[0]) == 0


def test_random_edges_pair_subset_equals_full_run():
    X = datagen.blobs(n=500, d=5, n_clusters=6, seed=8)
    nbr, _ = oracle.knn_exact(X, 1)
    comp, comps = oracle.components(oracle.undirected_graph(nbr))
    t = len(comps)
    assert t >= 6
    full = oracle.random_edges(X, comps, 3, seed=4)
    sub = [(t - 2, t - 1), (0, 1), (1, t - 1), (0, t - 1)]
    part = oracle.random_edges(X, comps, 3, seed=4, pairs=sub)
    for a, b in sub:
        m = (full.a == a) & (full.b == b)
        p = (part.a == a) & (part.b == b)
        assert np.array_equal(full.u[m], part.u[p]) and np.array_equal(full.v[m], part.v[p])
        assert np.array_equal(full.s[m], part.s[p])
