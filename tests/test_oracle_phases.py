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


@pytest.mark.parametrize("seed", range(6))
def test_components_match_reachability_closure(seed):
    # brute force on small random graphs: u and v share a component exactly
    # when the transitive closure of the adjacency matrix joins them
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 40))
    nbr = rng.integers(0, n, size=(n, 1))
    keep = rng.random(n) < 0.7
    nbr[~keep, 0] = np.flatnonzero(~keep)          # self entries add no edge
    G = oracle.undirected_graph(nbr)
    R = np.eye(n, dtype=bool)
    for i in range(n):
        R[i, G[i]] = True
    for _ in range(n):
        R = (R.astype(np.int64) @ R.astype(np.int64)) > 0
    comp, comps = oracle.components(G)
    for u in range(n):
        for v in range(n):
            assert (comp[u] == comp[v]) == R[u, v]
    mins = [int(R[i].argmax()) for i in range(n)]  # smallest vertex reachable from i
    order = sorted(set(mins))
    assert [order.index(m) for m in mins] == comp.tolist()


def test_components_long_path_shuffled_ids():
    # a path whose ids are shuffled: the smallest id must travel the whole path
    rng = np.random.default_rng(7)
    n = 3000
    ids = rng.permutation(n)
    nbr = np.empty((n, 1), dtype=np.int64)
    nbr[ids[:-1], 0] = ids[1:]
    nbr[ids[-1], 0] = ids[-2]
    comp, comps = oracle.components(oracle.undirected_graph(nbr))
    assert len(comps) == 1 and np.all(comp == 0) and np.array_equal(comps[0], np.arange(n))


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
def test_refine_round_properties(seed):
    # one round of Alg. 4 stated as properties of each output edge, checked
    # by enumerating the neighbours: u* is u or a same-component neighbour of
    # u other than v, no such neighbour is strictly closer to v than u*, and
    # among equally close ones u* has the smallest id (likewise v* from u*,
    # skipping the original u); a move happens only on a strict decrease
    X = datagen.blobs(n=500, d=5, n_clusters=4, seed=seed)
    nbr, _ = oracle.knn_exact(X, 2)
    G = oracle.undirected_graph(nbr)
    comp, comps = oracle.components(G)
    E = oracle.random_edges(X, comps, 3, seed=seed)
    X64 = oracle.as64(X)
    for _ in range(4):
        R, delta = oracle.refine_edges(X, G, comp, E)
        moved = 0
        for e in range(len(E)):
            u, v, s0 = int(E.u[e]), int(E.v[e]), float(E.s[e])
            us, vs, s1 = int(R.u[e]), int(R.v[e]), float(R.s[e])
            cu = [int(w) for w in G[u] if comp[w] == E.a[e] and w != v]
            su = {w: oracle.sqdist(X64, w, v) for w in cu}
            if us == u:
                assert all(x >= s0 for x in su.values())
                mid = s0
            else:
                assert us in su and su[us] < s0
                assert all(x > su[us] or (x == su[us] and w >= us) for w, x in su.items())
                mid = su[us]
            cv = [int(w) for w in G[v] if comp[w] == E.b[e] and w != u]
            sv = {w: oracle.sqdist(X64, us, w) for w in cv}
            if vs == v:
                assert all(x >= mid for x in sv.values())
                assert s1 == mid
            else:
                assert vs in sv and sv[vs] < mid and s1 == sv[vs]
                assert all(x > sv[vs] or (x == sv[vs] and w >= vs) for w, x in sv.items())
            assert s1 == oracle.sqdist(X64, us, vs)
            moved += (us, vs) != (u, v)
        assert moved == delta
        E = R


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


def test_refine_tie_among_neighbours_takes_smaller_id():
    fn = oracle.refine_edges
    # u=0 at x=0; its neighbours 1 and 2 sit at the same distance from v=3
    X = np.array([[0.0, 0.0], [5.0, 1.0], [5.0, -1.0], [10.0, 0.0]], dtype=np.float32)
    G = [np.array([1, 2]), np.array([0]), np.array([0]), np.array([], dtype=np.int64)]
    comp = np.array([0, 0, 0, 1])
    E = oracle.EdgeSet(np.array([0]), np.array([3]), np.array([100.0]), np.array([0]), np.array([1]))
    R, delta = fn(X, G, comp, E)
    assert delta == 1 and int(R.u[0]) == 1 and float(R.s[0]) == 26.0


def test_refine_equal_to_incumbent_not_taken():
    fn = oracle.refine_edges
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


def _first_draws(comps, lam, seed, cloud=0):
    # with every point at the same place all samples tie, and the stable
    # selection keeps the first lambda draws of each pair in sample order
    n = 1 + max(int(max(c)) for c in comps)
    E = oracle.random_edges(np.zeros((n, 2)), comps, lam, seed, cloud)
    return E.u.reshape(-1, lam), E.v.reshape(-1, lam)


def test_random_edges_draws_uniform_and_independent():
    # Alg. 3 draws u uniformly from C_a and v uniformly from C_b, each sample
    # independently: the joint counts over C_a x C_b are flat, also for
    # component sizes that are not powers of two and members in any order
    from scipy.stats import chisquare
    Ca, Cb = np.array([7, 2, 9]), np.array([0, 4, 5, 11, 3])
    lam = 8
    joint = np.zeros((3, 5))
    same_all = 0
    for seed in range(1000):
        u, v = _first_draws([Ca, Cb], lam, seed)
        assert set(u[0].tolist()) <= set(Ca.tolist()) and set(v[0].tolist()) <= set(Cb.tolist())
        for a, b in zip(u[0], v[0]):
            joint[list(Ca).index(a), list(Cb).index(b)] += 1
        same_all += len(set(zip(u[0].tolist(), v[0].tolist()))) == 1
    assert chisquare(joint.ravel()).pvalue > 1e-3
    assert same_all <= 2
    # equal sizes: u's and v's positions agree a quarter of the time (they
    # would always agree if both came from one generator word)
    C4a, C4b = np.array([0, 1, 2, 3]), np.array([4, 5, 6, 7])
    agree, tot = 0, 0
    for seed in range(400):
        u, v = _first_draws([C4a, C4b], lam, seed)
        agree += int(np.sum(u[0] == v[0] - 4))
        tot += lam
    assert abs(agree / tot - 0.25) < 0.03


def test_random_edges_counters_separate_pairs_and_clouds():
    # every (pair, sample, cloud) has its own counter: other pairs and other
    # clouds see other draws
    comps = [np.arange(0, 50), np.arange(50, 100), np.arange(100, 150)]
    u0, v0 = _first_draws(comps, 6, seed=9, cloud=0)
    u1, v1 = _first_draws(comps, 6, seed=9, cloud=1)
    assert not np.array_equal(u0, u1) and not np.array_equal(v0, v1)
    # pairs (0,1) and (0,2) share C_0: their u draws differ
    assert not np.array_equal(u0[0], u0[1])
    # the same run twice is the same
    u2, v2 = _first_draws(comps, 6, seed=9, cloud=0)
    assert np.array_equal(u0, u2) and np.array_equal(v0, v2)
