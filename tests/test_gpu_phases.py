"""Phase 2 and Phase 3 parity: famst_connect (Alg. 2, Alg. 3) and
famst_refine (Alg. 4) against the oracle on the same neighbour lists."""
import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_2507_14261_amd as F

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def _connect(X, nbr, lam, seed, offs=None):
    G, E = F.connect(_dev(X, torch.float32), _dev(nbr, torch.int32), lam, seed, offs=offs)
    torch.cuda.synchronize()
    return G, E


def _edges_np(E):
    return tuple(t.cpu().numpy() for t in (E.u, E.v, E.w, E.a, E.b))


@pytest.mark.parametrize("k,n", [(1, 3000), (2, 3000), (10, 4000), (3, 1537)])
def test_graph_and_components_bit_exact(k, n):
    print(f"case k={k} n={n}", flush=True)
    X = datagen.blobs(n=n, d=32, n_clusters=10, seed=0)
    nbr, sq = oracle.knn_exact(X, k)
    G, E = _connect(X, nbr, 3, 0)
    Gref = oracle.undirected_graph(nbr)
    comp_ref, comps_ref = oracle.components(Gref)
    row_ptr = G.row_ptr.cpu().numpy()
    col = G.col.cpu().numpy()
    assert row_ptr[-1] == len(col) == sum(len(g) for g in Gref)
    for i in range(n):
        assert np.array_equal(col[row_ptr[i]:row_ptr[i + 1]], Gref[i])
    assert np.array_equal(G.comp.cpu().numpy(), comp_ref)
    assert G.n_comp == [len(comps_ref)]
    members = G.members.cpu().numpy()
    comp_ptr = G.comp_ptr.cpu().numpy()
    for c, m in enumerate(comps_ref):
        assert np.array_equal(members[comp_ptr[c]:comp_ptr[c + 1]], m)


def _pair_lists(u, v, a, b, w=None):
    """Per component pair, its entries in stored order: (u, v) and, with w,
    the weights (Alg. 3 keeps each pair's samples in ascending (s, q)
    order, so the lists are compared entry by entry)."""
    out, ws = {}, {}
    w = np.zeros(len(u)) if w is None else w
    for uu, vv, aa, bb, ww in zip(u.tolist(), v.tolist(), a.tolist(), b.tolist(), w.tolist()):
        out.setdefault((aa, bb), []).append((uu, vv))
        ws.setdefault((aa, bb), []).append(ww)
    return out, ws


def _check_pairs(got, ref, keys=None):
    (gp, gw), (rp, rw) = got, ref
    for key in (rp if keys is None else keys):
        assert gp[key] == rp[key], key
        np.testing.assert_allclose(gw[key], rw[key], rtol=1e-5)


@pytest.mark.parametrize("k,lam,seed,n", [(2, 5, 0, 2500), (1, 3, 7, 600), (10, 5, 0, 2500),
                                          (3, 10, 123456789012, 2500)])
def test_lambda_edges_match_oracle(k, lam, seed, n):
    print(f"case k={k} lam={lam} seed={seed} n={n}", flush=True)
    X = datagen.blobs(n=n, d=32, n_clusters=10, seed=1)
    nbr, sq = oracle.knn_exact(X, k)
    G, E = _connect(X, nbr, lam, seed)
    Gref = oracle.undirected_graph(nbr)
    comp_ref, comps_ref = oracle.components(Gref)
    t = len(comps_ref)
    if t > 200:
        pytest.skip("oracle sampling too slow for this t")
    Eref = oracle.random_edges(X, comps_ref, lam, seed)
    u, v, w, a, b = _edges_np(E)
    assert len(u) == len(Eref) == lam * t * (t - 1) // 2
    # entry order: pairs in (a, b) order, lambda entries each in ascending
    # (s, sample) order; every entry with its own weight
    assert np.array_equal(a, Eref.a) and np.array_equal(b, Eref.b)
    assert np.array_equal(u, Eref.u) and np.array_equal(v, Eref.v)
    np.testing.assert_allclose(w, np.sqrt(Eref.s), rtol=1e-5)


def test_lambda_edges_batched_use_cloud_counter():
    X, offs = datagen.clouds(n_clouds=3, lo=200, hi=400, d=16, seed=5)
    k, lam, seed = 2, 3, 9
    nbr = np.concatenate([oracle.knn_exact(X[offs[b]:offs[b + 1]], k)[0] + offs[b] for b in range(3)])
    G, E = _connect(X, nbr, lam, seed, offs=offs)
    u, v, w, a, b = _edges_np(E)
    comp = G.comp.cpu().numpy()
    base = 0
    got = _pair_lists(u, v, a, b, w)
    for cb in range(3):
        Xb = X[offs[cb]:offs[cb + 1]]
        nb_local = nbr[offs[cb]:offs[cb + 1]] - offs[cb]
        comp_ref, comps_ref = oracle.components(oracle.undirected_graph(nb_local))
        assert G.n_comp[cb] == len(comps_ref)
        np.testing.assert_array_equal(comp[offs[cb]:offs[cb + 1]], comp_ref + base)
        Eref = oracle.random_edges(Xb, comps_ref, lam, seed, cloud=cb)
        _check_pairs(got, _pair_lists(Eref.u + offs[cb], Eref.v + offs[cb], Eref.a + base, Eref.b + base,
                                      np.sqrt(Eref.s)))
        base += len(comps_ref)


@pytest.mark.parametrize("n_clouds", [255, 256, 600])
def test_connect_many_clouds(n_clouds):
    # more clouds than one block of threads: per-cloud component offsets
    # must be gathered for every cloud
    print(f"case n_clouds={n_clouds}", flush=True)
    X, offs = datagen.clouds(n_clouds=n_clouds, lo=6, hi=40, d=4, n_clusters=3, seed=n_clouds)
    k, lam, seed = 1, 2, 5
    nbr = np.concatenate([oracle.knn_exact(X[offs[b]:offs[b + 1]], k)[0] + offs[b]
                          for b in range(n_clouds)])
    G, E = _connect(X, nbr, lam, seed, offs=offs)
    comp = G.comp.cpu().numpy()
    u, v, w, a, b = _edges_np(E)
    got = _pair_lists(u, v, a, b, w)
    base, P = 0, 0
    for cb in range(n_clouds):
        sl = slice(offs[cb], offs[cb + 1])
        comp_ref, comps_ref = oracle.components(oracle.undirected_graph(nbr[sl] - offs[cb]))
        t = len(comps_ref)
        assert G.n_comp[cb] == t
        np.testing.assert_array_equal(comp[sl], comp_ref + base)
        if cb % 37 == 0:
            Eref = oracle.random_edges(X[sl], comps_ref, lam, seed, cloud=cb)
            _check_pairs(got, _pair_lists(Eref.u + offs[cb], Eref.v + offs[cb], Eref.a + base,
                                          Eref.b + base, np.sqrt(Eref.s)))
        base += t
        P += t * (t - 1) // 2
    assert len(u) == lam * P
    assert G.comp_ptr.cpu().numpy()[base] == len(X)


def _edges_to_oracle(u, v, w, a, b):
    return oracle.EdgeSet(u.astype(np.int64), v.astype(np.int64), (w.astype(np.float64)) ** 2,
                          a.astype(np.int64), b.astype(np.int64))


@pytest.mark.parametrize("k,lam,n", [(2, 5, 3000), (1, 2, 500), (10, 5, 3000)])
def test_refine_rounds_match_oracle(k, lam, n):
    print(f"case k={k} lam={lam} n={n}", flush=True)
    X = datagen.blobs(n=n, d=32, n_clusters=10, seed=2)
    nbr, sq = oracle.knn_exact(X, k)
    G, E = _connect(X, nbr, lam, 3)
    Gref = oracle.undirected_graph(nbr)
    comp_ref, comps_ref = oracle.components(Gref)
    Er = _edges_to_oracle(*_edges_np(E))
    Er.s = np.array([oracle.sqdist(oracle.as64(X), int(p), int(q)) for p, q in zip(Er.u, Er.v)])
    Xd = _dev(X, torch.float32)
    for r in range(12):
        rounds, deltas, conv = F.refine(Xd, G, E, max_rounds=1)
        Er, dref = oracle.refine_edges(X, Gref, comp_ref, Er)
        u, v, w, a, b = _edges_np(E)
        assert deltas[0] == dref, (r, deltas, dref)
        assert np.array_equal(u, Er.u) and np.array_equal(v, Er.v), r
        np.testing.assert_allclose(w, np.sqrt(Er.s), rtol=1e-5)
        if dref == 0:
            break
    assert dref == 0


def test_refine_multi_round_call_and_not_converged_warning():
    X = datagen.blobs(n=1500, d=32, n_clusters=10, seed=2)
    nbr, _ = oracle.knn_exact(X, 1)
    Xd = _dev(X, torch.float32)
    G, E = _connect(X, nbr, 4, 1)
    E2 = F.Edges(*(t.clone() for t in (E.u, E.v, E.w, E.a, E.b)))
    rounds, deltas, conv = F.refine(Xd, G, E, max_rounds=1)
    assert rounds == 1 and deltas[0] > 0 and not conv
    rounds, deltas, conv = F.refine(Xd, G, E2, max_rounds=50)
    assert conv and deltas[-1] == 0 and rounds == len(deltas)


@pytest.mark.parametrize("n,k,lam", [(1500, 1, 4), (3000, 1, 5)])
def test_refine_one_call_equals_round_by_round(n, k, lam):
    """All rounds in one call (every edge iterating on its own) give the same
    endpoints, weights and per-round change counts as one call per round;
    3000 points at k = 1 give over 32768 edges (the group-per-edge kernel)."""
    X = datagen.blobs(n=n, d=32, n_clusters=10, seed=n)
    nbr, _ = oracle.knn_exact(X, k)
    Xd = _dev(X, torch.float32)
    G, E = _connect(X, nbr, lam, 2)
    E2 = F.Edges(*(t.clone() for t in (E.u, E.v, E.w, E.a, E.b)))
    print(f"case refine one call n={n} k={k} lam={lam} edges={len(E.u)}", flush=True)
    rounds, deltas, conv = F.refine(Xd, G, E, max_rounds=50)
    assert conv
    per = []
    for _ in range(50):
        r1, d1, _ = F.refine(Xd, G, E2, max_rounds=1)
        per.append(d1[0])
        if d1[0] == 0:
            break
    assert list(deltas) == per
    for a, b in zip(_edges_np(E), _edges_np(E2)):
        assert np.array_equal(a, b)


def test_many_components_k1_sampled_pairs_and_edges():
    # the 10,000-point blobs with k = 1: about 1175 components, 6.9e5
    # component pairs and 1.7e7 lambda-samples.  Components are checked in
    # full; lambda-edges on sampled pairs and refinement on sampled edges
    # (each pair draws from its own counters, each edge refines from its own
    # endpoints, so a sample is checked exactly).
    n, k, lam, seed = 10_000, 1, 5, 0
    print(f"case blobs n={n} k={k} lam={lam}", flush=True)
    X = datagen.blobs(n=n, d=32, n_clusters=10, seed=0)
    Xd = _dev(X, torch.float32)
    nbr, dist = F.knn_graph(Xd, k, precision="fp32", exact=True)
    ref_nbr, _ = oracle.knn_exact(X, k)
    assert np.array_equal(np.sort(nbr.cpu().numpy(), axis=1), np.sort(ref_nbr, axis=1))
    G, E = F.connect(Xd, nbr, lam, seed)
    torch.cuda.synchronize()
    Gref = oracle.undirected_graph(ref_nbr)
    comp_ref, comps_ref = oracle.components(Gref)
    t = len(comps_ref)
    print("components", t, "edges", len(E), flush=True)
    assert t > 1000 and G.n_comp == [t]
    assert np.array_equal(G.comp.cpu().numpy(), comp_ref)
    u, v, w, a, b = _edges_np(E)
    assert len(u) == lam * t * (t - 1) // 2
    rng = np.random.default_rng(3)
    ai = rng.integers(0, t - 1, size=300)
    pairs = sorted({(int(x), int(rng.integers(x + 1, t))) for x in ai})
    Eref = oracle.random_edges(X, comps_ref, lam, seed, pairs=pairs)
    _check_pairs(_pair_lists(u, v, a, b, w), _pair_lists(Eref.u, Eref.v, Eref.a, Eref.b, np.sqrt(Eref.s)))
    # refinement: a sample of edges followed through the rounds the GPU ran
    pick = np.sort(rng.choice(len(u), size=3000, replace=False))
    Es = _edges_to_oracle(u[pick], v[pick], w[pick], a[pick], b[pick])
    Es.s = np.array([oracle.sqdist(oracle.as64(X), int(p), int(q)) for p, q in zip(Es.u, Es.v)])
    rounds, deltas, conv = F.refine(Xd, G, E, max_rounds=10)
    print("refine rounds", rounds, "deltas", deltas, flush=True)
    for _ in range(rounds):
        Es, _ = oracle.refine_edges(X, Gref, comp_ref, Es)
    u2, v2, w2, _, _ = _edges_np(E)
    assert np.array_equal(u2[pick], Es.u) and np.array_equal(v2[pick], Es.v)
    np.testing.assert_allclose(w2[pick], np.sqrt(Es.s), rtol=1e-5)
    # spanning tree over the kNN edges and the refined lambda-edges
    tu, tv, tw, W = F.mst(Xd, nbr, dist, E)
    tu, tv, tw = tu.cpu().numpy(), tv.cpu().numpy(), tw.cpu().numpy()
    assert len(tu) == n - 1
    ds = oracle.DisjointSet(n)
    assert all(ds.union(int(p), int(q)) for p, q in zip(tu, tv))
    assert abs(float(W[0]) - float(np.sum(tw.astype(np.float64)))) <= 1e-6 * float(W[0])
