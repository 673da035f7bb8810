"""Pins for the oracle's random generator and exact kNN (CPU only)."""
import os

import numpy as np
import pytest
from scipy.stats import chisquare
from sklearn.neighbors import NearestNeighbors

import datagen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((tuple(w[0:4]), tuple(w[4:6]), tuple(w[6:10])))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat_rows())
def test_philox_known_answers(ctr, key, out):
    assert oracle.philox4x32_10(ctr, key) == out


def test_philox_counter_sensitivity():
    base = oracle.philox4x32_10((1, 2, 3, 4), (5, 6))
    for pos in range(4):
        c = [1, 2, 3, 4]
        c[pos] ^= 1
        assert oracle.philox4x32_10(tuple(c), (5, 6)) != base
    assert oracle.philox4x32_10((1, 2, 3, 4), (5, 7)) != base


def test_uniform_index_range_and_uniformity():
    size = 7
    counts = np.zeros(size)
    for i in range(7000):
        r = oracle.philox4x32_10((i, 0, 0, 0), oracle.seed_key(0))
        j = oracle.uniform_index(r[0], size)
        assert 0 <= j < size
        counts[j] += 1
    assert chisquare(counts).pvalue > 1e-3
    assert oracle.uniform_index(0xFFFFFFFF, size) == size - 1
    assert oracle.uniform_index(0, size) == 0


def test_seed_key_split():
    assert oracle.seed_key(0x0123456789ABCDEF) == (0x89ABCDEF, 0x01234567)


def _sets(nbr):
    return [set(r.tolist()) for r in nbr]


def test_knn_bruteforce_definition_tiny():
    X = np.array([[0.0], [1.0], [3.0], [7.0]], dtype=np.float32)
    nbr, sq = oracle.knn_bruteforce(X, 2)
    assert nbr.tolist() == [[1, 2], [0, 2], [1, 0], [2, 1]]
    assert sq.tolist() == [[1.0, 9.0], [1.0, 4.0], [4.0, 9.0], [16.0, 36.0]]


def test_knn_ties_broken_by_index():
    # lattice: many exactly equal distances
    X = np.array([[x, y] for x in range(4) for y in range(4)], dtype=np.float32)
    nbr, sq = oracle.knn_bruteforce(X, 4)
    nbr2, sq2 = oracle.knn_exact(X, 4, margin=2)
    assert np.array_equal(nbr, nbr2) and np.array_equal(sq, sq2)
    # corner 0 = (0,0): neighbours at s=1 are ids 1 (0,1) and 4 (1,0), then s=2 id 5
    assert nbr[0].tolist() == [1, 4, 5, 2]


def test_knn_duplicates_are_neighbours():
    X = np.zeros((6, 3), dtype=np.float32)
    X[3:] = 1.0
    nbr, sq = oracle.knn_exact(X, 2, margin=1)
    assert nbr[0].tolist() == [1, 2] and sq[0].tolist() == [0.0, 0.0]
    assert nbr[4].tolist() == [3, 5]


@pytest.mark.parametrize("seed", [0, 1])
def test_knn_exact_matches_sklearn_bruteforce(seed):
    X = datagen.blobs(n=1500, d=16, n_clusters=5, seed=seed)
    nbr, sq = oracle.knn_exact(X, 10)
    nn = NearestNeighbors(n_neighbors=11, algorithm="brute").fit(X.astype(np.float64))
    dist, ind = nn.kneighbors(X.astype(np.float64))
    # sklearn includes the point itself first (distinct float data: no ties)
    assert np.array_equal(ind[:, 0], np.arange(len(X)))
    assert _sets(nbr) == _sets(ind[:, 1:])
    np.testing.assert_allclose(np.sqrt(sq), dist[:, 1:], rtol=1e-12, atol=1e-12)


def test_knn_exact_matches_bruteforce_integer_data():
    rng = np.random.default_rng(3)
    X = rng.integers(0, 4, size=(120, 3)).astype(np.float32)   # heavy ties, duplicates
    a = oracle.knn_bruteforce(X, 7)
    b = oracle.knn_exact(X, 7, block=50, margin=3)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_knn_exact_rows_subset():
    X = datagen.gamma_int(n=3000, d=32, n_clusters=10, seed=2)
    full = oracle.knn_exact(X, 5)
    rows = np.array([0, 17, 2999])
    part = oracle.knn_exact(X, 5, rows=rows)
    assert np.array_equal(full[0][rows], part[0])


def test_knn_k_equals_n_minus_1():
    X = datagen.blobs(n=40, d=4, n_clusters=2, seed=5)
    nbr, sq = oracle.knn_exact(X, 39)
    for i in range(40):
        assert sorted(nbr[i].tolist()) == [j for j in range(40) if j != i]
        assert np.all(np.diff(sq[i]) >= 0)
