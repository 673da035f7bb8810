"""Phase 1 parity: famst_knn_graph against the oracle's exact kNN."""
import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_2507_14261_amd as F

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _run(X, k, **kw):
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to(DEV)
    out = F.knn_graph(Xd, k, with_stats=True, **kw)
    torch.cuda.synchronize()
    return out[0].cpu().numpy(), out[1].cpu().numpy(), out[2]


def _check_exact(X, k, nbr, dist, rtol=1e-5):
    ref_n, ref_s = oracle.knn_exact(X, k)
    for i in range(len(X)):
        assert set(nbr[i].tolist()) == set(ref_n[i].tolist()), (i, nbr[i], ref_n[i])
    # distances: the GPU lists are sorted by the float32 value; compare sorted
    np.testing.assert_allclose(np.sort(dist, axis=1), np.sqrt(np.sort(ref_s, axis=1)), rtol=rtol, atol=1e-6)
    assert np.all(np.diff(dist, axis=1) >= 0)


@pytest.mark.parametrize("n,d,k", [(1000, 32, 10), (777, 17, 5), (2100, 3, 1), (513, 100, 20),
                                   (300, 128, 24), (97, 8, 40)])
def test_knn_fp32_exact_matches_oracle(n, d, k):
    print(f"case n={n} d={d} k={k}", flush=True)
    X = datagen.blobs(n=n, d=d, n_clusters=5, seed=n)
    nbr, dist, st = _run(X, k, precision="fp32", exact=True)
    _check_exact(X, k, nbr, dist)


def test_knn_blobs_paper_workload_subsample():
    X = datagen.blobs(n=4000, d=32, n_clusters=10, seed=0)
    nbr, dist, st = _run(X, 10, precision="fp32", exact=True)
    _check_exact(X, 10, nbr, dist)
    print("stats", st)


def test_knn_integer_data_bf16_equals_fp32_bitwise():
    X = datagen.gamma_int(n=3000, d=128, n_clusters=20, seed=1)
    a = _run(X, 20, precision="fp32", exact=True)
    b = _run(X, 20, precision="bf16", exact=True)
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1].view(np.uint32), b[1].view(np.uint32))
    _check_exact(X, 20, a[0], a[1])
    # integer data: every squared distance is an exact float32 integer
    ref_n, ref_s = oracle.knn_exact(X, 20)
    np.testing.assert_array_equal(np.sort(a[1] ** 2, axis=1).round(), np.sort(ref_s, axis=1))


def test_knn_bf16_screen_recall_and_exact_flag():
    X = datagen.blobs(n=2000, d=64, n_clusters=8, seed=4)
    ref_n, _ = oracle.knn_exact(X, 10)
    nbr, dist, st = _run(X, 10, precision="bf16", exact=False)
    rec = oracle.recall_at_k(nbr, ref_n)
    print("bf16 recall", rec, st)
    assert rec >= 0.99
    nbr2, dist2, st2 = _run(X, 10, precision="bf16", exact=True)
    _check_exact(X, 10, nbr2, dist2)


def test_knn_duplicates_and_ties():
    rng = np.random.default_rng(0)
    base = rng.integers(0, 3, size=(300, 4)).astype(np.float32)
    X = np.concatenate([base, base[:50]])
    nbr, dist, st = _run(X, 8, precision="fp32", exact=True)
    ref_n, ref_s = oracle.knn_exact(X, 8)
    # heavy exact ties: (s, j) order is unique, so the lists must be identical
    assert np.array_equal(nbr, ref_n)
    np.testing.assert_allclose(dist, np.sqrt(ref_s), rtol=1e-7)


def test_knn_batched_clouds():
    X, offs = datagen.clouds(n_clouds=5, lo=40, hi=700, d=24, seed=2)
    nbr, dist, st = _run(X, 7, precision="fp32", exact=True, offs=offs)
    for b in range(5):
        sl = slice(offs[b], offs[b + 1])
        ref_n, ref_s = oracle.knn_exact(X[sl], 7)
        got = nbr[sl] - offs[b]
        assert np.all(got >= 0) and np.all(got < offs[b + 1] - offs[b])
        for i in range(len(ref_n)):
            assert set(got[i].tolist()) == set(ref_n[i].tolist())


def test_knn_k_is_n_minus_1():
    X = datagen.blobs(n=41, d=6, n_clusters=2, seed=1)
    nbr, dist, st = _run(X, 40, precision="fp32", exact=True)
    for i in range(41):
        assert sorted(nbr[i].tolist()) == [j for j in range(41) if j != i]


def test_knn_deterministic():
    X = datagen.blobs(n=1500, d=32, n_clusters=4, seed=9)
    a = _run(X, 10, precision="fp32", exact=True)
    b = _run(X, 10, precision="fp32", exact=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("prec,d", [("fp32", 200), ("bf16", 300), ("fp8", 64), ("fp8", 130), ("bf16", 960)])
def test_knn_chunked_and_fp8_exact_mode_matches_oracle(prec, d):
    # d beyond the register-resident kernel, and float8 at any d, use the
    # streamed-operand kernel at k' = 32; exact mode must still give the
    # exact neighbour sets
    print(f"case prec={prec} d={d}", flush=True)
    X = datagen.blobs(n=1500, d=d, n_clusters=6, seed=d)
    nbr, dist, st = _run(X, 12, precision=prec, exact=True)
    print("stats", st)
    _check_exact(X, 12, nbr, dist)


def test_knn_lowrank_d960_precisions():
    # the 960-dimensional embedding-like workload at a size the oracle covers
    X = datagen.lowrank(n=6000, d=960, seed=0)
    ref_n, _ = oracle.knn_exact(X, 20)
    rec = {}
    for prec in ["fp32", "bf16", "fp8"]:
        nbr, dist, st = _run(X, 20, precision=prec, exact=False)
        rec[prec] = oracle.recall_at_k(nbr, ref_n)
        print(prec, "recall", rec[prec], st)
    assert rec["fp32"] == 1.0
    assert rec["bf16"] >= 0.98
    assert rec["fp8"] >= 0.9
    nbr, dist, st = _run(X, 20, precision="fp8", exact=True)
    _check_exact(X, 20, nbr, dist)


# Beyond 128 dimensions (bf16 or float32, k' = 32) queries and rows both
# stream through LDS by K-steps: ragged query blocks and tiles, dimensions
# just past the threshold and padded to a K-step, batched clouds.
@pytest.mark.parametrize("n,d,k,prec", [(1100, 150, 12, "bf16"), (257, 129, 20, "fp32"),
                                        (2000, 512, 16, "bf16"), (700, 960, 8, "fp32"),
                                        (513, 200, 24, "bf16")])
def test_knn_high_dim_matches_oracle(n, d, k, prec):
    print(f"case n={n} d={d} k={k} {prec}", flush=True)
    X = datagen.blobs(n=n, d=d, n_clusters=6, seed=n + d)
    nbr, dist, st = _run(X, k, precision=prec, exact=True)
    print("stats", st, flush=True)
    _check_exact(X, k, nbr, dist)


def test_knn_high_dim_batched_clouds():
    X, offs = datagen.clouds(n_clouds=4, lo=60, hi=600, d=200, seed=5)
    nbr, dist, st = _run(X, 9, precision="bf16", exact=True, offs=offs)
    for b in range(4):
        sl = slice(offs[b], offs[b + 1])
        ref_n, ref_s = oracle.knn_exact(X[sl], 9)
        got = nbr[sl] - offs[b]
        assert np.all(got >= 0) and np.all(got < offs[b + 1] - offs[b])
        for i in range(len(ref_n)):
            assert set(got[i].tolist()) == set(ref_n[i].tolist())


def test_knn_high_dim_integer_data_bf16_equals_fp32_bitwise():
    X = datagen.gamma_int(n=1500, d=256, n_clusters=10, seed=2)
    a = _run(X, 20, precision="fp32", exact=True)
    b = _run(X, 20, precision="bf16", exact=False)
    assert b[2]["uncertified"] == 0, b[2]
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1].view(np.uint32), b[1].view(np.uint32))
    _check_exact(X, 20, a[0], a[1])


# float8 e4m3 with per-row scales (k' = 32) runs on the streamed-operand
# kernel: one 128-dimension K-step per stage, scales applied in the filter.
@pytest.mark.parametrize("n,d,k", [(700, 200, 20), (1300, 64, 10), (520, 960, 16), (300, 129, 5)])
def test_knn_fp8_streamed_matches_oracle(n, d, k):
    print(f"case n={n} d={d} k={k} fp8", flush=True)
    X = datagen.blobs(n=n, d=d, n_clusters=5, seed=n + 3 * d)
    nbr, dist, st = _run(X, k, precision="fp8", exact=True)
    print("stats", st, flush=True)
    _check_exact(X, k, nbr, dist)


def test_knn_fp8_batched_clouds():
    X, offs = datagen.clouds(n_clouds=3, lo=80, hi=500, d=96, seed=7)
    nbr, dist, st = _run(X, 8, precision="fp8", exact=True, offs=offs)
    for b in range(3):
        sl = slice(offs[b], offs[b + 1])
        ref_n, ref_s = oracle.knn_exact(X[sl], 8)
        got = nbr[sl] - offs[b]
        for i in range(len(ref_n)):
            assert set(got[i].tolist()) == set(ref_n[i].tolist())


# One cloud of at least 4096 points on the streamed kernel: the rows are
# visited in a spatial order (pivots assigned on a 128-coordinate sketch),
# and the results are mapped back to the input order.
@pytest.mark.parametrize("prec,d", [("bf16", 200), ("fp32", 100), ("fp8", 128), ("fp8", 300)])
def test_knn_streamed_spatial_order_sampled_rows(prec, d):
    n, k = 40000, 10
    print(f"case n={n} d={d} k={k} {prec} spatial order", flush=True)
    X = datagen.blobs(n=n, d=d, n_clusters=20, seed=d + 11)
    nbr, dist, st = _run(X, k, precision=prec, exact=True)
    print("stats", st, flush=True)
    rows = np.sort(np.random.default_rng(d).choice(n, size=96, replace=False))
    ref_n, ref_s = oracle.knn_exact(X, k, rows=rows, block=32)
    for i, r in enumerate(rows):
        assert set(nbr[r].tolist()) == set(ref_n[i].tolist()), (r, nbr[r], ref_n[i])
    np.testing.assert_allclose(np.sort(dist[rows], axis=1), np.sqrt(np.sort(ref_s, axis=1)), rtol=1e-5, atol=1e-6)
    assert np.all(np.diff(dist, axis=1) >= 0)
    # every row's list holds k distinct other points
    srt = np.sort(nbr, axis=1)
    assert np.all(np.diff(srt, axis=1) > 0) and np.all(nbr != np.arange(n)[:, None])


# From 2,097,152 points in one cloud the pipelined kernel runs eight waves of
# 64 queries per block over tiles of 128 rows (512 queries per block): a
# ragged last tile and block, three K-block counts (bf16 d = 32, 96; float32
# d = 40; d = 128 in the test below), in the spatial order, and a batch whose
# small clouds share the launch with one large cloud (no spatial order
# there); sampled rows against the oracle.  The bf16 cases take integer
# coordinates (exact in bf16), so that exact mode certifies almost every row
# and the recomputation of the rest stays cheap at this size.
@pytest.mark.parametrize("prec,d,batched", [("bf16", 96, False), ("fp32", 40, False), ("bf16", 32, True)])
def test_knn_eight_wave_blocks_sampled_rows(prec, d, batched):
    k = 20 if d >= 96 else 10
    if batched:
        sizes = np.array([300, 2_100_000, 1000, 777])
        X, offs = datagen.clouds(n_clouds=len(sizes), d=d, seed=5, sizes=sizes)
        X = np.round(X * 8.0).astype(np.float32)
    elif prec == "bf16":
        X, offs = datagen.gamma_int(n=2_100_001, d=d, seed=d + 1), None
    else:
        X, offs = datagen.blobs(n=2_100_001, d=d, n_clusters=20, seed=d + 1), None
    n = len(X)
    print(f"case n={n} d={d} k={k} {prec} eight-wave blocks batched={batched}", flush=True)
    nbr, dist, st = _run(X, k, precision=prec, exact=True, **({"offs": offs} if batched else {}))
    print("stats", st, flush=True)
    rng = np.random.default_rng(d)
    rows = np.unique(np.concatenate([rng.choice(n, size=40, replace=False), [0, n - 1]]))
    if batched:
        rows = np.unique(np.concatenate([rows, offs[:-1], offs[1:] - 1, np.arange(300, 340)]))
        for b in range(len(sizes)):
            rb = rows[(rows >= offs[b]) & (rows < offs[b + 1])]
            if len(rb) == 0:
                continue
            Xb = X[offs[b]:offs[b + 1]]
            ref_n, ref_s = oracle.knn_exact(Xb, k, rows=rb - offs[b], block=32)
            for i, r in enumerate(rb):
                assert set(nbr[r].tolist()) == set((ref_n[i] + offs[b]).tolist()), (r, nbr[r], ref_n[i] + offs[b])
            np.testing.assert_allclose(np.sort(dist[rb], axis=1), np.sqrt(np.sort(ref_s, axis=1)), rtol=1e-5,
                                       atol=1e-6)
    else:
        ref_n, ref_s = oracle.knn_exact(X, k, rows=rows, block=32)
        for i, r in enumerate(rows):
            assert set(nbr[r].tolist()) == set(ref_n[i].tolist()), (r, nbr[r], ref_n[i])
        np.testing.assert_allclose(np.sort(dist[rows], axis=1), np.sqrt(np.sort(ref_s, axis=1)), rtol=1e-5,
                                   atol=1e-6)
    assert np.all(np.diff(dist, axis=1) >= 0)
    srt = np.sort(nbr, axis=1)
    assert np.all(np.diff(srt, axis=1) > 0) and np.all(nbr != np.arange(n)[:, None])


def test_knn_eight_wave_blocks_integer_data_bf16_equals_fp32():
    """Integer-valued features (exact in bf16): the bf16-screened lists equal
    the float32 ones entry for entry on the eight-wave kernel, and sampled rows
    equal the oracle's."""
    X = datagen.gamma_int(n=2_100_000, d=128, seed=4)
    print("case gamma-int n=2100000 d=128 k=20 bf16 vs fp32", flush=True)
    nb, db, _ = _run(X, 20, precision="bf16")
    nf, df, _ = _run(X, 20, precision="fp32", exact=True)
    assert np.array_equal(nb, nf) and np.array_equal(db, df)
    rows = np.sort(np.random.default_rng(2).choice(len(X), size=24, replace=False))
    ref_n, ref_s = oracle.knn_exact(X, 20, rows=rows, block=8)
    for i, r in enumerate(rows):
        assert set(nf[r].tolist()) == set(ref_n[i].tolist()), (r, nf[r], ref_n[i])


# A batch of uneven clouds (one of 12 points) on the pipelined kernel, every
# K-block count: every row of every cloud against the oracle, float32 and
# bf16 in exact mode, and bf16 in the default mode against float32 on
# integer coordinates.
@pytest.mark.parametrize("prec,d", [("fp32", 24), ("bf16", 24), ("bf16", 100), ("fp32", 48)])
def test_knn_batched_uneven_clouds_match_oracle(prec, d):
    sizes = np.array([600, 3001, 12, 1500, 257, 2100])
    X, offs = datagen.clouds(n_clouds=len(sizes), d=d, seed=d + 3, sizes=sizes)
    k = 8
    print(f"case batched {prec} d={d} sizes={sizes.tolist()}", flush=True)
    nbr, dist, st = _run(X, k, precision=prec, exact=True, offs=offs)
    print("stats", st, flush=True)
    for b in range(len(sizes)):
        sl = slice(offs[b], offs[b + 1])
        ref_n, ref_s = oracle.knn_exact(X[sl], k)
        got = nbr[sl] - offs[b]
        for i in range(len(got)):
            assert set(got[i].tolist()) == set(ref_n[i].tolist()), (b, i, got[i], ref_n[i])
        np.testing.assert_allclose(np.sort(dist[sl], axis=1), np.sqrt(np.sort(ref_s, axis=1)), rtol=1e-5,
                                   atol=1e-6)


# The first tiles of each block's scan merge their passing rows into the
# lists a query block at a time (four 64-row tiles in the pipelined kernel,
# without its software pipeline at four K-blocks; one 256-row tile in the
# float8 streamed kernel); later rows are inserted one at a time.  Clouds
# sized around those boundaries, with integer coordinates full of exact ties
# (so the (s, j) order fixes every list), give exactly the oracle's lists in
# every precision and kernel form.
@pytest.mark.parametrize("prec,d", [("fp32", 24), ("fp32", 64), ("bf16", 24), ("bf16", 64), ("fp8", 24),
                                    ("fp8", 96)])
def test_knn_merged_first_tiles_boundaries_match_oracle(prec, d):
    sizes = np.array([20, 32, 33, 255, 256, 257, 300, 511, 512, 513, 700])
    X, offs = datagen.clouds(n_clouds=len(sizes), d=d, seed=d + 11, sizes=sizes)
    X = np.round(X * 2.0).astype(np.float32)
    k = 16
    print(f"case merged-tiles {prec} d={d} sizes={sizes.tolist()}", flush=True)
    nbr, dist, st = _run(X, k, precision=prec, exact=True, offs=offs)
    print("stats", st, flush=True)
    for b in range(len(sizes)):
        sl = slice(offs[b], offs[b + 1])
        ref_n, ref_s = oracle.knn_exact(X[sl], k)
        assert np.array_equal(nbr[sl] - offs[b], ref_n), (prec, d, b)
        np.testing.assert_allclose(dist[sl], np.sqrt(ref_s), rtol=1e-6, atol=0)


# Past the merged tiles the one- and two-K-block kernels append passing
# elements to per-query LDS buffers and merge them when one would overflow:
# clouds of 300-3000 points with every row repeated three times (exact
# zero-distance ties) and integer coordinates in a small range (many equal
# distances) overflow the buffers often; the lists must still be exactly
# the oracle's (s, j)-ordered kNN.
@pytest.mark.parametrize("prec,d", [("fp32", 16), ("fp32", 32), ("bf16", 32), ("bf16", 64)])
def test_knn_buffered_updates_with_duplicates_match_oracle(prec, d):
    rng = np.random.default_rng(d + 101)
    sizes = np.array([300, 1203, 3000, 777])
    parts = []
    for m in sizes:
        base = rng.integers(-3, 4, size=(int(m) // 3 + 1, d)).astype(np.float32)
        parts.append(np.repeat(base, 3, axis=0)[rng.permutation(3 * len(base))][: int(m)])
    X = np.concatenate(parts)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    k = 16
    print(f"case buffered-dups {prec} d={d} sizes={sizes.tolist()}", flush=True)
    nbr, dist, st = _run(X, k, precision=prec, exact=True, offs=offs)
    print("stats", st, flush=True)
    for b in range(len(sizes)):
        sl = slice(offs[b], offs[b + 1])
        ref_n, ref_s = oracle.knn_exact(X[sl], k)
        assert np.array_equal(nbr[sl] - offs[b], ref_n), (prec, d, b)
        np.testing.assert_allclose(dist[sl], np.sqrt(ref_s), rtol=1e-6, atol=0)


def test_knn_batched_integer_bf16_equals_fp32():
    sizes = np.array([5000, 333, 2700])
    X, offs = datagen.clouds(n_clouds=len(sizes), d=40, seed=17, sizes=sizes)
    X = np.round(X * 4.0).astype(np.float32)
    nb, db, _ = _run(X, 10, precision="bf16", offs=offs)
    nf, df, _ = _run(X, 10, precision="fp32", exact=True, offs=offs)
    assert np.array_equal(nb, nf) and np.array_equal(db, df)


# k above 24 takes candidate lists of k' = 64: the LDS-list kernel up to 256
# dimensions (bf16) or 128 (fp32), also with fewer K-blocks than its
# template holds (d = 200 bf16, d = 100 fp32: 7 of 8), the K-chunked kernel
# beyond that and for float8; k = 64 is the largest k the entry point takes
@pytest.mark.parametrize("n,d,k,prec", [(1000, 32, 64, "fp32"), (777, 128, 64, "bf16"), (700, 200, 30, "bf16"),
                                        (400, 100, 48, "fp32"), (700, 300, 40, "bf16"), (513, 200, 64, "fp32"),
                                        (600, 64, 25, "fp8"), (900, 130, 64, "fp8")])
def test_knn_large_k_lists_match_oracle(n, d, k, prec):
    print(f"case n={n} d={d} k={k} {prec}", flush=True)
    X = datagen.blobs(n=n, d=d, n_clusters=5, seed=3 * n + d)
    nbr, dist, st = _run(X, k, precision=prec, exact=True)
    print("stats", st, flush=True)
    _check_exact(X, k, nbr, dist)


def test_famst_k64_end_to_end():
    X = datagen.blobs(n=1500, d=16, n_clusters=8, seed=21)
    print("case famst n=1500 d=16 k=64 lam=3", flush=True)
    ref = oracle.famst(X, 64, 3, seed=5)
    out = F.famst(torch.from_numpy(X).to(DEV), 64, 3, seed=5, precision="fp32")
    W = float(out.W[0].item())
    assert abs(W - ref.W) <= 1e-5 * ref.W
    assert out.deltas == ref.deltas and len(out.tu) == len(X) - 1


def _cancellation_inputs(kind, n, d, seed):
    """Inputs where |x|^2 + |y|^2 - 2 x.y cancels: a large common offset with
    sub-unit spread, near-duplicate clusters far from the origin (with exact
    copies), and half of the rows offset far from the other half."""
    rng = np.random.default_rng(seed)
    if kind == "offset":
        X = 1000.0 + 0.01 * rng.standard_normal((n, d))
    elif kind == "far_clusters":
        c = rng.standard_normal((20, d))
        c *= 100.0 / np.linalg.norm(c, axis=1, keepdims=True)
        X = c[rng.integers(0, 20, n)] + 1e-3 * rng.standard_normal((n, d))
        X[n // 2:n // 2 + 40] = X[:40]           # exact copies
    else:
        X = rng.standard_normal((n, d))
        X[n // 2:] = 500.0 + 0.05 * rng.standard_normal((n - n // 2, d))
    return np.ascontiguousarray(X, dtype=np.float32)


@pytest.mark.parametrize("kind", ["offset", "far_clusters", "mixed"])
@pytest.mark.parametrize("prec,d,k", [("fp32", 32, 10), ("fp32", 100, 10), ("bf16", 32, 10), ("bf16", 200, 10),
                                      ("fp8", 64, 10), ("bf16", 48, 30), ("fp32", 150, 30), ("fp8", 130, 30)])
def test_exact_mode_certificate_under_cancellation(kind, prec, d, k):
    # the exactness certificate rests on an error bound for the screened
    # expansion; where it cancels catastrophically, rows must fall back to
    # exact recomputation rather than be certified with wrong lists
    n = 2500
    print(f"case {kind} {prec} n={n} d={d} k={k}", flush=True)
    X = _cancellation_inputs(kind, n, d, seed=d + k)
    nbr, dist, st = _run(X, k, precision=prec, exact=True)
    print("stats", st, flush=True)
    _check_exact(X, k, nbr, dist)
    if kind == "offset":
        # the screening error dwarfs every distance: nothing can be certified
        assert st["uncertified"] == n and st["recomputed"] == n


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_exact_mode_certificate_spatial_order_offset(prec):
    # one cloud large enough for the spatially ordered scan, half of it with
    # a large offset; sampled rows against the oracle over all points
    n, d, k = 40_000, 32, 10
    print(f"case mixed-offset spatial {prec} n={n}", flush=True)
    X = _cancellation_inputs("mixed", n, d, seed=5)
    nbr, dist, st = _run(X, k, precision=prec, exact=True)
    print("stats", st, flush=True)
    rows = np.sort(np.random.default_rng(1).choice(n, 160, replace=False))
    ref_n, ref_s = oracle.knn_exact(X, k, rows=rows, block=32)
    for i, r in enumerate(rows):
        assert set(nbr[r].tolist()) == set(ref_n[i].tolist()), r
    np.testing.assert_allclose(np.sort(dist[rows], axis=1), np.sqrt(np.sort(ref_s, axis=1)), rtol=1e-5, atol=1e-6)
    assert st["uncertified"] >= n // 2 - 100
