"""Write tests/golden/oracle_weights.json: the CPU oracle's FAMST results on
the measured workloads (test infrastructure; imports only the oracle and
the seeded input generators).

For each workload the oracle runs Alg. 1 in float64 -- exact kNN, graph and
components (Alg. 2), lambda-edges (Alg. 3), refinement rounds (Alg. 4),
Kruskal -- and the file stores the tree weight W, the component count t,
the number of lambda-edges, the refinement rounds and the changed edges per
round.  Where it is affordable the exact minimum spanning tree weight (Prim
on the complete graph, float64) is stored too, for the relative error of
Eq. (1).  GPU tests and the benchmark compare against these numbers.

    python tests/golden/make_oracle_weights.py [--only NAME ...] [--workers P]
                                               [--cache DIR] [--knn-only]

The kNN stage (the only quadratic one) runs over row chunks in P worker
processes; with --cache DIR its output is kept in DIR and reused.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "oracle_weights.json")


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*", default=None)
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--cache", default=None)
    ap.add_argument("--knn-only", action="store_true")
    return ap.parse_args()


ARGS = _args() if __name__ == "__main__" else None
if ARGS is not None and ARGS.workers > 1:
    # one BLAS thread per worker process
    for v in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import multiprocessing as mp  # noqa: E402

import numpy as np  # noqa: E402

import datagen  # noqa: E402
import oracle  # noqa: E402


def _make(name):
    """(X float32, k, lam, recipe dict) of a workload; recipes name the
    generator call and the subsample exactly."""
    if name == "blobs-10k-d32":
        return datagen.blobs(n=10_000, d=32, seed=0), 10, 5, dict(gen="blobs(n=10000, d=32, seed=0)")
    if name == "gamma-int-1m-d128":
        return (datagen.gamma_int(n=1_000_000, d=128, seed=0), 20, 10,
                dict(gen="gamma_int(n=1000000, d=128, seed=0)"))
    if name == "vmf-4m-d96-sub100k":
        idx = datagen.subsample(4_000_000, 100_000, seed=1)
        X = np.ascontiguousarray(datagen.vmf(n=4_000_000, d=96, seed=0)[idx])
        return X, 16, 8, dict(gen="vmf(n=4000000, d=96, seed=0)[subsample(4000000, 100000, seed=1)]")
    if name == "lowrank-500k-d960-sub50k":
        idx = datagen.subsample(500_000, 50_000, seed=1)
        X = np.ascontiguousarray(datagen.lowrank(n=500_000, d=960, seed=0)[idx])
        return X, 20, 10, dict(gen="lowrank(n=500000, d=960, seed=0)[subsample(500000, 50000, seed=1)]")
    raise KeyError(name)


CLOUDS = "clouds-256-d64"
SINGLE = ["blobs-10k-d32", "vmf-4m-d96-sub100k", "lowrank-500k-d960-sub50k", "gamma-int-1m-d128"]
# exact trees where Prim's O(n^2 d) float64 run stays within minutes
WITH_EXACT = {"blobs-10k-d32"}

_X = None
_K = None


def _knn_rows(rows):
    return oracle.knn_exact(_X, _K, rows=rows, block=64)


def _prim_cloud(args):
    Xc, = args
    return oracle.prim_exact(Xc)[3]


def _famst_cloud(args):
    Xc, k, lam, b = args
    r = oracle.famst(Xc, min(k, len(Xc) - 1), lam, seed=0, max_rounds=10, cloud=b)
    return r.W, len(r.comps), len(r.E0), r.rounds, r.deltas


def knn_parallel(X, k, workers, cache=None, tag=""):
    global _X, _K
    path = os.path.join(cache, f"{tag}_knn_k{k}.npz") if cache else None
    if path and os.path.exists(path):
        z = np.load(path)
        return z["nbr"], z["sq"]
    t0 = time.time()
    n = len(X)
    _X, _K = X, k
    chunks = [np.arange(s, min(n, s + 4096)) for s in range(0, n, 4096)]
    if workers > 1:
        with mp.get_context("fork").Pool(workers) as pool:
            parts = []
            for i, part in enumerate(pool.imap(_knn_rows, chunks)):
                parts.append(part)
                if i % 10 == 0:
                    print(f"  {tag}: knn chunk {i + 1}/{len(chunks)} {time.time() - t0:.0f}s", flush=True)
    else:
        parts = [_knn_rows(c) for c in chunks]
    nbr = np.concatenate([p[0] for p in parts])
    sq = np.concatenate([p[1] for p in parts])
    print(f"  {tag}: knn {time.time() - t0:.0f}s", flush=True)
    if path:
        os.makedirs(cache, exist_ok=True)
        np.savez(path, nbr=nbr, sq=sq)
    return nbr, sq


def run_single(name, workers, cache, knn_only):
    X, k, lam, recipe = _make(name)
    print(f"{name}: n={len(X)} d={X.shape[1]} k={k} lambda={lam}", flush=True)
    nbr, sq = knn_parallel(X, k, workers, cache, name)
    if knn_only:
        return None
    t0 = time.time()
    r = oracle.famst(X, k, lam, seed=0, max_rounds=10, nbr=nbr, sq=sq)
    rec = dict(recipe, n=int(len(X)), d=int(X.shape[1]), k=k, lam=lam, seed=0, max_rounds=10,
               W=r.W, t=len(r.comps), n_edges=len(r.E0), rounds=r.rounds, deltas=[int(x) for x in r.deltas],
               spanning=bool(r.spanning))
    print(f"  {name}: W={r.W!r} t={rec['t']} |E|={rec['n_edges']} deltas={rec['deltas']} "
          f"({time.time() - t0:.0f}s)", flush=True)
    if name in WITH_EXACT:
        W_ex = oracle.prim_exact(X)[3]
        rec["W_exact"] = W_ex
        rec["rel_err_vs_exact"] = oracle.relative_error(r.W, W_ex)
    return rec


def run_clouds(workers):
    X, offs = datagen.clouds(n_clouds=256, d=64, seed=0)
    k, lam = 16, 5
    print(f"{CLOUDS}: {len(offs) - 1} clouds, n={len(X)}", flush=True)
    t0 = time.time()
    jobs = [(np.ascontiguousarray(X[offs[b]:offs[b + 1]]), k, lam, b) for b in range(len(offs) - 1)]
    # largest clouds first so the pool finishes evenly
    order = sorted(range(len(jobs)), key=lambda b: -len(jobs[b][0]))
    with mp.get_context("fork").Pool(workers) as pool:
        fam = dict(zip(order, pool.map(_famst_cloud, [jobs[b] for b in order], chunksize=1)))
        print(f"  {CLOUDS}: famst {time.time() - t0:.0f}s", flush=True)
        ex = dict(zip(order, pool.map(_prim_cloud, [(jobs[b][0],) for b in order], chunksize=1)))
    print(f"  {CLOUDS}: exact {time.time() - t0:.0f}s", flush=True)
    B = len(jobs)
    return dict(gen="clouds(n_clouds=256, d=64, seed=0)", n=int(len(X)), d=64, k=k, lam=lam, seed=0,
                max_rounds=10, W=[fam[b][0] for b in range(B)], t=[fam[b][1] for b in range(B)],
                n_edges=[fam[b][2] for b in range(B)], rounds=[fam[b][3] for b in range(B)],
                deltas=[[int(x) for x in fam[b][4]] for b in range(B)], W_exact=[ex[b] for b in range(B)])


def main():
    a = ARGS
    names = a.only if a.only else SINGLE + [CLOUDS]
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names:
        rec = run_clouds(a.workers) if name == CLOUDS else run_single(name, a.workers, a.cache, a.knn_only)
        if rec is None:
            continue
        data[name] = rec
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
            f.write("\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
