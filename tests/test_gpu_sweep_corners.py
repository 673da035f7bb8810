"""Parity at the corners of the parameter sweeps (bench.py --sweep): the
k x lambda grid on 10,000 x 32 blobs and the n x d grid, each corner's
pipeline against the oracle's FAMST on the same input (float32 exact path:
equal components, lambda-edge count and refinement deltas, W within 1e-5
relative)."""
import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_2507_14261_amd as F

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _check(X, k, lam, seed, precision="fp32"):
    ref = oracle.famst(X, k, lam, seed=seed, max_rounds=10)
    out = F.famst(torch.from_numpy(X).to(DEV), k, lam, seed=seed, max_rounds=10, precision=precision, exact=True)
    torch.cuda.synchronize()
    W = float(out.W[0])
    print(f"  W={W!r} oracle={ref.W!r} rel={(W - ref.W) / ref.W:.2e} t={len(ref.comps)} deltas={ref.deltas}",
          flush=True)
    assert abs(W - ref.W) <= 1e-5 * ref.W
    assert out.graph.n_comp[0] == len(ref.comps) and len(out.E) == len(ref.E0)
    assert out.deltas == ref.deltas


@pytest.mark.parametrize("k,lam", [(5, 1), (5, 10), (20, 1), (20, 10)])
def test_kl_sweep_corners(k, lam):
    print(f"case kl corner k={k} lambda={lam}", flush=True)
    _check(datagen.blobs(n=10_000, d=32, seed=1), k, lam, seed=0)


@pytest.mark.parametrize("d,precision", [(2, "fp32"), (784, "bf16"), (784, "fp32")])
def test_nd_sweep_small_n_corners(d, precision):
    # the smallest n of the grid at its smallest and largest d
    n = 32_768
    print(f"case nd corner n={n} d={d} {precision}", flush=True)
    _check(datagen.blobs(n=n, d=d, seed=0), 10, 5, seed=0, precision=precision)
