"""The package computes only through libfamst.so: without the library every
entry point raises, host tensors are refused rather than computed on the
CPU, and no module of the package refers to the oracle."""
import ast
import os

import numpy as np
import pytest
import torch

import paper_2507_14261_amd as F
from paper_2507_14261_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2507_14261_amd")


def _calls(X):
    nbr = torch.zeros((X.shape[0], 3), dtype=torch.int32)
    return [
        lambda: F.knn_graph(X, 3),
        lambda: F.connect(X, nbr, 2),
        lambda: F.mst(X, algo="prim"),
        lambda: F.mst_dense_fused(X),
        lambda: F.mst_backward(X, nbr[:-1, 0], nbr[:-1, 1], torch.ones(1)),
        lambda: F.famst(X, 3, 2),
        lambda: F.MSTWeight.apply(X, 3, 2),
    ]


def test_every_entry_point_raises_without_the_library(monkeypatch, tmp_path):
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "libfamst.so"))
    monkeypatch.setattr(L, "_lib", None)
    X = torch.from_numpy(np.random.default_rng(0).standard_normal((64, 4)).astype(np.float32))
    for i, call in enumerate(_calls(X)):
        with pytest.raises(RuntimeError, match="missing"):
            call()


def test_host_tensors_are_refused():
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libfamst.so not built")
    X = torch.from_numpy(np.random.default_rng(0).standard_normal((64, 4)).astype(np.float32))
    for call in _calls(X):
        with pytest.raises(TypeError, match="device tensor"):
            call()


def test_package_never_refers_to_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if not f.endswith(".py"):
                continue
            path = os.path.join(dirpath, f)
            tree = ast.parse(open(path).read(), path)
            for node in ast.walk(tree):
                if isinstance(node, ast.Import):
                    assert all("oracle" not in a.name for a in node.names), path
                elif isinstance(node, ast.ImportFrom):
                    assert "oracle" not in (node.module or ""), path
                elif isinstance(node, ast.Constant) and isinstance(node.value, str):
                    assert "oracle/" not in node.value and "oracle." not in node.value, path
