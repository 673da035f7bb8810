"""Python binding of libfamst: same call names as the C-ABI.

PyTorch supplies device memory and the current HIP stream; every step of
the method runs in the library's kernels.  Inputs must be CUDA (HIP)
tensors; nothing here computes on the host.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

_PREC = {"fp32": L.FAMST_FP32, "bf16": L.FAMST_BF16, "fp8": L.FAMST_FP8_E4M3}
_ALGO = {"boruvka": L.FAMST_BORUVKA, "kruskal": L.FAMST_KRUSKAL, "prim": L.FAMST_DENSE_PRIM}


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    return t.contiguous()


def _offs(offs, n):
    if offs is None:
        return None, 1
    o = np.ascontiguousarray(np.asarray(offs, dtype=np.int64))
    if o.ndim != 1 or len(o) < 2 or o[0] != 0 or o[-1] != n:
        raise ValueError("offs must be [0, ..., n]")
    return o, len(o) - 1


def _offs_ptr(o):
    return None if o is None else o.ctypes.data_as(L.PI64)


def _workspace(fn, *args):
    """Query the workspace size (ws = NULL), allocate it, run the call."""
    sz = ctypes.c_size_t(0)
    L.check(fn(*args, None, ctypes.byref(sz), _stream()), fn.__name__ + " (size query)")
    dev = torch.device("cuda", torch.cuda.current_device())
    ws = torch.empty(max(int(sz.value), 256), dtype=torch.uint8, device=dev)
    return fn(*args, _ptr(ws), ctypes.byref(sz), _stream()), ws


# ------------------------------------------------------------ Phase 1
def knn_graph(X, k: int, precision: str = "fp32", exact: bool = False, k_cand: int = 0,
              offs=None, with_stats: bool = False, algo: str = "exact"):
    """k nearest neighbours per point (Alg. 1 GetANNs): ``algo="exact"``
    (matrix-core screening + float32 re-rank) or ``"nndescent"``
    (approximate, float32).  Returns (nbr int32 [n, k], dist float32 [n, k])
    and, with ``with_stats``, a dict."""
    lib = L.load()
    X = _dev(X, torch.float32, "X")
    n, d = X.shape
    o, B = _offs(offs, n)
    nbr = torch.empty((n, k), dtype=torch.int32, device=X.device)
    dist = torch.empty((n, k), dtype=torch.float32, device=X.device)
    if algo not in ("exact", "nndescent"):
        raise ValueError("algo must be 'exact' or 'nndescent'")
    prec = _PREC[precision] | (L.FAMST_EXACT if exact else 0)
    if algo == "nndescent":
        prec = L.FAMST_FP32 | L.FAMST_NNDESCENT
    st = (ctypes.c_int64 * L.FAMST_NSTATS)() if with_stats else None
    code, _ = _workspace(lib.famst_knn_graph, _ptr(X), n, d, _offs_ptr(o), B, k, prec, k_cand,
                         _ptr(nbr), _ptr(dist), st)
    L.check(code, "famst_knn_graph")
    if with_stats:
        stats = {"uncertified": st[0], "recomputed": st[1], "near_ties": st[2], "k_cand": st[3],
                 "nnd_iterations": st[4], "nnd_updates": st[5]}
        return nbr, dist, stats
    return nbr, dist


# ------------------------------------------------------------ Phase 2
@dataclass
class Graph:
    row_ptr: torch.Tensor
    col: torch.Tensor
    comp: torch.Tensor
    members: torch.Tensor
    comp_ptr: torch.Tensor
    n_comp: list


@dataclass
class Edges:
    u: torch.Tensor
    v: torch.Tensor
    w: torch.Tensor
    a: torch.Tensor
    b: torch.Tensor

    def __len__(self):
        return int(self.u.numel())


def _empty_edges(m, dev):
    return Edges(torch.empty(m, dtype=torch.int32, device=dev), torch.empty(m, dtype=torch.int32, device=dev),
                 torch.empty(m, dtype=torch.float32, device=dev), torch.empty(m, dtype=torch.int32, device=dev),
                 torch.empty(m, dtype=torch.int32, device=dev))


def connect(X, nbr, lam: int, seed: int = 0, offs=None, e_cap: int | None = None):
    """Undirected graph, components and lambda-edges (Alg. 2, Alg. 3).
    Returns (Graph, Edges)."""
    lib = L.load()
    X = _dev(X, torch.float32, "X")
    nbr = _dev(nbr, torch.int32, "nbr")
    n, d = X.shape
    k = nbr.shape[1]
    o, B = _offs(offs, n)
    dev = X.device
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
    col = torch.empty(2 * n * k, dtype=torch.int32, device=dev)
    comp = torch.empty(n, dtype=torch.int32, device=dev)
    members = torch.empty(n, dtype=torch.int32, device=dev)
    comp_ptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
    n_col = ctypes.c_int64(0)
    n_comp = (ctypes.c_int32 * B)()
    n_edges = ctypes.c_int64(0)
    # first guess: a few dozen component pairs per cloud (too small a guess
    # costs a second pass over the graph, see the ECAPACITY retry below)
    cap = int(e_cap) if e_cap is not None else lam * (64 + 32 * B)
    E = _empty_edges(cap, dev)
    for attempt in range(2):
        code, _ = _workspace(lib.famst_connect, _ptr(X), n, d, _offs_ptr(o), B, _ptr(nbr), k, lam,
                             ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), _ptr(row_ptr), _ptr(col),
                             ctypes.byref(n_col), _ptr(comp), _ptr(members), _ptr(comp_ptr), n_comp,
                             _ptr(E.u), _ptr(E.v), _ptr(E.w), _ptr(E.a), _ptr(E.b), cap,
                             ctypes.byref(n_edges))
        if code == L.FAMST_ECAPACITY and attempt == 0:
            cap = int(n_edges.value)
            E = _empty_edges(max(cap, 1), dev)
            continue
        L.check(code, "famst_connect")
        break
    m = int(n_edges.value)
    E = Edges(E.u[:m], E.v[:m], E.w[:m], E.a[:m], E.b[:m])
    G = Graph(row_ptr, col[:int(n_col.value)], comp, members, comp_ptr, list(n_comp))
    return G, E


# ------------------------------------------------------------ Phase 3
def refine(X, G: Graph, E: Edges, max_rounds: int = 10):
    """Alg. 4 rounds in place on E until no change.  Returns (rounds,
    deltas, converged)."""
    lib = L.load()
    X = _dev(X, torch.float32, "X")
    n, d = X.shape
    rounds = ctypes.c_int32(0)
    deltas = (ctypes.c_int64 * max_rounds)()
    code, _ = _workspace(lib.famst_refine, _ptr(X), n, d, _ptr(G.row_ptr), _ptr(G.col), _ptr(G.comp),
                         _ptr(E.u), _ptr(E.v), _ptr(E.w), _ptr(E.a), _ptr(E.b), len(E), max_rounds,
                         ctypes.byref(rounds), deltas)
    L.check(code, "famst_refine")
    r = int(rounds.value)
    return r, [int(deltas[i]) for i in range(r)], code != L.FAMST_WNOTCONVERGED


# ------------------------------------------------------------ Phase 4
def mst(X, nbr=None, dist=None, E: Edges | None = None, algo: str = "boruvka", offs=None):
    """Spanning tree of N u E (or of the complete graph with algo="prim").
    Returns (tu, tv, tw, W) with W float32 [B]."""
    lib = L.load()
    X = _dev(X, torch.float32, "X")
    n, d = X.shape
    o, B = _offs(offs, n)
    dev = X.device
    k = 0 if nbr is None else nbr.shape[1]
    if nbr is not None:
        nbr = _dev(nbr, torch.int32, "nbr")
        dist = _dev(dist, torch.float32, "dist")
    ne = 0 if E is None else len(E)
    tu = torch.empty(n - B, dtype=torch.int32, device=dev)
    tv = torch.empty(n - B, dtype=torch.int32, device=dev)
    tw = torch.empty(n - B, dtype=torch.float32, device=dev)
    W = torch.empty(B, dtype=torch.float32, device=dev)
    eu = ev = ew = None
    if E is not None and ne:
        eu, ev, ew = (_dev(E.u, torch.int32, "eu"), _dev(E.v, torch.int32, "ev"),
                      _dev(E.w, torch.float32, "ew"))
    code, _ = _workspace(lib.famst_mst, _ptr(X), n, d, _offs_ptr(o), B, _ptr(nbr), _ptr(dist), k,
                         _ptr(eu), _ptr(ev), _ptr(ew), ne, _ALGO[algo], _ptr(tu), _ptr(tv), _ptr(tw),
                         _ptr(W))
    L.check(code, "famst_mst")
    return tu, tv, tw, W


def mst_backward(X, tu, tv, gW, offs=None):
    """d W / d X for the given tree, scaled per cloud by gW."""
    lib = L.load()
    X = _dev(X, torch.float32, "X")
    n, d = X.shape
    o, B = _offs(offs, n)
    gW = _dev(gW.reshape(-1).to(torch.float32), torch.float32, "gW")
    grad = torch.empty_like(X)
    code, _ = _workspace(lib.famst_mst_backward, _ptr(X), n, d, _offs_ptr(o), B,
                         _ptr(_dev(tu, torch.int32, "tu")), _ptr(_dev(tv, torch.int32, "tv")), _ptr(gW),
                         _ptr(grad))
    L.check(code, "famst_mst_backward")
    return grad


def mst_backward_noalloc(X, tu, tv, gW, offs=None, grad=None):
    """mst_backward on the library's fixed scratch array (no workspace is
    allocated by the call; ``grad`` may be given to allocate nothing at
    all).  Returns (grad, scratch bytes the call needed)."""
    lib = L.load()
    X = _dev(X, torch.float32, "X")
    n, d = X.shape
    o, B = _offs(offs, n)
    gW = _dev(gW.reshape(-1).to(torch.float32), torch.float32, "gW")
    grad = torch.empty_like(X) if grad is None else _dev(grad, torch.float32, "grad")
    need = ctypes.c_size_t(0)
    code = lib.famst_mst_backward_noalloc(_ptr(X), n, d, _offs_ptr(o), B, _ptr(_dev(tu, torch.int32, "tu")),
                                          _ptr(_dev(tv, torch.int32, "tv")), _ptr(gW), _ptr(grad),
                                          ctypes.byref(need), _stream())
    L.check(code, "famst_mst_backward_noalloc")
    return grad, int(need.value)


def mst_dense_fused(X, offs=None):
    """Exact tree of every cloud, its weight and the gradient in one
    persistent launch.  Returns (tu, tv, tw, W, G) with G = dW/dX."""
    lib = L.load()
    X = _dev(X, torch.float32, "X")
    n, d = X.shape
    o, B = _offs(offs, n)
    dev = X.device
    tu = torch.empty(n - B, dtype=torch.int32, device=dev)
    tv = torch.empty(n - B, dtype=torch.int32, device=dev)
    tw = torch.empty(n - B, dtype=torch.float32, device=dev)
    W = torch.empty(B, dtype=torch.float32, device=dev)
    G = torch.empty_like(X)
    code, _ = _workspace(lib.famst_mst_dense_fused, _ptr(X), n, d, _offs_ptr(o), B, _ptr(tu), _ptr(tv),
                         _ptr(tw), _ptr(W), _ptr(G))
    L.check(code, "famst_mst_dense_fused")
    return tu, tv, tw, W, G


# ------------------------------------------------------------ Alg. 1
@dataclass
class FamstOut:
    nbr: torch.Tensor
    dist: torch.Tensor
    graph: Graph
    E0: Edges | None
    E: Edges
    rounds: int
    deltas: list
    converged: bool
    tu: torch.Tensor
    tv: torch.Tensor
    tw: torch.Tensor
    W: torch.Tensor
    knn_stats: dict | None = None


def famst(X, k: int, lam: int, seed: int = 0, max_rounds: int = 10, precision: str = "fp32",
          exact: bool | None = None, algo: str = "boruvka", offs=None, keep_initial: bool = False,
          e_cap: int | None = None, with_stats: bool = False, knn: str = "exact") -> FamstOut:
    """The whole FAMST pipeline (Alg. 1) on the device; ``knn="nndescent"``
    builds Phase 1 by NN-Descent."""
    if exact is None:
        exact = precision == "fp32" and knn == "exact"
    r = knn_graph(X, k, precision=precision, exact=exact, offs=offs, with_stats=with_stats, algo=knn)
    nbr, dist = r[0], r[1]
    stats = r[2] if with_stats else None
    G, E = connect(X, nbr, lam, seed, offs=offs, e_cap=e_cap)
    E0 = Edges(*(t.clone() for t in (E.u, E.v, E.w, E.a, E.b))) if keep_initial else None
    rounds, deltas, conv = refine(X, G, E, max_rounds)
    tu, tv, tw, W = mst(X, nbr, dist, E, algo=algo, offs=offs)
    return FamstOut(nbr, dist, G, E0, E, rounds, deltas, conv, tu, tv, tw, W, stats)


class MSTWeight(torch.autograd.Function):
    """W (per cloud) of the FAMST tree of X; the backward pass runs the
    library's gradient kernel with the forward tree held fixed."""

    @staticmethod
    def forward(ctx, X, k, lam, seed=0, max_rounds=10, precision="fp32", offs=None, dense=False):
        Xd = X.detach().contiguous()
        ctx.offs = offs
        ctx.dense = dense
        if dense:
            # exact trees: weight and gradient come from the same persistent launch
            tu, tv, tw, W, G = mst_dense_fused(Xd, offs=offs)
            ctx.save_for_backward(G)
        else:
            out = famst(Xd, k, lam, seed, max_rounds, precision, offs=offs)
            tu, tv, W = out.tu, out.tv, out.W
            ctx.save_for_backward(Xd, tu, tv)
        return W

    @staticmethod
    def backward(ctx, gW):
        if ctx.dense:
            (G,) = ctx.saved_tensors
            n = G.shape[0]
            o, B = _offs(ctx.offs, n)
            sizes = torch.from_numpy(np.diff(o) if o is not None else np.array([n])).to(G.device)
            scale = torch.repeat_interleave(gW.reshape(-1).to(G.dtype), sizes)
            return G * scale[:, None], None, None, None, None, None, None, None
        Xd, tu, tv = ctx.saved_tensors
        grad = mst_backward(Xd, tu, tv, gW.contiguous(), offs=ctx.offs)
        return grad, None, None, None, None, None, None, None


def profile_enable(on: bool = True):
    L.load().famst_profile_enable(1 if on else 0)


def profile_reset():
    L.load().famst_profile_reset()


def profile_read(name: str):
    """(launches, total_ms) of a kernel since the last reset."""
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    L.check(L.load().famst_profile_read(name.encode(), ctypes.byref(n), ctypes.byref(ms)), "profile_read")
    return int(n.value), float(ms.value)
