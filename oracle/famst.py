"""Plain CPU oracle for FAMST -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the package smoke check and the benchmark's CPU
baseline may import this module.  It shares no code with the HIP library
and imports nothing from it.  Everything is computed in float64 with NumPy
(the input float32 coordinates widen to float64 exactly), step by step in
the order of the paper's Algorithm 1:

  Phase 1  GetANNs         -> exact k nearest neighbours (Sec. 3, Alg. 1;
                              the paper allows any method that yields the
                              neighbour lists N and distances D)
  Phase 2  Components      -> Alg. 2 (undirected graph G, DFS components)
           RandomEdges     -> Alg. 3 (lambda^2 samples per component pair,
                              keep the lambda shortest)
  Phase 3  RefineEdges     -> Alg. 4, repeated until no edge changes
  Phase 4  GetMST          -> Kruskal on N u E (Sec. 2.1, Sec. 3)

plus the exact minimum spanning tree by Prim on the complete graph, the
relative error of Eq. (1) (Sec. 5.2), the gradient of the tree weight
with respect to the coordinates and its central finite difference.

Readings of points the paper leaves open (listed with reasons in the
design notes of the repository):
  * distances are Euclidean; every comparison uses the squared distance s,
    emitted weights are w = sqrt(s);
  * a point is not its own neighbour; ties at the k-th neighbour are broken
    by the smaller index;
  * components are numbered by ascending minimum vertex (the order in which
    Alg. 2's outer loop over ascending vertices discovers them) and members
    are listed in ascending order;
  * the random endpoints of Alg. 3 are drawn with replacement by
    Philox4x32-10 with key = seed and counter = (a, b, sample, cloud), the
    32-bit words mapped to a member by multiply-shift; the sort of the
    lambda^2 candidates is stable (ties keep sample order);
  * Alg. 4 scans neighbours in ascending id with a strict "<"; the second
    loop measures from the updated u* but skips v' == u with the original
    u; the refinement loop is capped at R_max rounds;
  * Kruskal orders edges by (w, min endpoint, max endpoint).

Parity status: every function here is pinned by tests against a library
routine, a closed form or brute force.  The random-edge sampling's
individual draws are fixed only by the generator's definition (published
known answers pin the generator); their selection rule is pinned by
invariants and their distribution (uniform and independent over the two
components, separate per pair and cloud) by statistical tests.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .philox import philox4x32_10, seed_key, uniform_index

U64 = 2.0 ** -53


# ---------------------------------------------------------------- distances
def as64(X) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(X, dtype=np.float64))


def sqdist(X64: np.ndarray, u: int, v: int) -> float:
    """Squared Euclidean distance by direct difference (Alg. 3 and Alg. 4
    use ||X_u - X_v||; comparisons on the square give the same order)."""
    return float(sqdist_to(X64, u, [v])[0])


def sqdist_to(X64: np.ndarray, u: int, vs) -> np.ndarray:
    """Direct-difference squared distances from point u to each of vs."""
    vs = np.asarray(vs, dtype=np.int64)
    diff = X64[vs] - X64[u]
    return np.einsum("ij,ij->i", diff, diff)


# ---------------------------------------------------------- Phase 1: kNN
def knn_bruteforce(X, k: int):
    """Definition of the k nearest neighbours, written out: for each i the k
    indices j != i with the smallest (s(i, j), j).  O(n^2 d); tiny n only."""
    X64 = as64(X)
    n = X64.shape[0]
    if not 1 <= k <= n - 1:
        raise ValueError("need 1 <= k <= n-1")
    nbr = np.empty((n, k), dtype=np.int64)
    sq = np.empty((n, k), dtype=np.float64)
    for i in range(n):
        keys = []
        for j in range(n):
            if j != i:
                keys.append((sqdist(X64, i, j), j))
        keys.sort()
        nbr[i] = [j for _, j in keys[:k]]
        sq[i] = [s for s, _ in keys[:k]]
    return nbr, sq


def knn_exact(X, k: int, block: int = 512, margin: int = 16, rows=None):
    """Exact k nearest neighbours (Phase 1 of Alg. 1 with an exact search).

    Candidates are screened with the float64 expansion |x|^2+|y|^2-2x.y
    (one matrix product per row block), the k+margin best are recomputed by
    direct difference and ordered by (s, j).  The screen is verified: every
    non-candidate must exceed the k-th exact value by more than the
    expansion's rounding bound, otherwise the row is redone by direct
    difference over all points.  ``rows`` restricts the query rows.
    Returns (nbr int64 [m, k], s float64 [m, k]) with s squared distances.
    """
    X64 = as64(X)
    n, d = X64.shape
    if not 1 <= k <= n - 1:
        raise ValueError("need 1 <= k <= n-1")
    rows = np.arange(n) if rows is None else np.asarray(rows, dtype=np.int64)
    norms = np.einsum("ij,ij->i", X64, X64)
    max_norm = float(norms.max())
    gamma = 2.0 * (d + 4) * U64
    kc = min(n - 1, k + margin)
    nbr = np.empty((len(rows), k), dtype=np.int64)
    sq = np.empty((len(rows), k), dtype=np.float64)
    for s0 in range(0, len(rows), block):
        rb = rows[s0:s0 + block]
        S = norms[rb, None] + norms[None, :] - 2.0 * (X64[rb] @ X64.T)
        S[np.arange(len(rb)), rb] = np.inf
        if kc < n - 1:
            cand = np.argpartition(S, kc - 1, axis=1)[:, :kc]
        else:
            cand = np.argsort(S, axis=1)[:, :n - 1]
        for r, i in enumerate(rb):
            c = cand[r]
            s_c = sqdist_to(X64, i, c)
            order = np.lexsort((c, s_c))
            sel, s_sel = c[order[:k]], s_c[order[:k]]
            if kc < n - 1:
                screen_floor = S[r, c].max() - gamma * (norms[i] + max_norm)
                if not screen_floor > s_sel[-1]:
                    allj = np.delete(np.arange(n), i)
                    s_all = sqdist_to(X64, i, allj)
                    order = np.lexsort((allj, s_all))
                    sel, s_sel = allj[order[:k]], s_all[order[:k]]
            nbr[s0 + r] = sel
            sq[s0 + r] = s_sel
    return nbr, sq


# ------------------------------------------------- Phase 2: Alg. 2 (graph)
def undirected_graph(nbr, n: int | None = None):
    """Alg. 2, first loop: add (i, j) and (j, i) for every j in N[i].  Rows
    are returned sorted ascending without duplicates or self-loops."""
    nbr = np.asarray(nbr)
    n = nbr.shape[0] if n is None else n
    adj = [set() for _ in range(n)]
    for i in range(nbr.shape[0]):
        for j in nbr[i]:
            j = int(j)
            adj[i].add(j)
            adj[j].add(i)
    return [np.array(sorted(a - {i}), dtype=np.int64) for i, a in enumerate(adj)]


def components(G):
    """Alg. 2, DFS part: visit vertices in ascending order; each unvisited
    vertex starts a new component explored with an explicit stack.
    Returns (comp int64 [n], comps list of ascending member arrays)."""
    n = len(G)
    visited = np.zeros(n, dtype=bool)
    comp = np.full(n, -1, dtype=np.int64)
    comps = []
    for i in range(n):
        if visited[i]:
            continue
        members = []
        stack = [i]
        while stack:
            u = stack.pop()
            if not visited[u]:
                visited[u] = True
                members.append(u)
                stack.extend(int(w) for w in G[u] if not visited[w])
        members = np.array(sorted(members), dtype=np.int64)
        comp[members] = len(comps)
        comps.append(members)
    return comp, comps


# ------------------------------------------- Phase 2: Alg. 3 (lambda-edges)
@dataclass
class EdgeSet:
    """Inter-component edges E with their component pairs E_C (Alg. 3)."""
    u: np.ndarray
    v: np.ndarray
    s: np.ndarray           # squared length
    a: np.ndarray           # component of u
    b: np.ndarray           # component of v

    def __len__(self):
        return len(self.u)

    def copy(self):
        return EdgeSet(self.u.copy(), self.v.copy(), self.s.copy(), self.a.copy(), self.b.copy())


def random_edges(X, comps, lam: int, seed: int, cloud: int = 0, pairs=None) -> EdgeSet:
    """Alg. 3: for every component pair a < b draw lambda^2 endpoint pairs
    (u from C_a, v from C_b), sort them by distance (stable) and keep the
    first lambda.  Edges are listed in (a, b, rank) order.  ``pairs``
    restricts the work to the given (a, b) pairs, in the given order: every
    pair's draws come from its own counters, so a subset is computed exactly
    as in the full run."""
    X64 = as64(X)
    key = seed_key(seed)
    t = len(comps)
    if pairs is None:
        pairs = [(a, b) for a in range(t - 1) for b in range(a + 1, t)]
    out_u, out_v, out_s, out_a, out_b = [], [], [], [], []
    for a, b in pairs:
        Ca, Cb = comps[a], comps[b]
        cands = []
        for sample in range(lam * lam):
            r = philox4x32_10((a, b, sample, cloud), key)
            u = int(Ca[uniform_index(r[0], len(Ca))])
            v = int(Cb[uniform_index(r[1], len(Cb))])
            cands.append((sqdist(X64, u, v), u, v))
        cands.sort(key=lambda c: c[0])          # stable: ties keep sample order
        for s, u, v in cands[:lam]:
            out_u.append(u), out_v.append(v), out_s.append(s)
            out_a.append(a), out_b.append(b)
    i64 = lambda x: np.array(x, dtype=np.int64)
    return EdgeSet(i64(out_u), i64(out_v), np.array(out_s, dtype=np.float64), i64(out_a), i64(out_b))


# ------------------------------------------------ Phase 3: Alg. 4 (refine)
def refine_edges_literal(X, G, comp, E: EdgeSet):
    """Alg. 4 written out loop by loop (for small inputs)."""
    X64 = as64(X)
    R = E.copy()
    delta = 0
    for e in range(len(E)):
        u, v, d, a, b = int(E.u[e]), int(E.v[e]), float(E.s[e]), int(E.a[e]), int(E.b[e])
        us, vs, ds = u, v, d
        Nu = [int(w) for w in G[u] if comp[w] == a]
        Nv = [int(w) for w in G[v] if comp[w] == b]
        for up in Nu:
            if up != v:
                dp = sqdist(X64, up, v)
                if dp < ds:
                    us, ds = up, dp
        for vp in Nv:
            if vp != u:
                dp = sqdist(X64, us, vp)
                if dp < ds:
                    vs, ds = vp, dp
        if (us, vs) != (u, v):
            delta += 1
        R.u[e], R.v[e], R.s[e] = us, vs, ds
    return R, delta


def refine_edges(X, G, comp, E: EdgeSet):
    """Alg. 4, one round.  Each edge only reads X, G and its own endpoints,
    so edges are independent.  A scan in ascending order with a strict "<"
    ends at the first index attaining the minimum when that minimum beats
    the incumbent, which is what argmin returns; this vectorised form is
    checked against refine_edges_literal in the tests."""
    X64 = as64(X)
    R = E.copy()
    delta = 0
    for e in range(len(E)):
        u, v, d, a, b = int(E.u[e]), int(E.v[e]), float(E.s[e]), int(E.a[e]), int(E.b[e])
        us, vs, ds = u, v, d
        Nu = G[u][(comp[G[u]] == a) & (G[u] != v)]
        if len(Nu):
            su = sqdist_to(X64, v, Nu)
            m = int(np.argmin(su))
            if su[m] < ds:
                us, ds = int(Nu[m]), float(su[m])
        Nv = G[v][(comp[G[v]] == b) & (G[v] != u)]
        if len(Nv):
            sv = sqdist_to(X64, us, Nv)
            m = int(np.argmin(sv))
            if sv[m] < ds:
                vs, ds = int(Nv[m]), float(sv[m])
        if (us, vs) != (u, v):
            delta += 1
        R.u[e], R.v[e], R.s[e] = us, vs, ds
    return R, delta


# --------------------------------------------------- Phase 4: Kruskal / Prim
class DisjointSet:
    def __init__(self, n):
        self.p = list(range(n))

    def find(self, x):
        root = x
        while self.p[root] != root:
            root = self.p[root]
        while self.p[x] != root:
            self.p[x], x = root, self.p[x]
        return root

    def union(self, a, b):
        ra, rb = self.find(a), self.find(b)
        if ra == rb:
            return False
        if ra < rb:
            ra, rb = rb, ra
        self.p[ra] = rb
        return True


def canonical_edges(eu, ev, w):
    """Edges as (min, max, w) with duplicates on (min, max) removed (the
    first occurrence's weight is kept) and self-loops dropped."""
    seen = {}
    for a, b, x in zip(np.asarray(eu).tolist(), np.asarray(ev).tolist(), np.asarray(w).tolist()):
        if a == b:
            continue
        key = (a, b) if a < b else (b, a)
        if key not in seen:
            seen[key] = float(x)
    keys = sorted(seen)
    lo = np.array([k[0] for k in keys], dtype=np.int64)
    hi = np.array([k[1] for k in keys], dtype=np.int64)
    ww = np.array([seen[k] for k in keys], dtype=np.float64)
    return lo, hi, ww


def kruskal(n: int, eu, ev, w):
    """Kruskal (Sec. 2.1): sort edges ascending by (w, min, max), accept an
    edge when its endpoints are in different sets, stop at n-1 edges.
    Returns (tu, tv, tw, W, spanning) with the tree in acceptance order and
    W the exactly rounded sum of the accepted weights."""
    lo, hi, ww = canonical_edges(eu, ev, w)
    order = np.lexsort((hi, lo, ww))
    ds = DisjointSet(n)
    tu, tv, tw = [], [], []
    for e in order:
        if ds.union(int(lo[e]), int(hi[e])):
            tu.append(int(lo[e])), tv.append(int(hi[e])), tw.append(float(ww[e]))
            if len(tu) == n - 1:
                break
    return (np.array(tu, dtype=np.int64), np.array(tv, dtype=np.int64),
            np.array(tw, dtype=np.float64), math.fsum(tw), len(tu) == n - 1)


def prim_exact(X):
    """Exact MST of the complete Euclidean graph by Prim's algorithm in
    O(n^2 d) with direct-difference float64 distances.  Returns (tu, tv,
    tw, W) with (tu[i], tv[i]) = (parent, vertex) in insertion order."""
    X64 = as64(X)
    n = X64.shape[0]
    in_tree = np.zeros(n, dtype=bool)
    best = np.full(n, np.inf)
    parent = np.full(n, -1, dtype=np.int64)
    best[0] = 0.0
    tu, tv, tw = [], [], []
    for _ in range(n):
        cand = np.where(in_tree, np.inf, best)
        v = int(np.argmin(cand))
        in_tree[v] = True
        if parent[v] >= 0:
            tu.append(int(parent[v])), tv.append(v), tw.append(math.sqrt(best[v]))
        s = sqdist_to(X64, v, np.arange(n))
        upd = (~in_tree) & (s < best)
        best[upd] = s[upd]
        parent[upd] = v
    return (np.array(tu, dtype=np.int64), np.array(tv, dtype=np.int64),
            np.array(tw, dtype=np.float64), math.fsum(tw))


def relative_error(W_approx: float, W_exact: float) -> float:
    """Eq. (1): (W_approx - W_exact) / W_exact."""
    return (W_approx - W_exact) / W_exact


# ----------------------------------------------------------- Alg. 1 driver
@dataclass
class FamstResult:
    nbr: np.ndarray
    sq: np.ndarray
    G: list
    comp: np.ndarray
    comps: list
    E0: EdgeSet
    E: EdgeSet
    rounds: int
    deltas: list
    tu: np.ndarray
    tv: np.ndarray
    tw: np.ndarray
    W: float
    spanning: bool
    extra: dict = field(default_factory=dict)


def final_edges(nbr, sq, E: EdgeSet):
    """Edge list of the final graph: the kNN edges (i, N[i][m]) with their
    distances and the refined inter-component edges (Alg. 1, GetMST)."""
    n, k = nbr.shape
    iu = np.repeat(np.arange(n, dtype=np.int64), k)
    eu = np.concatenate([iu, E.u])
    ev = np.concatenate([nbr.reshape(-1), E.v])
    w = np.sqrt(np.concatenate([sq.reshape(-1), E.s]))
    return eu, ev, w


def famst(X, k: int, lam: int, seed: int = 0, max_rounds: int = 10, cloud: int = 0,
          nbr=None, sq=None) -> FamstResult:
    """Alg. 1: kNN -> components -> lambda-edges -> refine until no change
    (at most ``max_rounds`` rounds) -> Kruskal.  ``nbr``/``sq`` may supply
    Phase 1's output (e.g. to run the later phases on given lists)."""
    X64 = as64(X)
    n = X64.shape[0]
    if nbr is None:
        nbr, sq = knn_exact(X64, k)
    nbr = np.asarray(nbr, dtype=np.int64)
    if sq is None:
        sq = np.array([sqdist_to(X64, i, nbr[i]) for i in range(n)])
    G = undirected_graph(nbr, n)
    comp, comps = components(G)
    E0 = random_edges(X64, comps, lam, seed, cloud)
    E, deltas = E0, []
    for _ in range(max_rounds):
        E, delta = refine_edges(X64, G, comp, E)
        deltas.append(delta)
        if delta == 0:
            break
    eu, ev, w = final_edges(nbr, sq, E)
    tu, tv, tw, W, spanning = kruskal(n, eu, ev, w)
    return FamstResult(nbr, sq, G, comp, comps, E0, E, len(deltas), deltas, tu, tv, tw, W, spanning)


def famst_batched(X, offs, k, lam, seed=0, max_rounds=10):
    """One FAMST run per cloud (rows offs[b]:offs[b+1]); the cloud index
    enters the random-edge counter."""
    out = []
    for b in range(len(offs) - 1):
        Xb = np.asarray(X)[offs[b]:offs[b + 1]]
        kb = min(k, Xb.shape[0] - 1)
        out.append(famst(Xb, kb, lam, seed, max_rounds, cloud=b))
    return out


# ------------------------------------------------------------ gradients
def mst_weight_grad(X, tu, tv):
    """Gradient of W = sum over tree edges of ||x_i - x_j|| with the tree
    held fixed: each edge adds (x_i - x_j)/||x_i - x_j|| to row i and the
    negative to row j (zero for a zero-length edge)."""
    X64 = as64(X)
    g = np.zeros_like(X64)
    for i, j in zip(np.asarray(tu).tolist(), np.asarray(tv).tolist()):
        diff = X64[i] - X64[j]
        w = math.sqrt(float(np.dot(diff, diff)))
        if w > 0.0:
            g[i] += diff / w
            g[j] -= diff / w
    return g


def fd_grad(weight_fn, X, coords, h: float = 1e-6):
    """Central finite differences (W(X + h e) - W(X - h e)) / 2h of a
    float64 weight function at the listed (row, col) coordinates."""
    X64 = as64(X)
    out = np.empty(len(coords))
    for c, (i, j) in enumerate(coords):
        Xp = X64.copy()
        Xm = X64.copy()
        Xp[i, j] += h
        Xm[i, j] -= h
        out[c] = (weight_fn(Xp) - weight_fn(Xm)) / (2.0 * h)
    return out


def recall_at_k(nbr_test, nbr_exact) -> float:
    """Mean over rows of |N_test[i] & N_exact[i]| / k."""
    nbr_test = np.asarray(nbr_test)
    nbr_exact = np.asarray(nbr_exact)
    k = nbr_exact.shape[1]
    hits = sum(len(set(a.tolist()) & set(b.tolist())) for a, b in zip(nbr_test, nbr_exact))
    return hits / (k * nbr_exact.shape[0])
