"""Plain CPU oracle for FAMST -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the package smoke check and the benchmark's CPU
baseline may import this module.  It shares no code with the HIP library
and imports nothing from it.  Everything is computed in float64 with NumPy
(the input float32 coordinates widen to float64 exactly), step by step in
the order of the paper's Algorithm 1:

  Phase 1  GetANNs         -> exact k nearest neighbours (Sec. 3, Alg. 1;
                              the paper allows any method that yields the
                              neighbour lists N and distances D)
  Phase 2  Components      -> Alg. 2 (undirected graph G and its connected
                              components, computed from the definition of
                              reachability by minimum-label propagation)
           RandomEdges     -> Alg. 3 (per component pair, the lambda
                              shortest of lambda^2 random endpoint pairs)
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
    (one matrix product per row block) and the k+margin smallest screened
    values of each row are taken; they are recomputed by direct difference
    and ordered by (s, j).  The screen is verified: every non-candidate must
    exceed the k-th exact value by more than the expansion's rounding bound,
    otherwise the row is redone by direct difference over all points.
    ``rows`` restricts the query rows.
    Returns (nbr int64 [m, k], s float64 [m, k]) with s squared distances.

    Selecting the k+margin smallest of a row: the (k+margin)-th smallest
    value of any subset of the row's columns is at least the (k+margin)-th
    smallest of the whole row, so every one of the row's k+margin smallest
    values lies at or below it.  The subset is every stride-th column
    (all columns when n <= 32768); the values at or below its threshold
    are then partitioned exactly.
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
    stride = max(1, n // 32768)
    nbr = np.empty((len(rows), k), dtype=np.int64)
    sq = np.empty((len(rows), k), dtype=np.float64)
    S_buf = np.empty((min(block, len(rows)), n))          # reused: no large allocation per block
    M_buf = np.empty(S_buf.shape, dtype=bool)
    for s0 in range(0, len(rows), block):
        rb = rows[s0:s0 + block]
        S = S_buf[:len(rb)]
        np.matmul(X64[rb], X64.T, out=S)
        S *= -2.0
        S += norms[None, :]
        S += norms[rb, None]
        S[np.arange(len(rb)), rb] = np.inf
        if kc < n - 1:
            thr = np.partition(S[:, ::stride], kc - 1, axis=1)[:, kc - 1]
            M = M_buf[:len(rb)]
            np.less_equal(S, thr[:, None], out=M)
            rr, cc = np.nonzero(M)
            bounds = np.searchsorted(rr, np.arange(len(rb) + 1))
        else:
            cand = np.argsort(S, axis=1)[:, :n - 1]
        for r, i in enumerate(rb):
            if kc < n - 1:
                c = cc[bounds[r]:bounds[r + 1]]
                c = c[np.argpartition(S[r, c], kc - 1)[:kc]]
            else:
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
    """G of Alg. 2: the symmetric closure of the kNN relation, i.e. {i, j}
    is an edge when j is in N[i] or i is in N[j].  Rows are returned sorted
    ascending without duplicates or self-loops."""
    nbr = np.asarray(nbr, dtype=np.int64)
    m, k = nbr.shape
    n = m if n is None else n
    i = np.repeat(np.arange(m, dtype=np.int64), k)
    j = nbr.reshape(-1)
    src = np.concatenate([i, j])
    dst = np.concatenate([j, i])
    keep = src != dst
    key = np.unique(src[keep] * n + dst[keep])        # sorted by (row, column), unique
    rows, cols = key // n, key % n
    starts = np.searchsorted(rows, np.arange(n + 1))
    return [cols[starts[r]:starts[r + 1]] for r in range(n)]


def components(G):
    """Connected components of G (Alg. 2): u and v share a component when a
    path of G joins them.  Computed from that definition: every vertex starts
    with its own id as label and repeatedly takes the smallest label among
    itself and its neighbours.  Labels only shrink and stay ids of the
    vertex's component, so the iteration stops, and at the fixed point
    neighbours carry equal labels: each component carries one label, which
    is its minimum vertex (that vertex can never take a smaller one).
    Components are numbered by ascending minimum vertex; members are listed
    ascending.  Returns (comp int64 [n], comps list of member arrays)."""
    n = len(G)
    deg = np.array([len(g) for g in G], dtype=np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), deg)
    dst = np.concatenate([np.asarray(g, dtype=np.int64) for g in G]) if n else np.zeros(0, np.int64)
    lab = np.arange(n, dtype=np.int64)
    changed = np.ones(n, dtype=bool)
    while changed.any():
        e = changed[src]                                  # only labels that moved can lower others
        new = lab.copy()
        np.minimum.at(new, dst[e], lab[src[e]])
        changed = new < lab
        lab = new
    mins, comp = np.unique(lab, return_inverse=True)   # mins ascending -> numbering
    comp = comp.astype(np.int64)
    order = np.argsort(comp, kind="stable")            # ascending ids within each component
    bounds = np.searchsorted(comp[order], np.arange(len(mins) + 1))
    comps = [order[bounds[c]:bounds[c + 1]] for c in range(len(mins))]
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


def draw_pair_samples(comps, a: int, b: int, lam: int, key, cloud: int = 0):
    """The lambda^2 random endpoint pairs of component pair (a, b) (Alg. 3):
    sample q takes the first two words (r0, r1) of Philox4x32-10 at counter
    (a, b, q, cloud) and picks u = C_a[(r0 |C_a|) >> 32], v = C_b[(r1 |C_b|)
    >> 32], uniformly and independently, with replacement."""
    Ca, Cb = np.asarray(comps[a]), np.asarray(comps[b])
    words = np.array([philox4x32_10((a, b, q, cloud), key)[:2] for q in range(lam * lam)],
                     dtype=np.uint64).reshape(-1, 2)
    iu = (words[:, 0] * np.uint64(len(Ca))) >> np.uint64(32)
    iv = (words[:, 1] * np.uint64(len(Cb))) >> np.uint64(32)
    return Ca[iu.astype(np.int64)].astype(np.int64), Cb[iv.astype(np.int64)].astype(np.int64)


def random_edges(X, comps, lam: int, seed: int, cloud: int = 0, pairs=None) -> EdgeSet:
    """Alg. 3: the edges of component pair a < b are the lambda samples with
    the smallest (s, q) among its lambda^2 draws (draw_pair_samples), listed
    in that order -- the stable sort by distance of the paper's listing, cut
    after lambda.  Pairs are listed in (a, b) order.  ``pairs`` restricts the
    work to the given (a, b) pairs, in the given order: every pair's draws
    come from its own counters, so a subset is computed exactly as in the
    full run."""
    X64 = as64(X)
    key = seed_key(seed)
    t = len(comps)
    if pairs is None:
        pairs = [(a, b) for a in range(t - 1) for b in range(a + 1, t)]
    parts = []
    for a, b in pairs:
        u, v = draw_pair_samples(comps, a, b, lam, key, cloud)
        diff = X64[u] - X64[v]
        s = np.einsum("ij,ij->i", diff, diff)
        keep = np.lexsort((np.arange(len(s)), s))[:lam]    # smallest (s, q)
        parts.append((u[keep], v[keep], s[keep], np.full(lam, a), np.full(lam, b)))
    if not parts:
        z = np.zeros(0, dtype=np.int64)
        return EdgeSet(z, z.copy(), np.zeros(0), z.copy(), z.copy())
    cat = [np.concatenate([p[i] for p in parts]) for i in range(5)]
    return EdgeSet(cat[0].astype(np.int64), cat[1].astype(np.int64), cat[2].astype(np.float64),
                   cat[3].astype(np.int64), cat[4].astype(np.int64))


# ------------------------------------------------ Phase 3: Alg. 4 (refine)
def refine_edges(X, G, comp, E: EdgeSet):
    """Alg. 4, one round.  Each edge only reads X, G and its own endpoints,
    so edges are independent.  For edge (u, v) of pair (a, b):
      u* = the neighbour u' of u with comp(u') = a, u' != v that has the
           smallest (s(u', v), u'), taken only if s(u', v) < s(u, v);
      v* = the neighbour v' of v with comp(v') = b, v' != u that has the
           smallest (s(u*, v'), v'), taken only if it beats the length after
           the first step.
    This is what the paper's scans in ascending id with a strict "<" end
    at: the first index attaining the minimum, when that minimum beats the
    incumbent (argmin returns the first index)."""
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
    first occurrence's weight is kept) and self-loops dropped; returned in
    ascending (min, max) order."""
    eu, ev = np.asarray(eu, dtype=np.int64), np.asarray(ev, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    lo, hi = np.minimum(eu, ev), np.maximum(eu, ev)
    pos = np.flatnonzero(lo != hi)
    lo, hi, w = lo[pos], hi[pos], w[pos]
    order = np.lexsort((np.arange(len(lo)), hi, lo))   # by (min, max), then first occurrence
    lo, hi, w = lo[order], hi[order], w[order]
    first = np.ones(len(lo), dtype=bool)
    first[1:] = (lo[1:] != lo[:-1]) | (hi[1:] != hi[:-1])
    return lo[first], hi[first], w[first]


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
