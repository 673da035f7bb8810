/*
 * famst.h -- C-ABI of libfamst, the MI355X (gfx950) implementation of the
 * data-parallel hot path of FAMST (Fast Approximate Minimum Spanning Tree,
 * Almansoori & Telek, arXiv 2507.14261).
 *
 * The method (Alg. 1 of the paper) takes n points X in d dimensions, the
 * neighbourhood size k and the number of inter-component edges lambda, and
 * returns an approximate Euclidean minimum spanning tree:
 *   famst_knn_graph    Phase 1: k nearest neighbours N and distances D
 *   famst_connect      Phase 2: undirected graph G, connected components C
 *                      (Alg. 2) and lambda inter-component edges E per
 *                      component pair (Alg. 3)
 *   famst_refine       Phase 3: neighbourhood refinement of E (Alg. 4),
 *                      repeated until no edge changes
 *   famst_mst          Phase 4: spanning tree of N u E (Kruskal, Sec. 3;
 *                      Boruvka, Sec. 2.1, gives the same tree)
 *   famst_mst_backward gradient of the tree weight W = sum of edge lengths
 *                      (the quantity of Eq. (1)) with respect to X
 *
 * Conventions shared by every call
 *   - Return value: 0 = FAMST_OK, negative = error (nothing useful was
 *     written unless stated), positive = warning (outputs are valid).
 *     Arguments are validated before any work is queued.
 *   - Pointers are DEVICE pointers unless marked "host".  X is float32
 *     row-major [n][d].  Vertex ids are int32 global row indices (n < 2^31).
 *   - Batching: a call may process B >= 1 independent point clouds stored
 *     back to back; offs (host, int64 [B+1]) holds the row offsets, with
 *     offs[0] = 0 and offs[B] = n.  offs == NULL means one cloud (B = 1).
 *     Every cloud needs at least 2 points.
 *   - Workspace: every call takes (ws, ws_bytes).  With ws == NULL the call
 *     only stores the required size in *ws_bytes and returns FAMST_OK; with
 *     ws != NULL, *ws_bytes must be at least that size.  The library never
 *     allocates device memory and keeps no state between calls, so calls
 *     with distinct workspaces may run concurrently.  The workspace must be
 *     256-byte aligned.
 *   - stream is a hipStream_t (NULL = the null stream).  Work is queued on
 *     it; calls that return host scalars synchronise it before returning,
 *     the others are asynchronous.
 *   - Distances: all comparisons use the squared Euclidean distance s; all
 *     emitted weights are w = sqrtf(s) with s computed in float32 by direct
 *     difference in one fixed reduction order, so the same pair always gets
 *     the same bits.  Where two float32 values are too close for float32 to
 *     order them safely, the pair is re-evaluated in float64.
 */
#ifndef FAMST_H
#define FAMST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define FAMST_OK              0
#define FAMST_EINVAL        (-1)  /* bad size, count, pointer or flag          */
#define FAMST_ECAPACITY     (-2)  /* an output buffer is too small; the needed
                                     size was stored where documented          */
#define FAMST_EDISCONNECTED (-3)  /* the given edges do not span every cloud   */
#define FAMST_EHIP          (-4)  /* a HIP runtime call failed                  */
#define FAMST_ENOTIMPL      (-5)  /* combination not supported                 */
#define FAMST_ENONFINITE    (-6)  /* X holds a NaN or an infinity, or (kNN)
                                     a row with squared norm above 1e37, where
                                     float32 distances would overflow        */
#define FAMST_EWORKSPACE    (-7)  /* *ws_bytes smaller than required or ws
                                     misaligned                                */
#define FAMST_ETIMEOUT      (-8)  /* a bounded wait inside a kernel ran out;
                                     the outputs are not valid (a library
                                     fault: it does not happen in a correct
                                     build)                                    */
#define FAMST_WNOTCONVERGED   1   /* refinement stopped at max_rounds with
                                     edges still changing                      */

/* screening precision for famst_knn_graph (low byte) */
#define FAMST_FP32            0
#define FAMST_BF16            1
#define FAMST_FP8_E4M3        2
/* flag: rows whose screened candidate list cannot be proven to contain the
   exact k nearest neighbours are recomputed exactly */
#define FAMST_EXACT         0x100
/* flag: approximate neighbours by NN-Descent (Dong, Charikar and Li, WWW
   2011; the paper's Phase 1 is PyNNDescent, Sec. 3) instead of the exact
   screened scan; with FAMST_FP32 only (float32 direct-difference distances) */
#define FAMST_NNDESCENT     0x200

/* tree algorithms for famst_mst */
#define FAMST_BORUVKA         0
#define FAMST_KRUSKAL         1
#define FAMST_DENSE_PRIM      2

/* slots of the optional stats array of famst_knn_graph */
#define FAMST_STAT_UNCERTIFIED   0  /* rows not proven exact after re-ranking */
#define FAMST_STAT_RECOMPUTED    1  /* rows recomputed exactly (FAMST_EXACT)  */
#define FAMST_STAT_NEAR_TIES     2  /* rows whose k-boundary needed float64   */
#define FAMST_STAT_K_CAND        3  /* candidate-list length used             */
#define FAMST_STAT_NND_ITERS     4  /* NN-Descent iterations run               */
#define FAMST_STAT_NND_UPDATES   5  /* list entries changed by the last one    */
#define FAMST_NSTATS             8

const char* famst_strerror(int status);
int famst_version(void);   /* major * 10000 + minor * 100 + patch */

/*
 * Phase 1 (Alg. 1 GetANNs; Sec. 3 allows any method producing N and D).
 * For every point i of cloud b, nbr[i][0..k) are the k points j != i of the
 * same cloud with the smallest (s(i,j), j), listed in ascending (s, j)
 * order, and dist[i][m] = sqrtf(s(i, nbr[i][m])).
 *
 * All distances of a cloud are screened with the matrix-core expansion
 * |x|^2 + |y|^2 - 2 x.y in the precision given by the low byte of
 * `precision` (float32, bfloat16, or float8 e4m3 with a per-row scale), the
 * k_cand best candidates per row are kept, and the candidates are re-ranked
 * with the direct-difference float32 distance.  A row is "certified" when
 * the screening error bound proves that no point outside its candidate
 * list can be closer than its k-th neighbour.  With FAMST_EXACT set, rows
 * that are not certified are recomputed exactly, so nbr equals the exact k
 * nearest neighbours; without it they keep the re-ranked candidates.
 *
 *   X        [n][d] float32, finite
 *   k        1 <= k <= 64 and k <= n_b - 1 for every cloud
 *   k_cand   candidate list length, 0 = default (32 for k <= 24, else 64);
 *            must be 32 or 64 and >= k
 *   nbr      out [n][k] int32 (global row ids)
 *   dist     out [n][k] float32 Euclidean distances
 *   stats    host int64 [FAMST_NSTATS] or NULL; if given the stream is
 *            synchronised and the counters above are stored
 *
 * With FAMST_NNDESCENT (precision FAMST_FP32 | FAMST_NNDESCENT) the lists
 * are NN-Descent's instead: every point starts from the 32 points that
 * follow it in its cloud (cyclically) and the lists are refined by local
 * joins (up to 8 new and 8 old samples per list and as many reverse
 * samples, proposals beating a list's 32nd entry) until fewer than 0.1 % of
 * the entries change, at most 16 iterations; nbr[i] holds the k best found,
 * in ascending (s, j) order, with float32 direct-difference distances.
 * Deterministic; no certificate (the lists are approximate).  Needs
 * k <= 32, d <= 256, n < 2^30 (FAMST_ENOTIMPL otherwise).
 * Errors: EINVAL, ENONFINITE (checked on the device; the stream is then
 * synchronised), EWORKSPACE, EHIP; ECAPACITY in exact mode when more than
 * 2048 points of a cloud lie within float32 rounding of a recomputed row's
 * k-th distance (massive exact ties); ENOTIMPL when a launch would exceed
 * 2^32 - 1 work-items.
 */
int famst_knn_graph(const float* X, int64_t n, int32_t d,
                    const int64_t* offs, int32_t B,
                    int32_t k, int32_t precision, int32_t k_cand,
                    int32_t* nbr, float* dist, int64_t* stats,
                    void* ws, size_t* ws_bytes, void* stream);

/*
 * Phase 2 (Alg. 2 and Alg. 3).
 * G: the undirected graph with an edge {i, j} for every j in N[i], as CSR:
 *    row_ptr int64 [n+1], col int32 [2*n*k capacity]; rows ascending, no
 *    duplicates, no self-loops; *n_col (host) = number of entries.
 * C: comp int32 [n] numbers the connected components of G by ascending
 *    minimum vertex (so cloud b's components follow cloud b-1's);
 *    members int32 [n] lists the vertices sorted by (comp, id);
 *    comp_ptr int64 [n+1] holds the start of each component in members
 *    (entries past the last component are unspecified);
 *    n_comp (host int32 [B]) = number of components per cloud.
 * E: for every pair of components a < b of the same cloud, lambda^2
 *    endpoint pairs (u in C_a, v in C_b) are drawn with replacement:
 *    sample q uses Philox4x32-10 (Salmon et al., SC'11) with key = seed
 *    (low word first) and counter = (a_local, b_local, q, cloud), where
 *    a_local, b_local are the component indices within the cloud; words 0
 *    and 1 pick u = members[comp_ptr[a] + (r0 * |C_a|) >> 32] and v the
 *    same way.  The lambda samples with the smallest (s, q) are kept.
 *    Pair (a, b) writes entries [p*lambda, (p+1)*lambda) where p is the
 *    pair's index in (cloud, a, b) lexicographic order; within a pair the
 *    entries are in ascending (s, q) order.  eu, ev int32, ew float32
 *    Euclidean length, ea, eb int32 global component ids.
 *    *n_edges (host) = lambda * sum_b t_b (t_b - 1) / 2.
 *    If e_cap < *n_edges, or eu == NULL, the call returns FAMST_ECAPACITY
 *    (eu == NULL: FAMST_OK) after G and C are complete and E untouched.
 *   lambda  1 <= lambda <= 32
 * The stream is synchronised (the component count sizes E).
 */
int famst_connect(const float* X, int64_t n, int32_t d,
                  const int64_t* offs, int32_t B,
                  const int32_t* nbr, int32_t k, int32_t lambda, uint64_t seed,
                  int64_t* row_ptr, int32_t* col, int64_t* n_col,
                  int32_t* comp, int32_t* members, int64_t* comp_ptr,
                  int32_t* n_comp,
                  int32_t* eu, int32_t* ev, float* ew, int32_t* ea, int32_t* eb,
                  int64_t e_cap, int64_t* n_edges,
                  void* ws, size_t* ws_bytes, void* stream);

/*
 * Phase 3 (Alg. 4, repeated while edges change; Alg. 1).
 * One round updates every edge (u, v) with components (a, b) independently:
 *   u* = the neighbour u' of u in G with comp(u') == a, u' != v, that has
 *        the smallest (s(u', v), u'), taken only if s(u', v) < s(u, v);
 *   v* = the neighbour v' of v in G with comp(v') == b, v' != u, that has
 *        the smallest (s(u*, v'), v'), taken only if it beats the length
 *        after the first step (strict).
 * Rounds repeat until no edge changes or max_rounds rounds ran
 * (1 <= max_rounds <= FAMST_REFINE_MAX_ROUNDS, else FAMST_EINVAL).  Since a
 * round's update of an edge depends only on that edge's endpoints, every
 * edge runs its own rounds until it stops changing, all in one launch, and
 * the per-round counts are kept on the device; the workspace grows with
 * max_rounds (2 KiB per round).
 *   eu, ev, ew  in/out (updated in place); ea, eb in
 *   rounds_run  host int32: rounds executed
 *   deltas      host int64 [max_rounds] or NULL: changed edges per round
 * Returns FAMST_WNOTCONVERGED if the last round still changed edges.
 * The stream is synchronised once, at the end.
 */
#define FAMST_REFINE_MAX_ROUNDS 4096
int famst_refine(const float* X, int64_t n, int32_t d,
                 const int64_t* row_ptr, const int32_t* col, const int32_t* comp,
                 int32_t* eu, int32_t* ev, float* ew,
                 const int32_t* ea, const int32_t* eb,
                 int64_t n_edges, int32_t max_rounds,
                 int32_t* rounds_run, int64_t* deltas,
                 void* ws, size_t* ws_bytes, void* stream);

/*
 * Phase 4 (Alg. 1 GetMST).  Spanning tree of each cloud over the edges
 * {i, nbr[i][m]} with weights dist[i][m] (k may be 0 with nbr = dist =
 * NULL) and the n_edges edges (eu, ev, ew).  Edges are identified by
 * (min, max) endpoint (duplicates collapse) and ordered by (w, min, max);
 * under that strict order the minimum spanning tree is unique, so every
 * algorithm returns the same tree:
 *   FAMST_BORUVKA     Boruvka rounds on the device
 *   FAMST_KRUSKAL     Kruskal: sort, then a sequential union-find scan
 *   FAMST_DENSE_PRIM  exact tree of the complete graph of each cloud
 *                     (nbr and E ignored; X used), never storing n^2 edges
 * Output: the n - B tree edges in ascending (min, max) order, tu < tv,
 * tw their weights; W (device float32 [B]) the per-cloud sum of tw,
 * accumulated with compensation in a fixed order.
 * Errors: EDISCONNECTED when the edges do not span a cloud.
 * Edge endpoints must lie in the same cloud.
 */
int famst_mst(const float* X, int64_t n, int32_t d,
              const int64_t* offs, int32_t B,
              const int32_t* nbr, const float* dist, int32_t k,
              const int32_t* eu, const int32_t* ev, const float* ew, int64_t n_edges,
              int32_t algo,
              int32_t* tu, int32_t* tv, float* tw, float* W,
              void* ws, size_t* ws_bytes, void* stream);

/*
 * Gradient of W_b = sum over tree edges of |x_i - x_j| (Eq. (1)'s W) with
 * the tree held fixed:
 *   grad_X[i] = gW[b] * sum over tree edges (i, j) of (x_i - x_j) / |x_i - x_j|
 * (an edge of zero length contributes nothing).  tu, tv as returned by
 * famst_mst (n - B edges, cloud by cloud); gW device float32 [B];
 * grad_X out [n][d], overwritten.  Each row sums its edges in ascending
 * edge order, so the result is deterministic.
 */
int famst_mst_backward(const float* X, int64_t n, int32_t d,
                       const int64_t* offs, int32_t B,
                       const int32_t* tu, const int32_t* tv, const float* gW,
                       float* grad_X,
                       void* ws, size_t* ws_bytes, void* stream);

/*
 * famst_mst_backward for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with the workspace taken from
 * a fixed device array of FAMST_NOALLOC_SCRATCH_BYTES that the library
 * holds on every GPU it runs on until the process ends.  The call allocates
 * nothing; the caller still provides X, tu, tv, gW and grad_X, and the
 * current device must be the one that owns them and the stream.
 *   scratch_needed  host, may be NULL: the workspace bytes this call needs
 * Errors: as famst_mst_backward; FAMST_ECAPACITY when the call needs more
 * than FAMST_NOALLOC_SCRATCH_BYTES (about one million points: the bytes
 * grow as 64 n), with *scratch_needed set and nothing queued.
 * Every call on one GPU shares that GPU's array: calls that overlap on the
 * same GPU (other streams, other host threads) race and must be ordered by
 * the caller.  The stream is synchronised, as in famst_mst_backward.
 */
#define FAMST_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int famst_mst_backward_noalloc(const float* X, int64_t n, int32_t d,
                               const int64_t* offs, int32_t B,
                               const int32_t* tu, const int32_t* tv, const float* gW,
                               float* grad_X, size_t* scratch_needed, void* stream);

/*
 * Exact tree weight and its gradient for a batch of clouds in one
 * persistent launch (FAMST with k = n_b - 1 is the exact minimum spanning
 * tree, Sec. 2.1 / Prim).  Blocks take clouds from a work queue, largest
 * first; each runs dense Prim on the complete graph of its cloud, the
 * compensated tree weight W[b], and the rows of
 *   G = dW_b / dX = sum over tree edges (i, j) of (x_i - x_j)/|x_i - x_j|
 * for that cloud.  Tree edges are written cloud by cloud in Prim insertion
 * order as (tu, tv) = (parent, child); each row of G sums its parent edge
 * first, then its children in ascending id, so G is deterministic.
 *   tu, tv, tw  out [n - B];  W out [B];  grad_X out [n][d] (unscaled G)
 * Every cloud must hold at most 12288 points, and for d <= 64 the work
 * items (per cloud: one per 64 tiles of 64 x 64 pairs, plus one) must number
 * below 2^31 - 2^16 (FAMST_ENOTIMPL otherwise).
 * Distances: for d <= 64 the same launch first stores the squared distance
 * of every pair of a cloud (the library's canonical float32 bits, nb^2
 * floats per cloud in the workspace, tiles spread over all blocks) and
 * Prim then reads one matrix row per step; for d > 64 they are computed on
 * the fly.  Both give the same tree.  FAMST_ETIMEOUT if a block waiting for
 * a cloud's matrix gave up (a library fault; outputs invalid).  The size
 * query (ws == NULL) asks for all matrices at once; a workspace that holds
 * at least the fixed part plus the largest cloud's matrix is accepted too,
 * and the clouds then run in consecutive groups (largest first) whose
 * matrices fit, with the same results; less is FAMST_EWORKSPACE.
 */
int famst_mst_dense_fused(const float* X, int64_t n, int32_t d,
                          const int64_t* offs, int32_t B,
                          int32_t* tu, int32_t* tv, float* tw, float* W, float* grad_X,
                          void* ws, size_t* ws_bytes, void* stream);

/*
 * Kernel timing for measurement.  While enabled, every kernel the library
 * queues is bracketed by HIP events on its stream.  famst_profile_read
 * synchronises the recorded events and returns, for kernel name `name`,
 * the number of launches and their summed duration in milliseconds since
 * the last reset.  Not thread-safe; meant for benchmarks.
 */
int famst_profile_enable(int enable);
int famst_profile_reset(void);
int famst_profile_read(const char* name, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* FAMST_H */
