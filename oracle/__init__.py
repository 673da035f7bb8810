"""CPU oracle for FAMST (test infrastructure only).

May be imported only by the test suite, the package smoke check and the
benchmark's CPU-baseline leg; the HIP library never uses it.
"""
from .philox import philox4x32_10, seed_key, uniform_index  # noqa: F401
from .famst import *  # noqa: F401,F403
from .famst import (EdgeSet, FamstResult, as64, sqdist, sqdist_to, knn_bruteforce,  # noqa: F401
                    knn_exact, undirected_graph, components, random_edges,
                    refine_edges, draw_pair_samples, canonical_edges, kruskal,
                    prim_exact, relative_error, famst, famst_batched, final_edges,
                    mst_weight_grad, fd_grad, recall_at_k, DisjointSet)
