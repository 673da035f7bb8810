"""FAMST (Almansoori & Telek, arXiv 2507.14261) hot path on MI355X (gfx950).

The five phases of the method run in the HIP library libfamst.so behind a
C-ABI (include/famst.h); this package only marshals arguments:

    knn_graph     Phase 1, k nearest neighbours (exact, matrix-core screened)
    connect       Phase 2, graph, components (Alg. 2) and lambda-edges (Alg. 3)
    refine        Phase 3, edge refinement rounds (Alg. 4)
    mst           Phase 4, spanning tree (Boruvka / Kruskal / dense Prim)
    mst_backward  gradient of the tree weight
    famst         the whole pipeline (Alg. 1)
    MSTWeight     torch.autograd.Function around famst + mst_backward
"""
from .api import (Edges, FamstOut, Graph, MSTWeight, connect, famst, knn_graph, mst,  # noqa: F401
                  mst_backward, mst_backward_noalloc, mst_dense_fused, profile_enable, profile_read,
                  profile_reset, refine)
from ._lib import FamstError, load  # noqa: F401
