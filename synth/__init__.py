"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This package holds input generation only -- Gaussian-mixture vectors, query
sets, proximity-graph construction (index building, which the paper leaves
unspecified), product-quantisation codebook training (also index building)
and random-link sample graphs -- and none of the search method's
arithmetic: there is no best-first search, no candidate list and no result
selection here.  Both the GPU path and the oracle consume what it produces.
"""
from .gmm import WORKLOADS, Workload, make_base, make_queries, make_dataset  # noqa: F401
from .graph import build_graph, random_graph, medoid  # noqa: F401
from .pq import train_codebooks  # noqa: F401
