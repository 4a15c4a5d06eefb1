"""Seeded synthetic inputs (graphs, edge increments, request streams).

Shared by the tests, the benchmark and the oracle checks; contains no part of
the embedding arithmetic itself.
"""
from .dcsbm import (Graph, dcsbm, gaussian_features, random_edges, shuffled_increments,  # noqa: F401
                    with_hubs)
