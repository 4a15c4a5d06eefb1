"""Seeded synthetic inputs (graphs, edge increments, request streams).

Shared by the tests, the benchmark and the oracle checks; contains no part of
the embedding arithmetic itself.
"""
from .dcsbm import Graph, dcsbm, shuffled_increments, random_edges, gaussian_features  # noqa: F401
