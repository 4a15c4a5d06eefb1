"""InfraredGP's training-free feed-forward propagation on AMD MI355X.

Public API (thin wrappers over the C ABI in include/ifgp.h):
    Graph(src, dst, N)            build a graph resident in HBM
    Graph.embed(tau, K, d, seed)  one FFP -> N x d FP32 embedding (torch tensor)
    Graph.embed_x(tau, K, X)      FFP from a caller-supplied input
    Graph.stream_add(src, dst)    merge an edge increment
    embed_batch(graphs, ...)      several graphs, hops batched per launch
    Graph.job_begin / job_step    hop-by-hop driving for serving loops
    gaussian_input(N, d, seed)    the random input alone
    Birch(d, threshold)           BIRCH clustering of the embeddings (host
                                  CF-tree, device labelling)
"""
from ._lib import (BF16, E_DEVICE, E_INVALID, E_OOM, E_RANGE, E_STATE, F16, F32, F64, OK,  # noqa: F401
                   EXPORTS, Birch, Graph, IfgpError, debug_grid_x, debug_hop_depth,
                   embed_batch, empty_cache, footprint_bytes, gaussian_input, job_step, lib, params,
                   use_hip_allocator, use_torch_allocator, version)

from ._lib import LIB_PATH  # noqa: E402,F401
