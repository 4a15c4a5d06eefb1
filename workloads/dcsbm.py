"""Seeded degree-corrected stochastic block model (DC-SBM) graphs.

These graphs stand in for the IEEE HPEC Graph Challenge benchmark graphs the
paper evaluates on (Sec. IV-A, Table I): planted blocks with heterogeneous
sizes, power-law degrees, a fixed ratio of within- to between-block edges,
undirected and unweighted.  The Graph Challenge generator and its graphs are
not available here, so a Poisson DC-SBM in the style of Karrer & Newman (2011)
is sampled instead:

1. block proportions p ~ Dirichlet(alpha * 1_B); sizes ~ Multinomial(N, p),
   every block non-empty;
2. node ids are a seeded random permutation of the block-ordered nodes, so
   blocks are not contiguous in id space;
3. propensities theta_i = dmin * (1 - u)^(-1/(exponent - 1)) (pdf exponent
   `exponent`), capped at the structural cutoff sqrt(mean_deg * N)
   (Boguna, Pastor-Satorras & Vespignani 2004), rescaled to mean `mean_deg`;
4. M* = round(N * mean_deg / 2) undirected edges, a fraction
   ratio / (1 + ratio) of them within blocks;
5. within-block edges: block chosen proportional to kappa_b^2 with
   kappa_b = sum of theta over the block, endpoints proportional to theta
   inside the block;
6. between-block edges: endpoints proportional to theta over all nodes,
   pairs inside one block rejected;
7. sampling repeats until exactly the target number of distinct non-loop
   edges exists in each class (first occurrences kept, in draw order).

This module holds only input generation: none of the embedding arithmetic.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Graph:
    N: int
    src: np.ndarray      # int64, one entry per undirected edge
    dst: np.ndarray      # int64
    labels: np.ndarray   # int32 planted block of each node
    theta: np.ndarray    # float64 degree propensities
    B: int

    @property
    def num_edges(self) -> int:
        return int(self.src.shape[0])


def _block_sizes(rng, N, B, alpha):
    p = rng.dirichlet(np.full(B, float(alpha)))
    sizes = rng.multinomial(N, p).astype(np.int64)
    # Every block gets at least one node: move nodes from the largest block.
    while (sizes == 0).any():
        z = int(np.flatnonzero(sizes == 0)[0])
        big = int(np.argmax(sizes))
        sizes[big] -= 1
        sizes[z] += 1
    return sizes


def _unique_pairs(u, v, N):
    """Undirected keys min*N+max with self-loops removed (draw order kept)."""
    keep = u != v
    u, v = u[keep], v[keep]
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    return lo * np.int64(N) + hi


def _collect(rng, draw, target, N):
    """Draw batches until `target` distinct keys exist; keep first occurrences."""
    keys = np.empty(0, dtype=np.int64)
    if target <= 0:
        return keys
    while True:
        need = target - keys.shape[0]
        batch = int(need * 1.25) + 1024
        u, v = draw(batch)
        keys = np.concatenate([keys, _unique_pairs(u, v, N)])
        _, first = np.unique(keys, return_index=True)
        first.sort()
        keys = keys[first]
        if keys.shape[0] >= target:
            return keys[:target]


def dcsbm(N: int, B: int, mean_deg: float = 20.0, ratio: float = 2.5,
          exponent: float = 2.5, dmin: float = 5.0, alpha: float = 2.0,
          seed: int = 0) -> Graph:
    """Sample a DC-SBM graph; deterministic for a given argument tuple."""
    if N < 2 or B < 1 or B > N:
        raise ValueError("need N >= 2 and 1 <= B <= N")
    rng = np.random.default_rng(seed)
    sizes = _block_sizes(rng, N, B, alpha)
    block_of_slot = np.repeat(np.arange(B, dtype=np.int32), sizes)
    node_of_slot = rng.permutation(N).astype(np.int64)
    labels = np.empty(N, dtype=np.int32)
    labels[node_of_slot] = block_of_slot

    u = rng.random(N)
    th = dmin * (1.0 - u) ** (-1.0 / (exponent - 1.0))
    th = np.minimum(th, np.sqrt(mean_deg * N))
    th *= mean_deg / th.mean()
    theta = np.empty(N)
    theta[node_of_slot] = th

    # Cumulative propensity over slots (block-ordered nodes).
    th_slot = theta[node_of_slot]
    cum = np.cumsum(th_slot)
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    ends = starts + sizes
    cum0 = np.concatenate([[0.0], cum])
    c_lo = cum0[starts]
    c_hi = cum0[ends]
    kappa = c_hi - c_lo
    pb = kappa ** 2
    pb /= pb.sum()
    total = cum[-1]

    # Inverse-CDF lookup through a guide table (Chen & Asau 1974): bucket b of
    # width h starts the search at the first slot whose cumulative propensity
    # exceeds b*h; a few vectorised forward steps finish it.  Same result as
    # searchsorted(cum, vals, side="right").
    h = total / N
    guide = np.searchsorted(cum, np.arange(N) * h, side="right")

    def pick(vals):
        b = np.clip((vals / h).astype(np.int64) - 1, 0, N - 1)
        idx = guide[b]
        while True:
            m = np.flatnonzero((idx < N - 1) & (cum[np.minimum(idx, N - 1)] <= vals))
            if m.size == 0:
                break
            idx[m] += 1
        return node_of_slot[np.minimum(idx, N - 1)]

    def draw_within(n):
        b = rng.choice(B, size=n, p=pb)
        lo, w = c_lo[b], kappa[b]
        a = pick(lo + rng.random(n) * w)
        c = pick(lo + rng.random(n) * w)
        return a, c

    def draw_between(n):
        a = pick(rng.random(n) * total)
        c = pick(rng.random(n) * total)
        ok = labels[a] != labels[c]
        return a[ok], c[ok]

    m_total = int(round(N * mean_deg / 2.0))
    m_in = int(round(m_total * ratio / (1.0 + ratio)))
    m_out = m_total - m_in
    k_in = _collect(rng, draw_within, m_in, N)
    k_out = _collect(rng, draw_between, m_out, N) if B > 1 else np.empty(0, np.int64)
    keys = np.concatenate([k_in, k_out])
    src = keys // N
    dst = keys % N
    # Randomise listing order and orientation so that no consumer can rely on
    # sorted input.
    order = rng.permutation(keys.shape[0])
    flip = rng.random(keys.shape[0]) < 0.5
    s, t = src[order], dst[order]
    s2 = np.where(flip, t, s)
    t2 = np.where(flip, s, t)
    return Graph(N=N, src=s2.astype(np.int64), dst=t2.astype(np.int64),
                 labels=labels, theta=theta, B=B)


def shuffled_increments(g: Graph, parts: int, seed: int):
    """Split the edge list of `g`, shuffled with `seed`, into `parts` equal
    increments (the streaming workload: edges arrive, N fixed)."""
    rng = np.random.default_rng(seed)
    order = rng.permutation(g.num_edges)
    chunks = np.array_split(order, parts)
    return [(g.src[c], g.dst[c]) for c in chunks]


def random_edges(N: int, E: int, seed: int, self_loops: float = 0.0,
                 dup: float = 0.0):
    """Uniform random pairs with optional self-loops and duplicate pairs, for
    edge-case tests of the graph build."""
    rng = np.random.default_rng(seed)
    u = rng.integers(0, N, size=E, dtype=np.int64)
    v = rng.integers(0, N, size=E, dtype=np.int64)
    if self_loops > 0 and E > 0:
        m = rng.random(E) < self_loops
        v[m] = u[m]
    if dup > 0 and E > 1:
        m = rng.random(E) < dup
        src_idx = rng.integers(0, E, size=int(m.sum()))
        sw = rng.random(src_idx.shape[0]) < 0.5
        u2, v2 = u[src_idx].copy(), v[src_idx].copy()
        u[m] = np.where(sw, v2, u2)
        v[m] = np.where(sw, u2, v2)
    return u, v


def gaussian_features(N: int, d: int, seed: int) -> np.ndarray:
    """Plain seeded Gaussian matrix (N x d, variance 1/d) for tests that feed
    a caller-supplied input; the method's own noise is drawn by each side
    from its counter-based generator."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((N, d)) / np.sqrt(d)


def with_hubs(g: Graph, hubs=(9000, 5000), medium=60, seed: int = 105):
    """`g` plus star edges that give the hop kernel's row classes rows to
    work on: node N-1-k joined to hubs[k] random other nodes (hub rows), and
    `medium` random nodes joined to 150, 158, 166, ... random nodes each
    (medium rows; some pairs may repeat, which the build merges)."""
    rng = np.random.default_rng(seed)
    N = g.N
    srcs, dsts = [g.src], [g.dst]
    for k, size in enumerate(hubs):
        srcs.append(np.full(size, N - 1 - k, dtype=np.int64))
        dsts.append(rng.choice(N - len(hubs), size=size, replace=False).astype(np.int64))
    for i, m in enumerate(rng.choice(N - len(hubs), size=medium, replace=False)):
        size = 150 + 8 * i
        srcs.append(np.full(size, m, dtype=np.int64))
        dsts.append(rng.integers(0, N, size=size, dtype=np.int64))
    return np.concatenate(srcs), np.concatenate(dsts)
