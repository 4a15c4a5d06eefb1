"""Seeded request streams of independent DC-SBM graphs (the serving mix).

Graph sizes are log-uniform in [n_min, n_max], planted blocks ~ N^0.33, mean
degree uniform in [10, 30], within/between ratio uniform in [2, 5], width
d in {32, 64}; arrivals form a Poisson process.  To keep host-side generation
bounded, requests draw their graph from a seeded pool of `pool` distinct
graphs; every request is still built and embedded from its own edge list.
Input generation only: none of the embedding arithmetic.
"""
from __future__ import annotations

import concurrent.futures as cf
import os

import numpy as np

from .dcsbm import dcsbm


def _pool_params(pool, n_min, n_max, seed):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(pool):
        N = int(round(np.exp(rng.uniform(np.log(n_min), np.log(n_max)))))
        out.append(dict(N=N, B=max(2, int(round(N ** 0.33))),
                        mean_deg=float(rng.uniform(10.0, 30.0)),
                        ratio=float(rng.uniform(2.0, 5.0)), seed=int(seed * 100003 + k)))
    return out


def _make(p):
    g = dcsbm(p["N"], p["B"], mean_deg=p["mean_deg"], ratio=p["ratio"], seed=p["seed"])
    return g


def graph_pool(pool=32, n_min=1000, n_max=500_000, seed=3, workers=None):
    params = _pool_params(pool, n_min, n_max, seed)
    workers = workers or min(16, os.cpu_count() or 1)
    if workers <= 1:
        return [_make(p) for p in params]
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_make, params))


def request_stream(graphs, n_requests, rate, seed=3, tau=-1.0, K=8, storage="bf16"):
    """[(arrival_s, graph, d, seed)]: Poisson arrivals at `rate` per second
    (rate = inf puts every request at t = 0: a closed-loop backlog)."""
    rng = np.random.default_rng(seed + 1)
    if np.isinf(rate):
        t = np.zeros(n_requests)
    else:
        t = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
        t -= t[0]
    pick = rng.integers(0, len(graphs), size=n_requests)
    ds = rng.choice([32, 64], size=n_requests)
    return [dict(arrival=float(t[i]), graph=graphs[pick[i]], d=int(ds[i]), seed=int(i),
                 tau=tau, K=K, storage=storage) for i in range(n_requests)]
