"""Benchmark of InfraredGP's FFP hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--storage bf16|f16|f32]

Workload (default): DC-SBM graph with N = 2,000,000 nodes, 200 planted blocks,
power-law degrees (exponent 2.5), mean degree 20 (nnz = 40,000,000 stored
entries), within/between ratio 2.5, seed 0; Gaussian input N x 64 (seed 1),
tau = -1, K = 8 hops, BF16 feature storage with FP32 accumulation.

One step = the whole path on one synthetic graph already resident in HBM as
an edge list: ifgp_build_graph (ingest, sort, dedupe, CSR, degree plan) then
ifgp_embed (scales, noise, K fused hops with column statistics, epilogue).
value = nnz * d * K / step time.  One JSON line on stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published


def hop_bytes(N, nnz, Dp, b, blocks):
    """Algorithmic bytes one hop launch moves if no gathered row is reused
    from cache: colidx 4 nnz, rowptr 8 (N+1), node info 16 N, own row read and
    new row written 2 b N Dp, neighbour rows b nnz Dp, block statistics."""
    return 4 * nnz + 8 * (N + 1) + 16 * N + 2 * b * N * Dp + b * nnz * Dp + 16 * Dp * blocks


def hop_bytes_compulsory(N, nnz, Dp, b, blocks):
    """The same with every feature row read from HBM once."""
    return 4 * nnz + 8 * (N + 1) + 16 * N + 2 * b * N * Dp + 16 * Dp * blocks


def hop_blocks(N, deg):
    hub = int((deg >= 4096).sum())
    med = int((deg >= 256).sum()) - hub
    return hub + -(-med // 4) + -(-(N - hub - med) // 256)


def cpu_info():
    model = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model


def cpu_baseline(g, rp, ci, tau, K, d, cols):
    """The FP64 oracle, as it stands, on a column sample of the same workload
    (the FFP is column-separable: each column's output depends on that column
    of the input only), timed on one host core."""
    from oracle import ffp
    t0 = time.perf_counter()
    X = ffp.gaussian_input(g.N, d, seed=1, cols=np.arange(cols))
    ffp.ffp_from_input(rp, ci, g.N, tau, K, X)
    t = time.perf_counter() - t0
    nnz = int(rp[-1])
    return {"value": nnz * cols * K / t, "unit": "nnz*d*K/s", "cores": 1, "kind": "oracle",
            "sample": f"NumPy/SciPy FP64 oracle (noise, {K} hops, sigmoid) on {cols} of {d} "
                      f"columns of the same graph; {t:.1f} s; host CPU: {cpu_info()}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--storage", default="bf16")
    ap.add_argument("--N", type=int, default=2_000_000)
    ap.add_argument("--blocks", type=int, default=200)
    ap.add_argument("--d", type=int, default=64)
    ap.add_argument("--K", type=int, default=8)
    ap.add_argument("--tau", type=float, default=-1.0)
    ap.add_argument("--cpu-cols", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate", action="store_true",
                    help="also run a plain 1 GiB copy kernel (reads 1 GiB, writes 1 GiB) so "
                         "that profiler byte counters can be scaled against known traffic")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(see the sharding note in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2508_19737_amd as ifgp
    from oracle import ffp
    from workloads import dcsbm

    def say(m):
        print(m, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    ifgp.use_torch_allocator()
    if a.calibrate:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        del x, y
    say(f"generating DC-SBM N={a.N} B={a.blocks}")
    g = dcsbm(a.N, a.blocks, mean_deg=20.0, ratio=2.5, seed=0)
    src = torch.as_tensor(g.src, device="cuda")
    dst = torch.as_tensor(g.dst, device="cuda")
    out = torch.empty((a.N, a.d), dtype=torch.float32, device="cuda")
    kw = dict(storage=a.storage)

    def step():
        G = ifgp.Graph(src, dst, a.N)
        G.embed(a.tau, a.K, a.d, 1, out=out, **kw)
        return G

    say("warmup")
    for _ in range(a.warmup):
        step().destroy()
    torch.cuda.synchronize()
    say(f"timing {a.steps} steps")
    graphs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        graphs.append(step())
        if len(graphs) > 1:
            graphs.pop(0).destroy()
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / a.steps
    G = graphs[-1]
    info = G.info()
    nnz = info["nnz"]

    # embed only (graph resident), and the hop kernel timed with HIP events
    # on the stream it runs on
    for _ in range(2):
        G.embed(a.tau, a.K, a.d, 1, out=out, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        G.embed(a.tau, a.K, a.d, 1, out=out, **kw)
    torch.cuda.synchronize()
    t_embed = (time.perf_counter() - t0) / a.steps
    G.timing(True)
    for _ in range(a.steps):
        G.embed(a.tau, a.K, a.d, 1, out=out, **kw)
    torch.cuda.synchronize()
    n_hops, hop_ms = G.timing_read()
    G.timing(False)
    hop_ms_avg = hop_ms / max(n_hops, 1)
    say(f"step {t_step*1e3:.3f} ms, embed {t_embed*1e3:.3f} ms, hop {hop_ms_avg:.4f} ms x {n_hops}")

    _, _, deg = G.export_csr()
    blocks = hop_blocks(a.N, deg)
    Dp = max(8, 1 << (a.d - 1).bit_length())
    b = {"bf16": 2, "f16": 2, "f32": 4}[a.storage]
    bytes_hop = hop_bytes(a.N, nnz, Dp, b, blocks)
    achieved = bytes_hop / (hop_ms_avg * 1e-3) / 1e9
    comp = hop_bytes_compulsory(a.N, nnz, Dp, b, blocks) / (hop_ms_avg * 1e-3) / 1e9

    cpu = None
    if not a.no_cpu_baseline:
        say("cpu baseline (oracle)")
        rp_, ci_, _ = G.export_csr()
        cpu = cpu_baseline(g, rp_, ci_.astype(np.int64), a.tau, a.K, a.d, a.cpu_cols)
    for x in graphs:
        x.destroy()

    work = nnz * a.d * a.K
    rec = {
        "metric": "FFP embed throughput (nnz*d*K/s)",
        "value": work / t_step,
        "unit": "nnz*d*K/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": a.storage,
        "data": "synthetic",
        "config": {"workload": f"DC-SBM N={a.N} nnz={nnz} d={a.d} tau={a.tau} K={a.K} "
                               f"{a.storage} storage; step = build graph + embed",
                   "N": a.N, "nnz": nnz, "d": a.d, "K": a.K, "tau": a.tau,
                   "storage": a.storage, "global_batch": 1, "parallelism": "none"},
        "embed_only": {"ms": t_embed * 1e3, "value": work / t_embed,
                       "build_ms": (t_step - t_embed) * 1e3},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "hop_kernel", "bytes_per_launch": bytes_hop,
                     "launch_ms": hop_ms_avg, "model": "no gathered row reused from cache",
                     "achieved_compulsory": comp},
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
