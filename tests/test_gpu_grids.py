"""Launch grids past the x dimension's limit, through the C ABI.

A launch holds at most 2^32 - 1 work items per grid dimension.  The kernels
with one thread per entry of an N x d matrix, or one block per few rows, pass
that on graphs of several hundred million nodes, so their grids continue in y
once x reaches a cap.  Two checks:

* with the cap lowered to a few blocks (ifgp_debug_grid_x), a mid-sized
  workload runs every such kernel on a two-dimensional grid: every result is
  bit-identical to the default launches;
* at N = 600,000,000 nodes, where the default grids are two-dimensional and
  several kernels have more than 2^32 threads, the build and an edge
  increment give the canonical CSR and the embedding matches the FP64 oracle
  (FP32 storage)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import cref, ffp  # noqa: E402
from workloads import dcsbm, random_edges  # noqa: E402


@pytest.fixture(scope="module")
def ifgp():
    import torch
    import paper_2508_19737_amd as m
    assert torch.cuda.is_available()
    m.use_torch_allocator()
    return m


def mid_workload():
    """DC-SBM with 60,000 nodes (more than 2^19 edges, so the build's side
    stream is used) plus a star of 9,000 leaves (a hub row and an oversized
    bucket); increments of the second half of the edges and of new nodes."""
    g = dcsbm(60_000, 40, seed=5)
    leaves = np.arange(100, 9100, dtype=np.int64)
    src = np.concatenate([g.src, np.full(leaves.size, 11, dtype=np.int64)])
    dst = np.concatenate([g.dst, leaves])
    return g.N, src, dst


def run_everything(ifgp, N, src, dst, birch):
    import torch
    S = torch.as_tensor(src, device="cuda")
    D = torch.as_tensor(dst, device="cuda")
    r = {}
    G = ifgp.Graph(S, D, N)
    r["csr"] = G.export_csr()
    for storage in ("f32", "bf16", "f16"):
        r["emb_" + storage] = G.embed(-1.0, 3, 64, 7, storage=storage).cpu()
    r["emb_d20"] = G.embed(0.5, 2, 20, 7, storage="bf16").cpu()
    X = torch.as_tensor(ffp.gaussian_input(N, 48, 3).astype(np.float32), device="cuda")
    r["emb_x"] = G.embed_x(-2.0, 3, X, storage="f32").cpu()
    r["scales"] = G.export_scales(-1.0)
    r["gauss_bf16"] = ifgp.gaussian_input(N, 36, 9, dtype="bf16").cpu()
    r["gauss_f64"] = ifgp.gaussian_input(N, 5, 9, dtype="f64").cpu()
    half = src.size // 2
    H = ifgp.Graph(S[:half], D[:half], N)
    H.stream_add(S[half:], D[half:])
    r["merge_csr"] = H.export_csr()
    r["merge_emb"] = H.embed(-1.0, 3, 32, 2, storage="bf16").cpu()
    ns, nd = random_edges(N + 5000, 20_000, seed=4)
    H.stream_add(ns, nd, new_N=N + 5000)
    r["snow_csr"] = H.export_csr()
    small = ifgp.Graph(*random_edges(3000, 12_000, seed=6), 3000)
    outs = ifgp.embed_batch([G, small, H], [-1.0, -1.0, 0.0], [3, 3, 2], [64, 64, 64],
                            [1, 2, 3], storage="bf16")
    for i, o in enumerate(outs):
        r[f"batch_{i}"] = o.cpu()
    Z = G.embed(-1.0, 4, 32, 5, storage="bf16")
    r["labels"] = birch.predict(Z).cpu()
    for h in (G, H, small):
        h.destroy()
    return r


def same(a, b):
    """Bit-identical (arrays, tensors, or tuples of them)."""
    import torch
    if isinstance(a, tuple):
        return all(same(x, y) for x, y in zip(a, b))
    if isinstance(a, np.ndarray):
        return a.shape == b.shape and a.tobytes() == b.tobytes()
    ints = {1: torch.uint8, 2: torch.int16, 4: torch.int32, 8: torch.int64}[a.element_size()]
    return a.shape == b.shape and torch.equal(a.contiguous().view(ints), b.contiguous().view(ints))


def test_two_dimensional_grids_match(ifgp):
    N, src, dst = mid_workload()
    G = ifgp.Graph(src, dst, N)
    birch = ifgp.Birch(32, 0.5)
    birch.partial_fit(G.embed(-1.0, 4, 32, 5, storage="bf16"))
    G.destroy()
    print(f"BIRCH clusters {birch.info()['clusters']}", flush=True)
    ref = run_everything(ifgp, N, src, dst, birch)
    for cap in (3, 64):
        prev = ifgp.debug_grid_x(cap)
        try:
            got = run_everything(ifgp, N, src, dst, birch)
        finally:
            ifgp.debug_grid_x(prev)
        bad = [k for k in ref if not same(ref[k], got[k])]
        print(f"x cap {cap} blocks: {len(ref)} results, differing: {bad}", flush=True)
        assert not bad
    birch.destroy()


def x_input(N, d):
    """A deterministic input exact in FP32 on both sides: entry (i, c) is
    ((i * 2654435761 + c * 40503) mod 2^24) / 2^24 - 1/2."""
    i = np.arange(N, dtype=np.int64)[:, None]
    c = np.arange(d, dtype=np.int64)[None, :]
    return (((i * 2654435761 + c * 40503) % (1 << 24)).astype(np.float32) / np.float32(1 << 24)
            - np.float32(0.5))


def x_input_device(N, d):
    import torch
    i = torch.arange(N, dtype=torch.int64, device="cuda")[:, None]
    c = torch.arange(d, dtype=torch.int64, device="cuda")[None, :]
    return ((i * 2654435761 + c * 40503) % (1 << 24)).to(torch.float32) / float(1 << 24) - 0.5


def test_six_hundred_million_nodes(ifgp):
    """N = 6e8 (ids need 30 bits, so a bucket holds 4 rows: 150M bucket
    blocks), 2M random edges, a star of 10,000 leaves and 20 rows of 300
    neighbours; an increment of 1M more edges; embedding of width 1 (padded
    to 8), K = 2, tau = -1, FP32 storage, from a caller-supplied input
    (N x 8 = 4.8e9 threads in its first kernel)."""
    import torch
    N = 600_000_000
    rng = np.random.default_rng(11)
    e_rand = rng.integers(0, N, size=(2, 2_000_000), dtype=np.int64)
    star = np.stack([np.full(10_000, 123_456_789, dtype=np.int64),
                     rng.integers(0, N, size=10_000, dtype=np.int64)])
    med = np.stack([np.repeat(rng.integers(0, N, size=20, dtype=np.int64), 300),
                    rng.integers(0, N, size=6000, dtype=np.int64)])
    src = np.concatenate([e_rand[0], star[0], med[0]])
    dst = np.concatenate([e_rand[1], star[1], med[1]])
    inc = rng.integers(0, N, size=(2, 1_000_000), dtype=np.int64)
    print("N = 6e8: building", flush=True)
    G = ifgp.Graph(torch.as_tensor(src, device="cuda"), torch.as_tensor(dst, device="cuda"), N)
    plan = G.plan_info()
    print(f"plan {plan}", flush=True)
    assert plan["hub_rows"] == 1 and plan["medium_rows"] >= 20
    rp, ci, _, _ = ffp.canonical_csr(src, dst, N)
    grp, gci, gdeg = G.export_csr()
    assert np.array_equal(grp, rp) and np.array_equal(gci.astype(np.int64), ci)
    del grp, gci, gdeg
    print("N = 6e8: CSR equal; merging an increment", flush=True)
    G.stream_add(torch.as_tensor(inc[0], device="cuda"), torch.as_tensor(inc[1], device="cuda"))
    rp, ci, _, _ = ffp.canonical_csr(np.concatenate([src, inc[0]]),
                                     np.concatenate([dst, inc[1]]), N)
    grp, gci, gdeg = G.export_csr()
    assert np.array_equal(grp, rp) and np.array_equal(gci.astype(np.int64), ci)
    del grp, gci, gdeg
    print("N = 6e8: merged CSR equal; embedding", flush=True)
    X = x_input_device(N, 1)
    out = G.embed_x(-1.0, 2, X, storage="f32")
    del X
    got = out.cpu().numpy()[:, 0]
    del out
    G.destroy()
    ref = cref.ffp_from_input(rp, ci, N, -1.0, 2, x_input(N, 1).astype(np.float64))[:, 0]
    err = ffp.rel_frobenius(got[:, None], ref[:, None])
    print(f"N = 6e8: rel_frobenius {err:.3e}", flush=True)
    assert err <= 1e-5
    assert np.all(np.isfinite(got)) and got.min() > 0 and got.max() < 1
