"""The allocation-free embedding (ifgp_embed_noalloc) through the C ABI.

It runs the kernels of ifgp_embed in the library's static device scratch
array instead of the handle's buffers, so its output must equal ifgp_embed's
bit for bit.  Calls follow each other on one stream, the later ones on
smaller inputs than the first, so that stale scratch contents from an earlier
call would show.  One FP32 case is also held to the FP64 oracle (relative
Frobenius error <= 1e-5)."""
import ctypes
import sys

import pytest

pytestmark = pytest.mark.gpu

from oracle import ffp  # noqa: E402
from workloads import dcsbm, random_edges  # noqa: E402


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ifgp():
    import torch
    import paper_2508_19737_amd as m
    assert torch.cuda.is_available()
    m.use_torch_allocator()
    return m


def _pair(ifgp, G, tau, K, d, seed, storage):
    import torch
    ref = G.embed(tau, K, d, seed, storage=storage)
    out = torch.full_like(ref, float("nan"))
    G.embed_noalloc(tau, K, d, seed, out, storage=storage)
    torch.cuda.synchronize()
    return ref, out


def test_noalloc_equals_embed_on_shrinking_inputs(ifgp):
    import torch
    big = dcsbm(150_000, 60, mean_deg=20.0, ratio=2.5, seed=11)
    small = dcsbm(3_000, 12, mean_deg=20.0, ratio=2.5, seed=12)
    Gb = ifgp.Graph(big.src, big.dst, big.N)
    Gs = ifgp.Graph(small.src, small.dst, small.N)
    # (graph, tau, K, d, seed, storage): a large BF16 call first, then smaller ones
    cases = [(Gb, -1.0, 8, 64, 1, "bf16"), (Gs, -1.5, 5, 20, 2, "f32"),
             (Gs, 0.0, 3, 7, 3, "f16"), (Gs, -1.0, 0, 16, 4, "bf16")]
    for G, tau, K, d, seed, st in cases:
        log(f"noalloc: N={G.N} tau={tau} K={K} d={d} seed={seed} storage={st}")
        ref, out = _pair(ifgp, G, tau, K, d, seed, st)
        assert torch.equal(ref, out), (G.N, tau, K, d, st)
    Gb.destroy()
    Gs.destroy()


def test_noalloc_against_oracle(ifgp):
    import torch
    g = dcsbm(1_000, 11, mean_deg=20.0, ratio=2.5, seed=0)
    G = ifgp.Graph(g.src, g.dst, g.N)
    out = torch.empty((g.N, 32), dtype=torch.float32, device="cuda")
    log("noalloc vs oracle: N=1000 d=32 tau=-1 K=8 fp32")
    G.embed_noalloc(-1.0, 8, 32, 1, out)
    ref = ffp.embed(g.src, g.dst, g.N, -1.0, 8, 32, 1)
    err = ffp.rel_frobenius(out.cpu().numpy(), ref)
    log(f"  rel_frobenius={err:.3e}")
    assert err <= 1e-5, err
    G.destroy()


def test_noalloc_table_path_and_handle_cache_untouched(ifgp):
    """A graph of 2^19 nodes or more takes the neighbour-sum table path (its
    table also lives in the scratch array); the handle's cached scales for
    another tau stay valid across the call."""
    import torch
    N = 600_000
    src, dst = random_edges(N, 3_000_000, seed=21)
    G = ifgp.Graph(src, dst, N)
    a = G.embed(-1.0, 4, 8, 5, storage="bf16")          # caches tau = -1
    log(f"noalloc: N={N} tau=-2 K=4 d=8 bf16 (table path)")
    ref, out = _pair(ifgp, G, -2.0, 4, 8, 5, "bf16")     # ref re-caches tau = -2
    assert torch.equal(ref, out)
    out2 = torch.empty_like(out)
    G.embed_noalloc(-1.0, 4, 8, 5, out2, storage="bf16")  # handle holds tau = -2
    b = G.embed(-2.0, 4, 8, 5, storage="bf16")           # cache still -2, used as is
    torch.cuda.synchronize()
    assert torch.equal(a, out2)
    assert torch.equal(b, ref)
    G.destroy()


def test_noalloc_rejects_graphs_beyond_the_scratch(ifgp):
    import torch
    N = 400_000
    src, dst = random_edges(N, 1_000_000, seed=22)
    G = ifgp.Graph(src, dst, N)
    out = torch.zeros((N, 64), dtype=torch.float32, device="cuda")
    log(f"noalloc: N={N} d=64 bf16 must be refused (host-side size check)")
    with pytest.raises(ifgp.IfgpError) as ei:
        G.embed_noalloc(-1.0, 8, 64, 1, out, storage="bf16")
    assert ei.value.status == ifgp.E_INVALID
    assert "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(out)) == 0            # nothing was enqueued
    # the handle still embeds normally afterwards
    ok = torch.empty((N, 8), dtype=torch.float32, device="cuda")
    G.embed_noalloc(-1.0, 2, 8, 1, ok, storage="bf16")
    ref = G.embed(-1.0, 2, 8, 1, storage="bf16")
    torch.cuda.synchronize()
    assert torch.equal(ok, ref)
    G.destroy()


def test_noalloc_argument_errors(ifgp):
    lib = ifgp.lib
    assert lib.ifgp_embed_noalloc(None, -1.0, 8, 32, 1, None, None, None) == ifgp.E_INVALID
    g = dcsbm(500, 5, seed=3)
    G = ifgp.Graph(g.src, g.dst, g.N)
    assert lib.ifgp_embed_noalloc(G.handle, -1.0, 8, 300, 1, None,
                                  ctypes.c_void_p(16), None) == ifgp.E_INVALID
    assert lib.ifgp_embed_noalloc(G.handle, float("nan"), 8, 32, 1, None,
                                  ctypes.c_void_p(16), None) == ifgp.E_INVALID
    assert lib.ifgp_embed_noalloc(G.handle, -1.0, 8, 32, 1, None, None, None) == ifgp.E_INVALID
    G.destroy()
