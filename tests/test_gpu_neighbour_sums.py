"""Neighbour sums r_i = sum of s_j over row i's neighbours, through the C ABI.

From 2^19 nodes the kernel takes s_j from a table in LDS (one value per
bucket of consecutive internal ids of one degree; internal ids are sorted by
degree and s depends on the degree alone) and gathers it from memory only in
buckets that mix degrees.  The sums enter every hop from the second on, so
the embedding checks them against the FP64 oracle."""
import pytest

pytestmark = pytest.mark.gpu

from oracle import cref, ffp  # noqa: E402
from workloads import dcsbm  # noqa: E402
import fp32_plain  # noqa: E402


@pytest.fixture(scope="module")
def ifgp():
    import torch
    import paper_2508_19737_amd as m
    assert torch.cuda.is_available()
    m.use_torch_allocator()
    return m


@pytest.fixture(scope="module")
def g600k():
    g = dcsbm(600_000, 120, mean_deg=20.0, ratio=2.5, seed=3)
    rp, ci, _, _ = ffp.canonical_csr(g.src, g.dst, g.N)
    return g, rp, ci


@pytest.mark.parametrize("tau,K", [(-80.0, 1), (-80.0, 2), (-80.0, 4), (-1.0, 4), (0.0, 4),
                                   (2.5, 4)])
def test_neighbour_sums_from_the_s_table(ifgp, g600k, tau, K):
    """From 2^19 nodes the neighbour sums take s from a per-degree-run table
    in LDS (mixed runs gather it); 600,000 nodes, so the table covers buckets
    of 256 internal ids.  FP32 storage against the FP64 oracle on sampled
    columns (the sums enter from the second hop), for tau that clamps most
    nodes (-80: D_tau = eps below degree 81, s = 31.6), that shifts them (-1,
    2.5) and that leaves D as it is (0).

    The bound is 1e-5 relative Frobenius, or the error of a plain FP32
    evaluation of the same formulas on the CPU where that is larger: at tau =
    -80 the map amplifies any perturbation by an order of magnitude per hop
    (the FP64 oracle itself moves by 3e-6 at K = 2 when its input is perturbed
    at FP32's rounding), so FP32 arithmetic cannot meet 1e-5 there beyond the
    first hops, and the HIP path is held to doing no worse than plain FP32."""
    import torch
    cols = [0, 5]
    g, rp, ci = g600k
    assert g.N >= 2**19
    X = ffp.gaussian_input(g.N, 8, 4, cols=cols)
    ref = cref.ffp_from_input(rp, ci, g.N, tau, K, X)
    G = ifgp.Graph(torch.as_tensor(g.src, device="cuda"), torch.as_tensor(g.dst, device="cuda"), g.N)
    out = G.embed(tau, K, 8, 4, storage="f32").cpu().numpy()
    G.destroy()
    err = ffp.rel_frobenius(out[:, cols], ref)
    bound = 1e-5
    if tau <= -30:
        plain = ffp.rel_frobenius(fp32_plain.ffp_fp32(rp, ci, g.N, tau, K, X), ref)
        bound = max(bound, plain)
        print(f"600k nodes tau={tau} K={K}: plain FP32 evaluation {plain:.3e}", flush=True)
    print(f"600k nodes tau={tau} K={K}: rel_frobenius {err:.3e} (bound {bound:.1e})", flush=True)
    assert err <= bound
