"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Integer work (CSR, degrees, counts) must be bit-exact; FP64 scales and the FP64
random input must agree to a few ulp; FP32 embeddings within 1e-5 relative
Frobenius error, BF16/FP16-storage embeddings within 1e-2 (the targets the
method's GPU path is held to); CPU-BIRCH NMI within 0.01 of the oracle's."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import cref, ffp  # noqa: E402
from workloads import dcsbm, gaussian_features, random_edges  # noqa: E402

FP32_TOL = 1e-5
HALF_TOL = 1e-2


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


@pytest.fixture(scope="module")
def config1():
    g = dcsbm(1000, 11, mean_deg=20.0, ratio=2.5, seed=0)
    rp, ci, _, _ = ffp.canonical_csr(g.src, g.dst, g.N)
    return g, rp, ci


@pytest.fixture(scope="module")
def config2():
    g = dcsbm(50_000, 44, mean_deg=20.0, ratio=2.5, seed=0)
    rp, ci, _, _ = ffp.canonical_csr(g.src, g.dst, g.N)
    X = ffp.gaussian_input(g.N, 64, seed=1)
    return g, rp, ci, X


def hub_graph():
    """DC-SBM plus a star centre joined to 6000 nodes and a second hub of 300:
    exercises the block-per-row and wave-per-row classes of the hop kernel."""
    g = dcsbm(20_000, 30, seed=5)
    rng = np.random.default_rng(7)
    a = rng.choice(g.N - 2, size=6000, replace=False)
    b = rng.choice(g.N - 2, size=300, replace=False)
    src = np.concatenate([g.src, np.full(6000, g.N - 1), np.full(300, g.N - 2)])
    dst = np.concatenate([g.dst, a, b])
    return src, dst, g.N


# --------------------------------------------------------------------------- CSR
def csr_cases():
    yield "config1", lambda: (lambda g: (g.src, g.dst, g.N))(dcsbm(1000, 11, seed=0))
    yield "loops_dups", lambda: (*random_edges(300, 5000, 1, self_loops=0.1, dup=0.3), 300)
    yield "empty", lambda: (np.zeros(0, np.int64), np.zeros(0, np.int64), 5)
    yield "single_node_loop", lambda: (np.array([0]), np.array([0]), 1)
    yield "all_loops", lambda: (np.arange(50), np.arange(50), 64)
    yield "pow2_N", lambda: (*random_edges(1024, 8000, 2, dup=0.1), 1024)
    yield "star", lambda: (np.zeros(9999, np.int64), np.arange(1, 10000), 10000)
    yield "hubs", hub_graph
    yield "ragged_tail", lambda: (*random_edges(4097, 4097 * 3 + 13, 3), 4097)
    yield "giant_hub", giant_hub_graph
    yield "dup_heavy", lambda: (*random_edges(8, 100_000, 4, self_loops=0.05, dup=0.9), 8)
    yield "sparse_large_N", sparse_large_graph


def sparse_large_graph():
    """30M nodes (25-bit ids), 6,000 edges: almost every bucket of rows is
    empty; ids 0 and N - 1 take part."""
    N = 30_000_000
    s, d = random_edges(N, 6000, 13, self_loops=0.01, dup=0.2)
    return np.concatenate([s, [0, N - 1, N - 1]]), np.concatenate([d, [N - 1, 0, 5]]), N


def giant_hub_graph():
    """A row of 30,000 neighbours (each edge given twice, once reversed) among
    random edges: the row's key range is larger than one block sorts in LDS."""
    rng = np.random.default_rng(11)
    N = 40_000
    leaves = rng.permutation(np.arange(1, N))[:30_000]
    rs, rd = random_edges(N, 60_000, 12, dup=0.2)
    src = np.concatenate([np.zeros(30_000, np.int64), leaves, rs])
    dst = np.concatenate([leaves, np.zeros(30_000, np.int64), rd])
    p = rng.permutation(src.size)
    return src[p], dst[p], N


@pytest.mark.parametrize("name,make", list(csr_cases()))
@pytest.mark.parametrize("on_device", [False, True])
def test_csr_bit_exact(ifgp, name, make, on_device):
    import torch
    src, dst, N = make()
    log(f"csr case {name} N={N} E={len(src)} device={on_device}")
    rp, ci, loops, dups = ffp.canonical_csr(src, dst, N)
    if on_device:
        g = ifgp.Graph(torch.as_tensor(src, device="cuda"), torch.as_tensor(dst, device="cuda"), N)
    else:
        g = ifgp.Graph(src, dst, N)
    grp, gci, gdeg = g.export_csr()
    assert np.array_equal(grp, rp)
    assert np.array_equal(gci.astype(np.int64), ci)
    assert np.array_equal(gdeg.astype(np.int64), np.diff(rp))
    info = g.info()
    assert info == {"N": N, "nnz": int(rp[-1]), "self_loops_dropped": loops, "dups_dropped": dups}
    g.destroy()


def test_out_of_range_ids_rejected(ifgp):
    with pytest.raises(ifgp.IfgpError) as e:
        ifgp.Graph(np.array([0, 1, 7]), np.array([1, 2, 3]), 5)
    assert e.value.status == -2
    with pytest.raises(ifgp.IfgpError) as e:
        ifgp.Graph(np.array([0, -1]), np.array([1, 2]), 5)
    assert e.value.status == -2


@pytest.mark.parametrize("on_device", [False, True])
@pytest.mark.parametrize("where,bad", [(0, 1000), (12_345, -1), (19_999, 1000)])
def test_out_of_range_ids_rejected_large(ifgp, on_device, where, bad):
    """Enough edges that the build's first radix pass makes the keys from the
    edge lists itself: one id out of range anywhere still fails the build
    with IFGP_E_RANGE, and a valid list of the same size builds."""
    import torch
    src, dst = random_edges(1000, 20_000, 5)
    src, dst = src.copy(), dst.copy()
    (dst if where % 2 else src)[where] = bad
    if on_device:
        src, dst = torch.as_tensor(src, device="cuda"), torch.as_tensor(dst, device="cuda")
    with pytest.raises(ifgp.IfgpError) as e:
        ifgp.Graph(src, dst, 1000)
    assert e.value.status == -2
    good_s, good_d = random_edges(1000, 20_000, 5)
    g = ifgp.Graph(good_s, good_d, 1000)
    rp, ci, _, _ = ffp.canonical_csr(good_s, good_d, 1000)
    grp, gci, _ = g.export_csr()
    assert np.array_equal(grp, rp) and np.array_equal(gci.astype(np.int64), ci)
    g.destroy()


# --------------------------------------------------------------------------- scales, noise
@pytest.mark.parametrize("tau", [-1.0, -1.5, 0.0, 2.5, -80.0, -3.0])
def test_scales_fp64(ifgp, config1, tau):
    g_, rp, _ = config1
    g = ifgp.Graph(g_.src, g_.dst, g_.N)
    got = g.export_scales(tau)
    want = ffp.scales(ffp.degrees(rp), tau)
    ulp = np.spacing(want)
    assert np.all(np.abs(got - want) <= ulp), np.max(np.abs(got - want) / ulp)
    g.destroy()


@pytest.mark.parametrize("N,d,seed", [(1000, 32, 1), (3001, 17, 2**63 + 11), (7, 1, 0)])
def test_gaussian_input(ifgp, N, d, seed):
    want = ffp.gaussian_input(N, d, seed)
    got = ifgp.gaussian_input(N, d, seed, "f64").cpu().numpy()
    # the integer stream must match exactly; the transcendental functions may
    # differ by a few ulp from the host library
    assert np.all(np.abs(got - want) <= 8 * np.spacing(np.abs(want)) + 1e-300)
    g32 = ifgp.gaussian_input(N, d, seed, "f32").cpu().numpy()
    assert np.all(np.abs(g32 - want.astype(np.float32)) <= np.spacing(np.abs(want).astype(np.float32)))
    gb = ifgp.gaussian_input(N, d, seed, "bf16").float().cpu().numpy()
    # BF16 unit roundoff 2^-8, plus the FP32 rounding on the way
    assert np.all(np.abs(gb - want) <= np.abs(want) * (2.0**-8 + 2.0**-23) + 1e-30)


# --------------------------------------------------------------------------- embeddings
def embed_gpu(ifgp, src, dst, N, tau, K, d, seed, storage="f32", **kw):
    g = ifgp.Graph(src, dst, N)
    out = g.embed(tau, K, d, seed, storage=storage, **kw).cpu().numpy()
    g.destroy()
    return out


def test_config1_fp32(ifgp, config1):
    g, rp, ci = config1
    ref = ffp.ffp_from_input(rp, ci, g.N, -1.0, 8, ffp.gaussian_input(g.N, 32, 1))
    got = embed_gpu(ifgp, g.src, g.dst, g.N, -1.0, 8, 32, 1)
    err = ffp.rel_frobenius(got, ref)
    log(f"config1 fp32 rel_frobenius={err:.3e}")
    assert err <= FP32_TOL


@pytest.mark.parametrize("storage,tol", [("bf16", HALF_TOL), ("f16", HALF_TOL)])
def test_config1_half(ifgp, config1, storage, tol):
    g, rp, ci = config1
    ref = ffp.ffp_from_input(rp, ci, g.N, -1.0, 8, ffp.gaussian_input(g.N, 32, 1))
    got = embed_gpu(ifgp, g.src, g.dst, g.N, -1.0, 8, 32, 1, storage=storage)
    err = ffp.rel_frobenius(got, ref)
    log(f"config1 {storage} rel_frobenius={err:.3e}")
    assert err <= tol


@pytest.mark.parametrize("tau", [0.0, -1.0, -1.5])
@pytest.mark.parametrize("storage,tol", [("f32", FP32_TOL), ("bf16", HALF_TOL), ("f16", HALF_TOL)])
def test_config2(ifgp, config2, tau, storage, tol):
    g, rp, ci, X = config2
    ref = cref.ffp_from_input(rp, ci, g.N, tau, 8, X)
    got = embed_gpu(ifgp, g.src, g.dst, g.N, tau, 8, 64, 1, storage=storage)
    err = ffp.rel_frobenius(got, ref)
    log(f"config2 tau={tau} {storage} rel_frobenius={err:.3e}")
    assert err <= tol


@pytest.mark.parametrize("storage,tol", [("f32", FP32_TOL), ("bf16", HALF_TOL)])
def test_hub_rows(ifgp, storage, tol):
    src, dst, N = hub_graph()
    rp, ci, _, _ = ffp.canonical_csr(src, dst, N)
    assert np.diff(rp).max() >= 6000
    ref = cref.ffp_from_input(rp, ci, N, -1.0, 8, ffp.gaussian_input(N, 32, 3))
    got = embed_gpu(ifgp, src, dst, N, -1.0, 8, 32, 3, storage=storage)
    err = ffp.rel_frobenius(got, ref)
    log(f"hubs {storage} rel_frobenius={err:.3e}")
    assert err <= tol


@pytest.mark.parametrize("d", [1, 5, 20, 100, 256])
def test_any_width(ifgp, config1, d):
    g, rp, ci = config1
    ref = ffp.ffp_from_input(rp, ci, g.N, -1.0, 4, ffp.gaussian_input(g.N, d, 9))
    got = embed_gpu(ifgp, g.src, g.dst, g.N, -1.0, 4, d, 9)
    assert got.shape == (g.N, d)
    assert ffp.rel_frobenius(got, ref) <= FP32_TOL


@pytest.mark.parametrize("kw", [dict(ddof=1), dict(alpha=0.5, theta=0.3), dict(alpha=-0.4, theta=0.9),
                                dict(eps=0.01)])
@pytest.mark.parametrize("tau", [-1.0, 2.0])
def test_parameters(ifgp, config1, kw, tau):
    g, rp, ci = config1
    ref = ffp.ffp_from_input(rp, ci, g.N, tau, 6, ffp.gaussian_input(g.N, 16, 4),
                             alpha=kw.get("alpha", 1.0), theta=kw.get("theta", 0.1),
                             eps=kw.get("eps", 1e-3), ddof=kw.get("ddof", 0))
    got = embed_gpu(ifgp, g.src, g.dst, g.N, tau, 6, 16, 4, **kw)
    assert ffp.rel_frobenius(got, ref) <= FP32_TOL


@pytest.mark.parametrize("K", [0, 1, 2])
def test_few_hops(ifgp, config1, K):
    g, rp, ci = config1
    X = ffp.gaussian_input(g.N, 32, 1)
    ref = ffp.ffp_from_input(rp, ci, g.N, -1.0, K, X)
    got = embed_gpu(ifgp, g.src, g.dst, g.N, -1.0, K, 32, 1)
    assert ffp.rel_frobenius(got, ref) <= FP32_TOL


@pytest.mark.parametrize("storage,tol", [("bf16", 2.0 ** -8), ("f16", 2.0 ** -10)])
def test_half_storage_noise(ifgp, config1, storage, tol):
    """K = 0 returns sigma(Z^(0)): the 2-byte storage path's own noise (top
    23 bits of each word, FP32 Box-Muller) against the oracle's FP64 noise,
    entry by entry within the storage rounding."""
    g, rp, ci = config1
    ref = ffp.sigmoid(ffp.gaussian_input(g.N, 32, 1))
    got = embed_gpu(ifgp, g.src, g.dst, g.N, -1.0, 0, 32, 1, storage=storage)
    err = np.abs(got - ref).max()
    log(f"{storage} K=0 max abs error {err:.2e}")
    assert err <= tol


def test_embed_x_matches_oracle(ifgp, config1):
    import torch
    g_, rp, ci = config1
    X = gaussian_features(g_.N, 24, seed=11)
    g = ifgp.Graph(g_.src, g_.dst, g_.N)
    got = g.embed_x(-1.5, 8, torch.as_tensor(X, dtype=torch.float32)).cpu().numpy()
    ref = ffp.ffp_from_input(rp, ci, g_.N, -1.5, 8, X.astype(np.float32).astype(np.float64))
    assert ffp.rel_frobenius(got, ref) <= FP32_TOL
    g.destroy()


@pytest.mark.parametrize("case", ["N1", "no_edges", "isolated_tau0", "two_nodes", "sparse_large"])
def test_degenerate_graphs(ifgp, case):
    if case == "N1":
        src, dst, N = np.zeros(0, np.int64), np.zeros(0, np.int64), 1
    elif case == "no_edges":
        src, dst, N = np.zeros(0, np.int64), np.zeros(0, np.int64), 37
    elif case == "isolated_tau0":
        src, dst = random_edges(200, 150, 4)
        N = 260
    elif case == "sparse_large":     # 1M nodes, nearly all isolated, ragged size
        N = 1_000_003
        src, dst = random_edges(N, 5000, 6)
    else:
        src, dst, N = np.array([0]), np.array([1]), 2
    rp, ci, _, _ = ffp.canonical_csr(src, dst, N)
    # Two degree-1 nodes at tau = -1 get s^2 = 1/eps = 1000: tanh saturates and
    # FP32 returns exactly +-1 for both rows where FP64 still keeps a spread of
    # ~1e-9 that ZNorm expands to +-1; that case is outside FP32's reach.
    # (the same holds for the random pairs of the sparse graph)
    taus = (0.0,) if case in ("two_nodes", "sparse_large") else (0.0, -1.0)
    for tau in taus:
        ref = ffp.ffp_from_input(rp, ci, N, tau, 3, ffp.gaussian_input(N, 8, 2))
        got = embed_gpu(ifgp, src, dst, N, tau, 3, 8, 2)
        assert np.all(np.isfinite(got))
        if case == "N1":
            # one row: zero spread, ZNorm gives 0 and sigma gives 1/2
            assert np.array_equal(got, np.full((1, 8), 0.5, np.float32))
        assert ffp.rel_frobenius(got, ref) <= FP32_TOL


def test_deterministic(ifgp, config2):
    g_, _, _, _ = config2
    g = ifgp.Graph(g_.src, g_.dst, g_.N)
    a = g.embed(-1.0, 8, 64, 1, storage="bf16").cpu().numpy()
    b = g.embed(-1.0, 8, 64, 1, storage="bf16").cpu().numpy()
    assert np.array_equal(a, b)
    g.destroy()


def test_column_separability(ifgp, config1):
    import torch
    g_, _, _ = config1
    g = ifgp.Graph(g_.src, g_.dst, g_.N)
    X = torch.as_tensor(gaussian_features(g_.N, 32, seed=3), dtype=torch.float32)
    full = g.embed_x(-1.0, 8, X).cpu().numpy()
    cols = [0, 7, 19, 31]
    part = g.embed_x(-1.0, 8, X[:, cols]).cpu().numpy()
    assert np.abs(part - full[:, cols]).max() < 1e-5
    g.destroy()


def test_trivial_eigenvector_closed_form_large(ifgp):
    """tau = 0, Z^(0)[:, c] = sqrt(deg): one layer gives
    sigma(ZNorm(tanh(1.1 sqrt(deg)))) elementwise, at any size."""
    import torch
    import scipy.special
    gr = dcsbm(400_000, 90, seed=1)
    g = ifgp.Graph(gr.src, gr.dst, gr.N)
    _, _, deg = g.export_csr()
    sq = np.sqrt(deg.astype(np.float64))
    X = torch.as_tensor(np.repeat(sq[:, None], 64, axis=1), dtype=torch.float32)
    t = np.tanh(1.1 * sq)
    want = scipy.special.expit((t - t.mean()) / t.std())
    # Storage rounds T by at most u |T| <= u (unit roundoff u = 2^-8 BF16,
    # 2^-11 FP16), ZNorm
    # scales that by 1/sigma and the sigmoid's slope is at most 1/4; FP32
    # keeps ~1e-7 relative error through the same steps.
    sd = t.std()
    bound = {"f32": 2e-6, "bf16": 1.5 * 0.25 * 2.0**-8 / sd, "f16": 1.5 * 0.25 * 2.0**-11 / sd}
    for storage, tol in bound.items():
        got = g.embed_x(0.0, 1, X, storage=storage).cpu().numpy()
        err = np.abs(got - want[:, None]).max()
        log(f"trivial eigvec {storage} max abs err {err:.2e} (bound {tol:.2e})")
        assert err <= tol
    g.destroy()


def test_nmi_gate(ifgp, config1):
    """CPU BIRCH on the GPU embedding and on the oracle's: NMI against the
    planted blocks within 0.01."""
    from sklearn.cluster import Birch
    from sklearn.metrics import normalized_mutual_info_score as nmi
    g, rp, ci = config1
    ref = ffp.ffp_from_input(rp, ci, g.N, -1.0, 8, ffp.gaussian_input(g.N, 32, 1))
    for storage in ("f32", "bf16"):
        got = embed_gpu(ifgp, g.src, g.dst, g.N, -1.0, 8, 32, 1, storage=storage)
        lab_o = Birch(n_clusters=None, threshold=0.7).fit_predict(ref)
        lab_g = Birch(n_clusters=None, threshold=0.7).fit_predict(got.astype(np.float64))
        n_o, n_g = nmi(g.labels, lab_o), nmi(g.labels, lab_g)
        log(f"NMI {storage}: oracle {n_o:.4f} gpu {n_g:.4f}")
        assert abs(n_o - n_g) <= 0.01
