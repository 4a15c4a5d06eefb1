"""Pins of the FP64 oracle against what the paper and mathematics fix.

None of these compares the oracle with itself: each check goes through an
independent route (the paper's printed worked example, the spectral
definition the spatial hop is derived from, a closed form, a library routine,
brute force, or a theorem the paper states)."""
import json
import os

import networkx as nx
import numpy as np
import pytest
import scipy.special
import scipy.stats

from oracle import cref, dense, ffp
from workloads import dcsbm, random_edges

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny_graph(seed, N=40, E=70, isolated=2):
    """Random tiny graph with a few isolated nodes, several components and
    degree-1 nodes (the awkward cases of Eq. (1))."""
    rng = np.random.default_rng(seed)
    active = N - isolated
    u = rng.integers(0, active, size=E)
    v = rng.integers(0, active, size=E)
    # a pendant path attached to node 0, and a separate 2-node component
    u = np.concatenate([u, [0, active - 3, active - 2]])
    v = np.concatenate([v, [active - 3, active - 4, active - 1]])
    rp, ci, _, _ = ffp.canonical_csr(u, v, N)
    return rp, ci


# --------------------------------------------------------------------------
# Counter-based generator and the Gaussian input
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1, 12345, 2**63 + 5, 2**64 - 1])
def test_philox_matches_numpy_library(seed):
    # numpy's Philox increments its 256-bit counter before producing a block,
    # so numpy counter (i, c, 0, 0) yields the block for (i + 1, c, 0, 0).
    for i, c in [(0, 0), (5, 3), (999_999, 63), (2**40, 7), (2**64 - 2, 1)]:
        bg = np.random.Philox(key=np.array([seed, 0], dtype=np.uint64),
                              counter=np.array([i, c, 0, 0], dtype=np.uint64))
        ref = bg.random_raw(4)
        one = lambda x: np.array([x], dtype=np.uint64)  # noqa: E731
        got = ffp.philox4x64_10(one(i + 1), one(c), one(0), one(0), seed, 0)
        assert np.array_equal(np.array([g[0] for g in got], dtype=np.uint64), ref)
        assert np.array_equal(cref.philox4x64_10([i + 1, c, 0, 0], seed, 0), ref)


def test_gaussian_input_uses_all_four_words():
    """Columns 4q..4q+3 of row i come from numpy's Philox block (i+1, q):
    (cos, sin) of the Box-Muller pair on words 0-1, then on words 2-3."""
    seed, d = 99, 12
    X = ffp.gaussian_input(5, d, seed)
    for i in range(5):
        for q in range(d // 4):
            bg = np.random.Philox(key=np.array([seed, 0], dtype=np.uint64),
                                  counter=np.array([i, q, 0, 0], dtype=np.uint64))
            w = bg.random_raw(4)
            u = ((w >> np.uint64(11)).astype(np.float64) + 0.5) / 2.0**53
            for p_ in range(2):
                r = np.sqrt(-2 * np.log(u[2 * p_]))
                ang = 2 * np.pi * u[2 * p_ + 1]
                assert X[i, 4 * q + 2 * p_] == r * np.cos(ang) / np.sqrt(d)
                assert X[i, 4 * q + 2 * p_ + 1] == r * np.sin(ang) / np.sqrt(d)
    # cos and sin halves of one pair are uncorrelated
    Y = ffp.gaussian_input(20000, 4, 5)
    assert abs(np.corrcoef(Y[:, 0], Y[:, 1])[0, 1]) < 0.03
    assert abs(np.corrcoef(Y[:, 0], Y[:, 2])[0, 1]) < 0.03


def test_gaussian_input_distribution():
    d = 16
    X = ffp.gaussian_input(4000, d, seed=7)
    z = X.ravel() * np.sqrt(d)
    assert abs(z.mean()) < 0.02
    assert abs(z.var() - 1.0) < 0.02
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3
    # columns are not copies of each other; rows neither
    assert abs(np.corrcoef(X[:, 0], X[:, 1])[0, 1]) < 0.1


def test_gaussian_input_entry_depends_only_on_index():
    X = ffp.gaussian_input(50, 8, seed=3)
    sub = ffp.gaussian_input(50, 8, seed=3, rows=[7, 41], cols=[2, 5])
    assert np.array_equal(sub, X[np.ix_([7, 41], [2, 5])])
    assert not np.array_equal(ffp.gaussian_input(50, 8, seed=4), X)
    # same (i, c) entry under a different d differs only by the d^{-1/2} factor
    X16 = ffp.gaussian_input(50, 16, seed=3)
    assert np.allclose(X16[:, :8] * 4.0, X * np.sqrt(8.0), rtol=1e-15, atol=0)
    assert np.allclose(cref.gaussian_input(50, 8, 3), X, rtol=1e-14, atol=1e-15)


# --------------------------------------------------------------------------
# Laplacian: the paper's worked example (Sec. I, Fig. 1)
# --------------------------------------------------------------------------
def test_karate_printed_eigenvectors():
    gold = json.load(open(os.path.join(GOLDEN, "karate_fig1.json")))
    G = nx.karate_club_graph()
    A = nx.to_numpy_array(G, nodelist=range(34), weight=None)
    N = A.shape[0]
    src, dst = np.nonzero(np.triu(A))
    rp, ci, _, _ = ffp.canonical_csr(src, dst, N)
    # the oracle's CSR is the same graph
    assert np.array_equal(dense.dense_adjacency(rp, ci, N), A)
    # tau = 0 with no isolated node: D_tau = D exactly, so L_tau = L
    assert np.array_equal(ffp.dtau(ffp.degrees(rp), 0.0), A.sum(axis=1))
    lam, U = dense.eig(dense.laplacian_tau(A, 0.0))
    assert abs(lam[0]) < 1e-12 and lam[-1] <= 2.0 + 1e-12
    u0, u1, u33 = U[:, 0], U[:, 1], U[:, 33]
    assert gold["u0_entries_share_one_sign"] and (np.all(u0 > 0) or np.all(u0 < 0))
    dec = gold["u33_printed_decimals"]
    sign = np.sign(u33[33]) * np.sign(gold["u33_printed"]["34"])
    for node, val in gold["u33_printed"].items():
        assert round(float(sign * u33[int(node) - 1]), dec) == val
    near_zero = set((np.argsort(np.abs(u1))[:4] + 1).tolist())
    assert near_zero == set(gold["u1_entries_close_to_zero"])


# --------------------------------------------------------------------------
# Eq. (1) and the spectra it produces
# --------------------------------------------------------------------------
def test_dtau_eq1_cases():
    deg = np.array([0, 1, 2, 3, 5, 40, 100], dtype=np.int64)
    eps = 1e-3
    # tau > 0: D + tau I
    assert np.array_equal(ffp.dtau(deg, 2.5), deg + 2.5)
    # tau = 0: D, except isolated nodes which get eps
    assert np.array_equal(ffp.dtau(deg, 0.0), np.where(deg == 0, eps, deg).astype(float))
    for tau in [-1.0, -1.5, -3.0, -80.0]:
        got = ffp.dtau(deg, tau)
        want = np.maximum(deg - abs(tau), eps)
        # literal Eq. (1) equals max(deg - |tau|, eps) up to one rounding of deg - eps
        assert np.all(np.abs(got - want) <= np.maximum(deg, 1) * 2.0**-52)
        assert np.all(got > 0)
    # the literal evaluation, not max(): deg = 1, tau = -1 lands one ulp-ish above eps
    assert ffp.dtau(np.array([1]), -1.0)[0] == 1.0 - (1.0 - 1e-3)
    assert ffp.dtau(np.array([40]), -80.0)[0] == 40.0 - (40.0 - 1e-3)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("tau", [-1.5, -1.0, -0.3, 0.0, 2.0, 10.0])
def test_gershgorin_contains_spectrum(seed, tau):
    rp, ci = tiny_graph(seed)
    N = len(rp) - 1
    A = dense.dense_adjacency(rp, ci, N)
    lam = np.linalg.eigvalsh(dense.laplacian_tau(A, tau))
    lo, hi = dense.gershgorin_interval(A, tau)
    assert lam.min() >= lo - 1e-9 and lam.max() <= hi + 1e-9
    if tau >= 0:
        # conventional range [0, 2] (Sec. I)
        assert lam.min() >= -1e-9 and lam.max() <= 2 + 1e-9


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("tau", [-0.5, -1.0, -1.5, -5.0])
def test_negative_tau_gives_infrared(seed, tau):
    """tau < 0 puts frequencies below 0 (Sec. I, 'infrared'): with
    x_i = (D_tau)_ii^{1/2} on non-isolated nodes, x^T (S A S) x = 2M and
    x^T x = sum (D_tau)_ii < 2M, so lambda_min(L_tau) <= 1 - 2M / sum (D_tau)_ii < 0."""
    rp, ci = tiny_graph(seed)
    N = len(rp) - 1
    A = dense.dense_adjacency(rp, ci, N)
    deg = A.sum(axis=1)
    Dt = ffp.dtau(deg, tau)
    bound = 1.0 - A.sum() / Dt[deg > 0].sum()
    lam = np.linalg.eigvalsh(dense.laplacian_tau(A, tau))
    assert bound < 0
    assert lam.min() <= bound + 1e-9


def test_positive_tau_pushes_frequencies_to_one():
    G = nx.karate_club_graph()
    A = nx.to_numpy_array(G, nodelist=range(34), weight=None)
    spans = []
    for tau in [0.0, 5.0, 10.0, 100.0]:
        lam = np.linalg.eigvalsh(dense.laplacian_tau(A, tau))
        spans.append(max(abs(lam.min() - 1), abs(lam.max() - 1)))
    assert spans == sorted(spans, reverse=True) and spans[-1] < 0.2


def test_zero_eigenvalue_multiplicity_is_component_count():
    # Sec. I footnote; L needs deg > 0, so isolated nodes (which Eq. (1) at
    # tau = 0 maps to eps, giving them eigenvalue 1) are not counted.
    # three disjoint pieces: a random graph on 0..19, a path 20-21-22, an edge 23-24
    rng = np.random.default_rng(0)
    u = np.concatenate([rng.integers(0, 20, 60), [20, 21, 23]])
    v = np.concatenate([rng.integers(0, 20, 60), [21, 22, 24]])
    N = 26   # node 25 isolated
    rp, ci, _, _ = ffp.canonical_csr(u, v, N)
    A = dense.dense_adjacency(rp, ci, N)
    comps = nx.connected_components(nx.from_numpy_array(A))
    ncomp = sum(1 for c in comps if len(c) > 1)
    assert ncomp >= 3
    lam = np.linalg.eigvalsh(dense.laplacian_tau(A, 0.0))
    assert int((np.abs(lam) < 1e-10).sum()) == ncomp


# --------------------------------------------------------------------------
# The hop: spatial Eq. (3) against the spectral definition (Eq. (2))
# --------------------------------------------------------------------------
@pytest.mark.parametrize("alpha,theta", [(1.0, 0.1), (-0.5, 0.3), (0.7, 0.0)])
@pytest.mark.parametrize("tau", [-1.5, -1.0, 0.0, 3.0])
def test_linear_hops_match_spectral_filter(alpha, theta, tau):
    rp, ci = tiny_graph(11)
    N = len(rp) - 1
    A_sp = ffp.adjacency(rp, ci, N)
    A = dense.dense_adjacency(rp, ci, N)
    s = ffp.scales(ffp.degrees(rp), tau)
    X = np.random.default_rng(0).standard_normal((N, 5))
    Z = X.copy()
    K = 4
    for _ in range(K):
        Z = ffp.conv(A_sp, s, Z, alpha, theta)
    ref = dense.spectral_conv(dense.laplacian_tau(A, tau), X, alpha, theta, power=K)
    assert np.abs(Z - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("tau,ddof", [(-1.0, 0), (-1.5, 1), (0.0, 0), (2.0, 0)])
def test_full_ffp_matches_spectral_route(seed, tau, ddof):
    rp, ci = tiny_graph(seed)
    N = len(rp) - 1
    A = dense.dense_adjacency(rp, ci, N)
    X = ffp.gaussian_input(N, 6, seed=seed + 10)
    got = ffp.ffp_from_input(rp, ci, N, tau, 5, X, ddof=ddof)
    ref = dense.spectral_ffp(A, tau, 5, X, ddof=ddof)
    assert np.abs(got - ref).max() < 1e-10


def test_trivial_eigenvector_closed_form():
    """tau = 0, connected components without isolated nodes: D^{1/2} 1 is an
    eigenvector of L with eigenvalue 0 (Sec. I footnote), so one linear hop maps
    it to (theta + alpha) D^{1/2} 1 = 1.1 D^{1/2} 1, and one full layer gives
    sigma(ZNorm(tanh(1.1 sqrt(deg)))) elementwise."""
    g = dcsbm(600, 5, seed=4)
    rp, ci, _, _ = ffp.canonical_csr(g.src, g.dst, g.N)
    deg = ffp.degrees(rp)
    keep = deg > 0
    # restrict to nodes with degree >= 1 by relabelling
    idx = np.flatnonzero(keep)
    remap = -np.ones(g.N, dtype=np.int64)
    remap[idx] = np.arange(idx.size)
    rows = np.repeat(np.arange(g.N), deg)
    src, dst = remap[rows], remap[ci]
    rp2, ci2, _, _ = ffp.canonical_csr(src, dst, idx.size)
    deg2 = ffp.degrees(rp2).astype(float)
    X = np.repeat(np.sqrt(deg2)[:, None], 3, axis=1)
    A = ffp.adjacency(rp2, ci2, idx.size)
    s = ffp.scales(deg2, 0.0)
    assert np.allclose(ffp.conv(A, s, X), 1.1 * X, rtol=1e-13, atol=0)
    t = np.tanh(1.1 * np.sqrt(deg2))
    want = scipy.special.expit((t - t.mean()) / t.std())
    got = ffp.ffp_from_input(rp2, ci2, idx.size, 0.0, 1, X)
    assert np.allclose(got, want[:, None], rtol=1e-13, atol=1e-15)


# --------------------------------------------------------------------------
# ZNorm, sigma, structure
# --------------------------------------------------------------------------
@pytest.mark.parametrize("ddof", [0, 1])
def test_znorm_postconditions(ddof):
    T = np.tanh(np.random.default_rng(5).standard_normal((300, 7)) * 2 + 0.3)
    Z = ffp.znorm(T, ddof)
    assert np.abs(Z.mean(axis=0)).max() < 1e-13
    assert np.abs(Z.std(axis=0, ddof=ddof) - 1).max() < 1e-13
    T[:, 3] = 0.25
    Z = ffp.znorm(T, ddof)
    assert np.all(Z[:, 3] == 0)
    assert np.array_equal(ffp.znorm(T[:1], 0), np.zeros((1, 7)))
    x = np.linspace(-30, 30, 101)
    assert np.allclose(ffp.sigmoid(x), scipy.special.expit(x), rtol=1e-15, atol=0)


def test_column_separability_and_permutation_equivariance():
    g = dcsbm(300, 4, seed=2)
    N = g.N
    rp, ci, _, _ = ffp.canonical_csr(g.src, g.dst, N)
    X = ffp.gaussian_input(N, 8, seed=9)
    full = ffp.ffp_from_input(rp, ci, N, -1.0, 6, X)
    cols = [1, 4, 6]
    part = ffp.ffp_from_input(rp, ci, N, -1.0, 6, X[:, cols])
    assert np.allclose(part, full[:, cols], rtol=0, atol=1e-14)
    p = np.random.default_rng(1).permutation(N)   # new id of old node i is p[i]
    rp2, ci2, _, _ = ffp.canonical_csr(p[g.src], p[g.dst], N)
    Xp = np.empty_like(X)
    Xp[p] = X
    fullp = ffp.ffp_from_input(rp2, ci2, N, -1.0, 6, Xp)
    assert np.allclose(fullp[p], full, rtol=0, atol=1e-12)


# --------------------------------------------------------------------------
# Graph construction, brute force
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(5))
def test_csr_matches_python_sets(seed):
    N = 30
    u, v = random_edges(N, 120, seed, self_loops=0.1, dup=0.2)
    rp, ci, loops, dups = ffp.canonical_csr(u, v, N)
    adj = [set() for _ in range(N)]
    und = set()
    nloop = 0
    for a, b in zip(u.tolist(), v.tolist()):
        if a == b:
            nloop += 1
            continue
        adj[a].add(b)
        adj[b].add(a)
        und.add((min(a, b), max(a, b)))
    assert loops == nloop
    assert dups == (len(u) - nloop) - len(und)
    for i in range(N):
        row = ci[rp[i]:rp[i + 1]].tolist()
        assert row == sorted(adj[i])
    assert rp[-1] == 2 * len(und) == ffp.degrees(rp).sum()


def test_csr_rejects_out_of_range():
    with pytest.raises(ValueError):
        ffp.canonical_csr([0, 5], [1, 2], 5)
    with pytest.raises(ValueError):
        ffp.canonical_csr([-1], [1], 5)
    rp, ci, loops, dups = ffp.canonical_csr([], [], 4)
    assert rp.tolist() == [0, 0, 0, 0, 0] and ci.size == 0


# --------------------------------------------------------------------------
# The plain-C oracle against the NumPy one
# --------------------------------------------------------------------------
@pytest.mark.parametrize("tau,ddof,K", [(-1.0, 0, 8), (0.0, 1, 3), (1.5, 0, 2), (-1.5, 0, 0)])
def test_c_oracle_matches_numpy(tau, ddof, K):
    g = dcsbm(1000, 11, seed=0)
    rp, ci, _, _ = ffp.canonical_csr(g.src, g.dst, g.N)
    X = ffp.gaussian_input(g.N, 32, seed=1)
    Xc = cref.gaussian_input(g.N, 32, 1)
    assert np.abs(Xc - X).max() < 1e-14
    a = ffp.ffp_from_input(rp, ci, g.N, tau, K, X, ddof=ddof)
    b = cref.ffp_from_input(rp, ci, g.N, tau, K, X, ddof=ddof)
    assert ffp.rel_frobenius(b, a) < 1e-12


# --------------------------------------------------------------------------
# Planted mistakes: each one must be caught by a pin above
# --------------------------------------------------------------------------
def test_planted_mistakes_are_caught(monkeypatch):
    rp, ci = tiny_graph(3)
    N = len(rp) - 1
    A = dense.dense_adjacency(rp, ci, N)
    X = ffp.gaussian_input(N, 4, seed=1)
    ref = dense.spectral_ffp(A, -1.0, 3, X)

    def close():
        return np.abs(ffp.ffp_from_input(rp, ci, N, -1.0, 3, X) - ref).max() < 1e-10

    assert close()
    good_conv = ffp.conv
    mistakes = {
        "theta sign": lambda A_, s, Z, a=1.0, t=0.1: good_conv(A_, s, Z, a, -t),
        "one-sided scale": lambda A_, s, Z, a=1.0, t=0.1: t * Z + a * (s[:, None] ** 2 * (A_ @ Z)),
        "alpha/theta swapped": lambda A_, s, Z, a=1.0, t=0.1: good_conv(A_, s, Z, t, a),
    }
    for name, bad in mistakes.items():
        monkeypatch.setattr(ffp, "conv", bad)
        assert not close(), name
        monkeypatch.setattr(ffp, "conv", good_conv)
    good_dtau = ffp.dtau
    monkeypatch.setattr(ffp, "dtau", lambda deg, tau, eps=1e-3: np.maximum(np.asarray(deg, float) + tau, 1.0))
    assert not close(), "clamp to 1 instead of eps"
    monkeypatch.setattr(ffp, "dtau", good_dtau)
    good_znorm = ffp.znorm
    monkeypatch.setattr(ffp, "znorm", lambda T, ddof=0: good_znorm(T, 1 - ddof))
    assert not close(), "std divisor"
    monkeypatch.setattr(ffp, "znorm", good_znorm)
    assert close()
