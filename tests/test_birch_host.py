"""BIRCH (the clustering step after the FFP): the oracle pinned against
scikit-learn's Birch, the oracle's own invariants, and the library's host
CF-tree against the oracle.  CPU only: the CF-tree is host logic, reached
through the C ABI with host input."""
import warnings

import numpy as np
import pytest

from oracle import birch, ffp
from workloads import dcsbm


def blobs(n, d, k, spread, seed):
    rng = np.random.default_rng(seed)
    c = rng.normal(size=(k, d)) * 3.0
    return c[rng.integers(0, k, size=n)] + rng.normal(size=(n, d)) * spread


def embedding(N=1000, d=32):
    g = dcsbm(N, 11, seed=0)
    rp, ci, _, _ = ffp.canonical_csr(g.src, g.dst, g.N)
    return ffp.ffp_from_input(rp, ci, g.N, -1.0, 8, ffp.gaussian_input(g.N, d, 1))


CASES = [  # (name, data, threshold, branching factor)
    ("blobs_2d", lambda: blobs(300, 2, 6, 0.5, 0), 0.5, 5),
    ("blobs_8d", lambda: blobs(2000, 8, 20, 0.3, 1), 0.5, 50),
    ("blobs_16d_b3", lambda: blobs(1500, 16, 10, 0.2, 2), 0.6, 3),
    ("embedding", lambda: embedding(), 0.7, 50),
    ("embedding_b10", lambda: embedding(), 0.5, 10),
]


@pytest.mark.parametrize("name,make,thr,B", CASES)
def test_oracle_matches_sklearn(name, make, thr, B):
    """Same partition and the same set of cluster centroids as scikit-learn's
    Birch(n_clusters=None).  (The numbering of the clusters may differ: the
    library breaks the farthest-pair choice of a split on rounding.)"""
    from sklearn.cluster import Birch
    from sklearn.metrics import adjusted_rand_score
    X = make()
    o = birch.Birch(thr, B).fit(X)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        sk = Birch(n_clusters=None, threshold=thr, branching_factor=B).fit(X)
    co, cs = o.centers(), sk.subcluster_centers_
    assert co.shape == cs.shape
    assert np.allclose(co[np.lexsort(co.T)], cs[np.lexsort(cs.T)], rtol=0, atol=1e-12)
    assert adjusted_rand_score(o.predict(X), sk.labels_) == 1.0


def leaves(o):
    out, leaf = [], o.first_leaf
    while leaf is not None:
        out.append(leaf)
        leaf = leaf.next_leaf
    return out


def walk(node, depth, acc):
    acc.append((node, depth))
    for ch in node.child:
        if ch is not None:
            walk(ch, depth + 1, acc)
    return acc


@pytest.mark.parametrize("name,make,thr,B", CASES)
def test_oracle_invariants(name, make, thr, B):
    """CF bookkeeping and the tree's shape: every point counted once, linear
    and squared sums add up, every node holds at most B entries, inner
    entries summarise their child, all leaves at one depth, the leaf list
    holds exactly the tree's leaves, and absorbed entries keep their radius
    within the threshold."""
    X = make()
    o = birch.Birch(thr, B).fit(X)
    nodes = walk(o.root, 0, [])
    leaf_nodes = [n for n, _ in nodes if n.leaf]
    assert {id(n) for n in leaf_nodes} == {id(n) for n in leaves(o)}
    assert len({dep for n, dep in nodes if n.leaf}) == 1
    for n, _ in nodes:
        assert 1 <= len(n.n) <= B
        if not n.leaf:
            for k, ch in enumerate(n.child):
                assert n.n[k] == sum(ch.n)
                assert np.allclose(n.ls[k], ch.ls.sum(axis=0), rtol=1e-12, atol=1e-9)
                assert abs(n.ss[k] - sum(ch.ss)) <= 1e-9 * max(1.0, abs(n.ss[k]))
    n_all = sum(sum(lf.n) for lf in leaf_nodes)
    ls_all = sum(lf.ls.sum(axis=0) for lf in leaf_nodes)
    assert n_all == X.shape[0]
    assert np.allclose(ls_all, X.sum(axis=0), rtol=1e-10, atol=1e-8)
    for lf in leaf_nodes:
        for k in range(len(lf.n)):
            if lf.n[k] > 1:
                c = lf.ls[k] / lf.n[k]
                assert lf.ss[k] / lf.n[k] - c @ c <= thr * thr + 1e-9


def test_oracle_degenerate():
    X = np.ones((50, 4))
    o = birch.Birch(0.0, 5).fit(X)          # identical points merge even at threshold 0
    assert o.centers().shape == (1, 4)
    assert (o.predict(X) == 0).all()
    Y = np.arange(40, dtype=np.float64)[:, None] * np.ones((1, 3))
    o = birch.Birch(0.0, 2).fit(Y)          # distinct points never merge; B = 2 splits often
    assert o.centers().shape == (40, 3)
    assert sorted(o.centers()[:, 0]) == list(range(40))
    assert np.array_equal(np.sort(o.predict(Y)), np.arange(40))


def test_oracle_partial_fit_is_sequential_fit():
    """Alg. 2 fits new nodes' embeddings into the existing tree: inserting in
    parts equals inserting everything in the same order."""
    X = blobs(900, 8, 12, 0.4, 3)
    a = birch.Birch(0.5, 10).fit(X)
    b = birch.Birch(0.5, 10)
    for lo in range(0, 900, 250):
        b.partial_fit(X[lo:lo + 250])
    assert np.array_equal(a.centers(), b.centers())


def test_planted_mistake_in_split_breaks_the_pin():
    """A split that sends ties and near entries to the wrong seed changes the
    clusters found, so the sklearn pin would catch it."""
    from sklearn.cluster import Birch
    X = blobs(2000, 8, 20, 0.3, 1)

    class Wrong(birch.Birch):
        def _split(self, node):
            a, b = super()._split(node)
            if len(a.n) > 1 and len(b.n) > 0:   # move one entry across
                b.append(a.n.pop(), a.ls[-1], a.ss.pop(), a.child.pop())
                a.ls = a.ls[:-1]
            return a, b
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        sk = Birch(n_clusters=None, threshold=0.5, branching_factor=5).fit(X)
    w = Wrong(0.5, 5).fit(X).centers()
    cs = sk.subcluster_centers_
    assert w.shape != cs.shape or not np.allclose(w[np.lexsort(w.T)], cs[np.lexsort(cs.T)])


# ---------------------------------------------------------------- library CF-tree
@pytest.fixture(scope="module")
def ifgp():
    import paper_2508_19737_amd as m
    return m


@pytest.mark.parametrize("name,make,thr,B", CASES)
def test_library_tree_equals_oracle(ifgp, name, make, thr, B):
    """The host CF-tree behind ifgp_birch_partial_fit takes the oracle's
    decisions: the same clusters in the same order, centroids to the last
    bit (both FP64, same operations)."""
    X = make().astype(np.float32)
    o = birch.Birch(thr, B).fit(X.astype(np.float64))
    b = ifgp.Birch(X.shape[1], thr, B)
    for lo in range(0, X.shape[0], 333):      # in parts: partial fits chain
        b.partial_fit(X[lo:lo + 333])
    info = b.info()
    assert info["points"] == X.shape[0]
    c = b.centers()
    assert c.shape == o.centers().shape == (info["clusters"], X.shape[1])
    assert np.array_equal(c, o.centers())
    b.destroy()


def test_library_birch_argument_errors(ifgp):
    with pytest.raises(ifgp.IfgpError) as e:
        ifgp.Birch(0, 0.5)
    assert e.value.status == -1
    with pytest.raises(ifgp.IfgpError):
        ifgp.Birch(4, -1.0)
    with pytest.raises(ifgp.IfgpError):
        ifgp.Birch(4, 0.5, 1)
    b = ifgp.Birch(4, 0.5)
    with pytest.raises(ifgp.IfgpError):
        b.partial_fit(np.zeros((3, 5), np.float32))
    assert b.info() == {"points": 0, "clusters": 0, "height": 1}
    b.destroy()
    with pytest.raises(ifgp.IfgpError):
        b.info()
