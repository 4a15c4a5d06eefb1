"""The seeded DC-SBM generator delivers the shape it promises."""
import numpy as np

from workloads import dcsbm, shuffled_increments


def test_dcsbm_shape_and_determinism():
    g = dcsbm(5000, 20, mean_deg=20.0, ratio=2.5, seed=0)
    h = dcsbm(5000, 20, mean_deg=20.0, ratio=2.5, seed=0)
    assert np.array_equal(g.src, h.src) and np.array_equal(g.dst, h.dst)
    assert g.num_edges == 50_000                      # mean degree exactly 20
    assert np.all(g.src != g.dst)                     # no self-loops
    key = np.minimum(g.src, g.dst) * g.N + np.maximum(g.src, g.dst)
    assert np.unique(key).size == key.size            # no duplicate pairs
    assert np.bincount(g.labels, minlength=g.B).min() >= 1
    within = (g.labels[g.src] == g.labels[g.dst]).sum()
    assert within == round(50_000 * 2.5 / 3.5)        # within/between ratio 2.5
    deg = np.bincount(np.concatenate([g.src, g.dst]), minlength=g.N)
    assert deg.max() > 5 * deg.mean()                 # heavy tail
    # blocks are spread over id space, not contiguous
    assert np.abs(np.diff(g.labels)).sum() > g.N // 2


def test_increments_partition_edges():
    g = dcsbm(2000, 8, seed=0)
    parts = shuffled_increments(g, 10, seed=2)
    assert len(parts) == 10
    s = np.concatenate([p[0] for p in parts])
    t = np.concatenate([p[1] for p in parts])
    k1 = np.sort(np.minimum(s, t) * g.N + np.maximum(s, t))
    k2 = np.sort(np.minimum(g.src, g.dst) * g.N + np.maximum(g.src, g.dst))
    assert np.array_equal(k1, k2)
