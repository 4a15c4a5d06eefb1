"""The row-level tolerance (tests/errbound.py) on the CPU: it is not vacuous,
and the row mistakes a hop kernel can make break it.

A reference with a planted mistake stands in for a HIP path with that bug:
each planted output must leave the bound of the correct reference on the
affected row, for 2-byte (BF16) and FP32 storage, at one and two hops."""
import numpy as np
import pytest

from oracle import ffp
from workloads import dcsbm, gaussian_features, with_hubs
import errbound


@pytest.fixture(scope="module")
def hubby():
    g = dcsbm(20_000, 30, mean_deg=20.0, ratio=2.5, seed=5)
    src, dst = with_hubs(g, hubs=(6000,), medium=30)
    rp, ci, _, _ = ffp.canonical_csr(src, dst, g.N)
    X = gaussian_features(g.N, 64, 1).astype(np.float32)
    return rp, ci, g.N, X


def _row_y(ctx, i, keep=None):
    """y of row i recomputed with only the neighbours `keep` (a mask)."""
    A, s, W, a, b = ctx["A"], ctx["s"], ctx["Wprev"], ctx["a"], ctx["b"]
    lo, hi = A.indptr[i], A.indptr[i + 1]
    nb = A.indices[lo:hi]
    if keep is not None:
        nb = nb[keep]
    agg = a[0] * W[nb].sum(axis=0) + b[0] * s[nb].sum()
    return ctx["theta"] * ctx["Zn"][i] + ctx["alpha"] * s[i] * agg


def _store(ctx, i, y):
    W, _, _ = errbound.grid_round(ctx["s"][i] * np.tanh(y), ctx["storage"])
    ctx["W"][i] = W


@pytest.mark.parametrize("storage,K", [("bf16", 1), ("bf16", 2), ("f32", 1), ("f32", 2)])
def test_planted_row_mistakes_break_the_bound(hubby, storage, K):
    rp, ci, N, X = hubby
    deg = np.diff(rp)
    ref, B = errbound.reference_and_bound(rp, ci, N, -1.0, K, X, storage)
    cls = errbound.row_classes(deg)
    hub = int(np.flatnonzero(cls["hub"])[0])
    med = np.flatnonzero(cls["medium"])[:2]
    rng = np.random.default_rng(3)
    light = rng.choice(np.flatnonzero(cls["light"] & (deg >= 2)), size=200, replace=False)
    last = K - 1

    def plant_hub(hop, ctx):            # one wave's quarter of the hub's neighbours lost
        if hop == last:
            keep = np.arange(deg[hub]) % 4 != 3
            _store(ctx, hub, _row_y(ctx, hub, keep))

    def plant_swap(hop, ctx):           # a medium row written with another's result
        if hop == last:
            ctx["W"][med[0]] = ctx["W"][med[1]] * ctx["s"][med[0]] / ctx["s"][med[1]]

    def plant_drop(hop, ctx):           # each sampled light row loses its last neighbour
        if hop == last:
            for i in light:
                keep = np.arange(deg[i]) != deg[i] - 1
                _store(ctx, i, _row_y(ctx, i, keep))

    def plant_shift(hop, ctx):          # a light row's columns moved by one 16-byte lane
        if hop == last:
            ctx["W"][light[0]] = np.roll(ctx["W"][light[0]], 8)

    def caught(plant, rows):
        bad, _ = errbound.reference_and_bound(rp, ci, N, -1.0, K, X, storage, plant=plant,
                                              with_bound=False)
        return np.array([np.any(np.abs(bad[i] - ref[i]) > B[i]) for i in np.atleast_1d(rows)])

    assert caught(plant_hub, hub).all()
    assert caught(plant_swap, med[0]).all()
    assert caught(plant_shift, light[0]).all()
    frac = caught(plant_drop, light).mean()
    print(f"{storage} K={K}: dropped neighbour caught on {frac:.1%} of light rows")
    assert frac >= 0.95


def test_bound_is_tight_where_storage_rounding_is_exact(hubby):
    """Light rows of the first hop: the stored input is reproduced exactly, so
    what is left is FP32 arithmetic and the rare stored value that may round
    the other way (whose whole unit in the last place enters the column
    statistics): a few 1e-6 (FP32) to 1e-5 (BF16) on outputs in (0, 1)."""
    rp, ci, N, X = hubby
    deg = np.diff(rp)
    for storage in ("f32", "bf16", "f16"):
        _, B = errbound.reference_and_bound(rp, ci, N, -1.0, 1, X, storage)
        light = errbound.row_classes(deg)["light"]
        print(storage, "light-row bound: median", np.median(B[light]), "max", B[light].max())
        assert np.median(B[light]) < 3e-5


def test_grid_round_matches_the_types():
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-9, 4, 20000),
                        [0.0, 1.0, -2.0, 65504.0, 2.0 ** -24, 3 * 2.0 ** -26]])
    r16, _, d16 = errbound.grid_round(v, "f16")
    assert np.array_equal(r16, v.astype(np.float16).astype(np.float64))
    r32, _, _ = errbound.grid_round(v, "f32")
    assert np.array_equal(r32, v.astype(np.float32).astype(np.float64))
    # bf16: round to nearest even on the top 16 bits of the float32 pattern
    f = v.astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    bf = u.astype(np.uint32).view(np.float32).astype(np.float64)
    rb, _, _ = errbound.grid_round(f.astype(np.float64), "bf16")
    assert np.array_equal(rb, bf)
    # the distance to the nearest rounding boundary: nudging v by less than it
    # never changes the rounded value
    for st in ("f16", "bf16", "f32"):
        r, _, dist = errbound.grid_round(v, st)
        for sgn in (-1, 1):
            r2, _, _ = errbound.grid_round(v + sgn * 0.999 * dist, st)
            assert np.array_equal(r2, r), st
