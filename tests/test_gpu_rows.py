"""Row-level parity of the hop kernel: every row class (hub: >= 4096
neighbours, one 256-thread block per row; medium: >= 128, one wave; light: one
lane group), every gather depth (neighbour rows in flight per lane: 8, 4 --
rows of 64 columns or more -- and 16; 2-byte storage) and every storage type,
element by element.

At one and two hops every element of every hub and medium row and of a
sample of light rows must lie within the bound of tests/errbound.py around
the reference that applies the storage type's rounding exactly to the FP64
formulas (Eq. (3), (4)); the reference itself differs from the FP64 oracle
only by that rounding (printed).  At eight hops the trajectories of any two
roundings drift apart, so there each class's largest error against the FP64
oracle must be of the size the exact storage rounding alone produces: at most
3x the reference's largest error on that class, plus 1e-6 (1e-5 for FP32
storage, whose arithmetic rounds as coarsely as its storage)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import ffp  # noqa: E402
from workloads import dcsbm, gaussian_features, with_hubs  # noqa: E402
import errbound  # noqa: E402

TAU = -1.0
DEPTHS = {"8 rows": 0, "4 rows": 1, "16 rows": 2}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ifgp():
    import torch
    import paper_2508_19737_amd as m
    assert torch.cuda.is_available()
    m.use_torch_allocator()
    yield m
    m.debug_hop_depth(-1)


@pytest.fixture(scope="module")
def hubby(ifgp):
    g = dcsbm(40_000, 40, mean_deg=20.0, ratio=2.5, seed=5)
    src, dst = with_hubs(g, hubs=(9000, 5000), medium=60)
    rp, ci, _, _ = ffp.canonical_csr(src, dst, g.N)
    deg = np.diff(rp)
    cls = errbound.row_classes(deg)
    G = ifgp.Graph(src, dst, g.N)
    plan = G.plan_info()
    assert plan["hub_rows"] == cls["hub"].sum() == 2
    assert plan["medium_rows"] == cls["medium"].sum() >= 60
    rng = np.random.default_rng(9)
    rows = {"hub": np.flatnonzero(cls["hub"]), "medium": np.flatnonzero(cls["medium"]),
            "light": rng.choice(np.flatnonzero(cls["light"]), size=4000, replace=False)}
    X = gaussian_features(g.N, 64, 1).astype(np.float32)
    yield G, rp, ci, g.N, X, rows
    G.destroy()


_refs = {}


def reference(rp, ci, N, X, storage, width, K, with_bound=True):
    key = (storage, width, K, with_bound)
    if key not in _refs:
        _refs[key] = errbound.reference_and_bound(rp, ci, N, TAU, K, X[:, :width], storage,
                                                  with_bound=with_bound)
    return _refs[key]


def run(ifgp, G, X, K, width, storage, depth):
    import torch
    prev = ifgp.debug_hop_depth(depth)
    try:
        out = G.embed_x(TAU, K, torch.as_tensor(X[:, :width]), storage=storage)
        torch.cuda.synchronize()
    finally:
        ifgp.debug_hop_depth(prev)
    return out.cpu().numpy().astype(np.float64)


CASES = ([("f32", "8 rows", 64)]
         + [(st, dn, 64) for st in ("bf16", "f16") for dn in DEPTHS]
         + [("bf16", "8 rows", 32), ("bf16", "16 rows", 32), ("f16", "16 rows", 32)])


@pytest.mark.parametrize("storage,depth,width", CASES)
@pytest.mark.parametrize("K", [1, 2])
def test_rows_within_bound(ifgp, hubby, storage, depth, width, K):
    G, rp, ci, N, X, rows = hubby
    log(f"rows: storage={storage} depth={depth} width={width} K={K}")
    out = run(ifgp, G, X, K, width, storage, DEPTHS[depth])
    ref, B = reference(rp, ci, N, X, storage, width, K)
    orc = ffp.ffp_from_input(rp, ci, N, TAU, K, X[:, :width].astype(np.float64))
    for name, idx in rows.items():
        dev = np.abs(out[idx] - ref[idx])
        used = (dev / B[idx]).max()
        log(f"  {name:6s} rows {len(idx):5d}: max |gpu - ref| {dev.max():.2e}, "
            f"{used:.2f} of the bound; max |ref - oracle| {np.abs(ref[idx] - orc[idx]).max():.2e}, "
            f"max |gpu - oracle| {np.abs(out[idx] - orc[idx]).max():.2e}")
        bad = np.argwhere(dev > B[idx])
        assert bad.size == 0, (name, idx[bad[:5, 0]], bad[:5, 1])


@pytest.mark.parametrize("storage,depth", [("f32", "8 rows")] +
                         [(st, dn) for st in ("bf16", "f16") for dn in DEPTHS])
def test_rows_eight_hops(ifgp, hubby, storage, depth):
    G, rp, ci, N, X, rows = hubby
    K, width = 8, 64
    log(f"rows, 8 hops: storage={storage} depth={depth}")
    out = run(ifgp, G, X, K, width, storage, DEPTHS[depth])
    ref, _ = reference(rp, ci, N, X, storage, width, K, with_bound=False)
    key = ("oracle", K)
    if key not in _refs:
        _refs[key] = ffp.ffp_from_input(rp, ci, N, TAU, K, X[:, :width].astype(np.float64))
    orc = _refs[key]
    for name, idx in rows.items():
        e_gpu = np.abs(out[idx] - orc[idx]).max(axis=1)
        e_ref = np.abs(ref[idx] - orc[idx]).max(axis=1)
        log(f"  {name:6s}: max |gpu - oracle| {e_gpu.max():.2e}, "
            f"max |ref - oracle| {e_ref.max():.2e}")
        assert e_gpu.max() <= 3 * e_ref.max() + (1e-5 if storage == "f32" else 1e-6), name
