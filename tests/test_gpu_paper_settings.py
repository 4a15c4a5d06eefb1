"""The paper's own parameter settings (Table II: tau far below zero, many
hops, narrow embeddings) and a sweep of tau from -100 to 100 (Fig. 4's range)
at 5,000 and 100,000 nodes.

Parity is judged on what the method is for: the partition that BIRCH
(Sec. III, Alg. 1; scikit-learn, as in Sec. IV) derives from the embedding,
scored against the planted blocks by NMI.  The HIP path's embedding and the
FP64 oracle's, clustered the same way, must score within 0.01 of each other.

The random input Z^(0) is part of the method, so the NMI of one seed is one
draw of a random variable.  At these settings that variable is very sensitive
to perturbations of the embedding: the HIP path with 2-byte storage rounds
every hop's features at 2^-8 (BF16) or 2^-11 (FP16), and the FP64 oracle
itself, given an input perturbed by that much, moves its own single-seed NMI
by up to 0.06-0.08 at tau = -80, K = 40 (threshold 1.0) and by more than 0.01
elsewhere too (BIRCH's radius threshold makes the partition a discontinuous
function of the points).  A single draw therefore cannot separate a correct
2-byte path from a wrong one, and the 2-byte gate is on the NMI averaged over a
fixed set of seeds (the same seeds for the oracle and the HIP path).  FP32
storage stays below the level where draws flip and is gated on every draw
(within 0.005).  Per-draw differences are printed.

Graphs are the seeded DC-SBM stand-in for the benchmark graphs, with the
benchmark's mean degree of about 40 and round(N^0.35) blocks."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import cref, ffp  # noqa: E402
from workloads import dcsbm  # noqa: E402

FP32_NMI_TOL = 0.005   # every draw
HALF_NMI_TOL = 0.01    # mean over the seeds


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


_graphs = {}


def graph(N):
    if N not in _graphs:
        g = dcsbm(N, int(round(N ** 0.35)), mean_deg=40.0, ratio=2.5, seed=0)
        rp, ci, _, _ = ffp.canonical_csr(g.src, g.dst, g.N)
        _graphs[N] = (g, rp, ci)
    return _graphs[N]


def nmi_of(labels, E, threshold):
    from sklearn.cluster import Birch
    from sklearn.metrics import normalized_mutual_info_score as nmi
    return nmi(labels, Birch(n_clusters=None, threshold=threshold).fit_predict(E))


def check(ifgp, N, tau, K, d, thresholds, seeds):
    g, rp, ci = graph(N)
    G = ifgp.Graph(g.src, g.dst, g.N)
    delta = {(st, thr): [] for st in ("f32", "bf16", "f16") for thr in thresholds}
    try:
        for seed in seeds:
            ref = cref.ffp_from_input(rp, ci, g.N, tau, K, cref.gaussian_input(g.N, d, seed))
            base = {thr: nmi_of(g.labels, ref, thr) for thr in thresholds}
            for st in ("f32", "bf16", "f16"):
                got = G.embed(tau, K, d, seed, storage=st).cpu().numpy().astype(np.float64)
                err = ffp.rel_frobenius(got, ref)
                for thr in thresholds:
                    n_g = nmi_of(g.labels, got, thr)
                    delta[(st, thr)].append(n_g - base[thr])
                    log(f"N={N} tau={tau} K={K} d={d} seed={seed} {st} threshold={thr}: "
                        f"rel_frobenius={err:.2e} NMI oracle {base[thr]:.4f} gpu {n_g:.4f}")
    finally:
        G.destroy()
    for (st, thr), dl in delta.items():
        dl = np.array(dl)
        log(f"N={N} tau={tau} {st} threshold={thr}: NMI gpu - oracle over {len(dl)} seeds: "
            f"mean {dl.mean():+.4f}, largest draw {np.abs(dl).max():.4f}")
        if st == "f32":
            assert np.abs(dl).max() <= FP32_NMI_TOL, (st, thr, dl)
        else:
            assert abs(dl.mean()) <= HALF_NMI_TOL, (st, thr, dl)


@pytest.mark.parametrize("N,tau,K,d,seeds", [(5000, -6.0, 10, 64, 8), (5000, -80.0, 40, 32, 16),
                                             (50000, -80.0, 40, 32, 4)])
def test_paper_settings_nmi(ifgp, N, tau, K, d, seeds):
    check(ifgp, N, tau, K, d, (0.5, 1.0), range(1, seeds + 1))


@pytest.mark.parametrize("tau", [-100.0, -30.0, -10.0, -3.0, -1.0, 0.0, 1.0, 10.0, 30.0, 100.0])
def test_tau_sweep_nmi(ifgp, tau):
    check(ifgp, 5000, tau, 10, 64, (0.5,), range(1, 5))


@pytest.mark.parametrize("tau", [-100.0, -10.0, -1.0, 0.0, 10.0, 100.0])
def test_tau_sweep_nmi_100k(ifgp, tau):
    check(ifgp, 100_000, tau, 10, 64, (1.0,), range(1, 5))
