"""The continuous-batching serving loop: every result equals the same graph
embedded alone, bit for bit, while requests arrive during others' hops."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from workloads.serving import graph_pool, request_stream  # noqa: E402


def make_requests(serve, specs):
    return [serve.Request(rid=i, arrival=s["arrival"], src=s["graph"].src, dst=s["graph"].dst,
                          N=s["graph"].N, tau=s["tau"], K=s["K"], d=s["d"], seed=s["seed"],
                          storage=s["storage"]) for i, s in enumerate(specs)]


@pytest.mark.parametrize("max_slots,budget", [(16, None), (1, None), (3, 64 << 20)])
def test_served_equals_alone(max_slots, budget):
    import torch
    import paper_2508_19737_amd as ifgp
    from paper_2508_19737_amd import serve
    pool = graph_pool(pool=8, n_min=1000, n_max=60_000, seed=3, workers=1)
    specs = request_stream(pool, 24, rate=2000.0, seed=3)
    reqs = make_requests(serve, specs)
    srv = serve.Server(max_slots=max_slots, budget_bytes=budget)
    done = srv.run(reqs)
    srv.close()
    assert sorted(r.rid for r in done) == list(range(24))
    for r in done:
        G = ifgp.Graph(r.src, r.dst, r.N)
        alone = G.embed(r.tau, r.K, r.d, r.seed, storage=r.storage)
        assert torch.equal(r.out, alone), r.rid
        G.destroy()
        assert r.t_done >= r.t_start >= r.t_admit >= r.arrival - 1e-9
    if max_slots == 1:
        # one slot: strict arrival order of completion
        assert [r.rid for r in done] == list(range(24))
    st = serve.summarize(done)
    assert st["graphs"] == 24 and st["p99_ms"] >= st["p50_ms"] > 0


def test_sequential_path_matches_fp32_alone():
    import torch
    import paper_2508_19737_amd as ifgp
    from paper_2508_19737_amd import serve
    pool = graph_pool(pool=3, n_min=1000, n_max=20_000, seed=4, workers=1)
    reqs = make_requests(serve, request_stream(pool, 6, rate=float("inf"), seed=4))
    done = serve.sequential(reqs, storage="f32")
    for r in done:
        G = ifgp.Graph(r.src, r.dst, r.N)
        assert torch.equal(r.out, G.embed(r.tau, r.K, r.d, r.seed, storage="f32"))
        G.destroy()
