"""Failure paths forced from the host: allocation failures through the
allocator hook (IFGP_E_OOM with the graph left unchanged), allocator switches
while graphs are alive, and argument errors that reach the device entry
points."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from workloads import dcsbm, random_edges  # noqa: E402


class Budget:
    """Allocator hook backed by torch's caching allocator that refuses any
    request beyond a byte budget (the library then reports IFGP_E_OOM)."""

    def __init__(self, ifgp):
        import torch
        self.ifgp = ifgp
        self.left = 1 << 62
        raw_alloc = torch._C._cuda_cudaCachingAllocator_raw_alloc
        raw_delete = torch._C._cuda_cudaCachingAllocator_raw_delete

        def _alloc(size, stream, ctx):
            if size > self.left:
                return None
            self.left -= size
            return raw_alloc(int(size), int(stream or 0))

        def _free(ptr, stream, ctx):
            raw_delete(int(ptr))

        self.hooks = (ifgp._lib._ALLOC_T(_alloc), ifgp._lib._FREE_T(_free))

    def __enter__(self):
        self.ifgp._lib.check(self.ifgp.lib.ifgp_set_allocator(
            ctypes.cast(self.hooks[0], ctypes.c_void_p),
            ctypes.cast(self.hooks[1], ctypes.c_void_p), None))
        return self

    def __exit__(self, *exc):
        self.ifgp.use_hip_allocator()


@pytest.fixture(scope="module")
def ifgp():
    import paper_2508_19737_amd as m
    return m


def test_oom_on_build_embed_and_stream_add(ifgp):
    g = dcsbm(5000, 10, seed=1)
    with Budget(ifgp) as b:
        b.left = 4096
        with pytest.raises(ifgp.IfgpError) as e:
            ifgp.Graph(g.src, g.dst, g.N)
        assert e.value.status == -3
        b.left = 1 << 62
        half = g.num_edges // 2
        G = ifgp.Graph(g.src[:half], g.dst[:half], g.N)
        ref = G.embed(-1.0, 8, 32, 3, storage="bf16").cpu().numpy()
        before = G.export_csr()
        b.left = 4096
        with pytest.raises(ifgp.IfgpError) as e:
            G.stream_add(g.src[half:], g.dst[half:])
        assert e.value.status == -3
        assert all(np.array_equal(x, y) for x, y in zip(before, G.export_csr()))
        # an embedding at a new width needs new buffers: refused, then fine
        with pytest.raises(ifgp.IfgpError) as e:
            G.embed(-1.0, 8, 128, 3, storage="f32")
        assert e.value.status == -3
        b.left = 1 << 62
        again = G.embed(-1.0, 8, 32, 3, storage="bf16").cpu().numpy()
        assert np.array_equal(again, ref)
        G.stream_add(g.src[half:], g.dst[half:])
        assert G.info()["nnz"] == 2 * g.num_edges
        G.destroy()


def test_allocator_switch_with_live_graphs(ifgp):
    src, dst = random_edges(3000, 20000, 5)
    ifgp.use_torch_allocator()
    A = ifgp.Graph(src, dst, 3000)
    a1 = A.embed(-1.0, 4, 16, 1).cpu().numpy()
    ifgp.use_hip_allocator()
    B = ifgp.Graph(src, dst, 3000)
    b1 = B.embed(-1.0, 4, 16, 1).cpu().numpy()
    A.stream_add(np.array([1, 2]), np.array([3, 4]))       # rebuilt under the other allocator
    a2 = A.embed(-1.0, 4, 16, 1).cpu().numpy()
    assert np.array_equal(a1, b1)
    assert not np.array_equal(a1, a2)
    A.destroy()
    B.destroy()
    ifgp.empty_cache()


def test_device_entry_point_argument_errors(ifgp):
    import torch
    src, dst = random_edges(100, 300, 6)
    G = ifgp.Graph(src, dst, 100)
    out = torch.empty((100, 8), dtype=torch.float32, device="cuda")
    for kw in (dict(storage="f64"), dict(ddof=2), dict(eps=0.0), dict(alpha=float("nan"))):
        with pytest.raises(ifgp.IfgpError) as e:
            G.embed(-1.0, 4, 8, 1, out=out, **kw)
        assert e.value.status == -1
    with pytest.raises(ifgp.IfgpError):
        G.embed(float("inf"), 4, 8, 1, out=out)
    with pytest.raises(ifgp.IfgpError):
        G.embed(-1.0, -1, 8, 1, out=out)
    with pytest.raises(ValueError):
        G.embed_x(-1.0, 4, torch.zeros((99, 8)))
    with pytest.raises(ifgp.IfgpError) as e:
        ifgp.job_step([G])                      # no job begun
    assert e.value.status == -5
    with pytest.raises(ifgp.IfgpError):
        ifgp.embed_batch([G, G], [-1.0, -1.0], [4, 4], [8, 8], [1, 2])
    G.destroy()
    with pytest.raises(ifgp.IfgpError):
        G.info()


def test_label_update_after_allocation_failures(ifgp):
    """An update that fails part-way (here: a device allocation refused at
    different points of it) must not leave labels or entries stale: the next
    update gives the full FP64 labelling's labels exactly."""
    import torch
    rng = np.random.default_rng(7)
    d, total = 16, 12000
    X = torch.as_tensor((0.3 * rng.standard_normal((total, d))).astype(np.float32), device="cuda")
    b = ifgp.Birch(d, 0.5, 50)
    labels = torch.empty(total, dtype=torch.int32, device="cuda")
    n = 3000
    b.partial_fit(X[:n])
    b.predict_update(X[:n], out=labels[:n])
    failures = 0
    with Budget(ifgp) as bud:
        for budget in [0, 256, 4096, 1 << 14, 1 << 16, 1 << 18, 1 << 20, 0, 1 << 12]:
            m = n + 1000
            b.partial_fit(X[n:m])
            n = m
            bud.left = budget
            try:
                b.predict_update(X[:n], out=labels[:n])
            except ifgp.IfgpError as e:
                assert e.status == -3
                failures += 1
            bud.left = 1 << 62
            b.predict_update(X[:n], out=labels[:n])
            full = b.predict(X[:n])
            torch.cuda.synchronize()
            assert torch.equal(full, labels[:n]), f"budget {budget}: labels differ after a failed update"
    assert failures >= 3
    b.destroy()


def test_handle_on_two_streams(ifgp):
    """One handle used on two streams in order (the second waits for the
    first), under both allocators: the blocks the second stream's calls
    replace (a wider embedding's workspace, the build's survivors when the
    canonical column indices are made) are released after that stream's
    work, and every result equals the one-stream result."""
    import torch
    g = dcsbm(6000, 12, seed=4)
    R = ifgp.Graph(g.src, g.dst, g.N)
    ref16 = R.embed(-1.0, 6, 16, 2).cpu()
    ref64 = R.embed(-1.0, 6, 64, 2).cpu()
    ref_csr = R.export_csr()
    R.destroy()
    for hook in (True, False):
        if hook:
            ifgp.use_torch_allocator()
        A, B = torch.cuda.Stream(), torch.cuda.Stream()
        with torch.cuda.stream(A):
            G = ifgp.Graph(g.src, g.dst, g.N, stream=A)
            z16 = G.embed(-1.0, 6, 16, 2, stream=A)
        B.wait_stream(A)
        with torch.cuda.stream(B):
            z64 = G.embed(-1.0, 6, 64, 2, stream=B)
            csr = G.export_csr()
        B.synchronize()
        assert torch.equal(z16.cpu(), ref16) and torch.equal(z64.cpu(), ref64)
        assert all(np.array_equal(x, y) for x, y in zip(csr, ref_csr))
        G.destroy()
        ifgp.use_hip_allocator()
    ifgp.empty_cache()
