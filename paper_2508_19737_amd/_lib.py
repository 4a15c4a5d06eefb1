"""ctypes binding of libifgp (include/ifgp.h): argument marshalling only.

Every computation runs in the HIP kernels of libifgp.so; this module passes
pointers, sizes and the current torch stream, turns status codes into
exceptions, and lets torch's caching allocator provide device memory.
There is no fallback: if the library is missing, importing fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# IFGP_LIBRARY may name another build of the same library (the sanitizer
# build, libifgp_san.so); by default the one built in this directory.
LIB_PATH = os.environ.get("IFGP_LIBRARY") or os.path.join(_HERE, "libifgp.so")

OK, E_INVALID, E_RANGE, E_OOM, E_DEVICE, E_STATE = 0, -1, -2, -3, -4, -5
F32, BF16, F16, F64 = 0, 1, 2, 3
DTYPES = {"f32": F32, "fp32": F32, "float32": F32, "bf16": BF16, "bfloat16": BF16,
          "f16": F16, "fp16": F16, "float16": F16, "f64": F64, "float64": F64}

# Every entry point that include/ifgp.h declares.
EXPORTS = [
    "ifgp_default_params", "ifgp_build_graph", "ifgp_embed", "ifgp_embed_noalloc",
    "ifgp_embed_x",
    "ifgp_gaussian_input", "ifgp_stream_add", "ifgp_embed_batch", "ifgp_job_begin",
    "ifgp_job_step", "ifgp_graph_info", "ifgp_plan_info", "ifgp_export_csr",
    "ifgp_export_scales",
    "ifgp_footprint_bytes", "ifgp_set_allocator", "ifgp_empty_cache", "ifgp_timing_enable",
    "ifgp_timing_read", "ifgp_debug_grid_x", "ifgp_debug_hop_depth",
    "ifgp_destroy", "ifgp_last_error", "ifgp_version",
    "ifgp_birch_create", "ifgp_birch_partial_fit", "ifgp_birch_info", "ifgp_birch_centers",
    "ifgp_birch_predict", "ifgp_birch_predict_update", "ifgp_birch_update_stats",
    "ifgp_birch_destroy",
]


class Params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("theta", ctypes.c_double), ("eps", ctypes.c_double),
                ("znorm_ddof", ctypes.c_int32), ("storage", ctypes.c_int32)]


class IfgpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"[{status}] {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python paper_2508_19737_amd/build.py`")
    # torch ships its own HIP runtime.  Load it first so that libifgp binds to
    # that same runtime (same soname) instead of a second copy from /opt/rocm:
    # two HIP runtimes in one process do not share the device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, i64, i32, u64, f64 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                             ctypes.c_double)
    PP = ctypes.POINTER(Params)
    sig = {
        "ifgp_default_params": [PP],
        "ifgp_build_graph": [P, P, i64, i64, ctypes.c_int, P, ctypes.POINTER(P)],
        "ifgp_embed": [P, f64, i32, i32, u64, PP, P, P],
        "ifgp_embed_noalloc": [P, f64, i32, i32, u64, PP, P, P],
        "ifgp_embed_x": [P, f64, i32, i32, P, PP, P, P],
        "ifgp_gaussian_input": [i64, i32, u64, i32, P, P],
        "ifgp_stream_add": [P, P, P, i64, i64, ctypes.c_int, P],
        "ifgp_embed_batch": [P, i32, P, P, P, P, PP, P, P],
        "ifgp_job_begin": [P, f64, i32, i32, u64, PP, P, P],
        "ifgp_job_step": [P, i32, P, P],
        "ifgp_graph_info": [P, P, P, P, P],
        "ifgp_plan_info": [P, P, P, P, P],
        "ifgp_export_csr": [P, P, P, P],
        "ifgp_export_scales": [P, f64, f64, P],
        "ifgp_footprint_bytes": [i64, i64, i32, i32, P],
        "ifgp_set_allocator": [P, P, P],
        "ifgp_empty_cache": [],
        "ifgp_timing_enable": [P, ctypes.c_int],
        "ifgp_timing_read": [P, P, P],
        "ifgp_debug_grid_x": [i64, P],
        "ifgp_debug_hop_depth": [i32, P],
        "ifgp_destroy": [P],
        "ifgp_birch_create": [i32, f64, i32, ctypes.POINTER(P)],
        "ifgp_birch_partial_fit": [P, P, i64, ctypes.c_int, P],
        "ifgp_birch_info": [P, P, P, P],
        "ifgp_birch_centers": [P, P],
        "ifgp_birch_predict": [P, P, i64, P, P],
        "ifgp_birch_predict_update": [P, P, i64, P, P],
        "ifgp_birch_update_stats": [P, P, P, P, P],
        "ifgp_birch_destroy": [P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.ifgp_last_error.argtypes = []
    lib.ifgp_last_error.restype = ctypes.c_char_p
    lib.ifgp_version.argtypes = []
    lib.ifgp_version.restype = ctypes.c_char_p
    return lib


lib = _load()


def check(status):
    if status != OK:
        raise IfgpError(status, lib.ifgp_last_error().decode())


def params(alpha=1.0, theta=0.1, eps=1e-3, ddof=0, storage="f32") -> Params:
    p = Params()
    check(lib.ifgp_default_params(ctypes.byref(p)))
    p.alpha, p.theta, p.eps, p.znorm_ddof = float(alpha), float(theta), float(eps), int(ddof)
    p.storage = DTYPES[storage] if isinstance(storage, str) else int(storage)
    return p


def version() -> str:
    return lib.ifgp_version().decode()


def footprint_bytes(N, nnz, d, storage="bf16") -> int:
    out = ctypes.c_int64()
    st = DTYPES[storage] if isinstance(storage, str) else int(storage)
    check(lib.ifgp_footprint_bytes(int(N), int(nnz), int(d), st, ctypes.byref(out)))
    return int(out.value)


# ---------------------------------------------------------------- torch glue
def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


_ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
_hooks = None


def use_torch_allocator():
    """Route libifgp's device allocations through torch's caching allocator."""
    global _hooks
    if _hooks is not None:
        return
    torch = _torch()
    raw_alloc = torch._C._cuda_cudaCachingAllocator_raw_alloc
    raw_delete = torch._C._cuda_cudaCachingAllocator_raw_delete

    owner = {}   # block -> the stream it was allocated on

    def _alloc(size, stream, ctx):
        try:
            p = raw_alloc(int(size), int(stream or 0))
        except Exception:   # out of memory: the library reports IFGP_E_OOM
            return None
        owner[p] = int(stream or 0)
        return p

    def _free(ptr, stream, ctx):
        # torch hands a released block out again at once to allocations on
        # the stream it was allocated on; released on another stream (the
        # one that used it last), that stream's work must finish first
        if owner.pop(int(ptr), None) != int(stream or 0):
            torch.cuda.synchronize()
        raw_delete(int(ptr))

    hooks = (_ALLOC_T(_alloc), _FREE_T(_free))
    check(lib.ifgp_set_allocator(ctypes.cast(hooks[0], ctypes.c_void_p),
                                 ctypes.cast(hooks[1], ctypes.c_void_p), None))
    _hooks = hooks


def use_hip_allocator():
    """Back to the library's own caching allocator (the default)."""
    global _hooks
    check(lib.ifgp_set_allocator(None, None, None))
    _hooks = None


def empty_cache():
    """Return the library allocator's cached blocks to the device."""
    check(lib.ifgp_empty_cache())


def debug_grid_x(max_x_blocks: int) -> int:
    """Test hook: cap the x dimension of the size-dependent grids at
    max_x_blocks blocks (0 = the default); returns the previous cap."""
    prev = ctypes.c_int64()
    check(lib.ifgp_debug_grid_x(int(max_x_blocks), ctypes.byref(prev)))
    return prev.value


def debug_hop_depth(depth: int) -> int:
    """Test hook: force the hop's gather depth for 2-byte storage (0: 8 rows
    in flight, 1: 4, 2: 16; -1: chosen per graph); returns the previous."""
    prev = ctypes.c_int32()
    check(lib.ifgp_debug_hop_depth(int(depth), ctypes.byref(prev)))
    return prev.value


def _edges(src, dst):
    """(ptr_src, ptr_dst, E, on_device, keepalive)."""
    torch = _torch()
    if isinstance(src, torch.Tensor):
        s = src.to(torch.int64).contiguous()
        t = dst.to(device=s.device, dtype=torch.int64).contiguous()
        if s.shape != t.shape:
            raise ValueError("src/dst length mismatch")
        return (ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(t.data_ptr()), s.numel(),
                int(s.is_cuda), (s, t))
    s = np.ascontiguousarray(np.asarray(src, dtype=np.int64).ravel())
    t = np.ascontiguousarray(np.asarray(dst, dtype=np.int64).ravel())
    if s.shape != t.shape:
        raise ValueError("src/dst length mismatch")
    return (s.ctypes.data_as(ctypes.c_void_p), t.ctypes.data_as(ctypes.c_void_p), s.size, 0,
            (s, t))


class Graph:
    """A graph resident in HBM (ifgp_build_graph)."""

    def __init__(self, src, dst, N, stream=None):
        ps, pd, E, on_dev, keep = _edges(src, dst)
        h = ctypes.c_void_p()
        check(lib.ifgp_build_graph(ps, pd, E, int(N), on_dev, _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        del keep

    @property
    def handle(self):
        if self._h is None:
            raise IfgpError(E_STATE, "graph was destroyed")
        return self._h

    def info(self):
        v = [ctypes.c_int64() for _ in range(4)]
        check(lib.ifgp_graph_info(self.handle, *[ctypes.byref(x) for x in v]))
        N, nnz, loops, dups = (int(x.value) for x in v)
        return {"N": N, "nnz": nnz, "self_loops_dropped": loops, "dups_dropped": dups}

    def plan_info(self):
        v = [ctypes.c_int64() for _ in range(3)]
        md = ctypes.c_int32()
        check(lib.ifgp_plan_info(self.handle, *[ctypes.byref(x) for x in v], ctypes.byref(md)))
        return {"hub_rows": int(v[0].value), "medium_rows": int(v[1].value),
                "hop_blocks": int(v[2].value), "max_degree": int(md.value)}

    @property
    def N(self):
        return self.info()["N"]

    @property
    def nnz(self):
        return self.info()["nnz"]

    def export_csr(self):
        inf = self.info()
        rowptr = np.empty(inf["N"] + 1, dtype=np.int64)
        colidx = np.empty(max(inf["nnz"], 1), dtype=np.int32)
        deg = np.empty(inf["N"], dtype=np.int32)
        check(lib.ifgp_export_csr(self.handle, rowptr.ctypes.data_as(ctypes.c_void_p),
                                  colidx.ctypes.data_as(ctypes.c_void_p),
                                  deg.ctypes.data_as(ctypes.c_void_p)))
        return rowptr, colidx[:inf["nnz"]], deg

    def export_scales(self, tau, eps=1e-3):
        s = np.empty(self.N, dtype=np.float64)
        check(lib.ifgp_export_scales(self.handle, float(tau), float(eps),
                                     s.ctypes.data_as(ctypes.c_void_p)))
        return s

    def _out(self, d, out):
        torch = _torch()
        N = self.N
        if out is None:
            out = torch.empty((N, d), dtype=torch.float32, device="cuda")
        if out.dtype != torch.float32 or not out.is_cuda or not out.is_contiguous() \
                or tuple(out.shape) != (N, d):
            raise ValueError("out must be a contiguous float32 CUDA tensor of shape (N, d)")
        return out

    def embed(self, tau, K, d, seed, out=None, stream=None, **kw):
        out = self._out(d, out)
        p = params(**kw)
        check(lib.ifgp_embed(self.handle, float(tau), int(K), int(d), ctypes.c_uint64(int(seed)),
                             ctypes.byref(p), ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def embed_noalloc(self, tau, K, d, seed, out, stream=None, **kw):
        """ifgp_embed_noalloc: as embed, in the library's static device
        scratch array (no device allocation; `out` must be given)."""
        out = self._out(d, out)
        p = params(**kw)
        check(lib.ifgp_embed_noalloc(self.handle, float(tau), int(K), int(d),
                                     ctypes.c_uint64(int(seed)), ctypes.byref(p),
                                     ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def embed_x(self, tau, K, X, out=None, stream=None, **kw):
        torch = _torch()
        X = X.to(device="cuda", dtype=torch.float32).contiguous()
        if X.dim() != 2 or X.shape[0] != self.N:
            raise ValueError("X must have shape (N, d)")
        d = X.shape[1]
        out = self._out(d, out)
        p = params(**kw)
        check(lib.ifgp_embed_x(self.handle, float(tau), int(K), int(d),
                               ctypes.c_void_p(X.data_ptr()), ctypes.byref(p),
                               ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def stream_add(self, src, dst, new_N=None, stream=None):
        ps, pd, E, on_dev, keep = _edges(src, dst)
        nN = self.N if new_N is None else int(new_N)
        check(lib.ifgp_stream_add(self.handle, ps, pd, E, nN, on_dev, _stream_ptr(stream)))
        del keep

    def job_begin(self, tau, K, d, seed, out=None, stream=None, **kw):
        out = self._out(d, out)
        p = params(**kw)
        check(lib.ifgp_job_begin(self.handle, float(tau), int(K), int(d),
                                 ctypes.c_uint64(int(seed)), ctypes.byref(p),
                                 ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def timing(self, enable=True):
        check(lib.ifgp_timing_enable(self.handle, int(bool(enable))))

    def timing_read(self):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        check(lib.ifgp_timing_read(self.handle, ctypes.byref(n), ctypes.byref(ms)))
        return int(n.value), float(ms.value)

    def destroy(self):
        if getattr(self, "_h", None) is not None:
            check(lib.ifgp_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _handles(graphs):
    arr = (ctypes.c_void_p * len(graphs))(*[g.handle.value for g in graphs])
    return arr


def embed_batch(graphs, taus, Ks, ds, seeds, outs=None, stream=None, **kw):
    torch = _torch()
    n = len(graphs)
    if outs is None:
        outs = [torch.empty((g.N, int(d)), dtype=torch.float32, device="cuda")
                for g, d in zip(graphs, ds)]
    p = params(**kw)
    tau = (ctypes.c_double * n)(*[float(t) for t in taus])
    K = (ctypes.c_int32 * n)(*[int(k) for k in Ks])
    d = (ctypes.c_int32 * n)(*[int(x) for x in ds])
    seed = (ctypes.c_uint64 * n)(*[int(s) for s in seeds])
    op = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    check(lib.ifgp_embed_batch(_handles(graphs), n, tau, K, d, seed, ctypes.byref(p), op,
                               _stream_ptr(stream)))
    return outs


def job_step(graphs, stream=None):
    n = len(graphs)
    flags = (ctypes.c_int32 * max(n, 1))()
    check(lib.ifgp_job_step(_handles(graphs), n, flags, _stream_ptr(stream)))
    return [bool(flags[i]) for i in range(n)]


def gaussian_input(N, d, seed, dtype="f64", out=None, stream=None):
    torch = _torch()
    tdt = {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16, F16: torch.float16}
    code = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    if out is None:
        out = torch.empty((int(N), int(d)), dtype=tdt[code], device="cuda")
    check(lib.ifgp_gaussian_input(int(N), int(d), ctypes.c_uint64(int(seed)), code,
                                  ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


class Birch:
    """BIRCH with no preset number of clusters (the clustering step after the
    FFP; rules in include/ifgp.h).  The CF-tree lives in the library (host);
    predict runs on the device."""

    def __init__(self, d, threshold, branching_factor=50):
        self.d = int(d)
        h = ctypes.c_void_p()
        check(lib.ifgp_birch_create(self.d, float(threshold), int(branching_factor),
                                    ctypes.byref(h)))
        self._h = h

    def _live(self):
        if not self._h:
            raise IfgpError(E_INVALID, "BIRCH tree already destroyed")
        return self._h

    def partial_fit(self, Z, stream=None):
        """Insert the rows of Z (n x d; a torch tensor on the GPU or any host
        array), in order."""
        torch = _torch()
        if isinstance(Z, torch.Tensor) and Z.is_cuda:
            Zt = Z.detach().to(torch.float32).contiguous()
            if Zt.dim() != 2 or Zt.shape[1] != self.d:
                raise IfgpError(E_INVALID, f"Z must be n x {self.d}")
            check(lib.ifgp_birch_partial_fit(self._live(), ctypes.c_void_p(Zt.data_ptr()),
                                             Zt.shape[0], 1, _stream_ptr(stream)))
        else:
            Zh = np.ascontiguousarray(np.asarray(Z, dtype=np.float32))
            if Zh.ndim != 2 or Zh.shape[1] != self.d:
                raise IfgpError(E_INVALID, f"Z must be n x {self.d}")
            check(lib.ifgp_birch_partial_fit(self._live(), Zh.ctypes.data_as(ctypes.c_void_p),
                                             Zh.shape[0], 0, None))
        return self

    def info(self):
        n = ctypes.c_int64()
        m = ctypes.c_int64()
        h = ctypes.c_int32()
        check(lib.ifgp_birch_info(self._live(), ctypes.byref(n), ctypes.byref(m), ctypes.byref(h)))
        return {"points": n.value, "clusters": m.value, "height": h.value}

    def centers(self):
        m = self.info()["clusters"]
        out = np.empty((m, self.d), dtype=np.float64)
        check(lib.ifgp_birch_centers(self._live(), out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def predict(self, Z, out=None, stream=None):
        """Labels (device int32) of the rows of Z (a GPU tensor, n x d)."""
        torch = _torch()
        Zt = Z.detach().to(torch.float32).contiguous()
        if Zt.dim() != 2 or Zt.shape[1] != self.d or not Zt.is_cuda:
            raise IfgpError(E_INVALID, f"Z must be a GPU tensor n x {self.d}")
        if out is None:
            out = torch.empty(Zt.shape[0], dtype=torch.int32, device=Zt.device)
        if out.dtype != torch.int32 or not out.is_cuda or not out.is_contiguous() \
                or tuple(out.shape) != (Zt.shape[0],):
            raise ValueError("out must be a contiguous int32 CUDA tensor of shape (n,)")
        check(lib.ifgp_birch_predict(self._live(), ctypes.c_void_p(Zt.data_ptr()), Zt.shape[0],
                                     ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def predict_update(self, Z, out=None, stream=None):
        """ifgp_birch_predict_update: the labels predict gives, for rows that
        extend those of the previous call of this method (Algorithm 2)."""
        torch = _torch()
        Zt = Z.detach().to(torch.float32).contiguous()
        if Zt.dim() != 2 or Zt.shape[1] != self.d or not Zt.is_cuda:
            raise IfgpError(E_INVALID, f"Z must be a GPU tensor n x {self.d}")
        if out is None:
            out = torch.empty(Zt.shape[0], dtype=torch.int32, device=Zt.device)
        if out.dtype != torch.int32 or not out.is_cuda or not out.is_contiguous() \
                or tuple(out.shape) != (Zt.shape[0],):
            raise ValueError("out must be a contiguous int32 CUDA tensor of shape (n,)")
        check(lib.ifgp_birch_predict_update(self._live(), ctypes.c_void_p(Zt.data_ptr()),
                                            Zt.shape[0], ctypes.c_void_p(out.data_ptr()),
                                            _stream_ptr(stream)))
        return out

    def update_stats(self):
        """ifgp_birch_update_stats: {"new_entries", "fp32_rows", "fp64_rows",
        "fp64_full_rows"} of the last predict_update."""
        v = [ctypes.c_int64() for _ in range(4)]
        check(lib.ifgp_birch_update_stats(self._live(), *[ctypes.byref(x) for x in v]))
        return dict(new_entries=v[0].value, fp32_rows=v[1].value, fp64_rows=v[2].value,
                    fp64_full_rows=v[3].value)

    def fit_predict(self, Z, stream=None):
        return self.partial_fit(Z, stream).predict(Z, stream=stream)

    def destroy(self):
        if self._h:
            check(lib.ifgp_birch_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
