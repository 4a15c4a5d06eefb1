"""The C ABI library loads, exports every entry point include/ifgp.h declares,
and rejects bad arguments before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "ifgp.h")).read()
    return sorted(set(re.findall(r"IFGP_API\s+[\w\s\*]*?\b(ifgp_\w+)\s*\(", src)))


def test_header_and_binding_agree():
    import paper_2508_19737_amd as ifgp
    decl = declared_symbols()
    assert len(decl) >= 19
    assert sorted(ifgp.EXPORTS) == decl


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2508_19737_amd", "libifgp.so"))
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_host_side_argument_checks():
    import paper_2508_19737_amd as ifgp
    lib = ifgp.lib
    h = ctypes.c_void_p()
    assert lib.ifgp_build_graph(None, None, 0, 0, 0, None, ctypes.byref(h)) == -1
    assert b"N" in lib.ifgp_last_error()
    assert lib.ifgp_build_graph(None, None, -1, 10, 0, None, ctypes.byref(h)) == -1
    assert lib.ifgp_build_graph(None, None, 5, 10, 0, None, ctypes.byref(h)) == -1   # NULL edges
    assert lib.ifgp_build_graph(None, None, 0, 2**31, 0, None, ctypes.byref(h)) == -1
    assert lib.ifgp_default_params(None) == -1
    assert lib.ifgp_embed(None, -1.0, 8, 32, 1, None, None, None) == -1
    assert lib.ifgp_graph_info(None, None, None, None, None) == -1
    assert lib.ifgp_gaussian_input(10, 0, 1, 0, None, None) == -1
    assert lib.ifgp_gaussian_input(10, 4, 1, 9, None, None) == -1
    assert lib.ifgp_destroy(None) == 0
    assert lib.ifgp_set_allocator(ctypes.c_void_p(1), None, None) == -1
    assert lib.ifgp_set_allocator(None, None, None) == 0
    assert lib.ifgp_job_step(None, -1, None, None) == -1
    assert ifgp.version().startswith("ifgp")


def test_default_params_are_the_papers():
    import paper_2508_19737_amd as ifgp
    p = ifgp.params()
    assert (p.alpha, p.theta, p.eps, p.znorm_ddof, p.storage) == (1.0, 0.1, 1e-3, 0, ifgp.F32)


def test_footprint_bytes():
    import paper_2508_19737_amd as ifgp
    b16 = ifgp.footprint_bytes(2_000_000, 40_000_000, 64, "bf16")
    b32 = ifgp.footprint_bytes(2_000_000, 40_000_000, 64, "f32")
    # graph ~ 2 * (16 MB + 160 MB); two BF16 feature buffers 512 MB
    assert 0.85e9 < b16 < 1.2e9
    assert b32 - b16 == 2 * 2_000_000 * 64 * 2
    assert ifgp.footprint_bytes(1000, 0, 20, "bf16") == ifgp.footprint_bytes(1000, 0, 32, "bf16")
    with pytest.raises(ifgp.IfgpError):
        ifgp.footprint_bytes(10, 10, 300, "bf16")
    with pytest.raises(ifgp.IfgpError):
        ifgp.footprint_bytes(10, 10, 3, "f64")


def test_debug_grid_x_round_trip():
    import paper_2508_19737_amd as ifgp
    lib = ifgp.lib
    prev = ctypes.c_int64()
    assert lib.ifgp_debug_grid_x(-1, ctypes.byref(prev)) == -1
    assert ifgp.debug_grid_x(7) == 2**21       # the default cap
    assert ifgp.debug_grid_x(0) == 7           # 0 restores the default
    assert ifgp.debug_grid_x(0) == 2**21
