"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU): the ABI and BIRCH host tests pass against the instrumented build, and
the instrumentation is live -- a host buffer one row too small for
ifgp_birch_centers is reported as a heap-buffer-overflow.  Device code is not
instrumented."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2508_19737_amd")

pytestmark = pytest.mark.skipif(bool(os.environ.get("IFGP_LIBRARY")),
                                reason="already inside a run against another build")


@pytest.fixture(scope="module")
def san():
    sys.path.insert(0, PKG)
    import build as b
    import sanitize_check as sc
    srcs = [os.path.join(PKG, "csrc", f) for f in os.listdir(os.path.join(PKG, "csrc"))]
    if (not os.path.exists(b.LIB_SAN)
            or os.path.getmtime(b.LIB_SAN) < max(os.path.getmtime(f) for f in srcs)):
        b.build(out=b.LIB_SAN, sanitize=True)
    env = dict(os.environ, IFGP_LIBRARY=b.LIB_SAN, LD_PRELOAD=sc.preload_with_asan(),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    return env


def test_host_code_clean_under_sanitizers(san):
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                        "tests/test_abi.py", "tests/test_birch_host.py"],
                       cwd=ROOT, env=san, capture_output=True, text=True, timeout=600)
    print(r.stdout[-2000:], r.stderr[-2000:])
    assert r.returncode == 0
    assert "passed" in r.stdout


def test_instrumentation_reports_a_host_overflow(san):
    code = textwrap.dedent("""
        import ctypes, numpy as np
        import paper_2508_19737_amd as ifgp
        assert ifgp.LIB_PATH.endswith("libifgp_san.so"), ifgp.LIB_PATH
        b = ifgp.Birch(4, 0.1, 10)
        b.partial_fit(np.random.default_rng(0).normal(size=(50, 4)))
        m = b.info()["clusters"]
        short = np.empty((m - 1) * 4, dtype=np.float64)     # one row too small
        ifgp.lib.ifgp_birch_centers(b._live(), short.ctypes.data_as(ctypes.c_void_p))
        print("NOT CAUGHT")
    """)
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=san, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr
    assert "NOT CAUGHT" not in r.stdout
