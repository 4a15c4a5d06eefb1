"""Run tests against the host-sanitized build of libifgp: the library's host
code (argument checks, handle lifecycle, staging, the caching allocator, the
BIRCH CF-tree) compiled with AddressSanitizer and UndefinedBehaviorSanitizer,
device code as usual.

    python paper_2508_19737_amd/sanitize_check.py [--no-build] [--ubsan] [pytest args]

Default pytest arguments: -x -q -m "not gpu" tests/.  The clang ASan runtime is
preloaded (Python itself is not instrumented), leak detection is off (the
interpreter keeps its allocations until exit) and any report stops the run
with a non-zero status.  --ubsan runs against the UBSan-only build instead
(libifgp_ubsan.so, its runtime found through the library path): ASan's shadow
memory needs address-space reservations that a process driving the GPU may
not be granted, UBSan needs none, so the GPU tests can run under it.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def asan_runtime() -> str:
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise SystemExit("clang ASan runtime not found under /opt/rocm/lib/llvm")
    return hits[-1]


def preload_with_asan() -> str:
    """LD_PRELOAD for a sanitised child: the ASan runtime first (it must come
    first in the library list), then whatever the environment preloads."""
    rest = os.environ.get("LD_PRELOAD", "")
    return asan_runtime() + (":" + rest if rest else "")


def ubsan_dir() -> str:
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/"
                            "libclang_rt.ubsan_standalone-x86_64.so"))
    if not hits:
        raise SystemExit("clang UBSan runtime not found under /opt/rocm/lib/llvm")
    return os.path.dirname(hits[-1])


def main(argv):
    build = "--no-build" not in argv
    ub = "--ubsan" in argv
    args = [a for a in argv if a not in ("--no-build", "--ubsan")] or ["-x", "-q", "-m", "not gpu",
                                                                       "tests/"]
    sys.path.insert(0, HERE)
    import build as b
    if ub:
        if build:
            b.build(out=b.LIB_UBSAN, sanitize="ub")
        nm = subprocess.run(["nm", "-D", b.LIB_UBSAN], capture_output=True, text=True).stdout
        if "__ubsan_handle" not in nm:
            raise SystemExit(f"{b.LIB_UBSAN} is not instrumented")
        lp = ubsan_dir() + (":" + os.environ["LD_LIBRARY_PATH"] if os.environ.get("LD_LIBRARY_PATH") else "")
        env = dict(os.environ, IFGP_LIBRARY=b.LIB_UBSAN, LD_LIBRARY_PATH=lp,
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        print(f"sanitizer run: IFGP_LIBRARY={b.LIB_UBSAN}", flush=True)
        return subprocess.call([sys.executable, "-m", "pytest", *args], cwd=ROOT, env=env)
    if build:
        b.build(out=b.LIB_SAN, sanitize=True)
    nm = subprocess.run(["nm", "-D", b.LIB_SAN], capture_output=True, text=True).stdout
    if "__asan_report" not in nm or "__ubsan_handle" not in nm:
        raise SystemExit(f"{b.LIB_SAN} is not instrumented")
    env = dict(os.environ, IFGP_LIBRARY=b.LIB_SAN, LD_PRELOAD=preload_with_asan(),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    print(f"sanitizer run: IFGP_LIBRARY={b.LIB_SAN}", flush=True)
    return subprocess.call([sys.executable, "-m", "pytest", *args], cwd=ROOT, env=env)


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
