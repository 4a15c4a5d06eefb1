"""Compile libifgp.so (HIP, gfx950) in-tree.

    python paper_2508_19737_amd/build.py [--jobs N]

(run by path: importing the package loads the library this script builds)

Objects go to _build/ at the repository root; the shared library is written
next to this file.  Every call recompiles.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libifgp.so")
SOURCES = ["primitives.hip", "graph.hip", "ffp.hip", "api.hip", "birch.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
    "-I", INCLUDE, "-I", CSRC,
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer (device code is
# built as usual): each flag applies to the host pass only.
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all",
            "-Xarch_host", "-g"]
LIB_SAN = os.path.join(HERE, "libifgp_san.so")
# UndefinedBehaviorSanitizer alone (no shadow memory: usable where ASan's
# address-space reservations are not, e.g. next to the GPU runtime)
UBSAN = ["-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all",
         "-Xarch_host", "-g"]
LIB_UBSAN = os.path.join(HERE, "libifgp_ubsan.so")


def _compile(src: str, objdir: str = OBJDIR, defines=(), extra=()) -> str:
    obj = os.path.join(objdir, os.path.splitext(os.path.basename(src))[0] + ".o")
    cmd = [HIPCC, *FLAGS, *extra, *[f"-D{d}" for d in defines], "-c", os.path.join(CSRC, src),
           "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    # the host pass does not know the device feature above: that warning is expected
    noise = [ln for ln in r.stderr.splitlines()
             if ln.strip() and "packed-fp32-ops" not in ln and "warning generated" not in ln]
    if noise:
        sys.stderr.write("\n".join(noise) + "\n")
    return obj


def build(jobs: int | None = None, out: str = LIB, defines=(), sanitize: bool | str = False) -> str:
    """Compile and link; `defines` (NAME=VALUE) override the kernels' tuning
    constants (IFGP_HOP_UNROLL, IFGP_LIGHT_ROWS, IFGP_MED_DEGREE,
    IFGP_HUB_DEGREE).  sanitize=True builds the host code with ASan and
    UBSan (load it with the clang ASan runtime preloaded), sanitize="ub" with
    UBSan alone (the UBSan runtime on the library path); see
    sanitize_check.py."""
    extra = UBSAN if sanitize == "ub" else SANITIZE if sanitize else []
    tag = "ubsan" if sanitize == "ub" else "san"
    objdir = OBJDIR if out == LIB and not sanitize else os.path.join(
        OBJDIR, "variant_" + (tag if sanitize else str(abs(hash(out)))))
    os.makedirs(objdir, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, objdir, defines, extra), SOURCES))
    tmp = out + ".tmp"
    link_extra = (["-Xarch_host", "-fsanitize=undefined", "-shared-libsan"] if sanitize == "ub"
                  else ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                        "-shared-libsan"] if sanitize else [])
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *link_extra, *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--out", default=LIB)
    ap.add_argument("--define", action="append", default=[])
    ap.add_argument("--sanitize", action="store_true",
                    help="host code with ASan + UBSan, written to libifgp_san.so")
    ap.add_argument("--ubsan", action="store_true",
                    help="host code with UBSan alone, written to libifgp_ubsan.so")
    a = ap.parse_args()
    if a.sanitize:
        print(build(a.jobs, LIB_SAN, a.define, sanitize=True))
    elif a.ubsan:
        print(build(a.jobs, LIB_UBSAN, a.define, sanitize="ub"))
    else:
        print(build(a.jobs, os.path.abspath(a.out), a.define))
