"""The host index of twin leaf entries (centroids equal bit for bit) that the
BIRCH update labelling keeps: its source, cut out of birch.hip, compiled with
g++ under AddressSanitizer and UndefinedBehaviorSanitizer and driven at
random against a plain model (tests/twin_groups_fuzz.cpp)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "paper_2508_19737_amd", "csrc", "birch.hip")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_twin_group_index(tmp_path):
    s = open(SRC).read()
    a = s.index("struct TwinGroups {")
    b = s.index("\n};\n", a) + 4
    (tmp_path / "twins.inc").write_text(s[a:b])
    exe = tmp_path / "fuzz"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", str(tmp_path),
                    os.path.join(HERE, "twin_groups_fuzz.cpp"), "-o", str(exe)], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "twin groups: ok" in r.stdout
