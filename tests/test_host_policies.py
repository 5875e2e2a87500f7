"""Host-side policies that need no GPU: the request server's admission
accounting (refusal by in-flight matrices and by admitted bytes) and the
bounded, pin-aware LRU that holds the convenience entry points' plans.  Both
live in HIP-free headers of the library; this test compiles them into a small
checker with g++ (address and undefined-behaviour sanitizers on) and runs it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2604_27325_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "host", "policies_check.cpp")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_admission_and_cache_policies(tmp_path):
    exe = str(tmp_path / "policies_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", CSRC, SRC, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr:
        cmd = [c for c in cmd if not c.startswith("-fsanitize") and c != "-fno-sanitize-recover=all"]
        r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([exe], capture_output=True, text=True)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "admission ok" in out.stdout and "lru ok" in out.stdout
