"""Host-only checks of the serving form's resident-subtree bookkeeping
(arena, LRU eviction, pins, run ends), built from the library's header with
the host compiler and run on the CPU."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2103_07512_amd", "csrc")


@pytest.mark.parametrize("sanitize", [False, True])
def test_subtree_cache_bookkeeping(tmp_path, sanitize):
    exe = str(tmp_path / "cache_sim")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-I", CSRC, os.path.join(HERE, "cache_sim.cpp"),
           "-o", exe]
    if sanitize:
        cmd[1:1] = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout + r.stderr
