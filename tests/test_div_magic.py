"""Host check of the multiply-shift division by invariant divisors that the
interpreter uses to turn case indices into grid coordinates
(paper_2103_07512_amd/csrc/div_magic.h, see tests/div_check.cpp)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2103_07512_amd", "csrc")


def test_div_magic_exact(tmp_path):
    exe = str(tmp_path / "div_check")
    r = subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-I", CSRC, os.path.join(HERE, "div_check.cpp"),
                        "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout + r.stderr
