"""Host check of the FP64-carried pow the device interpreter uses
(paper_2103_07512_amd/csrc/pow_fp64.h, compiled here for the CPU): C99
special cases against the C library's powf, random operands against the C
library's FP64 pow rounded once (see tests/pow_check.cpp)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2103_07512_amd", "csrc")


def test_pow_fp64_against_libm(tmp_path):
    exe = str(tmp_path / "pow_check")
    r = subprocess.run(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-Wall", "-I", CSRC,
                        os.path.join(HERE, "pow_check.cpp"), "-o", exe, "-lm"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout[-2000:])
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout[-4000:] + r.stderr
