"""Host check of the FP32 operator implementations the device interpreter
uses (paper_2103_07512_amd/csrc/fp32_math.h, compiled here for the CPU):
sin(pi x), cos(pi x), tan(pi x), pow (with every C99 special case bit for
bit against the C library's powf), sstep, sstepp, len and lerp, each against
its exact value in FP64 over millions of seeded operands, in ulps and
against the accuracy the parity classifier assumes (tests/fp32_math_check.cpp)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2103_07512_amd", "csrc")


def test_fp32_math_against_libm(tmp_path):
    exe = str(tmp_path / "fp32_math_check")
    r = subprocess.run(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-I", CSRC,
                        os.path.join(HERE, "fp32_math_check.cpp"), "-o", exe, "-lm"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout[-3000:])
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout[-4000:] + r.stderr
