"""Host check of the evaluation planner (tests/planner_check.cpp): random
populations hash-consed into DAGs, planned with the sequential and the
level-parallel decision passes at stack depths that force spills, and every
emitted program run on a host stack machine against direct evaluation of
its root node.  Compiled with hipcc for the CPU (the planner's source uses
the HIP headers) and linked against the built library; no device call."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_2103_07512_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_planner_programs_and_decisions(tmp_path):
    from paper_2103_07512_amd import tgp
    assert os.path.exists(tgp.LIBRARY), "build the library first (__graft_entry__.build())"
    exe = str(tmp_path / "planner_check")
    r = subprocess.run([HIPCC, "-O2", "-std=c++17", "-w", "-I", os.path.join(ROOT, "include"),
                        "-I", os.path.join(PKG, "csrc"), os.path.join(HERE, "planner_check.cpp"), "-o", exe,
                        "-L", PKG, "-ltgp", f"-Wl,-rpath,{PKG}", "-lpthread"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(r.stdout[-3000:])
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout[-4000:] + r.stderr[-2000:]
