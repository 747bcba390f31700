"""CPU checks of the C ABI boundary: the library loads and exports every
function include/tgp.h declares, and the binding's view of it matches."""
import os
import re
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tgp.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tgp_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    from paper_2103_07512_amd import tgp
    lib = tgp.lib()
    names = _declared()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", tgp.LIBRARY], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (tgp_\w+)", out))
    assert set(names) <= exported


def test_binding_covers_header():
    from paper_2103_07512_amd import tgp
    assert sorted(n for n, _, _ in tgp.SIGNATURES) == _declared()


def test_token_layout():
    from paper_2103_07512_amd import popgen, tgp
    assert tgp.TOKEN_DTYPE.itemsize == 8
    assert popgen.TOKEN_DTYPE == tgp.TOKEN_DTYPE
    text = open(HEADER).read()
    for name, code in popgen.OP_CODE.items():
        if name == "mul":
            continue
        m = re.search(rf"TGP_{name.upper()}\s*=\s*(\d+)", text)
        assert m and int(m.group(1)) == code, name


def test_no_gpu_gives_clean_error():
    """Without a GPU the library reports an error code instead of crashing."""
    import ctypes
    from paper_2103_07512_amd import tgp
    try:
        import torch
        if torch.cuda.is_available():
            return
    except ImportError:
        pass
    h = ctypes.c_void_p()
    st = tgp.lib().tgp_ctx_create(0, None, ctypes.byref(h))
    assert st == -6 and not h.value
    assert tgp.lib().tgp_last_error(None)


def test_generated_interpreter_is_current():
    gen = os.path.join(ROOT, "paper_2103_07512_amd", "csrc", "gen_interp.py")
    assert subprocess.run([sys.executable, gen, "--check"]).returncode == 0


def test_library_built_for_gfx950_only():
    from paper_2103_07512_amd import tgp
    data = open(tgp.LIBRARY, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data
    for other in (b"gfx942", b"gfx90a", b"gfx908", b"gfx1100"):
        assert other not in data


def test_header_is_plain_c(tmp_path):
    """include/tgp.h is a C header: it compiles as strict C99 (no C++ or HIP
    types cross the boundary)."""
    src = tmp_path / "abi.c"
    src.write_text('#include "tgp.h"\nint main(void) { tgp_ctx c = 0; (void)c; return 0; }\n')
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                        os.path.join(ROOT, "include"), "-c", str(src), "-o", str(tmp_path / "abi.o")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
