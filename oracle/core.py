"""ctypes wrapper of oracle.c (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

STABLE = 1             # finite case whose value is insensitive to FP32 rounding
NONFINITE_STABLE = 2   # every FP32 variant gives the same non-finite class
ENVELOPE = 4           # finite, clear of every discontinuity, bound above the stable limit

_TOKEN = np.dtype([("op", "u1"), ("var", "u1"), ("pad", "<u2"), ("value", "<f4")])
_lib = None
# A test that plants a mistake in a copy of oracle.c points this at the
# mutant's library (the pins must then fail).
_OVERRIDE = os.environ.get("TGP_ORACLE_LIBRARY")


def library_path() -> str:
    return _OVERRIDE or _LIB


def build(src: str = _SRC, out: str = _LIB) -> str:
    """Compile oracle.c (or a copy of it) with gcc (plain -O2, no fast-math, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-Wall", src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _load():
    global _lib
    if _lib is None:
        if not _OVERRIDE and not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(library_path())
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.orc_eval.argtypes = [P, P, i64, ctypes.c_int, P, P, P, P, i64, P, P, P, P, ctypes.c_int]
        lib.orc_eval.restype = ctypes.c_int
        lib.orc_fitness.argtypes = [P, P, i64, ctypes.c_int, i64, ctypes.c_int, P]
        lib.orc_fitness.restype = ctypes.c_int
        lib.orc_coords.argtypes = [i64, ctypes.c_double, ctypes.c_double, P]
        lib.orc_coords.restype = ctypes.c_int
        lib.orc_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def max_threads() -> int:
    return int(_load().orc_max_threads())


def coords(n: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    out = np.empty(n, dtype=np.float32)
    if _load().orc_coords(n, lo, hi, _ptr(out)) != 0:
        raise ValueError("bad axis")
    return out


def evaluate(tokens, offsets, shape, lo=None, hi=None, cases=None, variants=False,
             nthreads: int = 0, bound=False):
    """Per-case values of every tree.

    Returns v64 [n_roots][n_cases] (float64); with variants=True the tuple
    (v64, v32r, stab) with the O32r values and the uint8 stability flags, and
    with bound=True as well, (v64, v32r, stab, ebound) with the running error
    bound of every root.
    """
    tokens = np.ascontiguousarray(tokens, dtype=_TOKEN)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    shape = np.ascontiguousarray(shape, dtype=np.int64)
    nd = len(shape)
    lo = np.ascontiguousarray(lo if lo is not None else [-1.0] * nd, dtype=np.float64)
    hi = np.ascontiguousarray(hi if hi is not None else [1.0] * nd, dtype=np.float64)
    n_roots = len(offsets) - 1
    if cases is None:
        n_cases = int(np.prod(shape))
        cptr = None
    else:
        cases = np.ascontiguousarray(cases, dtype=np.int64)
        n_cases = len(cases)
        cptr = cases
    v64 = np.empty((n_roots, n_cases), dtype=np.float64)
    variants = variants or bound
    v32 = np.empty_like(v64) if variants else None
    st = np.empty((n_roots, n_cases), dtype=np.uint8) if variants else None
    eb = np.empty_like(v64) if bound else None
    rc = _load().orc_eval(_ptr(tokens), _ptr(offsets), n_roots, nd, _ptr(shape), _ptr(lo),
                          _ptr(hi), _ptr(cptr), n_cases, _ptr(v64), _ptr(v32), _ptr(st),
                          _ptr(eb), int(nthreads))
    if rc == -1000000000:
        raise ValueError("bad domain or case list")
    if rc < 0:
        raise ValueError(f"malformed tree {-rc - 1}")
    if bound:
        return v64, v32, st, eb
    return (v64, v32, st) if variants else v64


def fitness(values, target, n_ind: int, n_ch: int = 1, loss: str = "rmse") -> np.ndarray:
    """FP64 RMSE ('rmse') or MSE ('mse') per individual; non-finite -> +inf."""
    values = np.ascontiguousarray(values, dtype=np.float64)
    target = np.ascontiguousarray(target, dtype=np.float32)
    n_cases = values.shape[-1]
    if values.size != n_ind * n_ch * n_cases or target.size != n_ch * n_cases:
        raise ValueError("shape mismatch")
    out = np.empty(n_ind, dtype=np.float64)
    rc = _load().orc_fitness(_ptr(values), _ptr(target), n_ind, n_ch, n_cases,
                             0 if loss == "rmse" else 1, _ptr(out))
    if rc != 0:
        raise ValueError("bad fitness arguments")
    return out


def render_target(trees, shape, lo=None, hi=None):
    """Render target trees (one per channel) in O64 and round to FP32.

    Returns float32 [n_ch][cases], or None when any value is non-finite.
    """
    lens = [len(t) for t in trees]
    offsets = np.zeros(len(trees) + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    toks = np.concatenate(trees).astype(_TOKEN)
    v = evaluate(toks, offsets, shape, lo, hi)
    with np.errstate(over="ignore", invalid="ignore"):
        t = v.astype(np.float32)
    if not np.all(np.isfinite(t)):
        return None
    return t


def target_renderer(shape, lo=None, hi=None):
    """render(tree) for popgen.pick_target: O64 rounded to FP32, None if non-finite."""
    def render(tree):
        t = render_target([tree], shape, lo, hi)
        return None if t is None else t[0]
    return render
