"""The oracle's pins must catch plausible mistakes: each test plants one
mistake (a swapped operand, a dropped term, a wrong sign or protection, a
wrong accuracy constant or margin in the stability classifier) in a copy of
oracle.c, builds it on the CPU, and runs the pin suites (tests/test_oracle.py
and tests/test_oracle_stability.py) against it in a fresh process; they must
fail.  The identity rewrites of the oracle's DAG builder (dag.py) get the same
treatment against tests/test_oracle_rewrite.py."""
import os
import shutil
import subprocess
import sys

import pytest

from oracle import core

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "oracle.c")

MUTANTS = [
    ("sub operands swapped", "case OV_SUB: return a - b;", "case OV_SUB: return b - a;"),
    ("div protection gives 1", "return b == 0.0 ? 0.0 : a / b;", "return b == 0.0 ? 1.0 : a / b;"),
    ("sin and cos swapped", "case OV_SIN: sincospi64(a, &s, &co); return s;",
     "case OV_SIN: sincospi64(a, &s, &co); return co;"),
    ("pi prescale dropped", "double st = sin(M_PI * t), ct = cos(M_PI * t);",
     "double st = sin(t), ct = cos(t);"),
    ("log protection value", "return a < 0.0 ? -1.0 : log(a);", "return a < 0.0 ? 0.0 : log(a);"),
    ("pow(0, 0) = 1", "return (a == 0.0 && b == 0.0) ? 0.0 : pow(a, b);",
     "return (a == 0.0 && b == 0.0) ? 1.0 : pow(a, b);"),
    ("mod truncated", "if (r != 0.0 && ((r < 0.0) != (y < 0.0)))", "if (0)"),
    ("clip bounds swapped", "case OV_CLIP: return max_num(min_num(a, c), b);",
     "case OV_CLIP: return max_num(min_num(a, b), c);"),
    ("mdist not halved", "case OV_MDIST: return (a + b) / 2.0;", "case OV_MDIST: return (a + b);"),
    ("sstepp term dropped", "return a * a * a * (a * (6.0 * a - 15.0) + 10.0);",
     "return a * a * a * (a * (6.0 * a - 15.0));"),
    ("sign flipped", "return (double)((a > 0.0) - (a < 0.0));", "return (double)((a < 0.0) - (a > 0.0));"),
    ("sqrt protection", "return a < 0.0 ? 0.0 : sqrt(a);", "return a < 0.0 ? sqrt(-a) : sqrt(a);"),
    ("grid endpoint", "lo + (hi - lo) * (double)i / (double)(n - 1)", "lo + (hi - lo) * (double)i / (double)n"),
    ("rmse without the root", "(loss == 0 ? sqrt(s / N) : s / N)", "(loss == 0 ? s / N : s / N)"),
    ("xor computed as or", "(ia ^ ib)", "(ia | ib)"),
    ("integers rounded, not truncated", "return (int32_t)trunc(x);", "return (int32_t)rint(x);"),
    ("warp axes swapped", "warp_coords(d, ev64(d, n, p->kid[1], xyz), ev64(d, n, p->kid[2], xyz), xyz, at);",
     "warp_coords(d, ev64(d, n, p->kid[2], xyz), ev64(d, n, p->kid[1], xyz), xyz, at);"),
    ("warp rounds halves down", "(d->hi[k] - d->lo[k])) + 0.5;", "(d->hi[k] - d->lo[k])) + 0.4999;"),
    ("min of signed zeros by operand order", "        return signbit(a) ? a : b;\n    return fmin(a, b);",
     "        return b;\n    return fmin(a, b);"),
    # the stability classifier (error bound and flags)
    ("correctly rounded accuracy x10", "#define U_CR 1.1920928955078125e-07", "#define U_CR 1.1920928955078125e-06"),
    ("library accuracy x10", "#define U_LIB 4.76837158203125e-07", "#define U_LIB 4.76837158203125e-06"),
    ("discontinuity margin 40 bounds", "#define MARGIN 4.0", "#define MARGIN 40.0"),
    ("mult bound drops a derivative", "err = contrib(b, ea) + contrib(a, eb) + rnd(ucr, av);",
     "err = contrib(b, ea) + rnd(ucr, av);"),
    ("sin bound drops its derivative", "err = contrib(M_PI * co, ea) + rnd(exact_in", "err = rnd(exact_in"),
    ("no subnormal floor", "u * (av > 0x1p-126 ? av : 0x1p-126)", "u * av"),
    ("0^b sign of b not checked", "if (a == 0.0 && !clear_of(b, 0.0, eb)) *ok = 0;", ""),
    ("phase of sin unguarded", "        if (M_PI * ea > LINEAR) *ok = 0;       /* phase error not small against the period */\n", ""),
    ("overflow edge unchecked", "    else if (!clear_of(av, FLT_OVERFLOW, err))\n        *ok = 0;", ""),
    ("stable limit x10", "e <= 5e-6 * sc && fabs(r32 - v) <= 5e-6 * sc", "e <= 5e-5 * sc && fabs(r32 - v) <= 5e-6 * sc"),
    ("exactness without exact operands", "const double ucr = exact_in && (double)(float)val == val ? 0.0 : U_CR;",
     "const double ucr = (double)(float)val == val ? 0.0 : U_CR;"),
    ("min/max bound of the other operand", "return val == x ? ex : ey;", "return val == x ? ey : ex;"),
    ("envelope limit x10", "e <= 0.0625 * sc &&", "e <= 0.625 * sc &&"),
]


def _run_pins(tmp_path, text):
    src = tmp_path / "oracle_copy.c"
    src.write_text(text)
    lib = core.build(str(src), str(tmp_path / "liboracle_copy.so"))
    env = dict(os.environ, TGP_ORACLE_LIBRARY=lib)
    return subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                           os.path.join(HERE, "test_oracle.py"), os.path.join(HERE, "test_oracle_stability.py")],
                          env=env, capture_output=True, text=True, timeout=600)


def test_unmodified_copy_passes(tmp_path):
    """Control: the same procedure on an unmodified copy passes every pin."""
    with open(SRC) as f:
        r = _run_pins(tmp_path, f.read())
    assert r.returncode == 0, r.stdout[-3000:]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new):
    with open(SRC) as f:
        text = f.read()
    assert text.count(old) == 1, f"mutation site not unique or missing: {old!r}"
    r = _run_pins(tmp_path, text.replace(old, new))
    assert r.returncode != 0, f"planted mistake '{name}' passed every pin:\n{r.stdout[-2000:]}"


DAG = os.path.join(os.path.dirname(HERE), "oracle", "dag.py")
DAG_MUTANTS = [
    ("sub(x, -0) rewritten", "if op == _SUB and const_bits(kids[1]) == _POS_ZERO:",
     "if op == _SUB and const_bits(kids[1]) in (_POS_ZERO, _NEG_ZERO):"),
    ("add(x, +0) rewritten", "        if const_bits(kids[1]) == _NEG_ZERO:\n            return kids[0]",
     "        if const_bits(kids[1]) in (_NEG_ZERO, _POS_ZERO):\n            return kids[0]"),
    ("neg(neg(x)) to the inner neg", "return node_key[kids[0]][2][0]", "return kids[0]"),
    ("min/max of different operands", "if op in (_MIN, _MAX) and kids[0] == kids[1]:", "if op in (_MIN, _MAX):"),
    ("if(c, y, y) to the condition", "if op == _IF and kids[1] == kids[2]:\n        return kids[1]",
     "if op == _IF and kids[1] == kids[2]:\n        return kids[0]"),
    ("rewritten token not counted", "                    mult[target] += 1\n", ""),
    ("mult by -1 rewritten", "        if const_bits(kids[1]) == _ONE:\n            return kids[0]\n        if const_bits(kids[0]) == _ONE:",
     "        if const_bits(kids[1]) in (_ONE, 0xBF800000):\n            return kids[0]\n        if const_bits(kids[0]) == _ONE:"),
]


def _run_rewrite_pins(tmp_path, text):
    pkg = tmp_path / "oracle"
    shutil.copytree(os.path.dirname(DAG), pkg, ignore=shutil.ignore_patterns("__pycache__"))
    (pkg / "dag.py").write_text(text)
    env = dict(os.environ, PYTHONPATH=os.pathsep.join([str(tmp_path), HERE, os.path.dirname(HERE)]))
    return subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                           os.path.join(HERE, "test_oracle_rewrite.py")],
                          env=env, capture_output=True, text=True, timeout=600, cwd=str(tmp_path))


def test_rewrite_control_passes(tmp_path):
    with open(DAG) as f:
        r = _run_rewrite_pins(tmp_path, f.read())
    assert r.returncode == 0, r.stdout[-3000:]


@pytest.mark.parametrize("name,old,new", DAG_MUTANTS, ids=[m[0] for m in DAG_MUTANTS])
def test_rewrite_pins_catch_planted_mistake(tmp_path, name, old, new):
    with open(DAG) as f:
        text = f.read()
    assert text.count(old) == 1, f"mutation site not unique or missing: {old!r}"
    r = _run_rewrite_pins(tmp_path, text.replace(old, new))
    assert r.returncode != 0, f"planted mistake '{name}' passed every pin:\n{r.stdout[-2000:]}"
