"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Every check here compares the oracle with something other than itself:
hand-derived values (tests/golden, each citing Table 1 or Eq. 1), closed
forms, algebraic identities, library routines (numpy) and brute force over
all small trees with an independent numpy evaluator written in the style of
the paper's serial EVAL baseline (Sec. 4.1).
"""
import glob
import itertools
import math
import os

import numpy as np
import pytest

import oracle
from paper_2103_07512_amd import popgen as pg

GOLD = os.path.join(os.path.dirname(__file__), "golden")
G5 = (5, 5)


def ev(text, shape=G5, variants=False, **kw):
    t = pg.parse(text)
    off = np.array([0, len(t)], np.int64)
    out = oracle.evaluate(t, off, shape, variants=variants, **kw)
    return tuple(a[0] for a in out) if variants else out[0]


def ev1(text):
    """Value of a constant tree (domain of one point)."""
    return ev(text, (1,))[0]


# --------------------------------------------------------------- golden grids
def _load_golden(path):
    tree, rows = None, []
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("tree:"):
            tree = line[5:].strip()
            continue
        rows.append([float(w) for w in line.split()])
    return tree, np.array(rows, np.float64)


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(GOLD, "g*.txt"))),
                         ids=lambda p: os.path.basename(p))
def test_golden_5x5(path):
    tree, want = _load_golden(path)
    got = ev(tree).reshape(5, 5)
    assert np.array_equal(np.isnan(got), np.isnan(want))
    m = ~np.isnan(want)
    inf = np.isinf(want) & m
    assert np.array_equal(got[inf], want[inf])
    fin = m & ~inf
    np.testing.assert_allclose(got[fin], want[fin], rtol=1e-15, atol=0)


# ------------------------------------------------------------- Table 1 points
@pytest.mark.parametrize("text,want", [
    ("div(0.5, 0.0)", 0.0), ("div(0.5, -0.0)", 0.0), ("div(-0.75, 0.5)", -1.5),
    ("log(-0.5)", -1.0), ("log(0.0)", -math.inf), ("log(1.0)", 0.0),
    ("sqrt(-0.25)", 0.0), ("sqrt(0.25)", 0.5),
    ("pow(0.0, 0.0)", 0.0), ("pow(0.5, 2.0)", 0.25), ("pow(-0.5, 2.0)", 0.25),
    ("pow(0.0, -1.0)", math.inf), ("pow(-0.5, 3.0)", -0.125),
    ("sign(-0.3)", -1.0), ("sign(0.0)", 0.0), ("sign(-0.0)", 0.0), ("sign(0.7)", 1.0),
    ("abs(-0.5)", 0.5), ("neg(0.25)", -0.25),
    ("clip(0.5, -0.25, 0.25)", 0.25), ("clip(-0.5, -0.25, 0.25)", -0.25),
    ("clip(0.1, -0.25, 0.25)", float(np.float32(0.1))), ("clip(0.1, 0.5, -0.5)", 0.5),
    ("mod(0.75, 0.5)", 0.25), ("mod(-0.75, 0.5)", 0.25), ("mod(0.75, -0.5)", -0.25),
    ("mod(-0.75, -0.5)", -0.25), ("mod(0.3, 0.0)", 0.0),
    ("frac(-0.25)", 0.75), ("frac(0.75)", 0.75), ("frac(1.0)", 0.0), ("frac(-1.0)", 0.0),
    ("if(0.0, 0.5, -0.5)", -0.5), ("if(-0.0, 0.5, -0.5)", -0.5), ("if(0.1, 0.5, -0.5)", 0.5),
    ("if(pow(-0.5, 0.5), 0.5, -0.5)", 0.5),                 # NaN condition counts as true
    ("sin(0.5)", 1.0), ("sin(1.0)", 0.0), ("sin(-0.5)", -1.0), ("sin(2.5)", 1.0),
    ("sin(-3.5)", 1.0), ("cos(1.0)", -1.0), ("cos(0.5)", 0.0), ("cos(0.0)", 1.0),
    ("cos(-1.0)", -1.0), ("cos(3.0)", -1.0), ("cos(16777216.0)", 1.0), ("sin(16777215.0)", 0.0),
    ("exp(0.0)", 1.0), ("min(0.5, -0.25)", -0.25), ("max(0.5, -0.25)", 0.5),
    ("min(pow(-0.5, 0.5), 0.5)", 0.5), ("max(0.5, pow(-0.5, 0.5))", 0.5),
    ("mdist(0.5, -0.25)", 0.125), ("step(-0.1)", -1.0), ("step(0.0)", 1.0),
    ("sstep(0.5)", 0.5), ("sstepp(0.5)", 0.5), ("len(0.75, 1.0)", 1.25),
    ("lerp(0.0, 1.0, 0.25)", 0.25), ("lerp(0.0, 1.0, 1.25)", 0.25), ("lerp(0.0, 1.0, -0.75)", 0.25),
    # bitwise on truncated integers: 3 | 1, -2 ^ 1, -1 & 5, NaN -> 0, saturation
    ("or(3.7, 1.2)", 3.0), ("xor(-2.5, 1.0)", -1.0), ("and(-1.0, 5.9)", 5.0),
    ("or(pow(-0.5, 0.5), 6.0)", 6.0), ("and(exp(100.0), 1.0)", 1.0),
    ("or(neg(exp(100.0)), 0.0)", -2147483648.0), ("xor(0.9, -0.9)", 0.0),
])
def test_table1_points(text, want):
    got = ev1(text)
    if math.isinf(want):
        assert got == want
    else:
        assert got == want, (text, got, want)


def test_min_max_signed_zeros():
    """min and max order -0 below +0, in either operand order (the device's
    fminf / fmaxf do, and a zero's sign decides pow(0, -1) = +-inf)."""
    for text, want in (("min(0.0, neg(0.0))", -0.0), ("min(neg(0.0), 0.0)", -0.0),
                       ("max(0.0, neg(0.0))", 0.0), ("max(neg(0.0), 0.0)", 0.0),
                       ("pow(min(0.0, neg(0.0)), -1.0)", -math.inf), ("pow(max(neg(0.0), 0.0), -1.0)", math.inf),
                       ("clip(neg(0.0), 0.0, 0.5)", 0.0), ("clip(0.0, neg(0.5), neg(0.0))", -0.0)):
        got = ev1(text)
        assert got == want and math.copysign(1, got) == math.copysign(1, want), (text, got)


def test_nan_rules():
    assert math.isnan(ev1("pow(-0.5, 0.5)"))
    assert ev1("sign(pow(-0.5, 0.5))") == 0.0
    assert math.isnan(ev1("sin(div(1.0, 0.0))")) is False          # div protects: sin(0) = 0
    assert math.isnan(ev1("sin(exp(exp(exp(1.0))))")) is False     # huge finite argument
    assert math.isnan(ev1("cos(pow(0.0, -1.0))"))                  # cos(inf) is NaN


def test_trig_against_library():
    """sin(pi x), cos(pi x), tan(pi x) match numpy on generic points."""
    xs = [float(v) for v in np.float32(np.linspace(-3.3, 3.3, 97))]
    for name, fn in (("sin", np.sin), ("cos", np.cos), ("tan", np.tan)):
        got = np.array([ev1(f"{name}({x!r})") for x in xs])
        want = fn(np.pi * np.array(xs))
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-13)


def test_unary_against_library():
    xs = [float(v) for v in np.float32(np.linspace(-2.5, 2.5, 41))]
    for x in xs:
        assert ev1(f"exp({x!r})") == pytest.approx(np.exp(x), rel=1e-15, abs=0)
        assert ev1(f"log({x!r})") == pytest.approx(-1.0 if x < 0 else np.log(x), rel=1e-15)
        assert ev1(f"sqrt({x!r})") == (0.0 if x < 0 else np.sqrt(x))
        assert ev1(f"frac({x!r})") == x - np.floor(x)
        for y in (-1.5, -0.75, 0.5, 2.0):
            assert ev1(f"mod({x!r}, {y!r})") == np.mod(x, y)       # numpy's mod is floored
            want = 0.0 if x == 0 and y == 0 else np.power(abs(x), y)
            assert ev1(f"pow({abs(x)!r}, {y!r})") == pytest.approx(want, rel=1e-15, abs=0)


# ---------------------------------------------------------- coordinates, grid
def test_coordinates():
    assert oracle.coords(5).tolist() == [-1.0, -0.5, 0.0, 0.5, 1.0]
    c4 = oracle.coords(4)
    assert c4.tolist() == [-1.0, float(np.float32(-1 / 3)), float(np.float32(1 / 3)), 1.0]
    assert oracle.coords(1, -0.7, 2.0).tolist() == [float(np.float32(-0.7))]
    c = oracle.coords(1024)
    assert c[0] == -1.0 and c[-1] == 1.0 and np.all(np.diff(c) > 0)
    # antisymmetric grid: c[i] = -c[n-1-i]
    assert np.array_equal(c, -c[::-1])


def test_axis_order():
    """Axis 0 (x) is the slow axis, the last axis is fastest (row-major)."""
    got = ev("x", (2, 3))
    assert got.tolist() == [-1, -1, -1, 1, 1, 1]
    got = ev("y", (2, 3))
    assert got.tolist() == [-1, 0, 1, -1, 0, 1]
    got = ev("z", (2, 2, 3))
    assert got.tolist() == [-1, 0, 1] * 4
    got = ev("y", (2, 2, 3))
    assert got.tolist() == [-1, -1, -1, 1, 1, 1] * 2


def test_case_subset_matches_full():
    pop, dom, _ = pg.workload_c1()
    full = oracle.evaluate(pop.tokens, pop.offsets, dom.shape)
    idx = np.array([0, 5, 4095, 77, 1000], np.int64)
    sub = oracle.evaluate(pop.tokens, pop.offsets, dom.shape, cases=idx)
    assert np.array_equal(sub, full[:, idx])


def test_threads_do_not_change_values():
    pop, dom, _ = pg.workload_c1()
    a = oracle.evaluate(pop.tokens, pop.offsets, dom.shape, nthreads=1)
    b = oracle.evaluate(pop.tokens, pop.offsets, dom.shape, nthreads=4)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


# ------------------------------------------------------------ closed forms
def test_pagie_closed_form():
    """Eq. 1 written as a tree equals x^4/(1+x^4) + y^4/(1+y^4) on a 64x64 grid."""
    tree = "add(div(1.0, add(1.0, pow(x, -4.0))), div(1.0, add(1.0, pow(y, -4.0))))"
    got = ev(tree, (64, 64)).reshape(64, 64)
    c = oracle.coords(64).astype(np.float64)
    X, Y = np.meshgrid(c, c, indexing="ij")
    want = X ** 4 / (1 + X ** 4) + Y ** 4 / (1 + Y ** 4)
    np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-16)


def test_polynomial_closed_form():
    tree = "sub(mult(mult(x, x), y), add(x, mult(0.5, y)))"
    got = ev(tree, (33, 17)).reshape(33, 17)
    X, Y = np.meshgrid(oracle.coords(33).astype(float), oracle.coords(17).astype(float), indexing="ij")
    np.testing.assert_array_equal(got, X * X * Y - (X + 0.5 * Y))


# ------------------------------------------------------------- identities
RNG = np.random.default_rng(7)


def _random_subtrees(n, depth=3, functions=pg.F18, seed=11):
    mk = pg.TreeMaker(pg.Rng(seed), functions, 2)
    return [pg.to_text(mk.tree(depth, bool(i % 2))) for i in range(n)]


@pytest.mark.parametrize("t", _random_subtrees(12))
def test_identities(t):
    g = (16, 16)
    v = ev(t, g)
    fin = np.isfinite(v)
    assert np.all(ev(f"sub({t}, {t})", g)[fin] == 0)
    assert np.all(ev(f"div({t}, sub(y, y))", g) == 0)
    np.testing.assert_array_equal(ev(f"mod({t}, 1.0)", g)[fin], ev(f"frac({t})", g)[fin])
    c = ev(f"clip({t}, -0.25, 0.5)", g)
    assert np.all((c[~np.isnan(v)] >= -0.25) & (c[~np.isnan(v)] <= 0.5))
    s2c2 = ev(f"add(mult(sin({t}), sin({t})), mult(cos({t}), cos({t})))", g)
    np.testing.assert_allclose(s2c2[fin], 1.0, atol=1e-14)
    np.testing.assert_array_equal(ev(f"max({t}, {t})", g)[fin], v[fin])
    np.testing.assert_array_equal(ev(f"pow({t}, 1.0)", g)[fin], v[fin])
    np.testing.assert_array_equal(ev(f"mult(sign({t}), abs({t}))", g)[fin], v[fin])
    np.testing.assert_array_equal(ev(f"neg(neg({t}))", g)[fin], v[fin])
    np.testing.assert_array_equal(ev(f"if(0.0, x, {t})", g)[fin], v[fin])
    np.testing.assert_array_equal(ev(f"mdist({t}, {t})", g)[fin], v[fin])


# ---------------------------------------------- brute force vs EVAL-style numpy
def _np_eval(text, X, Y):
    """Independent evaluator: the tree text becomes a numpy expression evaluated by eval()."""
    def div(a, b):
        with np.errstate(all="ignore"):
            return np.where(b == 0, 0.0, a / np.where(b == 0, 1.0, b))

    def sinpi(a):
        with np.errstate(all="ignore"):
            r = np.sin(np.pi * np.asarray(a, float))
        a = np.asarray(a, float)
        return np.where(np.isfinite(a) & (a == np.round(a)), 0.0, r)

    def cospi(a):
        with np.errstate(all="ignore"):
            a = np.asarray(a, float)
            r = np.cos(np.pi * a)
        half = (a * 2 == np.round(a * 2)) & (a != np.round(a))
        return np.where(half, 0.0, r)

    def log(a):
        with np.errstate(all="ignore"):
            return np.where(a < 0, -1.0, np.log(np.where(a < 0, 1.0, a)))

    def sqrt(a):
        with np.errstate(all="ignore"):
            return np.where(a < 0, 0.0, np.sqrt(np.where(a < 0, 0.0, a)))

    def pw(a, b):
        with np.errstate(all="ignore"):
            return np.where((a == 0) & (b == 0), 0.0, np.power(a, b))

    def mod(a, b):
        with np.errstate(all="ignore"):
            return np.where(b == 0, 0.0, np.mod(a, np.where(b == 0, 1.0, b)))

    def sign(a):
        return np.where(np.isnan(a), 0.0, np.sign(a))

    def min_num(a, b):  # -0 below +0
        a, b = np.broadcast_arrays(np.asarray(a, float), np.asarray(b, float))
        return np.where((a == 0) & (b == 0), np.where(np.signbit(a), a, b), np.fmin(a, b))

    def max_num(a, b):
        a, b = np.broadcast_arrays(np.asarray(a, float), np.asarray(b, float))
        return np.where((a == 0) & (b == 0), np.where(np.signbit(a), b, a), np.fmax(a, b))

    def frac(a):
        return a - np.floor(a)

    def tanpi(a):
        with np.errstate(all="ignore"):
            return sinpi(a) / cospi(a)

    def ex(a):
        with np.errstate(all="ignore"):
            return np.exp(a)

    env = dict(
        add=lambda a, b: a + b, sub=lambda a, b: a - b, mult=lambda a, b: a * b, div=div,
        sin=sinpi, cos=cospi, tan=tanpi, exp=ex, log=log, pow=pw, min=min_num, max=max_num,
        mdist=lambda a, b: (a + b) / 2, neg=lambda a: -a, sqrt=sqrt, sign=sign, abs=np.abs,
        clip=lambda a, b, c: max_num(min_num(a, c), b), mod=mod, frac=frac,
        step=lambda a: np.where(a < 0, -1.0, 1.0), sstep=lambda a: a * a * (3 - 2 * a),
        sstepp=lambda a: a ** 3 * (a * (6 * a - 15) + 10),
        len=lambda a, b: np.where(np.isnan(a) | np.isnan(b), np.nan, np.hypot(a, b)),
        lerp=lambda a, b, c: a + (b - a) * frac(c), x=X, y=Y, inf=np.inf, nan=np.nan,
        np=np)
    env["if"] = lambda a, b, c: np.where(a != 0, b, c)

    def to_int(a):
        a = np.asarray(a, dtype=np.float64)
        with np.errstate(all="ignore"):
            t = np.where(np.isnan(a), 0.0, np.clip(np.trunc(a), -2.0 ** 31, 2.0 ** 31 - 1))
        return t.astype(np.int64)

    def warp(a, b, c):
        A, B, C = (np.broadcast_to(np.asarray(v, float), X.shape) for v in (a, b, c))

        def idx(t, n):
            with np.errstate(all="ignore"):
                u = (t + 1.0) * (n - 1) / 2.0 + 0.5
            return np.floor(np.where(np.isnan(u), 0.0, np.clip(u, 0, n - 1))).astype(int)
        return A[idx(B, X.shape[0]), idx(C, X.shape[1])]

    env["warp"] = warp
    env["or"] = lambda a, b: (to_int(a) | to_int(b)).astype(float)
    env["xor"] = lambda a, b: (to_int(a) ^ to_int(b)).astype(float)
    env["and"] = lambda a, b: (to_int(a) & to_int(b)).astype(float)
    code = text.replace("if(", "env['if'](").replace("xor(", "env['xor'](")
    code = code.replace("and(", "env['and'](").replace(" or(", " env['or'](")
    if code.startswith("or("):
        code = "env['or'](" + code[3:]
    code = code.replace("(or(", "(env['or'](")
    env["env"] = env
    with np.errstate(all="ignore"):
        return np.broadcast_to(eval(code, {"__builtins__": {}}, env), X.shape).astype(float)


TERMS = ["x", "y", "-1.0", "-0.5", "0.0", "0.5", "1.0"]
OPS1 = [n for n, a in pg.OPS if a == 1]
OPS2 = [n for n, a in pg.OPS if a == 2]
OPS3 = [n for n, a in pg.OPS if a == 3]


def _all_depth1():
    out = list(TERMS)
    out += [f"{o}({a})" for o in OPS1 for a in TERMS]
    out += [f"{o}({a}, {b})" for o in OPS2 for a in TERMS for b in TERMS]
    out += [f"{o}({a}, {b}, {c})" for o in OPS3 for a in TERMS for b in TERMS for c in TERMS]
    return out


def _compare(got, want, text):
    assert np.array_equal(np.isnan(got), np.isnan(want)), text
    m = ~np.isnan(got)
    big = m & ((np.abs(got) > 1e12) | (np.abs(want) > 1e12))
    # near tan's poles the numpy evaluator rounds pi: compare sign and magnitude only
    assert np.array_equal(np.sign(got[big]), np.sign(want[big])), text
    ok = m & ~big
    np.testing.assert_allclose(got[ok], want[ok], rtol=1e-12, atol=1e-12, err_msg=text)


def test_brute_force_depth1():
    """Every tree of depth <= 1 over the operators and 7 terminals, on the 4x4 grid."""
    trees = _all_depth1()
    assert len(trees) == 7 + 13 * 7 + 13 * 49 + 4 * 343
    c = oracle.coords(4).astype(float)
    X, Y = np.meshgrid(c, c, indexing="ij")
    toks = [pg.parse(t) for t in trees]
    pop = pg.Population.from_trees(toks)
    got = oracle.evaluate(pop.tokens, pop.offsets, (4, 4))
    for i, t in enumerate(trees):
        _compare(got[i], _np_eval(t, X, Y).ravel(), t)


def test_brute_force_depth2_sample():
    """A seeded sample of depth-2 compositions of depth-1 trees."""
    d1 = _all_depth1()
    rng = np.random.default_rng(3)
    names = OPS1 + OPS2 + OPS3
    trees = []
    for _ in range(3000):
        o = names[rng.integers(len(names))]
        a = dict(pg.OPS)[o]
        trees.append(f"{o}({', '.join(d1[rng.integers(len(d1))] for _ in range(a))})")
    c = oracle.coords(4).astype(float)
    X, Y = np.meshgrid(c, c, indexing="ij")
    pop = pg.Population.from_trees([pg.parse(t) for t in trees])
    got = oracle.evaluate(pop.tokens, pop.offsets, (4, 4))
    for i, t in enumerate(trees):
        _compare(got[i], _np_eval(t, X, Y).ravel(), t)


# ----------------------------------------------------------------- warp
def test_warp_gather_rules():
    """warp read as a gather at the nearest grid point (Sec. 3.2, Table 1)."""
    g = ev("add(x, mult(y, 3.0))").reshape(5, 5)
    # identity: each case reads its own point
    assert np.array_equal(ev("warp(add(x, mult(y, 3.0)), x, y)").reshape(5, 5), g)
    # transpose: t0 = y, t1 = x
    assert np.array_equal(ev("warp(add(x, mult(y, 3.0)), y, x)").reshape(5, 5), g.T)
    # halves round up: position (0.25 + 1) * 2 = 2.5 -> point 3; -0.25 -> 1.5 -> point 2
    assert np.all(ev("warp(x, 0.25, y)") == 0.5) and np.all(ev("warp(x, -0.25, y)") == 0.0)
    # clamping to the axis and NaN -> first point
    assert np.all(ev("warp(add(x, y), 7.0, -7.0)") == 1.0 + -1.0)
    assert np.all(ev("warp(x, pow(-0.5, 0.5), y)") == -1.0)
    # a 1-D domain ignores t1; a 3-D domain keeps the case's own z point
    assert np.array_equal(ev("warp(x, neg(x), 0.0)", (7,)), -ev("x", (7,)))
    z = ev("z", (3, 3, 3))
    assert np.array_equal(ev("warp(z, 1.0, -1.0)", (3, 3, 3)), z)
    assert np.all(ev("warp(add(x, y), 1.0, -1.0)", (3, 3, 3)) == 0.0)
    # a one-point axis always reads its point; t1 = 0 names the middle of axis 1
    assert np.array_equal(ev("warp(y, 0.3, y)", (1, 5)), ev("y", (1, 5)))
    assert np.all(ev("warp(y, 0.3, 0.0)", (1, 5)) == 0.0)


# ----------------------------------------------------------------- fitness
def test_fitness_closed_forms():
    # constant vs constant: RMSE = |c - d|
    v = ev("0.25", G5)[None, :]
    t = np.full((1, 25), -0.5, np.float32)
    assert oracle.fitness(v, t, 1)[0] == 0.75
    assert oracle.fitness(v, t, 1, loss="mse")[0] == 0.5625
    # x against a zero target: sqrt(mean x^2) = sqrt(0.5) on the 5x5 grid
    v = ev("x", G5)[None, :]
    z = np.zeros((1, 25), np.float32)
    assert oracle.fitness(v, z, 1)[0] == math.sqrt(0.5)
    # two channels: N counts both
    v2 = np.stack([ev("x", G5), ev("0.0", G5)])
    z2 = np.zeros((2, 25), np.float32)
    assert oracle.fitness(v2, z2, 1, 2, loss="mse")[0] == 0.25
    # non-finite values make the fitness +inf
    vb = ev("log(x)", G5)[None, :]
    assert oracle.fitness(vb, z, 1)[0] == math.inf
    vn = ev("pow(x, 0.5)", G5)[None, :]
    assert oracle.fitness(vn, z, 1)[0] == math.inf


def test_fitness_matches_numpy_sum():
    pop, dom, spec = pg.workload_c1()
    v = oracle.evaluate(pop.tokens, pop.offsets, dom.shape)
    _, T = pg.pick_target(spec, oracle.target_renderer(dom.shape))
    f = oracle.fitness(v, T, pop.n_individuals)
    with np.errstate(all="ignore"):
        want = np.sqrt(np.mean((v - T.astype(float)) ** 2, axis=1))
    want = np.where(np.isfinite(want), want, np.inf)
    np.testing.assert_allclose(f, want, rtol=1e-13)


# ------------------------------------------------------ stability classification
def test_stability_flags():
    v, v32, st = ev("sub(x, x)", (8, 8), variants=True)
    assert np.all(st == oracle.STABLE)
    v, v32, st = ev("div(1.0, sub(x, x))", (8, 8), variants=True)
    assert np.all(st == oracle.STABLE) and np.all(v == 0)
    # exp overflow: finite in FP64, +inf in every FP32 variant
    v, v32, st = ev("exp(88.75)", (1,), variants=True)
    assert np.isfinite(v[0]) and v32[0] == np.inf and st[0] == oracle.NONFINITE_STABLE
    # 3 * fl32(-1/3) rounds to -1 in FP32 but lies below -1 in FP64: frac flips
    v, v32, st = ev("frac(mult(x, 3.0))", (4,), variants=True)
    assert st[1] == 0 and v[1] > 0.99 and v32[1] == 0.0
    # the smooth Pagie tree is stable everywhere except where pow hits 0^-4
    v, v32, st = ev("add(div(1.0, add(1.0, pow(x, -4.0))), div(1.0, add(1.0, pow(y, -4.0))))",
                    (64, 64), variants=True)
    assert (st & oracle.STABLE).mean() == 1.0


def test_o32r_rounds_every_operator():
    # 0.1f + 0.2f in FP64 is not an FP32 value; O32r rounds it
    v, v32, st = ev("add(0.1, 0.2)", (1,), variants=True)
    assert v32[0] == float(np.float32(v[0])) and v32[0] != v[0]


# ------------------------------------------------------------------ DAG
def _subtree_strings(tree):
    sizes = pg.subtree_sizes(tree)
    out = set()
    for i in range(len(tree)):
        out.add(pg.to_text(tree[i - sizes[i] + 1:i + 1]))
    return out


def test_dag_counts_match_canonical_strings():
    pop, _, _ = pg.workload_c2(side=8)
    d = oracle.build_dag(pop.tokens, pop.offsets)
    strings = set()
    for t in pop.trees():
        strings |= _subtree_strings(t)
    assert d["dag_nodes"] == len(strings)
    assert d["tree_nodes"] == len(pop.tokens)
    assert d["multiplicity"].sum() == len(pop.tokens)
    # every child id is smaller than its parent's (topological first-occurrence order)
    ch = d["children"]
    ids = np.arange(d["dag_nodes"])[:, None]
    assert np.all((ch < ids) | (ch == -1))


def test_dag_small_exact():
    texts = ["add(x, y)", "mult(add(x, y), add(x, y))", "add(x, y)", "sub(x, 0.5)", "sub(x, -0.0)",
             "sub(x, 0.0)"]
    pop = pg.population_from_texts(texts)
    d = oracle.build_dag(pop.tokens, pop.offsets)
    # ids: x=0, y=1, add=2, mult=3, 0.5=4, sub(x,0.5)=5, -0=6, sub(x,-0)=7, +0=8, sub(x,0)=9
    assert d["dag_nodes"] == 10
    assert d["roots"].tolist() == [2, 3, 2, 5, 7, 9]
    assert d["multiplicity"].tolist() == [7, 4, 4, 1, 1, 1, 1, 1, 1, 1]
    assert d["indegree"].tolist() == [4, 1, 2, 0, 1, 0, 1, 0, 1, 0]
    assert d["children"][3].tolist() == [2, 2, -1]
    assert d["dag_internal"] == 5 and d["shared_internal"] == 1
    assert d["max_stack"] == 3


def test_dag_invariants():
    pop, _, _ = pg.workload_c1()
    d = oracle.build_dag(pop.tokens, pop.offsets)
    twice = pg.Population.from_trees(pop.trees() + pop.trees())
    d2 = oracle.build_dag(twice.tokens, twice.offsets)
    assert d2["tree_nodes"] == 2 * d["tree_nodes"]
    assert d2["dag_nodes"] == d["dag_nodes"]
    assert np.array_equal(d2["roots"][:50], d2["roots"][50:])
    rev = pg.Population.from_trees(pop.trees()[::-1])
    d3 = oracle.build_dag(rev.tokens, rev.offsets)
    for k in ("dag_nodes", "dag_internal", "shared_internal", "tree_nodes"):
        assert d3[k] == d[k]


def test_dag_commutative_identity():
    """Hash-consing up to the operand order of commuting operators: add, mult
    and min pairs merge, sub and pow pairs do not; a merged node keeps the
    child order of its first occurrence."""
    texts = ["add(x, y)", "add(y, x)", "sub(x, y)", "sub(y, x)", "min(x, y)", "min(y, x)",
             "mult(add(x, y), 2.0)", "mult(2.0, add(y, x))", "pow(x, y)", "pow(y, x)"]
    pop = pg.population_from_texts(texts)
    s = oracle.build_dag(pop.tokens, pop.offsets)
    c = oracle.build_dag(pop.tokens, pop.offsets, commutative=True)
    assert s["dag_nodes"] == 3 + 10 and c["dag_nodes"] == 3 + 1 + 2 + 1 + 1 + 2
    r = c["roots"].tolist()
    assert r[0] == r[1] and r[2] != r[3] and r[4] == r[5] and r[6] == r[7] and r[8] != r[9]
    assert c["children"][r[0]][:2].tolist() == [0, 1]          # add(x, y) as first met
    assert c["children"][r[6]][:2].tolist() == [r[0], c["children"][r[6]][1]]
    assert c["node_value"][c["children"][r[6]][1]] == 2.0
    # same trees in every order: the commutative DAG is never larger
    pop2, _, _ = pg.workload_c2(side=8)
    a = oracle.build_dag(pop2.tokens, pop2.offsets)
    b = oracle.build_dag(pop2.tokens, pop2.offsets, commutative=True)
    assert b["dag_nodes"] <= a["dag_nodes"] and b["tree_nodes"] == a["tree_nodes"]
    assert b["multiplicity"].sum() == len(pop2.tokens)


def test_commutative_set_is_exactly_the_bitwise_commuting_operators():
    """Every operator in the hashing identity's set gives the same bits (NaN
    positions aside) for both operand orders over operands that take signed
    zeros, infinities, NaN, subnormals and large values; every other binary
    operator differs in some case, so it cannot be in the set."""
    from oracle.dag import COMMUTATIVE
    subs = ["x", "y", "mult(x, 0.0)", "mult(y, 0.0)", "pow(x, 0.5)", "exp(mult(y, 1000.0))",
            "neg(exp(mult(x, 1000.0)))", "mult(x, 1e-40)", "mult(y, 3e38)", "add(x, 0.25)"]
    binary = [o for o in range(len(pg.OP_NAME)) if pg.ARITY[o] == 2 and pg.OP_NAME[o] != "warp"]
    for o in binary:
        name = pg.OP_NAME[o]
        texts = [f"{name}({a}, {b})" for a in subs for b in subs] + [f"{name}({b}, {a})" for a in subs
                                                                     for b in subs]
        pop = pg.population_from_texts(texts)
        v = oracle.evaluate(pop.tokens, pop.offsets, (9, 7))
        n = len(texts) // 2
        a, b = v[:n], v[n:]
        same = np.array_equal(np.isnan(a), np.isnan(b)) and np.array_equal(
            a[~np.isnan(a)].view(np.uint64), b[~np.isnan(b)].view(np.uint64))
        assert same == (o in COMMUTATIVE), name


def test_c2_sharing_in_range():
    pop, _, _ = pg.workload_c2(side=8)
    d = oracle.build_dag(pop.tokens, pop.offsets)
    share = 1 - d["dag_internal"] / d["tree_internal"]
    assert 0.30 <= share <= 0.60
    assert max(pg.tree_depth(t) for t in pop.trees()) <= 10
