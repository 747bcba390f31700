"""Pins of the oracle's stability classifier: the first-order error bound E of
every case and the flags (stable, envelope, non-finite stable) that decide
which cases the parity tests compare and how tightly.

The classifier (oracle.c, evb) propagates E analytically: each operator adds
|partial derivative| x operand bound for every operand plus the rounding an
FP32 implementation may add (Wilkinson's first-order forward analysis).  The
checks here derive the same quantities another way, with no derivative
written down: a numpy evaluator perturbs the result of every operator
occurrence by s_i u_i max(|v_i|, 2^-126) (v_i its FP64 value, s_i = +-1, u_i the
operator's assumed accuracy: 2^-23 for a correctly rounded operator, 2^-21
for a library function, 0 for an exact one) and enumerates all 2^n sign
patterns.  To first order the largest deviation of the root from O64 over
the patterns IS the bound, so

  * E must equal that largest deviation (up to second-order terms) on every
    case in the linear regime: a dropped or wrong derivative makes E too
    small, a wrong accuracy constant makes it too large;
  * the flags must equal those recomputed from the perturbation bounds with
    the documented rules: an operand of a discontinuous operator must lie
    more than 4 of its bounds from the discontinuity (or exactly on it with
    a zero bound), O32r must take O64's branch, a stable case has
    E <= 5e-6 max(|O64|, 1) and |O32r - O64| within the same, an envelope
    case is clear but has E above that and at most max(|O64|, 1) / 16.

Exactness, as in the reading the oracle implements: a correctly rounded
operator whose operands are exact adds nothing when its FP64 result is an
FP32 value, and sin(pi a) / cos(pi a) of an exact multiple of 1/2 are exact.
"""
import numpy as np
import pytest

import oracle
from paper_2103_07512_amd import popgen as pg

U_CR = 2.0 ** -23
U_LIB = 2.0 ** -21
MARGIN = 4.0
LINEAR = 0.0625
FLT_OVERFLOW = (2.0 - 2.0 ** -24) * 2.0 ** 127   # FLT_MAX plus half an ulp
STABLE_LIMIT = 5e-6
ENVELOPE_LIMIT = 1.0 / 16.0

CORRECTLY_ROUNDED = {"add", "sub", "mult", "div", "sqrt", "mdist", "frac", "mod"}
LIBRARY = {"sin", "cos", "tan", "exp", "log", "pow", "sstep", "sstepp", "len", "lerp"}
EXACT = {"min", "max", "neg", "abs", "clip", "if", "sign", "step"}
NAME = dict(enumerate(pg.OP_NAME))
ARITY = dict(pg.OPS)


def _quarter(a):
    """a = n/2 + t with n an integer and |t| <= 1/4 (exact in FP64)."""
    a = np.asarray(a, float)
    fin = np.isfinite(a)
    n = np.rint(2 * np.where(fin, a, 0.0))
    t = np.where(fin, a, 0.0) - 0.5 * n
    return fin, np.mod(n, 4), np.sin(np.pi * t), np.cos(np.pi * t)


def _sinpi(a):
    fin, q, s, c = _quarter(a)
    r = np.choose(q.astype(int), [s, c, -s, -c]) + 0.0
    return np.where(fin, r, np.nan)


def _cospi(a):
    fin, q, s, c = _quarter(a)
    r = np.choose(q.astype(int), [c, -s, -c, s]) + 0.0
    return np.where(fin, r, np.nan)


def _min_num(a, b):
    """minNum with -0 ordered below +0."""
    z = (a == 0) & (b == 0)
    return np.where(z, np.where(np.signbit(a), a, b), np.fmin(a, b))


def _max_num(a, b):
    """maxNum with +0 ordered above -0."""
    z = (a == 0) & (b == 0)
    return np.where(z, np.where(np.signbit(a), b, a), np.fmax(a, b))


def _value(name, a, b=None, c=None):
    """FP64 value of one operator (the readings of Table 1)."""
    if name == "add":
        return a + b
    if name == "sub":
        return a - b
    if name == "mult":
        return a * b
    if name == "div":
        return np.where(b == 0, 0.0, a / np.where(b == 0, 1.0, b))
    if name == "sin":
        return _sinpi(a)
    if name == "cos":
        return _cospi(a)
    if name == "tan":
        return _sinpi(a) / _cospi(a)
    if name == "exp":
        return np.exp(a)
    if name == "log":
        return np.where(a < 0, -1.0, np.log(np.where(a < 0, 1.0, a)))
    if name == "pow":
        return np.where((a == 0) & (b == 0), 0.0, np.power(a, b))
    if name == "min":
        return _min_num(a, b)
    if name == "max":
        return _max_num(a, b)
    if name == "mdist":
        return (a + b) / 2
    if name == "neg":
        return -a
    if name == "sqrt":
        return np.where(a < 0, 0.0, np.sqrt(np.where(a < 0, 0.0, a)))
    if name == "sign":
        return np.where(np.isnan(a), 0.0, np.sign(a))
    if name == "abs":
        return np.abs(a)
    if name == "clip":
        return _max_num(_min_num(a, c), b)
    if name == "mod":
        return np.where(b == 0, 0.0, np.mod(a, np.where(b == 0, 1.0, b)))
    if name == "frac":
        return a - np.floor(a)
    if name == "if":
        return np.where(a != 0, b, c)
    if name == "step":
        return np.where(a < 0, -1.0, 1.0)
    if name == "sstep":
        return a * a * (3 - 2 * a)
    if name == "sstepp":
        return a ** 3 * (a * (6 * a - 15) + 10)
    if name == "len":
        return np.where(np.isnan(a) | np.isnan(b), np.nan, np.hypot(a, b))
    if name == "lerp":
        return a + (b - a) * (c - np.floor(c))
    raise KeyError(name)


def _dist_int(x):
    return np.abs(x - np.rint(x))


def _clear(x, p, e):
    """x more than MARGIN bounds from p, or exactly on it with a zero bound."""
    return (e == 0) | (np.abs(x - p) > MARGIN * e)


def _branch(name, a, b, c):
    """Which side of its discontinuities an operator's operands are on."""
    if name == "div":
        return (b == 0).astype(float)
    if name in ("log", "sign"):
        return np.select([np.isnan(a), a < 0, a == 0], [3.0, 0.0, 1.0], 2.0)
    if name == "pow":
        integral = np.isfinite(b) & (np.floor(b) == b)
        zs = np.where(np.signbit(a), 10.0, 0.0)
        return np.select([np.isnan(a) | np.isnan(b), (a == 0) & (b == 0), (a == 0) & (b > 0), a == 0,
                          np.isinf(b) & (np.abs(a) < 1), np.isinf(b) & (np.abs(a) == 1), np.isinf(b),
                          (a < 0) & integral, a < 0],
                         [5.0, 0.0, 1.0 + zs, 6.0 + zs, 7.0, 8.0, 9.0, 2.0, 3.0], 4.0)
    if name == "mult":
        fin = np.where(np.isinf(a), b, a)
        return np.where(np.isinf(a) != np.isinf(b), np.sign(fin), 0.0)
    if name in ("sqrt", "step"):
        return (a < 0).astype(float)
    if name == "if":
        return (a != 0).astype(float)
    if name == "mod":
        opposite = (a != 0) & ((a < 0) != (b < 0))
        return np.select([(b == 0) | np.isnan(a) | np.isnan(b), np.isinf(b)],
                         [1e308, np.where(opposite, -1.0, 0.0)], np.floor(a / np.where(b == 0, 1.0, b)))
    if name == "frac":
        return np.where(np.isfinite(a), np.floor(a), -1.0)
    if name == "tan":
        return np.where(np.isfinite(a), np.floor(a + 0.5), -1.0)
    if name == "lerp":
        return np.where(np.isfinite(c), np.floor(c), -1.0)
    return np.zeros_like(a)


def _linear_ok(name, v, e, e_node):
    """The first-order regime: the change an operand's bound allows stays
    small on the scale on which the operator bends."""
    a, b = (v + [None])[:2]
    ea, eb = (e + [None])[:2]
    if name in ("sin", "cos", "tan"):
        return ~(np.pi * ea > LINEAR)
    if name == "exp":
        return ~(ea > LINEAR)
    if name == "pow":
        with np.errstate(all="ignore"):
            t = np.where(ea == 0, 0.0, np.abs(b / a) * ea) + np.where((eb == 0) | ~(a > 0), 0.0,
                                                                      np.abs(np.log(np.abs(a))) * eb)
        return ~((a != 0) & np.isfinite(_value("pow", a, b)) & (t > LINEAR))
    if name == "mult":
        return ~(ea * eb > LINEAR * e_node)
    if name == "sstep":
        return ~(ea > LINEAR * LINEAR / (1 + np.abs(a)))
    if name == "sstepp":
        return ~(ea > LINEAR * LINEAR / (1 + a ** 4))
    return np.ones_like(a, dtype=bool)


def _discontinuity_ok(name, v, e):
    """The operand checks of one operator; v, e: operand values and bounds."""
    a, b, c = (v + [None, None])[:3]
    ea, eb, ec = (e + [None, None])[:3]
    true = np.ones_like(a, dtype=bool)
    if name == "div":
        return np.where(b == 0, eb == 0, _clear(b, 0.0, eb))
    if name in ("log", "sqrt", "sign", "step", "if"):
        return _clear(a, 0.0, ea)
    if name == "pow":
        both0 = (a == 0) & (b == 0)
        ok = _clear(a, 0.0, ea) & ~((a < 0) & (eb != 0) & (_dist_int(b) <= MARGIN * eb))
        ok &= ~(a == 0) | _clear(b, 0.0, eb)
        ok &= ~np.isinf(b) | _clear(np.abs(a), 1.0, ea)
        return np.where(both0, (ea == 0) & (eb == 0), ok)
    if name == "mult":
        return (~np.isinf(a) | _clear(b, 0.0, eb)) & (~np.isinf(b) | _clear(a, 0.0, ea))
    if name == "mod":
        bb = np.where((b == 0) | np.isinf(b), 1.0, b)
        q = a / bb
        eq = (ea + np.abs(q) * eb) / np.abs(bb)
        generic = ~((eq != 0) & (_dist_int(q) <= MARGIN * eq))
        inf_b = ~np.isfinite(a) | _clear(a, 0.0, ea)
        return np.select([b == 0, np.isinf(b)], [eb == 0, inf_b], generic)
    if name == "frac":
        return ~((ea != 0) & (_dist_int(a) <= MARGIN * ea))
    if name == "tan":
        return _clear(np.abs(a - np.floor(a)), 0.5, ea)
    if name == "lerp":
        return ~((ec != 0) & (_dist_int(c) <= MARGIN * ec))
    return true


def _protected(name, v):
    """Cases where Table 1's protection returns its constant (exactly)."""
    a = v[0]
    if name == "log" or name == "sqrt":
        return a < 0
    if name == "div" or name == "mod":
        return v[1] == 0
    if name == "pow":
        return (a == 0) & (v[1] == 0)
    return np.zeros_like(a, dtype=bool)


def perturbation_classify(tree, coords):
    """Bound and flags of every case of one tree, by exhaustive perturbation.

    coords: list of per-axis FP64 coordinate arrays (one value per case).
    Returns (v64, bound, stable, envelope, nonfinite_stable) per case.
    """
    n_pert = sum(1 for t in tree if NAME[int(t["op"])] in CORRECTLY_ROUNDED | LIBRARY)
    assert n_pert <= 12, "too many operator occurrences to enumerate"
    P = 1 << n_pert
    signs = np.where((np.arange(P)[:, None] >> np.arange(max(n_pert, 1))[None, :]) & 1, 1.0, -1.0)
    C = len(coords[0])
    stack = []
    k = 0
    with np.errstate(all="ignore"):
        for t in tree:
            name = NAME[int(t["op"])]
            if name == "var":
                x = np.asarray(coords[int(t["var"])], float)
                stack.append(dict(v=x, r=x, pv=np.broadcast_to(x, (P, C)), ex=np.ones(C, bool),
                                  ok=np.ones(C, bool)))
                continue
            if name == "const":
                x = np.full(C, float(t["value"]))
                stack.append(dict(v=x, r=x, pv=np.broadcast_to(x, (P, C)), ex=np.ones(C, bool),
                                  ok=np.ones(C, bool)))
                continue
            ar = ARITY[name]
            ops = stack[-ar:]
            del stack[-ar:]
            v = _value(name, *[o["v"] for o in ops])
            r = _value(name, *[o["r"] for o in ops]).astype(np.float32).astype(float)
            pv = _value(name, *[o["pv"] for o in ops])
            ex = np.logical_and.reduce([o["ex"] for o in ops])
            ebs = [np.nanmax(np.abs(o["pv"] - o["v"][None, :]), axis=0) for o in ops]
            ebs = [np.where(o["ex"], 0.0, e) for o, e in zip(ops, ebs)]
            ok = np.logical_and.reduce([o["ok"] for o in ops])
            ok &= _discontinuity_ok(name, [o["v"] for o in ops], ebs)
            # an operand beyond FP32's range is +-inf in every FP32 evaluation
            for o in ops:
                ok &= ~(np.isfinite(o["v"]) & (np.abs(o["v"]) >= FLT_OVERFLOW))
            b64 = _branch(name, *([o["v"] for o in ops] + [None] * (3 - ar)))
            b32 = _branch(name, *([o["r"] for o in ops] + [None] * (3 - ar)))
            ok &= (b64 == b32) | (np.isnan(b64) & np.isnan(b32))
            if name in CORRECTLY_ROUNDED | LIBRARY:
                u = U_CR if name in CORRECTLY_ROUNDED else U_LIB
                if name in CORRECTLY_ROUNDED:
                    own_exact = ex & (v.astype(np.float32).astype(float) == v)
                elif name in ("sin", "cos"):
                    a = ops[0]["v"]
                    own_exact = ex & (2 * a == np.rint(2 * a))
                else:
                    own_exact = np.zeros(C, bool)
                own_exact = own_exact | _protected(name, [o["v"] for o in ops])
                # a non-finite result is an exact special value (its class is
                # what the parity contract compares)
                # below FP32's normal range one ulp is 2^-149 whatever the size
                delta = np.where(own_exact | ~np.isfinite(v) | (v == 0), 0.0,
                                 u * np.maximum(np.abs(v), 2.0 ** -126))
                pv = pv + signs[:, k:k + 1] * delta[None, :]
                k += 1
            # FP32 overflow: finite below FLT_MAX + half an ulp, inf from there on
            e_node = np.nanmax(np.abs(pv - v[None, :]), axis=0)
            ok &= _linear_ok(name, [o["v"] for o in ops], ebs, np.where(np.isfinite(e_node), e_node, 0.0))
            ok &= ~np.isfinite(v) | _clear(np.abs(v), FLT_OVERFLOW, np.where(np.isfinite(e_node), e_node, 0.0))
            # exact: no rounding pattern moves this node's value
            same = (pv == v[None, :]) | (np.isnan(pv) & np.isnan(v)[None, :])
            ex = np.all(same, axis=0)
            stack.append(dict(v=v, r=r, pv=pv, ex=ex, ok=ok))
        (root,) = stack
        v, r = root["v"], root["r"]
        fin = np.isfinite(v)
        e = np.where(root["ex"], 0.0, np.nanmax(np.abs(root["pv"] - v[None, :]), axis=0))
        e = np.where(fin, e, 0.0)
        sc = np.maximum(np.abs(v), 1.0)
        ok = root["ok"] & np.isfinite(e)
        base = ok & fin & np.isfinite(r)
        stable = base & (e <= STABLE_LIMIT * sc) & (np.abs(r - v) <= STABLE_LIMIT * sc)
        envelope = base & ~stable & (e <= ENVELOPE_LIMIT * sc) & (np.abs(r - v) <= e + STABLE_LIMIT * sc)
    return v, e, stable, envelope


def _random_trees(n, seed, functions, max_depth=3, max_pert=10):
    mk = pg.TreeMaker(pg.Rng(seed), functions, 2)
    out = []
    i = 0
    while len(out) < n:
        t = mk.tree(1 + i % max_depth, bool(i % 3 == 0))
        i += 1
        if sum(1 for x in t if NAME[int(x["op"])] in CORRECTLY_ROUNDED | LIBRARY) <= max_pert:
            out.append(t)
    return out


SMOOTH = ("add", "sub", "mult", "div", "sin", "cos", "exp", "log", "pow", "sqrt", "mdist", "len",
          "sstep", "sstepp", "tan", "min", "max", "abs", "neg", "clip")
ALL = SMOOTH + ("mod", "frac", "if", "sign", "step", "lerp")
GRID = (11, 13)


def _grid_coords(shape, lo=None, hi=None):
    lo = lo or [-1.0] * len(shape)
    hi = hi or [1.0] * len(shape)
    axes = [oracle.coords(n, l, h).astype(float) for n, l, h in zip(shape, lo, hi)]
    mesh = np.meshgrid(*axes, indexing="ij")
    return [m.ravel() for m in mesh]


def _oracle(tree, shape, lo=None, hi=None):
    off = np.array([0, len(tree)], np.int64)
    v64, v32, st, eb = oracle.evaluate(tree, off, shape, lo, hi, bound=True)
    return v64[0], v32[0], st[0], eb[0]


@pytest.mark.parametrize("functions,seed", [(SMOOTH, 101), (ALL, 202)], ids=["smooth", "all"])
def test_bound_equals_worst_perturbation(functions, seed):
    """E is the largest first-order deviation over all rounding patterns."""
    trees = _random_trees(160, seed, functions)
    coords = _grid_coords(GRID)
    compared = loose = 0
    for t in trees:
        v64, v32, st, eb = _oracle(t, GRID)
        v, e, _, _ = perturbation_classify(t, coords)
        np.testing.assert_allclose(v, v64, rtol=1e-12, atol=1e-300, equal_nan=True)
        sc = np.maximum(np.abs(v64), 1.0)
        linear = ((st & (oracle.STABLE | oracle.ENVELOPE)) != 0) & (eb <= 1e-4 * sc)
        # sound: no rounding pattern moves the root further than E (the
        # absolute slack covers second-order terms where a derivative
        # vanishes, e.g. cos at a multiple of pi)
        over = linear & ~(e <= eb * (1 + 2e-3) + 1e-8 * sc)
        assert not over.any(), (pg.to_text(t), np.argwhere(over)[:3].ravel(), eb[over][:3], e[over][:3])
        # tight: some pattern reaches E, except where min or max operands
        # lie within their bounds of each other (E then covers either pick)
        loose += int((linear & ~(e >= eb * (1 - 2e-3) - 1e-8 * sc)).sum())
        compared += int(linear.sum())
    assert compared > 0.5 * len(trees) * len(coords[0])
    assert loose <= 2e-3 * compared, (loose, compared)


def _flags_match(t, shape, lo=None, hi=None, allow=0.0):
    v64, v32, st, eb = _oracle(t, shape, lo, hi)
    v, e, stable, envelope = perturbation_classify(t, _grid_coords(shape, lo, hi))
    mism = (((st & oracle.STABLE) != 0) != stable) | (((st & oracle.ENVELOPE) != 0) != envelope)
    assert mism.mean() <= allow, (pg.to_text(t), np.argwhere(mism)[:5].ravel(), st[mism][:5],
                                  stable[mism][:5], envelope[mism][:5], eb[mism][:5], e[mism][:5])
    return stable, envelope


@pytest.mark.parametrize("seed", [303, 404])
def test_flags_equal_perturbation_classification(seed):
    """Stable and envelope flags recomputed from perturbation bounds agree
    with the oracle's on random trees over every operator with a
    discontinuity (a tie at a threshold is measure-zero: none are allowed
    beyond one case in a thousand)."""
    trees = _random_trees(200, seed, ALL, max_depth=4, max_pert=11)
    n = mism = 0
    lo, hi = [-4.0, -4.0], [4.0, 4.0]
    coords = _grid_coords(GRID, lo, hi)
    kinds = np.zeros(3, int)
    for t in trees:
        v64, v32, st, eb = _oracle(t, GRID, lo, hi)
        v, e, stable, envelope = perturbation_classify(t, coords)
        m = (((st & oracle.STABLE) != 0) != stable) | (((st & oracle.ENVELOPE) != 0) != envelope)
        mism += int(m.sum())
        n += m.size
        kinds += [int(stable.sum()), int(envelope.sum()), int((~stable & ~envelope).sum())]
    assert mism <= 1e-3 * n, (mism, n)
    # the random set exercises every class
    assert kinds.min() > 0.005 * n, kinds


def test_margin_of_four_bounds():
    """sqrt(a) with a = (x + 0.75) - 0.75: a equals x in FP64 but carries the
    rounding bound of both operators; along x in [1e-8, 5e-6] the distance of
    a from sqrt's discontinuity runs from under 1 to over 50 of its bounds.
    Cases are clear exactly where x > 4 bounds, with no case in doubt."""
    t = pg.parse("sqrt(sub(add(x, 0.75), 0.75))")
    shape, lo, hi = (997,), [1e-8], [5e-6]
    stable, envelope = _flags_match(t, shape, lo, hi)
    x = oracle.coords(997, 1e-8, 5e-6).astype(float)
    ea = np.array([U_CR * abs(xi + 0.75) if np.float32(xi + 0.75) != xi + 0.75 else 0.0 for xi in x])
    ea += np.where(np.float32(x) == x, 0.0, U_CR * np.abs(x))
    ratio = x / np.where(ea > 0, ea, np.inf)
    clear = stable | envelope
    assert ratio.min() < 2 and ratio.max() > 50
    assert np.all(clear[ratio > 4.05]) and not np.any(clear[(ratio < 3.95) & (ea > 0)])


def test_stable_limit():
    """1 / ((x + 0.3) - x) for x up to 100: the relative bound of the divisor
    grows with x, so the cases turn from stable to envelope where E crosses
    5e-6 max(|v|, 1) and leave the envelope where E passes max(|v|, 1) / 16."""
    t = pg.parse("div(1.0, sub(add(x, 0.3), x))")
    stable, envelope = _flags_match(t, (1001,), [0.0], [100.0])
    assert stable[:50].all() and envelope[-300:].all()
    # at the envelope's limit the second-order terms are a few percent of E,
    # so the two derivations may split a few cases there
    stable2, envelope2 = _flags_match(t, (1001,), [0.0], [3e6], allow=0.01)
    assert envelope2[1:10].all() and (~stable2 & ~envelope2)[-100:].all()
    assert (~stable2 & ~envelope2)[-100:].all()


def test_exactness_rules():
    """Correctly rounded operators on exact operands with representable
    results add nothing; sin and cos are exact at multiples of 1/2."""
    for text, shape in [("frac(mult(x, 2.0))", (5,)), ("sign(sub(x, y))", (5, 5)),
                        ("div(x, sin(cos(sub(x, x))))", (7,)), ("mod(add(x, 0.5), 0.25)", (9,))]:
        v64, v32, st, eb = _oracle(pg.parse(text), shape)
        assert np.all(eb == 0) and np.all((st & oracle.STABLE) != 0), text


def test_nonfinite_stable_class():
    """exp overflows FP32 but not FP64: O32r is +inf, the case is required to
    be +inf; exp of a bound-carrying argument near the overflow edge is not."""
    v64, v32, st, eb = _oracle(pg.parse("exp(88.75)"), (1,))
    assert st[0] == oracle.NONFINITE_STABLE
    v64, v32, st, eb = _oracle(pg.parse("exp(mult(add(x, 88.72283935546875), 1.0))"), (3,),
                               [0.0], [1e-6])
    assert np.all((st & oracle.NONFINITE_STABLE) == 0) or np.all(v32 == np.inf)


@pytest.mark.parametrize("text,lo,hi,why", [
    # a result below FP32's normal range: spacing 2^-149, not a relative ulp
    ("sign(exp(mult(x, 110.0)))", -0.96, -0.9, "subnormal"),
    # 0^b is 0 for b > 0 and +inf for b < 0: the sign of a bound-carrying b decides
    ("pow(0.0, sub(add(x, 0.3), 0.3))", -1e-6, 1e-6, "zero base"),
    # sin of an argument whose bound spans a good part of a period
    ("sin(div(1.0, sub(add(x, 0.5), 0.5)))", 1e-4, 1e-2, "phase"),
    # exp near FP32's overflow threshold: finite or inf is undecided
    ("exp(add(x, 88.72283935546875))", -1e-4, -5e-6, "overflow edge"),
    # a finite FP64 operand beyond FP32's range: inf * 0 is NaN in FP32
    ("max(mult(exp(mult(x, 100.0)), sub(x, x)), -0.5)", 0.8, 0.95, "operand overflow"),
])
def test_guards(text, lo, hi, why):
    """Each guard of the first-order analysis decides some cases of a domain
    that sweeps across its threshold; the oracle's flags there equal the
    independent classification."""
    t = pg.parse(text)
    stable, envelope = _flags_match(t, (1001,), [lo], [hi], allow=0.003)
    checked = stable | envelope
    assert 0.02 < checked.mean() < 0.98 or why in ("subnormal", "overflow edge"), (why, checked.mean())
    if why == "operand overflow":
        x = oracle.coords(1001, lo, hi).astype(float)
        assert not checked[100 * x > 88.73].any() and checked[100 * x < 88.7].all()
