"""Seeded populations full of the identity-rewrite patterns (tgp_ctx_set_rewrite):
random subtrees wrapped, and wrapped again, in neg(neg(.)), abs(abs(.)),
min(s, s), if(c, s, s), sub(s, +0), add(-0, s), mult(s, 1), div(s, 1) and the
like, among patterns that look alike but must stay (sub(s, -0), add(s, +0),
min(s, t) with s != t, mult(s, -1)).  Text generation only: no arithmetic of
the method lives here."""
import numpy as np

from paper_2103_07512_amd import popgen as pg

# (template, rewrites?) -- "{s}", "{t}" are subtrees, "{c}" a condition
WRAPS = [
    ("neg(neg({s}))", True), ("abs(abs({s}))", True), ("sign(sign({s}))", True), ("step(step({s}))", True),
    ("min({s}, {s})", True), ("max({s}, {s})", True), ("if({c}, {s}, {s})", True),
    ("sub({s}, 0.0)", True), ("add({s}, -0.0)", True), ("add(-0.0, {s})", True),
    ("mult({s}, 1.0)", True), ("mult(1.0, {s})", True), ("div({s}, 1.0)", True),
    ("neg({s})", False), ("abs(neg({s}))", False), ("sub({s}, -0.0)", False), ("add({s}, 0.0)", False),
    ("min({s}, {t})", False), ("mult({s}, -1.0)", False), ("div(1.0, {s})", False), ("if({c}, {s}, {t})", False),
]


def rewrite_texts(seed: int, n: int, depth: int = 5, funcs=pg.F18, nvars: int = 2):
    """n tree texts: random subtrees wrapped one to three times."""
    rng = np.random.default_rng(seed)
    base = pg.ramped_half_and_half(3 * n, 1, depth, seed, funcs, nvars)
    subs = [pg.to_text(base.tree(i)) for i in range(3 * n)]
    out = []
    for i in range(n):
        s = subs[i]
        for _ in range(int(rng.integers(1, 4))):
            tpl = WRAPS[int(rng.integers(len(WRAPS)))][0]
            s = tpl.format(s=s, t=subs[n + i], c=subs[2 * n + i])
        out.append(s)
    return out
