"""Pins of the oracle's genetic operators (oracle/breed.py) against what their
definitions fix: the generator's published outputs, a hand-derived worked
example, tree shapes by hand, brute-force enumeration of every valid
crossover and mutation outcome on tiny populations, the selection law of a
tournament, the depth limit and the independence of offspring streams."""
import math
import os

import numpy as np
import pytest

from oracle import breed as ob
from paper_2103_07512_amd import popgen as pg

GOLD = os.path.join(os.path.dirname(__file__), "golden")
F = [pg.OP_CODE[f] for f in pg.F18]


def test_splitmix64_known_answers():
    seen = 0
    with open(os.path.join(GOLD, "rng_splitmix64.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            head, vals = line.split(":")
            seed = int(head.split()[1])
            for n, v in enumerate(vals.split(), start=1):
                assert ob.splitmix64_output(seed, n) == int(v, 16)
                seen += 1
    assert seen == 9


def test_stream_draw_numbering():
    # offspring o, draw k is generator output o * 2^32 + k + 1
    st = ob.Stream(0, 0)
    assert [st.next() for _ in range(4)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                              0x06C45D188009454F, 0xF88BB8A8724C81EC]
    st = ob.Stream(1234567, 3)
    st.k = 7
    assert st.next() == ob.splitmix64_output(1234567, (3 << 32) + 8)


def test_draw_conversions():
    st = ob.Stream(0, 0)
    # below(m) is the top bits of the draw: 0xe2... / 2^64 * 4 = 3.53 -> 3
    assert st.below(4) == 3
    # uniform: 53 top bits; 0x6e789e6aa1b965f4 / 2^64 = 0.4315...
    assert st.uniform() == (0x6E789E6AA1B965F4 >> 11) / 2.0 ** 53
    # constant: 24 top bits u -> 2u - 1; 0x06c45d -> 2 * 0x06c45d / 2^24 - 1
    assert st.constant() == 2.0 * 0x06C45D / 2.0 ** 24 - 1.0


def test_worked_example_reproduction():
    """Seed 0, offspring 0, four parents of fitness (5, 1, 7, 3), tournament 3,
    p_crossover 0.8, p_mutation 0.05.  By hand from the generator's published
    outputs: u = 0xe220a839.../2^64 = 0.883 >= 0.85, so reproduction; the
    tournament draws below(4) = top two bits of 0x6e78..., 0x06c4..., 0xf88b...
    = 1, 0, 3 and keeps parent 1 (fitness 1); so offspring 0 is parent 1."""
    trees = [pg.parse(t) for t in ("x", "add(x, y)", "mult(y, 2.0)", "sin(x)")]
    pop = pg.Population.from_trees(trees, 1)
    toks, offs = ob.breed(pop.tokens, pop.offsets, 1, [5.0, 1.0, 7.0, 3.0], seed=0, n_offspring=1,
                          tournament=3, p_crossover=0.8, p_mutation=0.05, functions=F)
    assert list(offs) == [0, 3]
    assert np.array_equal(toks, trees[1])


def test_shape_by_hand():
    # add(x, mult(y, 2.0)) in postfix: x y 2.0 mult add
    t = pg.parse("add(x, mult(y, 2.0))")
    size, depth, height = ob.shape([int(o) for o in t["op"]])
    assert size == [1, 1, 1, 3, 5]
    assert depth == [1, 2, 2, 1, 0]
    assert height == [0, 0, 0, 1, 2]
    # if(x, neg(y), lerp(x, y, 0.5)): x y neg x y 0.5 lerp if
    t = pg.parse("if(x, neg(y), lerp(x, y, 0.5))")
    size, depth, height = ob.shape([int(o) for o in t["op"]])
    assert size == [1, 1, 2, 1, 1, 1, 4, 8]
    assert depth == [1, 2, 1, 2, 2, 2, 1, 0]
    assert height == [0, 0, 1, 0, 0, 0, 1, 2]
    with pytest.raises(ValueError):
        ob.shape([0, 0])


def _valid_tree(t):
    try:
        ob.shape([int(o) for o in t["op"]])
    except (ValueError, IndexError):
        return False
    return True


def _tiny_pop(seed, n=4, n_ch=2, d=2):
    return pg.ramped_half_and_half(n, 1, d, seed, pg.F18, 2, n_ch)


def _subtrees(t):
    size, _, _ = ob.shape([int(o) for o in t["op"]])
    return [(i, int(size[i])) for i in range(len(t))]


def test_crossover_outcomes_by_enumeration():
    """Every crossover child is, for one pair of parents shared by all channels
    of the offspring, a with one subtree replaced by one subtree of b (or a
    copy of a), within the depth limit."""
    for seed in (1, 2, 3):
        pop = _tiny_pop(seed)
        trees = pop.trees()
        n, nch = pop.n_individuals, pop.n_channels
        toks, offs = ob.breed(pop.tokens, pop.offsets, nch, None, seed=seed, n_offspring=12,
                              p_crossover=1.0, p_mutation=0.0, max_depth=4, functions=F)
        for o in range(12):
            kids = [toks[offs[o * nch + c]:offs[o * nch + c + 1]] for c in range(nch)]
            ok_pairs = []
            for p1 in range(n):
                for p2 in range(n):
                    good = True
                    for c in range(nch):
                        a, b = trees[p1 * nch + c], trees[p2 * nch + c]
                        cands = [a] + [np.concatenate([a[:i - sa + 1], b[j - sb + 1:j + 1], a[i + 1:]])
                                       for i, sa in _subtrees(a) for j, sb in _subtrees(b)]
                        if not any(len(k) == len(kids[c]) and np.array_equal(k, kids[c]) for k in cands):
                            good = False
                            break
                    if good:
                        ok_pairs.append((p1, p2))
            assert ok_pairs, (seed, o)
            for k in kids:
                assert _valid_tree(k) and pg.tree_depth(k) <= 4


def test_mutation_outcomes_by_enumeration():
    """Every mutation child is a parent tree with one subtree replaced by a
    valid tree of the function and terminal sets no deeper than the room left
    (and no deeper than max_mutation_depth)."""
    allowed = set(F) | {0, 1}
    for seed in (4, 5):
        pop = _tiny_pop(seed, n=3, n_ch=1, d=3)
        trees = pop.trees()
        toks, offs = ob.breed(pop.tokens, pop.offsets, 1, None, seed=seed, n_offspring=20,
                              p_crossover=0.0, p_mutation=1.0, max_depth=5, max_mutation_depth=2,
                              functions=F)
        for o in range(20):
            kid = toks[offs[o]:offs[o + 1]]
            assert set(int(x) for x in kid["op"]) <= allowed
            assert all(int(v) < 2 for v, op in zip(kid["var"], kid["op"]) if op == 0)
            found = False
            for a in trees:
                _, depth_a, _ = ob.shape([int(x) for x in a["op"]])
                for i, sa in _subtrees(a):
                    lo = i - sa + 1
                    tail = len(a) - i - 1
                    if len(kid) < lo + tail + 1:
                        continue
                    if not (np.array_equal(kid[:lo], a[:lo]) and np.array_equal(kid[len(kid) - tail:], a[i + 1:])):
                        continue
                    mid = kid[lo:len(kid) - tail]
                    if _valid_tree(mid) and pg.tree_depth(mid) <= min(5 - depth_a[i], 2):
                        found = True
                        break
                if found:
                    break
            assert found, (seed, o)


def test_reproduction_copies_whole_individuals():
    pop = _tiny_pop(6, n=5, n_ch=3)
    trees = pop.trees()
    toks, offs = ob.breed(pop.tokens, pop.offsets, 3, np.arange(5.0), seed=9, n_offspring=30,
                          p_crossover=0.0, p_mutation=0.0, functions=F)
    for o in range(30):
        kids = [toks[offs[o * 3 + c]:offs[o * 3 + c + 1]] for c in range(3)]
        assert any(all(np.array_equal(kids[c], trees[p * 3 + c]) for c in range(3)) for p in range(5))


def test_tournament_selection_law():
    """With distinct fitness, a size-t tournament with replacement picks the
    individual of rank r (0 = best) with probability ((n-r)/n)^t -
    ((n-r-1)/n)^t; checked on 6000 reproductions of 6 individuals whose trees
    are told apart by a constant."""
    n, t, m = 6, 3, 6000
    trees = [pg.parse(f"{float(k) + 0.5}") for k in range(n)]
    pop = pg.Population.from_trees(trees, 1)
    fit = np.array([3.0, 0.5, 2.0, 5.0, 1.0, 4.0])
    rank_of = {int(i): r for r, i in enumerate(np.argsort(fit))}
    toks, _ = ob.breed(pop.tokens, pop.offsets, 1, fit, seed=77, n_offspring=m, tournament=t,
                       p_crossover=0.0, p_mutation=0.0, functions=F)
    counts = np.zeros(n)
    for v in toks["value"]:
        counts[rank_of[int(v - 0.5)]] += 1
    for r in range(n):
        p = ((n - r) / n) ** t - ((n - r - 1) / n) ** t
        sd = math.sqrt(m * p * (1 - p))
        assert abs(counts[r] - m * p) < 5 * sd + 1, (r, counts, p)
    # a NaN or infinite fitness counts as +inf: such an individual wins only
    # when every draw of the tournament is one (probability (1/2)^6 here)
    fit2 = np.array([np.nan, np.inf, 1.0, 2.0, np.nan, 3.0])
    m2 = 4000
    toks, _ = ob.breed(pop.tokens, pop.offsets, 1, fit2, seed=5, n_offspring=m2, tournament=6,
                       p_crossover=0.0, p_mutation=0.0, functions=F)
    bad = sum(int(v - 0.5) in (0, 1, 4) for v in toks["value"])
    p = 0.5 ** 6
    assert abs(bad - m2 * p) < 5 * math.sqrt(m2 * p * (1 - p)) + 1, bad


def test_operator_rates():
    """The share of exact parent copies is the reproduction probability when
    crossover and mutation always change the tree (distinct constants per
    parent, points and new subtrees that never reproduce the old tree are
    overwhelmingly likely; allowed 5 standard deviations plus the rare ties)."""
    n = 40
    trees = [pg.parse(f"add(mult(x, {k + 0.25}), sub(y, {k + 0.75}))") for k in range(n)]
    pop = pg.Population.from_trees(trees, 1)
    m = 3000
    toks, offs = ob.breed(pop.tokens, pop.offsets, 1, None, seed=3, n_offspring=m, tournament=1,
                          p_crossover=0.5, p_mutation=0.3, max_depth=8, functions=F)
    copies = 0
    for o in range(m):
        kid = toks[offs[o]:offs[o + 1]]
        copies += any(len(kid) == len(t) and np.array_equal(kid, t) for t in trees)
    p = 0.2
    sd = math.sqrt(m * p * (1 - p))
    # crossover at the roots of two copies of the same tree, or a swap of
    # identical leaves (x for x), gives a copy too: at most a few per cent
    assert m * p - 5 * sd < copies < m * (p + 0.08) + 5 * sd, copies


def test_depth_limit_and_prefix_independence():
    pop = pg.ramped_half_and_half(30, 2, 6, 12, pg.F18, 2, 2)
    fit = np.linspace(1.0, 2.0, 30)
    kw = dict(tournament=3, p_crossover=0.7, p_mutation=0.2, max_depth=6, functions=F)
    t1, o1 = ob.breed(pop.tokens, pop.offsets, 2, fit, seed=21, n_offspring=25, **kw)
    t2, o2 = ob.breed(pop.tokens, pop.offsets, 2, fit, seed=21, n_offspring=40, **kw)
    assert np.array_equal(o1, o2[:51]) and np.array_equal(t1, t2[:o1[-1]])
    for r in range(80):
        k = t2[o2[r]:o2[r + 1]]
        assert _valid_tree(k) and pg.tree_depth(k) <= 6
    t3, _ = ob.breed(pop.tokens, pop.offsets, 2, fit, seed=22, n_offspring=25, **kw)
    assert not (len(t3) == len(t1) and np.array_equal(t3, t1))
