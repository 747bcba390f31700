"""Seeded synthetic GP populations: the shared input generator.

This module produces the inputs that both the HIP path and the oracle consume
and holds none of the method's arithmetic: it never evaluates a tree, never
hashes or merges subtrees and never computes a fitness.  It knows only the
token encoding (opcode numbers and arities of the primitive set of the paper's
Table 1), how to draw random trees from it, how to breed new trees by cutting
and splicing token ranges, and how to print and parse the text form.

Token encoding (one 8-byte record per node, trees stored in postfix order,
children before their parent; identical to ``tgp_token`` in include/tgp.h):
    op    uint8   opcode, numbering below
    var   uint8   axis index for VAR (0 = x, 1 = y, 2 = z)
    pad   uint16  zero
    value float32 the constant for CONST, else 0

Tree generation follows the ramped half-and-half method the paper uses for its
populations (Table 2), in the textbook form of Poli, Langdon and McPhee's field
guide cited by the paper: individual i gets depth d_min + (i mod n_depths) and
uses *full* when floor(i / n_depths) is even, *grow* otherwise.  Grow picks
uniformly from functions and terminals below the depth limit (each variable and
the ephemeral constant count as one terminal each) and terminals at the limit.
A terminal-only tree has depth 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------------------
# Token encoding (primitive set of Table 1, pointwise operators only)
# --------------------------------------------------------------------------
OPS = [
    # name     arity
    ("var", 0), ("const", 0),
    ("add", 2), ("sub", 2), ("mult", 2), ("div", 2),
    ("sin", 1), ("cos", 1), ("tan", 1),
    ("exp", 1), ("log", 1), ("pow", 2),
    ("min", 2), ("max", 2), ("mdist", 2), ("neg", 1),
    ("sqrt", 1), ("sign", 1), ("abs", 1), ("clip", 3),
    ("mod", 2), ("frac", 1), ("if", 3),
    ("step", 1), ("sstep", 1), ("sstepp", 1), ("len", 2), ("lerp", 3),
    ("or", 2), ("xor", 2), ("and", 2),      # bitwise (Table 1, Logic), appended
    ("warp", 3),                            # image transform (Table 1), appended
]
OP_CODE = {name: i for i, (name, _) in enumerate(OPS)}
OP_CODE["mul"] = OP_CODE["mult"]           # the configs spell it "mul"
OP_NAME = [name for name, _ in OPS]
ARITY = np.array([a for _, a in OPS], dtype=np.int64)
VAR, CONST = OP_CODE["var"], OP_CODE["const"]
AXIS_NAMES = ("x", "y", "z")

TOKEN_DTYPE = np.dtype([("op", "u1"), ("var", "u1"), ("pad", "<u2"), ("value", "<f4")])

# Function sets named by the workloads.
F6 = ("add", "sub", "mult", "div", "sin", "cos")
F18 = F6 + ("exp", "log", "sqrt", "pow", "abs", "min", "max", "mod", "sign",
            "frac", "clip", "if")

MASK64 = (1 << 64) - 1


# --------------------------------------------------------------------------
# PRNG: SplitMix64 seeding a xoshiro256** generator (Blackman & Vigna)
# --------------------------------------------------------------------------
def _rotl(x: int, k: int) -> int:
    return ((x << k) | (x >> (64 - k))) & MASK64


class Rng:
    """xoshiro256** seeded by SplitMix64; deterministic across platforms."""

    def __init__(self, seed: int):
        s = seed & MASK64
        st = []
        for _ in range(4):
            s = (s + 0x9E3779B97F4A7C15) & MASK64
            z = s
            z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
            z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
            st.append(z ^ (z >> 31))
        self.s = st

    def next_u64(self) -> int:
        s0, s1, s2, s3 = self.s
        result = (_rotl((s1 * 5) & MASK64, 7) * 9) & MASK64
        t = (s1 << 17) & MASK64
        s2 ^= s0
        s3 ^= s1
        s1 ^= s2
        s0 ^= s3
        s2 ^= t
        s3 = _rotl(s3, 45)
        self.s = [s0, s1, s2, s3]
        return result

    def below(self, n: int) -> int:
        """Uniform integer in [0, n) (Lemire's multiply-shift with rejection)."""
        if n <= 0:
            raise ValueError("below(n) needs n > 0")
        thresh = ((1 << 64) - n) % n
        while True:
            r = self.next_u64()
            m = r * n
            if (m & MASK64) >= thresh:
                return m >> 64

    def uniform(self) -> float:
        """Uniform double in [0, 1) with 53 random bits."""
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))

    def const_f32(self) -> float:
        """Ephemeral constant 2u-1, u = 24 random bits * 2^-24: exact in FP32, in [-1, 1)."""
        u = (self.next_u64() >> 40) * (1.0 / (1 << 24))
        return float(np.float32(2.0 * u - 1.0))

    def exponential(self, mean: float) -> float:
        return -mean * math.log(1.0 - self.uniform())


# --------------------------------------------------------------------------
# Population container
# --------------------------------------------------------------------------
@dataclass
class Population:
    """A population of n_individuals x n_channels postfix trees, tree-major.

    Tree r (individual r // n_channels, channel r % n_channels) occupies
    tokens[offsets[r]:offsets[r+1]].
    """
    tokens: np.ndarray                  # TOKEN_DTYPE[T]
    offsets: np.ndarray                 # int64[n_roots + 1]
    n_individuals: int
    n_channels: int = 1
    meta: dict = field(default_factory=dict)

    @property
    def n_roots(self) -> int:
        return self.n_individuals * self.n_channels

    def tree(self, r: int) -> np.ndarray:
        return self.tokens[self.offsets[r]:self.offsets[r + 1]]

    def trees(self) -> list:
        return [self.tree(r) for r in range(self.n_roots)]

    @staticmethod
    def from_trees(trees, n_channels: int = 1, meta=None) -> "Population":
        if len(trees) % n_channels:
            raise ValueError("tree count is not a multiple of n_channels")
        lens = np.array([len(t) for t in trees], dtype=np.int64)
        offsets = np.zeros(len(trees) + 1, dtype=np.int64)
        np.cumsum(lens, out=offsets[1:])
        tokens = (np.concatenate(trees) if trees else np.zeros(0, TOKEN_DTYPE)).astype(TOKEN_DTYPE)
        return Population(tokens, offsets, len(trees) // n_channels, n_channels, dict(meta or {}))


def make_tokens(items) -> np.ndarray:
    """items: iterable of (op, var, value) tuples in postfix order."""
    items = list(items)
    a = np.zeros(len(items), dtype=TOKEN_DTYPE)
    for i, (op, var, val) in enumerate(items):
        a[i] = (op, var, 0, val)
    return a


# --------------------------------------------------------------------------
# Random trees: full / grow / ramped half-and-half
# --------------------------------------------------------------------------
class TreeMaker:
    def __init__(self, rng: Rng, functions=F6, ndim: int = 2, use_const: bool = True):
        self.rng = rng
        self.functions = [OP_CODE[f] for f in functions]
        self.terminals = [("var", k) for k in range(ndim)]
        if use_const:
            self.terminals.append(("const", None))

    def _terminal(self, out):
        kind, k = self.terminals[self.rng.below(len(self.terminals))]
        if kind == "var":
            out.append((VAR, k, 0.0))
        else:
            out.append((CONST, 0, self.rng.const_f32()))

    def _build(self, depth: int, full: bool, out):
        # Pre-order choice, post-order emission (children first).
        if depth == 0:
            self._terminal(out)
            return
        nf, nt = len(self.functions), len(self.terminals)
        if full:
            op = self.functions[self.rng.below(nf)]
        else:
            j = self.rng.below(nf + nt)
            if j >= nf:
                kind, k = self.terminals[j - nf]
                if kind == "var":
                    out.append((VAR, k, 0.0))
                else:
                    out.append((CONST, 0, self.rng.const_f32()))
                return
            op = self.functions[j]
        for _ in range(ARITY[op]):
            self._build(depth - 1, full, out)
        out.append((op, 0, 0.0))

    def tree(self, depth: int, full: bool) -> np.ndarray:
        out = []
        self._build(depth, full, out)
        return make_tokens(out)


def ramped_half_and_half(n: int, d_min: int, d_max: int, seed: int, functions=F6,
                         ndim: int = 2, n_channels: int = 1) -> Population:
    """n individuals (each with n_channels trees) by ramped half-and-half.

    Individual i uses depth d_min + (i mod n_depths) and full when
    floor(i / n_depths) is even; all channels of an individual share the
    depth and method.
    """
    rng = Rng(seed)
    mk = TreeMaker(rng, functions, ndim)
    nd = d_max - d_min + 1
    trees = []
    for i in range(n):
        d = d_min + (i % nd)
        full = (i // nd) % 2 == 0
        for _ in range(n_channels):
            trees.append(mk.tree(d, full))
    return Population.from_trees(trees, n_channels,
                                 dict(kind="rhh", n=n, d_min=d_min, d_max=d_max, seed=seed,
                                      functions=list(functions), ndim=ndim))


def full_tree(depth: int, seed: int, functions=F6, ndim: int = 2) -> np.ndarray:
    return TreeMaker(Rng(seed), functions, ndim).tree(depth, True)


# --------------------------------------------------------------------------
# Tree structure helpers (shape only: sizes and depths of token ranges)
# --------------------------------------------------------------------------
def subtree_sizes(tree: np.ndarray) -> np.ndarray:
    """size[i] = number of tokens of the subtree whose root is token i."""
    ar = ARITY[tree["op"].astype(np.int64)]
    size = np.empty(len(tree), dtype=np.int64)
    stack = []
    for i, a in enumerate(ar):
        s = 1
        for _ in range(a):
            s += stack.pop()
        size[i] = s
        stack.append(s)
    if len(stack) != 1:
        raise ValueError("token range is not exactly one postfix tree")
    return size


def node_depths(tree: np.ndarray):
    """(depth-from-root of each token, height of each token's subtree)."""
    ar = ARITY[tree["op"].astype(np.int64)]
    n = len(tree)
    height = np.zeros(n, dtype=np.int64)
    parent = np.full(n, -1, dtype=np.int64)
    stack = []
    for i, a in enumerate(ar):
        h = 0
        for _ in range(a):
            c = stack.pop()
            parent[c] = i
            h = max(h, height[c] + 1)
        height[i] = h
        stack.append(i)
    depth = np.zeros(n, dtype=np.int64)
    for i in range(n - 2, -1, -1):       # parents come after children
        depth[i] = depth[parent[i]] + 1
    return depth, height


def tree_depth(tree: np.ndarray) -> int:
    return int(node_depths(tree)[1][-1])


# --------------------------------------------------------------------------
# Breeding: tournament selection, subtree crossover and subtree mutation
# --------------------------------------------------------------------------
def _splice(a: np.ndarray, i: int, size_a: int, b_sub: np.ndarray) -> np.ndarray:
    lo = i - size_a + 1
    return np.concatenate([a[:lo], b_sub, a[i + 1:]])


def breed(pop: Population, rng: Rng, functions=F18, ndim: int = 2, max_depth: int = 10,
          fitness=None, p_cross: float = 0.8, p_mut: float = 0.1, tournament: int = 3,
          retries: int = 8) -> Population:
    """One generation of subtree crossover / subtree mutation / reproduction.

    Parents come from a size-`tournament` tournament on `fitness` (lower is
    better, NaN counts as worst) when given, or are drawn uniformly otherwise.
    Offspring deeper than max_depth are rejected and redrawn up to `retries`
    times, after which the first parent is copied.  Every channel tree of an
    offspring is bred from the same channel of its parents.
    """
    nch = pop.n_channels
    n = pop.n_individuals
    fit = None if fitness is None else np.where(np.isfinite(fitness), fitness, np.inf)
    mk = TreeMaker(rng, functions, ndim)
    trees = pop.trees()
    info = {}

    def shape(r):
        if r not in info:
            t = trees[r]
            d, h = node_depths(t)
            info[r] = (subtree_sizes(t), d, h)
        return info[r]

    def select():
        if fit is None:
            return rng.below(n)
        best = rng.below(n)
        for _ in range(tournament - 1):
            c = rng.below(n)
            if fit[c] < fit[best]:
                best = c
        return best

    out = []
    for _ in range(n):
        u = rng.uniform()
        p1 = select()
        if u < p_cross:
            p2 = select()
            kids = []
            for ch in range(nch):
                ra, rb = p1 * nch + ch, p2 * nch + ch
                a, b = trees[ra], trees[rb]
                sa, da, _ = shape(ra)
                sb, _, hb = shape(rb)
                child = a
                for _ in range(retries):
                    i = rng.below(len(a))
                    j = rng.below(len(b))
                    if da[i] + hb[j] <= max_depth:
                        child = _splice(a, i, int(sa[i]), b[j - int(sb[j]) + 1:j + 1])
                        break
                kids.append(child)
            out.extend(kids)
        elif u < p_cross + p_mut:
            for ch in range(nch):
                ra = p1 * nch + ch
                a = trees[ra]
                sa, da, _ = shape(ra)
                child = a
                for _ in range(retries):
                    i = rng.below(len(a))
                    room = max_depth - int(da[i])
                    sub = mk.tree(rng.below(min(room, 4) + 1), rng.below(2) == 0)
                    child = _splice(a, i, int(sa[i]), sub)
                    break
                out.append(child)
        else:
            for ch in range(nch):
                out.append(trees[p1 * nch + ch].copy())
    return Population.from_trees(out, nch, dict(pop.meta))


# --------------------------------------------------------------------------
# Text form: op(a, b) with Table 1 abbreviations, terminals x/y/z and floats
# --------------------------------------------------------------------------
def _fmt_const(v: float) -> str:
    # repr of the double that equals the FP32 value round-trips exactly.
    return repr(float(np.float32(v)))


def to_text(tree: np.ndarray) -> str:
    stack = []
    for t in tree:
        op = int(t["op"])
        if op == VAR:
            stack.append(AXIS_NAMES[int(t["var"])])
        elif op == CONST:
            stack.append(_fmt_const(float(t["value"])))
        else:
            a = ARITY[op]
            args = stack[len(stack) - a:]
            del stack[len(stack) - a:]
            stack.append(f"{OP_NAME[op]}({', '.join(args)})")
    if len(stack) != 1:
        raise ValueError("not a single tree")
    return stack[0]


def parse(text: str) -> np.ndarray:
    """Parse the text form into postfix tokens (the inverse of to_text)."""
    s = text.strip()
    pos = 0
    out = []

    def skip():
        nonlocal pos
        while pos < len(s) and s[pos].isspace():
            pos += 1

    def expr():
        nonlocal pos
        skip()
        start = pos
        while pos < len(s) and (s[pos].isalnum() or s[pos] in "._+-"):
            if s[pos] in "+-" and pos > start and s[pos - 1] not in "eEpP":
                break
            pos += 1
        word = s[start:pos]
        if not word:
            raise ValueError(f"expected a term at {start} in {text!r}")
        skip()
        if pos < len(s) and s[pos] == "(":
            if word not in OP_CODE or OP_CODE[word] in (VAR, CONST):
                raise ValueError(f"unknown operator {word!r}")
            op = OP_CODE[word]
            pos += 1
            n = 0
            while True:
                skip()
                if pos < len(s) and s[pos] == ")":
                    pos += 1
                    break
                if n:
                    if s[pos] != ",":
                        raise ValueError(f"expected ',' at {pos} in {text!r}")
                    pos += 1
                expr()
                n += 1
            if n != ARITY[op]:
                raise ValueError(f"{word} takes {ARITY[op]} arguments, got {n}")
            out.append((op, 0, 0.0))
        elif word in AXIS_NAMES:
            out.append((VAR, AXIS_NAMES.index(word), 0.0))
        else:
            try:
                v = float.fromhex(word) if "0x" in word.lower() else float(word)
            except ValueError:
                raise ValueError(f"bad terminal {word!r}") from None
            out.append((CONST, 0, float(np.float32(v))))

    expr()
    skip()
    if pos != len(s):
        raise ValueError(f"trailing text at {pos} in {text!r}")
    return make_tokens(out)


def population_from_texts(texts, n_channels: int = 1) -> Population:
    return Population.from_trees([parse(t) for t in texts], n_channels)


# --------------------------------------------------------------------------
# Domains (shape only) and the named workloads
# --------------------------------------------------------------------------
@dataclass
class DomainSpec:
    shape: tuple
    lo: tuple = None
    hi: tuple = None

    def __post_init__(self):
        nd = len(self.shape)
        if self.lo is None:
            self.lo = (-1.0,) * nd
        if self.hi is None:
            self.hi = (1.0,) * nd

    @property
    def ndim(self):
        return len(self.shape)

    @property
    def cases(self):
        return int(np.prod(self.shape))


@dataclass
class TargetSpec:
    """A target tensor rendered from seeded full trees, one per channel.

    Channel c first tries seed + c; a tree whose rendering has a non-finite
    value is redrawn with the seed n_channels higher, until one is finite.
    """
    depth: int
    seed: int
    functions: tuple = F18
    ndim: int = 2
    n_channels: int = 1

    def tree(self, channel: int, attempt: int) -> np.ndarray:
        return full_tree(self.depth, self.seed + channel + attempt * self.n_channels,
                         self.functions, self.ndim)


def pick_target(spec: TargetSpec, render, max_attempts: int = 10000):
    """render(tree) -> 1-D float32 values over the domain, or None when any
    value is non-finite.  Returns (trees, float32 [n_channels][cases])."""
    trees, rows = [], []
    for c in range(spec.n_channels):
        for attempt in range(max_attempts):
            t = spec.tree(c, attempt)
            v = render(t)
            if v is not None:
                trees.append(t)
                rows.append(np.asarray(v, dtype=np.float32).reshape(-1))
                break
        else:
            raise RuntimeError("no finite target tree found")
    return trees, np.stack(rows)


def workload_c1(seed: int = 1):
    """50 ramped half-and-half trees, depths 2-6, F6, on a 64x64 grid in [-1, 1]."""
    pop = ramped_half_and_half(50, 2, 6, seed, F6, 2)
    return pop, DomainSpec((64, 64)), TargetSpec(4, seed + 1, F6, 2, 1)


def workload_c3(seed: int = 6, n: int = 1000, side: int = 1024):
    """1000 individuals x 3 channel trees, ramped half-and-half depths 2-12, F18, 1024x1024."""
    pop = ramped_half_and_half(n, 2, 12, seed, F18, 2, n_channels=3)
    return pop, DomainSpec((side, side)), TargetSpec(8, seed + 1, F18, 2, 3)


def workload_c2(seed: int = 3, generations: int = None, n: int = 500, side: int = 256):
    """500 trees bred by neutral subtree crossover/mutation from RHH depths 2-6, F18, depth <= 10."""
    if generations is None:
        generations = C2_GENERATIONS
    pop = ramped_half_and_half(n, 2, 6, seed, F18, 2)
    rng = Rng(seed + 1)
    for _ in range(generations):
        pop = breed(pop, rng, F18, 2, max_depth=10)
    pop.meta.update(kind="bred", generations=generations, seed=seed)
    return pop, DomainSpec((side, side)), TargetSpec(4, seed + 2, F18, 2, 1)


def workload_c4(seed: int = 10, n_pops: int = 64):
    """64 independent populations for one batched launch.

    Population p: size round(exp(U[ln 20, ln 2000])), maximum depth
    U{4..14}, ramped half-and-half from depth 2 over the 18-operator set; with
    probability 1/8 a 3-D 64^3 domain (terminals gain z), otherwise a 2-D grid
    of side 2^U{5..10}; target a full depth-4 tree.
    Returns a list of (population, DomainSpec, TargetSpec).
    """
    rng = Rng(seed)
    out = []
    for p in range(n_pops):
        size = int(round(math.exp(math.log(20) + rng.uniform() * (math.log(2000) - math.log(20)))))
        d_max = 4 + rng.below(11)
        three_d = rng.below(8) == 0
        if three_d:
            ndim, shape = 3, (64, 64, 64)
        else:
            side = 1 << (5 + rng.below(6))
            ndim, shape = 2, (side, side)
        pop_seed = seed * 1000 + 2 * p
        pop = ramped_half_and_half(size, 2, d_max, pop_seed, F18, ndim)
        out.append((pop, DomainSpec(shape), TargetSpec(4, pop_seed + 1, F18, ndim, 1)))
    return out


@dataclass
class RunSpec:
    """One GP run of the serving workload: its domain, first population,
    target, and the seeds of its breeding and of its think times."""
    run: int
    shape: tuple
    size: int
    pop_seed: int
    target: TargetSpec
    breed_seed: int
    think_seed: int
    max_depth: int = 12

    def first_population(self) -> Population:
        return ramped_half_and_half(self.size, 2, 6, self.pop_seed, F18, len(self.shape))


def workload_c5(seed: int = 11, n_runs: int = 16):
    """Concurrent GP runs sending one population per generation.

    Run r: grid side 512, 1024, 2048 or 4096 (n_runs / 4 runs each, in that
    order), population size round(exp(U[ln 200, ln 2000])) fixed for the run,
    generation 0 by ramped half-and-half depths 2-6 over the 18-operator set,
    later generations bred from the returned fitness (tournament of 3,
    crossover 0.8 / mutation 0.1 / copy 0.1, depth <= 12), target a full
    depth-4 tree, RMSE.
    """
    rng = Rng(seed)
    sides = (512, 1024, 2048, 4096)
    per = max(1, n_runs // len(sides))
    out = []
    for r in range(n_runs):
        side = sides[min(r // per, len(sides) - 1)]
        size = int(round(math.exp(math.log(200) + rng.uniform() * (math.log(2000) - math.log(200)))))
        base = seed * 1000 + 4 * r
        out.append(RunSpec(r, (side, side), size, base, TargetSpec(4, base + 1, F18, 2, 1), base + 2,
                           base + 3))
    return out


# The first generation of neutral breeding (seed 4 on the seed-3 start) at
# which the 500-tree population shares 30-60% of its internal nodes; chosen
# once and checked by a CPU test.
C2_GENERATIONS = 1
