"""Genetic operators between evaluations, computed plainly (test
infrastructure only).

TensorGP evaluates a population on the device and runs the genetic operators
on the host between evaluations (Sec. 4.2); the paper names its generation
method (ramped half-and-half, Table 2) but does not spell out selection or
variation.  This module fixes one reading, the textbook tree-GP operators
(Koza 1992: tournament selection, subtree crossover, subtree mutation,
reproduction), with every random decision drawn from a counter-based stream
so that each offspring can be bred independently:

* draw k of offspring o is output number o * 2^32 + k + 1 of SplitMix64
  (Steele, Lea & Flood 2014) started from `seed`, i.e. the SplitMix64 output
  function applied to seed + n * 0x9E3779B97F4A7C15 (mod 2^64);
* below(m) = floor(x * m / 2^64) (multiply-shift, no rejection), uniform()
  = (x >> 11) * 2^-53, a constant = fl32(2 u - 1) with u = (x >> 40) * 2^-24;
* offspring o: u = uniform(); p1 = tournament(); with u < p_crossover also
  p2 = tournament(); tournament(t) draws t individuals with replacement and
  keeps the first of the lowest fitness (a non-finite fitness counts as
  +inf); then for each channel tree a of p1 (and b, the same channel of p2):
    - crossover: up to `tries` attempts draw a point i of a and j of b
      (uniform over tokens) and accept when depth_a(i) + height_b(j) <=
      max_depth; the child is a with the subtree at i replaced by the subtree
      at j of b; with no accepted attempt the child is a copy of a;
    - mutation (p_crossover <= u < p_crossover + p_mutation): a point i of
      a, a depth d = below(min(max(max_depth - depth_a(i), 0),
      max_mutation_depth) + 1), full = below(2) == 0, and the subtree at i
      is replaced by a new random tree of depth d (full or grow);
    - reproduction (otherwise): a copy of a;
* a random tree chooses its nodes in pre-order and emits them in postfix: at
  depth 0 a terminal (below(n_terminals)); full: a function
  (below(n_functions)); grow: below(n_functions + n_terminals), a function
  when below n_functions, else that terminal; terminals are the variables
  0..ndim-1, then the constant when enabled (which draws its value).

Populations are (tokens, offsets, n_channels) with tokens a structured array
of (op u8, var u8, pad u16, value f32), postfix, tree-major.  Everything here
is written from the definitions above; nothing is shared with the library.
"""
from __future__ import annotations

import numpy as np

M64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15

# Arities by opcode, in Table 1 order (kept here independently of any other module).
_ARITY = [0, 0, 2, 2, 2, 2, 1, 1, 1, 1, 1, 2, 2, 2, 2, 1, 1, 1, 1, 3, 2, 1, 3, 1, 1, 1, 2, 3, 2, 2, 2, 3]
VAR, CONST = 0, 1


def splitmix64_output(seed: int, n: int) -> int:
    """Output n (n >= 1) of SplitMix64 started from seed."""
    z = (seed + n * GOLDEN) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


class Stream:
    """The draws of one offspring: draw k is output o * 2^32 + k + 1."""

    def __init__(self, seed: int, o: int):
        self.seed = seed & M64
        self.base = o << 32
        self.k = 0

    def next(self) -> int:
        x = splitmix64_output(self.seed, self.base + self.k + 1)
        self.k += 1
        return x

    def below(self, m: int) -> int:
        return (self.next() * m) >> 64

    def uniform(self) -> float:
        return (self.next() >> 11) * 2.0 ** -53

    def constant(self) -> float:
        u = (self.next() >> 40) * 2.0 ** -24
        return float(np.float32(2.0 * u - 1.0))


def shape(ops) -> tuple:
    """(size, depth, height) of every token of one postfix tree: the number of
    tokens of its subtree, its distance from the root, its subtree's height."""
    n = len(ops)
    size = [0] * n
    height = [0] * n
    parent = [-1] * n
    stack = []
    for i, op in enumerate(ops):
        s, h = 1, 0
        for _ in range(_ARITY[op]):
            c = stack.pop()
            parent[c] = i
            s += size[c]
            h = max(h, height[c] + 1)
        size[i], height[i] = s, h
        stack.append(i)
    if len(stack) != 1:
        raise ValueError("not a single postfix tree")
    depth = [0] * n
    for i in range(n - 2, -1, -1):  # a parent follows its children
        depth[i] = depth[parent[i]] + 1
    return size, depth, height


def random_tree(st: Stream, depth: int, full: bool, functions, ndim: int, use_const: bool) -> list:
    """Tokens (op, var, value) of a random tree of the given depth."""
    n_term = ndim + (1 if use_const else 0)
    out = []

    def terminal(t):
        if t < ndim:
            out.append((VAR, t, 0.0))
        else:
            out.append((CONST, 0, st.constant()))

    def node(d):
        if d == 0:
            terminal(st.below(n_term))
            return
        if full:
            op = functions[st.below(len(functions))]
        else:
            j = st.below(len(functions) + n_term)
            if j >= len(functions):
                terminal(j - len(functions))
                return
            op = functions[j]
        for _ in range(_ARITY[op]):
            node(d - 1)
        out.append((op, 0, 0.0))

    node(depth)
    return out


def _tokens(items) -> np.ndarray:
    t = np.zeros(len(items), dtype=[("op", "u1"), ("var", "u1"), ("pad", "<u2"), ("value", "<f4")])
    for i, (op, var, value) in enumerate(items):
        t[i] = (op, var, 0, value)
    return t


def breed(tokens, offsets, n_channels: int, fitness, seed: int, n_offspring: int, *,
          tournament: int = 3, p_crossover: float = 0.8, p_mutation: float = 0.1,
          max_depth: int = 10, max_mutation_depth: int = 4, tries: int = 8,
          functions=(), ndim: int = 2, use_const: bool = True):
    """One generation bred from the parents; returns (tokens, offsets) of the
    offspring (n_offspring individuals of n_channels trees, tree-major)."""
    offsets = np.asarray(offsets, dtype=np.int64)
    n_par = (len(offsets) - 1) // n_channels
    fit = None
    if fitness is not None:
        fit = [float(f) if np.isfinite(f) else float("inf") for f in np.asarray(fitness, dtype=np.float64)]
    trees = [tokens[int(offsets[r]):int(offsets[r + 1])] for r in range(len(offsets) - 1)]
    shapes = {}

    def shp(r):
        if r not in shapes:
            shapes[r] = shape([int(x) for x in trees[r]["op"]])
        return shapes[r]

    def select(st):
        best = st.below(n_par)
        for _ in range(tournament - 1):
            c = st.below(n_par)
            if fit is not None and fit[c] < fit[best]:
                best = c
        return best

    out = []
    for o in range(n_offspring):
        st = Stream(seed, o)
        u = st.uniform()
        p1 = select(st)
        cross = u < p_crossover
        mutate = not cross and u < p_crossover + p_mutation
        p2 = select(st) if cross else -1
        for ch in range(n_channels):
            ra = p1 * n_channels + ch
            a = trees[ra]
            size_a, depth_a, _ = shp(ra)
            child = a.copy()
            if cross:
                rb = p2 * n_channels + ch
                b = trees[rb]
                size_b, _, height_b = shp(rb)
                for _ in range(tries):
                    i = st.below(len(a))
                    j = st.below(len(b))
                    if depth_a[i] + height_b[j] <= max_depth:
                        child = np.concatenate([a[:i - size_a[i] + 1], b[j - size_b[j] + 1:j + 1], a[i + 1:]])
                        break
            elif mutate:
                i = st.below(len(a))
                room = max(max_depth - depth_a[i], 0)
                d = st.below(min(room, max_mutation_depth) + 1)
                full = st.below(2) == 0
                sub = _tokens(random_tree(st, d, full, functions, ndim, use_const))
                child = np.concatenate([a[:i - size_a[i] + 1], sub, a[i + 1:]])
            out.append(child)
    lens = np.array([len(t) for t in out], dtype=np.int64)
    offs = np.zeros(len(out) + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    toks = np.concatenate(out) if out else _tokens([])
    return toks, offs
