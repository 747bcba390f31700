"""Handley's population DAG, computed plainly (test infrastructure only).

Handley represents the population as a DAG in which structurally identical
subtrees are stored once (related-work section of the paper).  Here two nodes
are identical when their opcode, payload and (already canonical) children are
equal; the payload is the axis for a variable and the FP32 bit pattern for a
constant, and is empty for every function node.  Identifiers are handed out
in first-occurrence order of a postfix walk over the trees in population
order, so every child has a smaller id than its parents.
"""
from __future__ import annotations

import numpy as np

# Arities by opcode, in Table 1 order (kept here independently of any other module).
_ARITY = [0, 0, 2, 2, 2, 2, 1, 1, 1, 1, 1, 2, 2, 2, 2, 1, 1, 1, 1, 3, 2, 1, 3, 1, 1, 1, 2, 3, 2, 2, 2, 3]


def tree_stack_depth(ops) -> int:
    """Largest number of values on the stack in a left-to-right postfix walk."""
    d = best = 0
    for op in ops:
        d += 1 - _ARITY[op]
        best = max(best, d)
    return best


# Operators whose two operands may be swapped without changing a bit of the
# result (NaN payloads aside): IEEE addition and multiplication, min and max
# under the readings (-0 below +0, a NaN operand gives the other), the mean,
# the hypotenuse, the bitwise operators.
COMMUTATIVE = (2, 4, 12, 13, 14, 26, 28, 29, 30)


# Opcodes (Table 1 order) the rewrites name.
_ADD, _SUB, _MULT, _DIV, _MIN, _MAX, _NEG, _SIGN, _ABS, _IF, _STEP = 2, 3, 4, 5, 12, 13, 15, 17, 18, 22, 23
_POS_ZERO, _NEG_ZERO, _ONE = 0x00000000, 0x80000000, 0x3F800000


def rewrite_target(op, kids, node_key):
    """The node a token of operator op over canonical children kids stands
    for under the identity rewrites, or None.  Every rule maps to an
    existing node (a child or a grandchild) and holds bit for bit under the
    library's readings, NaN payloads aside (a NaN stays a NaN):

      neg(neg(x)) -> x          sign flipped twice
      abs(abs(x)) -> abs(x)     |x| is already non-negative
      sign(sign(x)) -> sign(x)  sign of -1, 0 (never -0) and 1
      step(step(x)) -> step(x)  step of -1 and 1
      min(x, x) -> x, max(x, x) -> x
      if(c, y, y) -> y          either branch is y
      sub(x, +0) -> x           x - (+0) = x, also for x = -0
      add(x, -0) -> x, add(-0, x) -> x
      mult(x, 1) -> x, mult(1, x) -> x, div(x, 1) -> x

    sub(x, -0) and add(x, +0) are not rewrites: -0 + (+0) is +0."""
    def const_bits(k):
        o, payload, _ = node_key[k]
        return payload if o == 1 else None

    if op in (_NEG,) and node_key[kids[0]][0] == _NEG:
        return node_key[kids[0]][2][0]
    if op in (_ABS, _SIGN, _STEP) and node_key[kids[0]][0] == op:
        return kids[0]
    if op in (_MIN, _MAX) and kids[0] == kids[1]:
        return kids[0]
    if op == _IF and kids[1] == kids[2]:
        return kids[1]
    if op == _SUB and const_bits(kids[1]) == _POS_ZERO:
        return kids[0]
    if op == _ADD:
        if const_bits(kids[1]) == _NEG_ZERO:
            return kids[0]
        if const_bits(kids[0]) == _NEG_ZERO:
            return kids[1]
    if op == _MULT:
        if const_bits(kids[1]) == _ONE:
            return kids[0]
        if const_bits(kids[0]) == _ONE:
            return kids[1]
    if op == _DIV and const_bits(kids[1]) == _ONE:
        return kids[0]
    return None


def build_dag(tokens, offsets, commutative=False, rewrite=False):
    """Canonicalise a population.

    With commutative=True, a node of a COMMUTATIVE operator is identified by
    the unordered pair of its children (its children stay in the order of
    its first occurrence).  With rewrite=True, a token that rewrite_target
    maps to an existing node stands for that node (no node of its own; it
    counts in that node's multiplicity).

    Returns a dict with
      node_op, node_var (uint8), node_value (float32), children (int32 [U][3], -1 = none),
      roots (int32 [R]), multiplicity (int32 [U], tokens mapped to each node),
      indegree (int32 [U], DAG edges (parent, slot) into each node),
      and the counts tree_nodes, tree_internal, dag_nodes, dag_internal,
      shared_internal, max_stack, max_height.
    """
    ops = tokens["op"].astype(np.int64)
    var = tokens["var"].astype(np.int64)
    bits = tokens["value"].view(np.uint32).astype(np.int64)
    table = {}
    node_key = []
    mult = []
    roots = []
    heights = []
    max_stack = 0
    for r in range(len(offsets) - 1):
        stack = []
        hstack = []
        ops_r = []
        for t in range(int(offsets[r]), int(offsets[r + 1])):
            op = int(ops[t])
            ops_r.append(op)
            a = _ARITY[op]
            if a:
                kids = tuple(stack[len(stack) - a:])
                del stack[len(stack) - a:]
                h = 1 + max(hstack[len(hstack) - a:])
                del hstack[len(hstack) - a:]
                key = (op, 0, tuple(sorted(kids)) if commutative and op in COMMUTATIVE else kids)
                first_kids = kids
                target = rewrite_target(op, kids, node_key) if rewrite else None
                if target is not None:
                    mult[target] += 1
                    stack.append(target)
                    hstack.append(h)
                    continue
            else:
                payload = int(var[t]) if op == 0 else int(bits[t])
                key = (op, payload, ())
                first_kids = ()
                h = 0
            nid = table.get(key)
            if nid is None:
                nid = len(node_key)
                table[key] = nid
                node_key.append((key[0], key[1], first_kids))
                mult.append(0)
            mult[nid] += 1
            stack.append(nid)
            hstack.append(h)
        if len(stack) != 1:
            raise ValueError(f"tree {r} is not a single postfix tree")
        roots.append(stack[0])
        heights.append(hstack[0])
        max_stack = max(max_stack, tree_stack_depth(ops_r))
    U = len(node_key)
    node_op = np.zeros(U, np.uint8)
    node_var = np.zeros(U, np.uint8)
    node_value = np.zeros(U, np.float32)
    children = np.full((U, 3), -1, np.int32)
    indeg = np.zeros(U, np.int32)
    for i, (op, payload, kids) in enumerate(node_key):
        node_op[i] = op
        if op == 0:
            node_var[i] = payload
        elif op == 1:
            node_value[i] = np.array([payload], np.uint32).view(np.float32)[0]
        for j, k in enumerate(kids):
            children[i, j] = k
            indeg[k] += 1
    mult = np.array(mult, np.int32)
    internal = np.array([_ARITY[k[0]] > 0 for k in node_key], bool)
    tree_internal = int(sum(1 for o in ops if _ARITY[o] > 0))
    return dict(node_op=node_op, node_var=node_var, node_value=node_value, children=children,
                roots=np.array(roots, np.int32), multiplicity=mult, indegree=indeg,
                tree_nodes=int(len(ops)), tree_internal=tree_internal, dag_nodes=U,
                dag_internal=int(internal.sum()),
                shared_internal=int((internal & (mult >= 2)).sum()),
                max_stack=int(max_stack), max_height=int(max(heights) if heights else 0))
