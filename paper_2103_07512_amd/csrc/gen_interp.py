#!/usr/bin/env python3
"""Writes interp_gen.inc: the stack-depth-specialised postfix interpreter.

The interpreter keeps the operand stack of a postfix program in registers.
One wave runs one program and each lane owns K fitness cases, so the stack
depth S before every instruction is the same for all lanes.  The stack
slots are plain named values s0..s{D-1} (each a vector of K lanes' cases),
and one dispatch loop switches on the pair (S, opcode): the case of an
operator of arity a at depth S reads s{S-a}..s{S-1} and writes s{S-a}, so no
register is ever indexed at run time.  The depth of every instruction is
known when the program is emitted, so the emitter writes the pair itself
into the instruction word, (S << 8) | code, and the loop switches on the
loaded word as it is: no depth is carried from one instruction to the next.  A single loop
around a single switch keeps the control flow simple for the compiler: with
one dispatch block per depth, jumping between blocks, the blocks became a
nest of loops whose multi-level exits the compiler implemented with boolean
flags in scalar registers (tens of scalar moves and register spills per
dispatched instruction); the flat loop costs a branch tree over the case
keys.

Superinstructions (Ertl and Gregg): a binary operator whose last-evaluated
operand is a terminal -- x, y, a constant or a cached subtree row -- reads
that operand itself (code FUSE_BASE + 16 * kind + v, v the index in FUSED),
which saves the terminal's own dispatch and the copy into a stack slot.

Operators with long bodies (transcendentals, floored modulo, the FP64 image
operators) are compiled once as out-of-line functions that take and return
the K-vectors by value in registers; the cheap operators are written into
every block.

The planner evaluates the children of a node in decreasing order of the
stack they need (Sethi and Ullman's order), which keeps programs within a
few slots.  An operator whose children were evaluated in another order than
left to right reads its operands from the permuted slots: non-commutative
binary operators have a reversed form (opcode REV_BASE + op) and the
ternary operators one form per permutation (PERM_BASE + 6 t + p, with t the
index in TERNARY and p the index of the evaluation order in PERMS).

Run:  python gen_interp.py          writes interp_gen.inc beside this file
      python gen_interp.py --check  exits 1 when interp_gen.inc is stale
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))

# (name, public opcode, arity) of the function operators, in Table 1 order.
FUNCS = [
    ("add", 2, 2), ("sub", 3, 2), ("mult", 4, 2), ("div", 5, 2),
    ("sin", 6, 1), ("cos", 7, 1), ("tan", 8, 1),
    ("exp", 9, 1), ("log", 10, 1), ("pow", 11, 2),
    ("min", 12, 2), ("max", 13, 2), ("mdist", 14, 2), ("neg", 15, 1),
    ("sqrt", 16, 1), ("sign", 17, 1), ("abs", 18, 1), ("clip", 19, 3),
    ("mod", 20, 2), ("frac", 21, 1), ("if", 22, 3),
    ("step", 23, 1), ("sstep", 24, 1), ("sstepp", 25, 1), ("len", 26, 2), ("lerp", 27, 3),
    ("or", 28, 2), ("xor", 29, 2), ("and", 30, 2),
]
FN_BASE = 8
REV_BASE = 40
PERM_BASE = 72
REVERSIBLE = ("sub", "div", "pow", "mod")
TERNARY = ("clip", "if", "lerp")
PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
# Operators compiled once, out of line.
CALLED = {"sin", "cos", "tan", "exp", "log", "pow", "mod", "sstep", "sstepp", "len", "lerp"}
# The bitwise operators share one opcode (that of "or"); the instruction's
# .y says which (0 or, 1 xor, 2 and).  They, warp (I_WARP) and the third
# axis (I_Z) are compiled only into the interpreters instantiated with
# EXT = true, so the others carry no z vector.
BITWISE = ("or", "xor", "and")
DEPTHS = [8]
ARGS = "abc"
# Fused forms: (operator, reversed) in the order of kFuseOps (tgp_internal.h);
# reversed means the terminal is the operator's first operand.
FUSE_BASE = 96
FUSED = [("add", False), ("sub", False), ("mult", False), ("div", False), ("pow", False),
         ("min", False), ("max", False), ("mdist", False), ("mod", False), ("len", False),
         ("sub", True), ("div", True), ("pow", True), ("mod", True)]
# terminal kinds of a fused operand: (code offset name, how to read case k)
FUSE_KINDS = [("kFuseX", "xv.v[k]"), ("kFuseY", "yv.v[k]"), ("kFuseConst", "c"), ("kFuseCache", "row_load(row, coff[k])")]


def fused_checks():
    """static_asserts tying FUSED to the C++ table the emitter uses."""
    L = ["// The fused forms' table as the emitter sees it (tgp_internal.h)."]
    for v, (name, rev) in enumerate(FUSED):
        op = dict((n, o) for n, o, _ in FUNCS)[name]
        L.append(f"static_assert(kFuseOps[{v}] == {op} && kFuseRev[{v}] == {'true' if rev else 'false'}, "
                 f"\"fused form {v}: {name}{' reversed' if rev else ''}\");")
    L.append(f"static_assert(kFuseBase == {FUSE_BASE} && kNumFused == {len(FUSED)}, \"fused form table\");")
    L.append("")
    return "\n".join(L)


def fused_case(e, key_expr, name, rev, kind, read, dst, ind, end):
    """One fused case: dst = name(dst, T) (or name(T, dst) when reversed),
    T the terminal operand of the given kind; ends with `end`.  With key_expr
    None only the braced body is written (the dispatch tree's leaves)."""
    e(f"{ind}case {key_expr}: {{" if key_expr is not None else f"{ind}{{")
    if kind == "kFuseConst":
        e(f"{ind}    const float c = __uint_as_float(ins.y);")
    if kind == "kFuseCache":
        e(f"{ind}    const Row row = row_at(cache, cache_stride, ins.y);")
    if name in CALLED:
        if kind in ("kFuseX", "kFuseY"):
            tv = "xv" if kind == "kFuseX" else "yv"
        else:
            e(f"{ind}    FV<K> tv;")
            e("#pragma unroll")
            e(f"{ind}    for (int k = 0; k < K; ++k) tv.v[k] = {read};")
            tv = "tv"
        args = f"{tv}, {dst}" if rev else f"{dst}, {tv}"
        e(f"{ind}    {dst} = vcall_{name}<K>({args});")
    else:
        if kind == "kFuseCache":
            e(f"{ind}    float tv[K];")
            e("#pragma unroll")
            e(f"{ind}    for (int k = 0; k < K; ++k) tv[k] = {read};")
            read = "tv[k]"
        a, b = (read, f"{dst}.v[k]") if rev else (f"{dst}.v[k]", read)
        e("#pragma unroll")
        e(f"{ind}    for (int k = 0; k < K; ++k) {dst}.v[k] = f_{name}({a}, {b});")
    e(f"{ind}    {end}")
    e(f"{ind}}}")


def fused_key(kind, v):
    return f"(kFuseBase + 16u * {kind} + {v}u)"


def called_functions():
    L = []
    e = L.append
    e("// Out-of-line operators on K-vectors (arguments and results in registers).")
    for name, _, ar in FUNCS:
        if name not in CALLED:
            continue
        params = ", ".join(f"FV<K> {ARGS[i]}" for i in range(ar))
        call = ", ".join(f"{ARGS[i]}.v[k]" for i in range(ar))
        e("template <int K>")
        e(f"__device__ __attribute__((noinline)) FV<K> vcall_{name}({params}) {{")
        e("    FV<K> r;")
        e("#pragma unroll")
        e(f"    for (int k = 0; k < K; ++k) r.v[k] = f_{name}({call});")
        e("    return r;")
        e("}")
    e("")
    return "\n".join(L)


# Numeric values of the instruction codes (tgp_internal.h; checked by the
# static_asserts of the generated file).
CODES = {"I_X": 0, "I_Y": 1, "I_Z": 2, "I_CONST": 3, "I_CACHE": 4, "I_END": 5, "I_WARP": 6}
KINDS = {"kFuseX": 0, "kFuseY": 1, "kFuseConst": 2, "kFuseCache": 3}


def code_checks():
    L = ["// Instruction codes as the dispatch tree below numbers them."]
    L += [f"static_assert({n} == {v}, \"code {n}\");" for n, v in CODES.items()]
    L += [f"static_assert({n} == {v}, \"fused kind {n}\");" for n, v in KINDS.items()]
    L.append(f"static_assert(kFnBase == {FN_BASE} && kRevBase == {REV_BASE} && kPermBase == {PERM_BASE}, \"bases\");")
    L.append("")
    return "\n".join(L)


def dispatch_weights():
    """Measured frequency of each instruction word (dispatch_weights.txt):
    key -> count.  Words it does not list weigh 1."""
    path = os.path.join(HERE, "dispatch_weights.txt")
    w = {}
    for line in open(path):
        line = line.split("#")[0].split()
        if len(line) == 2:
            w[int(line[0])] = float(line[1])
    return w


def tree(e, keys, bodies, weight, ind):
    """Binary search on the instruction word over the sorted keys, split
    where the weights on both sides balance (Mehlhorn's rule), so a frequent
    word is found after few comparisons; a leaf holds one case.  Every word
    the emitter writes is one of the keys, so a leaf does not test its key."""
    if len(keys) == 1:
        for line in bodies[keys[0]]:
            e(ind + line if not line.startswith("#") else line)
        return
    ws = [weight.get(k, 1.0) for k in keys]
    total, acc, best, m = sum(ws), 0.0, None, 1
    for i in range(1, len(keys)):
        acc += ws[i - 1]
        d = abs(2 * acc - total)
        if best is None or d < best:
            best, m = d, i
    # the split's probability, so the compiler's block frequencies (register
    # allocation, spill placement, layout) follow the measured ones
    p = min(max(sum(ws[:m]) / total, 0.001), 0.999)
    e(f"{ind}if (__builtin_expect_with_probability(ins.x < {keys[m]}u, 1, {p:.3f})) {{")
    tree(e, keys[:m], bodies, weight, ind + "    ")
    e(f"{ind}}} else {{")
    tree(e, keys[m:], bodies, weight, ind + "    ")
    e(f"{ind}}}")


def body_for_depth(D):
    L = []
    e = L.append
    e(f"// Stack of {D} register slots, one dispatch loop over (depth, opcode).")
    e("template <int K, bool EXT>")
    e(f"__device__ __forceinline__ void run_prog_d{D}(const uint2 *__restrict__ ip, const FV<K> &xv0,")
    e("        const FV<K> &yv0, const FV<K> &zv, const float *__restrict__ cache, int64_t cache_stride,")
    e("        const uint32_t (&coff)[K], const WarpGeom &wg, FV<K> &res)")
    e("{")
    e("    " + " ".join(f"FV<K> s{j};" for j in range(D)))
    e("    FV<K> xv = xv0, yv = yv0;")
    # One opaque pass before the loop as well: it waits for the coordinate
    # loads there, so the passes inside the loop find no load pending on
    # those registers and the loop head carries no wait for them.
    e("#pragma unroll")
    e("    for (int k = 0; k < K; ++k) {")
    e("        asm volatile(\"\" : \"+v\"(xv.v[k]));")
    e("        asm volatile(\"\" : \"+v\"(yv.v[k]));")
    e("    }")
    e("    uint2 ins;")
    e("    // one scalar load of the next whole word, issued a dispatch ahead,")
    e("    // through the constant address space at a 32-bit byte offset (one")
    e("    // scalar add per instruction)")
    e("    typedef const __attribute__((address_space(4))) char cchar;")
    e("    typedef const __attribute__((address_space(4))) uint64_t cword;")
    e("    cchar *const cb = (cchar *)ip;")
    e("    uint32_t off = 8;")
    e("    uint64_t nxt = *(cword *)(cb + off);")
    e("    for (;;) {")
    e("    ins = make_uint2((uint32_t)nxt, (uint32_t)(nxt >> 32));")
    # The coordinates pass through an empty asm at every dispatch, so the
    # compiler sees them redefined in the loop and does not hoist the cases'
    # expressions of them (x / 2 for mdist, x == 0 for div, ...) out of it
    # into registers that then spill: fewer VGPRs, no per-tile spill stores.
    e("#pragma unroll")
    e("    for (int k = 0; k < K; ++k) {")
    e("        asm volatile(\"\" : \"+v\"(xv.v[k]));")
    e("        asm volatile(\"\" : \"+v\"(yv.v[k]));")
    e("    }")
    e("    if (ins.x == ((1u << 8) | I_END)) break;")
    e("    __builtin_amdgcn_sched_barrier(0);")
    e("    off += 8;")
    e("    nxt = *(cword *)(cb + off);")
    bodies = {}

    def case(key, lines):
        assert key not in bodies
        bodies[key] = lines

    variants = []
    for name, op, ar in FUNCS:
        if name in BITWISE[1:]:
            continue
        variants.append((FN_BASE + op, name, ar, tuple(range(ar))))
        if name in REVERSIBLE:
            variants.append((REV_BASE + op, name, ar, (1, 0)))
        if name in TERNARY:
            t = TERNARY.index(name)
            for p, order in enumerate(PERMS):
                if p:
                    variants.append((PERM_BASE + 6 * t + p, name, ar, order))
    for S in range(D + 1):
        key = lambda c: (S << 8) | c
        if S < D:
            for name, reg in (("I_X", "xv"), ("I_Y", "yv")):
                case(key(CODES[name]), [f"s{S} = {reg};", "continue;"])
            # the third axis only in the extended interpreter (3-D domains)
            case(key(CODES["I_Z"]), ["if constexpr (EXT) {", f"    s{S} = zv;", "    continue;", "} else {",
                                     "    goto BAD;", "}"])
            case(key(CODES["I_CONST"]), ["const float c = __uint_as_float(ins.y);", "#pragma unroll",
                                         f"for (int k = 0; k < K; ++k) s{S}.v[k] = c;", "continue;"])
            case(key(CODES["I_CACHE"]), ["const Row row = row_at(cache, cache_stride, ins.y);",
                                         "#pragma unroll",
                                         f"for (int k = 0; k < K; ++k) s{S}.v[k] = row_load(row, coff[k]);",
                                         "continue;"])
        if S >= 2:
            case(key(CODES["I_WARP"]), [
                "if constexpr (EXT) {",
                "    const Row row = row_at(cache, cache_stride, ins.y);",
                "#pragma unroll",
                f"    for (int k = 0; k < K; ++k) s{S - 2}.v[k] = row_load(row, 4u * (uint32_t)warp_case(wg, s{S - 2}.v[k], s{S - 1}.v[k], (int32_t)(coff[k] >> 2)));",
                "    continue;",
                "} else {",
                "    goto BAD;",
                "}"])
        for c, name, ar, order in variants:
            if S < ar:
                continue
            dst = S - ar
            src = [f"s{dst + order.index(i)}" for i in range(ar)]
            if name == BITWISE[0]:
                case(key(c), [
                    "if constexpr (EXT) {",
                    "    const uint32_t kind = ins.y;",
                    "#pragma unroll",
                    f"    for (int k = 0; k < K; ++k) s{dst}.v[k] = f_bitop({src[0]}.v[k], {src[1]}.v[k], kind);",
                    "    continue;",
                    "} else {",
                    "    goto BAD;",
                    "}"])
            elif name in CALLED:
                case(key(c), [f"s{dst} = vcall_{name}<K>({', '.join(src)});", "continue;"])
            else:
                args = ", ".join(f"{x}.v[k]" for x in src)
                case(key(c), ["#pragma unroll", f"for (int k = 0; k < K; ++k) s{dst}.v[k] = f_{name}({args});",
                              "continue;"])
        if S >= 1:
            for kind, read in FUSE_KINDS:
                for v, (name, rev) in enumerate(FUSED):
                    lines = []
                    fused_case(lines.append, None, name, rev, kind, read, f"s{S - 1}", "", "continue;")
                    case(key(FUSE_BASE + 16 * KINDS[kind] + v), lines)
    tree(e, sorted(bodies), bodies, dispatch_weights(), "    ")
    e("    }")
    e("    res = s0;")
    e("    return;")
    e("BAD:")
    e("#pragma unroll")
    e("    for (int k = 0; k < K; ++k) res.v[k] = __builtin_nanf(\"\");")
    e("}")
    e("")
    return "\n".join(L)


def body_lds():
    """The interpreter with its operand stack in LDS.

    The top of the stack stays in registers (t); the values below it live in
    this wave's LDS rows, slot s of case k of lane l at sl[(s * K + k) * 64 +
    l] (consecutive lanes in consecutive banks).  A push stores t and moves
    the new value into t; the first push stores an unused value into slot 0,
    so a program of stack depth n uses slots 0 .. n - 1.  One dispatch loop
    serves every depth: the slot index is a run-time scalar, which LDS
    addressing allows and registers do not.
    """
    L = []
    e = L.append
    e("// Operand stack in LDS (top of stack in registers); see gen_interp.py.")
    e("template <int K>")
    e("__device__ __forceinline__ void lds_put(float *sl, uint32_t s, int lane, const FV<K> &v) {")
    e("#pragma unroll")
    e("    for (int k = 0; k < K; ++k) sl[(s * K + k) * 64 + lane] = v.v[k];")
    e("}")
    e("template <int K>")
    e("__device__ __forceinline__ FV<K> lds_get(const float *sl, uint32_t s, int lane) {")
    e("    FV<K> v;")
    e("#pragma unroll")
    e("    for (int k = 0; k < K; ++k) v.v[k] = sl[(s * K + k) * 64 + lane];")
    e("    return v;")
    e("}")
    e("template <int K>")
    e("__device__ __forceinline__ void run_prog_lds(const uint2 *__restrict__ ip, const FV<K> &xv,")
    e("        const FV<K> &yv, const FV<K> &zv, const float *__restrict__ cache, int64_t cache_stride,")
    e("        const uint32_t (&coff)[K], const WarpGeom &wg, float *sl, int lane, FV<K> &res)")
    e("{")
    e("    FV<K> t;")
    e("#pragma unroll")
    e("    for (int k = 0; k < K; ++k) t.v[k] = 0.0f;")
    e("    uint32_t sp = 0;  // values stored in LDS")
    e("    for (;;) {")
    e("        const uint2 ins = *ip;")
    e("        ++ip;")
    e("        switch (ins.x & 0xffu) {")
    for name, reg in (("I_X", "xv"), ("I_Y", "yv"), ("I_Z", "zv")):
        e(f"        case {name}: lds_put<K>(sl, sp++, lane, t); t = {reg}; break;")
    e("        case I_CONST: {")
    e("            lds_put<K>(sl, sp++, lane, t);")
    e("            const float c = __uint_as_float(ins.y);")
    e("#pragma unroll")
    e("            for (int k = 0; k < K; ++k) t.v[k] = c;")
    e("            break;")
    e("        }")
    e("        case I_CACHE: {")
    e("            lds_put<K>(sl, sp++, lane, t);")
    e("            const Row row = row_at(cache, cache_stride, ins.y);")
    e("#pragma unroll")
    e("            for (int k = 0; k < K; ++k) t.v[k] = row_load(row, coff[k]);")
    e("            break;")
    e("        }")
    e("        case I_END: res = t; return;")
    e("        case I_WARP: {")
    e("            const FV<K> t0 = lds_get<K>(sl, --sp, lane);")
    e("            const Row row = row_at(cache, cache_stride, ins.y);")
    e("#pragma unroll")
    e("            for (int k = 0; k < K; ++k) t.v[k] = row_load(row, 4u * (uint32_t)warp_case(wg, t0.v[k], t.v[k], (int32_t)(coff[k] >> 2)));")
    e("            break;")
    e("        }")
    for name, op, ar in FUNCS:
        if name in BITWISE[1:]:
            continue
        variants = [(FN_BASE + op, tuple(range(ar)))]
        if name in REVERSIBLE:
            variants.append((REV_BASE + op, (1, 0)))
        if name in TERNARY:
            t = TERNARY.index(name)
            variants += [(PERM_BASE + 6 * t + p, order) for p, order in enumerate(PERMS) if p]
        for c, order in variants:
            e(f"        case {c}: {{")
            # stack values in evaluation order: the deepest first, t last;
            # child order[i] is the i-th value
            names = [f"u{i}" for i in range(ar)]
            for i in range(ar - 1):
                e(f"            const FV<K> {names[i]} = lds_get<K>(sl, sp - {ar - 1 - i}, lane);")
            if ar > 1:
                e(f"            sp -= {ar - 1};")
            e(f"            const FV<K> {names[ar - 1]} = t;")
            args = [names[order.index(i)] for i in range(ar)]
            if name == BITWISE[0]:
                e("            const uint32_t kind = ins.y;")
                e("#pragma unroll")
                e(f"            for (int k = 0; k < K; ++k) t.v[k] = f_bitop({args[0]}.v[k], {args[1]}.v[k], kind);")
            elif name in CALLED:
                e(f"            t = vcall_{name}<K>({', '.join(args)});")
            else:
                e("#pragma unroll")
                e(f"            for (int k = 0; k < K; ++k) t.v[k] = f_{name}({', '.join(a + '.v[k]' for a in args)});")
            e("            break;")
            e("        }")
    for kind, read in FUSE_KINDS:
        for v, (name, rev) in enumerate(FUSED):
            fused_case(e, fused_key(kind, v), name, rev, kind, read, "t", "        ", "break;")
    e("        default:")
    e("#pragma unroll")
    e("            for (int k = 0; k < K; ++k) res.v[k] = __builtin_nanf(\"\");")
    e("            return;")
    e("        }")
    e("    }")
    e("}")
    e("")
    return "\n".join(L)


def generate():
    out = ["// interp_gen.inc -- GENERATED by gen_interp.py; do not edit.",
           "// Stack-depth-specialised postfix interpreters, one per stack size.",
           f"// Stack sizes: {', '.join(map(str, DEPTHS))}.",
           "",
           fused_checks(),
           code_checks(),
           called_functions()]
    for D in DEPTHS:
        out.append(body_for_depth(D))
    out.append(body_lds())
    return "\n".join(out) + "\n"


def main():
    path = os.path.join(HERE, "interp_gen.inc")
    text = generate()
    if len(sys.argv) > 1 and sys.argv[1] == "--check":
        cur = open(path).read() if os.path.exists(path) else ""
        sys.exit(0 if cur == text else 1)
    with open(path, "w") as f:
        f.write(text)


if __name__ == "__main__":
    main()
