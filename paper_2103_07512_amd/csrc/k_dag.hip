// k_dag.hip -- building Handley's population DAG on the GPU.
//
// The paper caches the results of structurally identical subtrees so that
// code shared between individuals is not executed again (Sec. 1, Sec. 3.1),
// generalising the trees to a DAG as in Handley's work (Sec. 2).  The DAG is
// built here by hash-consing, in three steps:
//   1. structure: one thread per tree scans its postfix tokens with a stack,
//      validates arities and opcodes, and records each token's children and
//      height (a terminal has height 0);
//   2. hash-consing, level by level in increasing height: a token's key is
//      (opcode, payload, classes of its children), whose children all lie on
//      lower, already finished levels.  Keys go into an open-addressing table
//      (linear probing, capacity >= 2 x tokens); equal keys are detected by
//      comparing the full key, never the hash alone.  While the levels run, a
//      token's class is the table slot of its key (a slot never moves, so the
//      keys built from classes stay put); the representative of a key is its
//      smallest token index (atomicMin over every level: with rewrites, one
//      key can occur at several tree heights), and a last pass replaces each
//      class by its representative, so the result does not depend on thread
//      timing;
//   3. compaction: representatives are numbered by an exclusive scan in token
//      order, which is the order of first occurrence in a postfix walk of the
//      trees in population order, so children get smaller ids than parents.
#include <hip/hip_runtime.h>

#include <string.h>
#include <stdio.h>
#include <vector>

#include "tgp_internal.h"

namespace tgp {

struct BuildStatus {
    unsigned long long first_error;  // (tree << 4) | code, min over trees; ~0 = none
    int32_t max_height;
    int32_t max_var;
    int32_t max_stack;
    int32_t n_internal;
    int32_t lost_key;  // nonzero when hash-consing found no slot for a key
};

enum { ERR_NONE = 0, ERR_OP = 1, ERR_PARSE = 2, ERR_RANGE = 3 };

__device__ __forceinline__ void report(BuildStatus *st, int64_t r, int code) {
    atomicMin(&st->first_error, ((unsigned long long)r << 4) | (unsigned long long)code);
}

// 1. Structure scan, one thread per tree: children, subtree heights, the
// postfix stack depth.  The operand stack of pending (token, height) pairs
// lives in LDS (kStructStack entries per thread); a tree whose stack needs
// more is rescanned with its stack in stk[off[r] .. off[r+1]) of global
// scratch.
constexpr int kStructStack = 32;

template <bool LDS>
__device__ __forceinline__ bool structure_scan(const uint2 *tok, int64_t o0, int64_t o1, int64_t r, int32_t *kid,
                                               int32_t *height, int32_t *stk_g, int2 (*stk_l)[64], int lane,
                                               BuildStatus *st, int32_t *out_maxsp, int32_t *out_internal,
                                               int32_t *out_maxvar) {
    int64_t sp = 0;
    int32_t maxsp = 0, internal = 0, maxvar = -1;
    int verdict = 0;  // 1 reported, 2 needs the global stack
    for_tokens<8, false>(tok, o0, o1, [&](int64_t t, uint2 w) {
        const uint32_t op = w.x & 0xffu;
        if (op >= TGP_NUM_OPS) {
            report(st, r, ERR_OP);
            verdict = 1;
            return false;
        }
        const int a = arity_of(op);
        if (sp < a) {
            report(st, r, ERR_PARSE);
            verdict = 1;
            return false;
        }
        int32_t h = 0;
        int32_t k3[3] = {-1, -1, -1};
        for (int j = a - 1; j >= 0; --j) {
            --sp;
            int32_t c, hc;
            if constexpr (LDS) {
                const int2 e = stk_l[sp][lane];
                c = e.x;
                hc = e.y + 1;
            } else {
                c = stk_g[o0 + sp];
                hc = height[c] + 1;
            }
            k3[j] = c;
            h = hc > h ? hc : h;
        }
        kid[3 * t + 0] = k3[0];
        kid[3 * t + 1] = k3[1];
        kid[3 * t + 2] = k3[2];
        height[t] = h;
        if constexpr (LDS) {
            if (sp == kStructStack) {
                verdict = 2;
                return false;
            }
            stk_l[sp][lane] = int2{(int32_t)t, h};
        } else {
            stk_g[o0 + sp] = (int32_t)t;
        }
        ++sp;
        if (sp > maxsp) maxsp = (int32_t)sp;
        if (a > 0) ++internal;
        if (op == TGP_VAR) {
            const int32_t v = (int32_t)((w.x >> 8) & 0xffu);
            maxvar = v > maxvar ? v : maxvar;
        }
        return true;
    });
    if (verdict == 1) return true;
    if (verdict == 2) return false;
    if (sp != 1) {
        report(st, r, ERR_PARSE);
        return true;
    }
    *out_maxsp = maxsp;
    *out_internal = internal;
    *out_maxvar = maxvar;
    return true;
}

__global__ __launch_bounds__(64) void k_structure(const uint2 *tok, const int64_t *off, int64_t R, int64_t T,
                                                  int32_t *kid, int32_t *height, int32_t *stk, int32_t *root_tok,
                                                  BuildStatus *st) {
    __shared__ int2 stk_l[kStructStack][64];
    const int lane = threadIdx.x;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + lane;
    if (r >= R) return;
    const int64_t o0 = off[r], o1 = off[r + 1];
    if (o0 < 0 || o1 > T || o1 < o0) {
        report(st, r, ERR_RANGE);
        return;
    }
    if (o1 == o0) {
        report(st, r, ERR_PARSE);
        return;
    }
    int32_t maxsp = -1, internal = 0, maxvar = -1;
    if (!structure_scan<true>(tok, o0, o1, r, kid, height, stk, stk_l, lane, st, &maxsp, &internal, &maxvar))
        structure_scan<false>(tok, o0, o1, r, kid, height, stk, stk_l, lane, st, &maxsp, &internal, &maxvar);
    if (maxsp < 0) return;  // reported
    root_tok[r] = (int32_t)(o1 - 1);
    atomicMax(&st->max_height, height[o1 - 1]);
    atomicMax(&st->max_stack, maxsp);
    atomicMax(&st->max_var, maxvar);
    atomicAdd(&st->n_internal, internal);
}

__global__ void k_level_hist(const int32_t *height, int64_t T, int32_t *cnt) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < T) atomicAdd(&cnt[height[t]], 1);
}

__global__ void k_level_scatter(const int32_t *height, int64_t T, int32_t *cursor, int32_t *list) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < T) {
        const int32_t pos = atomicAdd(&cursor[height[t]], 1);
        list[pos] = (int32_t)t;
    }
}

// The same two passes with the counters privatised in LDS (most tokens are
// leaves, so the global forms above serialise on one address).  A block
// takes kLvlPer tokens per thread and touches each global counter once.
// Used when the tallest tree has at most kLvlBins levels; the order of the
// tokens inside a level is not significant.
constexpr int kLvlBins = 512;
constexpr int kLvlPer = 16;

__global__ void __launch_bounds__(256) k_level_hist_lds(const int32_t *height, int64_t T, int32_t H,
                                                        int32_t *cnt) {
    __shared__ int32_t c[kLvlBins];
    for (int i = threadIdx.x; i < H; i += blockDim.x) c[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * blockDim.x * kLvlPer + threadIdx.x;
    for (int j = 0; j < kLvlPer; ++j) {
        const int64_t t = base + (int64_t)j * blockDim.x;
        if (t < T) atomicAdd(&c[height[t]], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < H; i += blockDim.x)
        if (c[i]) atomicAdd(&cnt[i], c[i]);
}

__global__ void __launch_bounds__(256) k_level_scatter_lds(const int32_t *height, int64_t T, int32_t H,
                                                           int32_t *cursor, int32_t *list) {
    __shared__ int32_t c[kLvlBins];
    for (int i = threadIdx.x; i < H; i += blockDim.x) c[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * blockDim.x * kLvlPer + threadIdx.x;
    int32_t h[kLvlPer], r[kLvlPer];
    for (int j = 0; j < kLvlPer; ++j) {
        const int64_t t = base + (int64_t)j * blockDim.x;
        h[j] = t < T ? height[t] : -1;
        r[j] = h[j] >= 0 ? atomicAdd(&c[h[j]], 1) : 0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < H; i += blockDim.x)
        c[i] = c[i] ? atomicAdd(&cursor[i], c[i]) : 0;
    __syncthreads();
    for (int j = 0; j < kLvlPer; ++j)
        if (h[j] >= 0) list[c[h[j]] + r[j]] = (int32_t)(base + (int64_t)j * blockDim.x);
}

// Key of token t: k0 = opcode | axis << 8 (the axis only for a variable);
// k1 = constant bits or first child's canonical id; k2, k3 = further
// children; unused fields are all-ones.
struct Key {
    uint32_t k0, k1, k2, k3;
};

// Operators whose operands commute bitwise in this library (see
// tgp_ctx_set_hashing).
__device__ __forceinline__ bool commutes(uint32_t op) {
    return op == TGP_ADD || op == TGP_MULT || op == TGP_MIN || op == TGP_MAX || op == TGP_MDIST ||
           op == TGP_LEN || op == TGP_OR || op == TGP_XOR || op == TGP_AND;
}

__device__ __forceinline__ Key key_of(int32_t t, const uint2 *tok, const int32_t *kid,
                                      const int32_t *canon, bool commute) {
    const uint2 w = tok[t];
    const uint32_t op = w.x & 0xffu;
    Key k{op, 0xffffffffu, 0xffffffffu, 0xffffffffu};
    if (op == TGP_VAR) {
        k.k0 = op | (w.x & 0xff00u);
    } else if (op == TGP_CONST) {
        k.k1 = w.y;
    } else {
        const int a = arity_of(op);
        k.k1 = (uint32_t)canon[kid[3 * t + 0]];
        if (a > 1) k.k2 = (uint32_t)canon[kid[3 * t + 1]];
        if (a > 2) k.k3 = (uint32_t)canon[kid[3 * t + 2]];
        if (commute && commutes(op) && k.k1 > k.k2) {
            const uint32_t x = k.k1;
            k.k1 = k.k2;
            k.k2 = x;
        }
    }
    return k;
}

__device__ __forceinline__ bool key_eq(const Key &a, const Key &b) {
    return a.k0 == b.k0 && a.k1 == b.k1 && a.k2 == b.k2 && a.k3 == b.k3;
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t key_hash(const Key &k, uint32_t hash_mask_bits) {
    uint64_t h = mix64(((uint64_t)k.k0 << 32) | k.k1);
    h = mix64(h ^ (((uint64_t)k.k2 << 32) | k.k3));
    if (hash_mask_bits) h &= ((1ull << hash_mask_bits) - 1);  // collision stress (tests)
    return h;
}

// Identity rewrites (tgp_ctx_set_rewrite; the algebraic equivalences of Wong
// and Zhang's subtree caching, Sec. 2, and the simplification the paper
// proposes as future work, Sec. 5), restricted to those that hold bit for bit
// under this library's readings (NaN payloads aside) and whose result is a
// node that already exists: the representative token that token t stands for,
// or -1 (as a class, like canon while the levels run).  The rules:
//   neg(neg(x)) -> x; abs(abs(x)) -> abs(x); sign(sign(x)) -> sign(x);
//   step(step(x)) -> step(x); min(x, x) -> x; max(x, x) -> x;
//   if(c, y, y) -> y; sub(x, +0) -> x; add(x, -0), add(-0, x) -> x;
//   mult(x, 1), mult(1, x) -> x; div(x, 1) -> x.
// The children are already canonical (lower levels), so a rule sees through
// earlier rewrites.
__device__ __forceinline__ int32_t rewrite_target(int32_t t, const uint2 *tok, const int32_t *kid,
                                                  const int32_t *canon, const int32_t *table) {
    const uint32_t op = tok[t].x & 0xffu;
    const int a = arity_of(op);
    if (a == 0) return -1;
    // classes (table slots) of the children; any token of a class (its
    // slot's current value) has the class's opcode, payload and children
    const int32_t c0 = canon[kid[3 * t]];
    const int32_t c1 = a > 1 ? canon[kid[3 * t + 1]] : -1;
    const int32_t c2 = a > 2 ? canon[kid[3 * t + 2]] : -1;
    auto op_of = [&](int32_t c) { return tok[table[c]].x & 0xffu; };
    auto is_const = [&](int32_t c, uint32_t bits) { return op_of(c) == TGP_CONST && tok[table[c]].y == bits; };
    switch (op) {
    case TGP_NEG: return op_of(c0) == TGP_NEG ? canon[kid[3 * table[c0]]] : -1;
    case TGP_ABS:
    case TGP_SIGN:
    case TGP_STEP: return op_of(c0) == op ? c0 : -1;
    case TGP_MIN:
    case TGP_MAX: return c0 == c1 ? c0 : -1;
    case TGP_IF: return c1 == c2 ? c1 : -1;
    case TGP_SUB: return is_const(c1, 0x00000000u) ? c0 : -1;
    case TGP_ADD: return is_const(c1, 0x80000000u) ? c0 : (is_const(c0, 0x80000000u) ? c1 : -1);
    case TGP_MULT: return is_const(c1, 0x3f800000u) ? c0 : (is_const(c0, 0x3f800000u) ? c1 : -1);
    case TGP_DIV: return is_const(c1, 0x3f800000u) ? c0 : -1;
    default: return -1;
    }
}

// 2a. Insert the tokens of one level; the slot of a key ends up holding the
// smallest token index with that key.  A rewritten token is not inserted.
__global__ void k_hash_insert(const int32_t *list, int32_t n, const uint2 *tok, const int32_t *kid,
                              const int32_t *canon, int32_t *table, uint64_t mask,
                              uint32_t hash_bits, bool commute, bool rewrite) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < n;
    int32_t t = live ? list[i] : -1;
    const Key k = live ? key_of(t, tok, kid, canon, commute) : Key{0xffffffffu, 0, 0, 0};
    const bool rewritten = live && rewrite && rewrite_target(t, tok, kid, canon, table) >= 0;
    // Leaves (x, y, z and the constants) repeat many times within one wave:
    // lanes holding the same leaf key (its first two words) insert once,
    // through the group's lowest lane, with the group's smallest token index.
    // Every lane of the wave takes part in the ballots and shuffles.
    const uint32_t op = k.k0 & 0xffu;
    const bool leaf = live && (op == TGP_VAR || op == TGP_CONST);
    bool insert = live && !leaf && !rewritten;
    const int lane = (int)(threadIdx.x & 63u);
    uint64_t todo = __ballot(leaf);
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const uint32_t l0 = __shfl(k.k0, leader), l1 = __shfl(k.k1, leader);
        const uint64_t same = __ballot(leaf && k.k0 == l0 && k.k1 == l1) & todo;
        int32_t m = ((same >> lane) & 1u) ? t : INT32_MAX;
        for (int d = 32; d > 0; d >>= 1) m = min(m, __shfl_xor(m, d));
        if (lane == leader) {
            t = m;
            insert = true;
        }
        todo &= ~same;
    }
    if (!insert) return;
    uint64_t s = key_hash(k, hash_bits) & mask;
    for (;;) {
        int32_t e = table[s];
        if (e < 0) {
            e = atomicCAS(&table[s], -1, t);
            if (e < 0) return;  // claimed an empty slot
        }
        if (key_eq(key_of(e, tok, kid, canon, commute), k)) {
            // A slot's value only decreases and its key never changes, so a
            // token that is not below the value it read (which may be stale,
            // never lower than the current one) cannot lower it.  Skipping
            // those leaves the atomics to the few tokens that can: without
            // this, every leaf x or y of the level updated one address.
            if (t < e) atomicMin(&table[s], t);
            return;
        }
        s = (s + 1) & mask;
    }
}

// 2b. Every token of the level looks its key up again and takes the
// representative.
__global__ void k_hash_resolve(const int32_t *list, int32_t n, const uint2 *tok, const int32_t *kid,
                               int32_t *canon, const int32_t *table, uint64_t mask,
                               uint32_t hash_bits, bool commute, bool rewrite, BuildStatus *st) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t t = list[i];
    if (rewrite) {
        const int32_t target = rewrite_target(t, tok, kid, canon, table);
        if (target >= 0) {
            canon[t] = target;
            return;
        }
    }
    const Key k = key_of(t, tok, kid, canon, commute);
    uint64_t s = key_hash(k, hash_bits) & mask;
    for (;;) {
        const int32_t e = table[s];
        if (e < 0) {
            // t itself was inserted before the first empty slot of its probe
            // sequence, so reaching one means the table is corrupt: the build
            // fails with an error instead of yielding a wrong DAG
            atomicOr(&st->lost_key, 1);
            canon[t] = (int32_t)s;  // an empty slot; the build fails with an error
            return;
        }
        if (key_eq(key_of(e, tok, kid, canon, commute), k)) {
            canon[t] = (int32_t)s;  // the class: the key's slot
            return;
        }
        s = (s + 1) & mask;
    }
}

// 2c. After the last level: every class becomes its representative, the
// smallest token index with that key.
__global__ void k_class_to_token(int32_t *canon, int64_t T, const int32_t *table) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < T) canon[t] = table[canon[t]];
}

__global__ void k_flags(const int32_t *canon, int64_t T, int32_t *flag) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < T) flag[t] = canon[t] == (int32_t)t ? 1 : 0;
}

// Exclusive scan, 1024 elements per block (256 threads x 4).
__global__ __launch_bounds__(256) void k_scan_block(const int32_t *in, int32_t *out, int64_t n,
                                                    int32_t *block_sums) {
    __shared__ int32_t sh[256];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * 1024 + tid * 4;
    int32_t v[4];
    int32_t sum = 0;
    for (int j = 0; j < 4; ++j) {
        v[j] = base + j < n ? in[base + j] : 0;
        sum += v[j];
    }
    sh[tid] = sum;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int32_t x = tid >= o ? sh[tid - o] : 0;
        __syncthreads();
        sh[tid] += x;
        __syncthreads();
    }
    int32_t run = sh[tid] - sum;  // exclusive prefix of this thread
    for (int j = 0; j < 4; ++j) {
        if (base + j < n) out[base + j] = run;
        run += v[j];
    }
    if (tid == 255 && block_sums) block_sums[blockIdx.x] = sh[255];
}

__global__ void k_scan_add(int32_t *out, int64_t n, const int32_t *block_off) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += block_off[i / 1024];
}

static hipError_t exclusive_scan(const int32_t *in, int32_t *out, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + 1023) / 1024;
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_block, dim3(1), dim3(256), 0, s, in, out, n, (int32_t *)nullptr);
        return hipGetLastError();
    }
    int32_t *sums = nullptr, *offs = nullptr;
    hipError_t e = hipMallocAsync((void **)&sums, nb * sizeof(int32_t), s);
    if (e != hipSuccess) return e;
    e = hipMallocAsync((void **)&offs, nb * sizeof(int32_t), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_block, dim3(nb), dim3(256), 0, s, in, out, n, sums);
    e = exclusive_scan(sums, offs, nb, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_scan_add, dim3((n + 255) / 256), dim3(256), 0, s, out, n, offs);
        e = hipGetLastError();
    }
    hipFreeAsync(sums, s);
    hipFreeAsync(offs, s);
    return e;
}

// 3a. Node fields of every representative.
__global__ void k_emit_nodes(const uint2 *tok, const int32_t *canon, const int32_t *pos,
                             const int32_t *height, int64_t T, int32_t *node_op, float *node_value,
                             int32_t *node_height) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T || canon[t] != (int32_t)t) return;
    const int32_t id = pos[t];
    const uint2 w = tok[t];
    const uint32_t op = w.x & 0xffu;
    node_op[id] = (int32_t)(op == TGP_VAR ? (op | (w.x & 0xff00u)) : op);
    node_value[id] = op == TGP_CONST ? __uint_as_float(w.y) : 0.0f;
    node_height[id] = height[t];
}

// 3b. Children ids, in-degrees and multiplicities.
// Block-level counts: an open-addressing table in LDS of (id, count), filled
// with LDS atomics and flushed to the device counters with one atomic per
// distinct id of the block.  An id that finds no free entry within a few
// probes goes straight to its device counter.
constexpr int kCountSlots = 1024;  // at most 256 + 768 distinct ids per block of 256
struct BlockCounts {
    int32_t id[kCountSlots];
    int32_t n[kCountSlots];
};

__device__ __forceinline__ void block_counts_clear(BlockCounts &c) {
    for (int e = threadIdx.x; e < kCountSlots; e += blockDim.x) {
        c.id[e] = -1;
        c.n[e] = 0;
    }
}

__device__ __forceinline__ void block_counts_add(BlockCounts &c, int32_t *counter, int32_t id, int32_t k) {
    uint32_t h = ((uint32_t)id * 2654435761u) & (kCountSlots - 1);
    for (int probe = 0; probe < 8; ++probe) {
        const int32_t prev = atomicCAS(&c.id[h], -1, id);
        if (prev == -1 || prev == id) {
            atomicAdd(&c.n[h], k);
            return;
        }
        h = (h + 1) & (kCountSlots - 1);
    }
    atomicAdd(&counter[id], k);
}

__device__ __forceinline__ void block_counts_flush(const BlockCounts &c, int32_t *counter) {
    for (int e = threadIdx.x; e < kCountSlots; e += blockDim.x)
        if (c.id[e] >= 0) atomicAdd(&counter[c.id[e]], c.n[e]);
}

// Adds 1 for every lane whose id >= 0: lanes of a wave with equal ids are
// grouped by ballots (the loop runs once per distinct id, wave-uniform) and
// add their count through the group's lowest lane into the block's table.
// The shared leaves (x, y and common constants) are counted by many tokens
// of every wave; one device atomic per lane serialised on their few
// addresses.
__device__ __forceinline__ void add_one_per_lane(BlockCounts &c, int32_t *counter, int32_t id) {
    const int lane = (int)(threadIdx.x & 63u);
    uint64_t todo = __ballot(id >= 0);
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int32_t lid = __shfl(id, leader);
        const uint64_t same = __ballot(id == lid) & todo;
        if (lane == leader) block_counts_add(c, counter, lid, (int32_t)__popcll(same));
        todo &= ~same;
    }
}

// Blocks of four waves: a block of many waves waits for that many free wave
// slots on one compute unit, which it rarely finds while a long evaluation
// kernel runs beside it (DAGs are built on side streams when serving).
constexpr int kEmitBlock = 256;

__global__ __launch_bounds__(kEmitBlock) void k_emit_edges(const int32_t *canon, const int32_t *pos,
                                                           const int32_t *kid, int64_t T, int32_t *node_kid,
                                                           int32_t *indeg, int32_t *mult) {
    __shared__ BlockCounts cm, ci;
    block_counts_clear(cm);
    block_counts_clear(ci);
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // every lane reaches the ballots and barriers; lanes past T take part
    // with id -1 (nothing to count)
    const int32_t c = t < T ? canon[t] : -1;
    const int32_t id = c >= 0 ? pos[c] : -1;
    add_one_per_lane(cm, mult, id);
    const bool rep = c == (int32_t)t && t < T;  // the token that represents node id
    for (int j = 0; j < 3; ++j) {
        const int32_t k = rep ? kid[3 * t + j] : -1;
        const int32_t kid_id = k < 0 ? -1 : pos[canon[k]];
        if (rep) node_kid[3 * id + j] = kid_id;
        add_one_per_lane(ci, indeg, kid_id);
    }
    __syncthreads();
    block_counts_flush(cm, mult);
    block_counts_flush(ci, indeg);
}

__global__ void k_emit_roots(const int32_t *root_tok, const int32_t *canon, const int32_t *pos,
                             int64_t R, int32_t *roots) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < R) roots[r] = pos[canon[root_tok[r]]];
}

static inline dim3 grid_for(int64_t n, int b = 256) { return dim3((unsigned)((n + b - 1) / b)); }

void dag_device_free(DagDevice *d, DevicePool &pool) {
    pool.release(d->blob);
    *d = DagDevice{};
}

#define DCHK(x)                                                                  \
    do {                                                                         \
        hipError_t _e = (x);                                                     \
        if (_e != hipSuccess) {                                                  \
            snprintf(err, errlen, "%s: %s", #x, hipGetErrorString(_e));          \
            res.status = TGP_EHIP;                                               \
            goto done;                                                           \
        }                                                                        \
    } while (0)

uint32_t g_debug_hash_bits = 0;  // set by tests to force hash collisions

DagBuildResult build_dag_device(const tgp_token *tok_dev, const int64_t *off_dev, int64_t R,
                                int64_t T, DagDevice *dev, DevicePool &pool, hipStream_t s,
                                char *err, size_t errlen, bool commute, bool rewrite) {
    DagBuildResult res{};
    res.status = TGP_OK;
    res.bad_tree = -1;
    res.T = T;
    const uint2 *tok = reinterpret_cast<const uint2 *>(tok_dev);
    int32_t *kid = nullptr, *height = nullptr, *stk = nullptr, *root_tok = nullptr;
    int32_t *canon = nullptr, *table = nullptr, *cnt = nullptr, *list = nullptr, *flag = nullptr,
            *pos = nullptr;
    BuildStatus *st = nullptr;
    BuildStatus hs{};
    std::vector<int32_t> hcnt;
    uint64_t cap = 1024;
    int64_t U = 0;
    *dev = DagDevice{};
    dev->T = T;
    dev->R = R;
    while (cap < (uint64_t)(2 * T)) cap <<= 1;

    DCHK(pool.alloc((void **)&kid, sizeof(int32_t) * 3 * T));
    DCHK(pool.alloc((void **)&height, sizeof(int32_t) * T));
    DCHK(pool.alloc((void **)&stk, sizeof(int32_t) * T));
    DCHK(pool.alloc((void **)&root_tok, sizeof(int32_t) * R));
    DCHK(pool.alloc((void **)&st, sizeof(BuildStatus)));
    hs.first_error = ~0ull;
    hs.max_height = 0;
    hs.max_var = -1;
    hs.max_stack = 0;
    hs.n_internal = 0;
    hs.lost_key = 0;
    DCHK(hipMemcpyAsync(st, &hs, sizeof(hs), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_structure, grid_for(R, 64), dim3(64), 0, s, tok, off_dev, R, T, kid,
                       height, stk, root_tok, st);
    DCHK(hipGetLastError());
    DCHK(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
    DCHK(hipStreamSynchronize(s));
    if (hs.first_error != ~0ull) {
        const int code = (int)(hs.first_error & 15ull);
        res.bad_tree = (int64_t)(hs.first_error >> 4);
        res.status = code == ERR_OP ? TGP_EOP : (code == ERR_PARSE ? TGP_EPARSE : TGP_EINVAL);
        snprintf(err, errlen, "tree %lld: %s", (long long)res.bad_tree,
                 code == ERR_OP ? "unknown opcode"
                                : (code == ERR_PARSE ? "token range is not exactly one postfix tree"
                                                     : "offsets out of range or decreasing"));
        goto done;
    }
    res.max_height = hs.max_height;
    res.max_stack = hs.max_stack;
    res.max_var = hs.max_var;
    res.tree_internal = hs.n_internal;
    {
        const int64_t H = hs.max_height + 1;
        DCHK(pool.alloc((void **)&cnt, sizeof(int32_t) * H));
        DCHK(hipMemsetAsync(cnt, 0, sizeof(int32_t) * H, s));
        const bool lds = H <= kLvlBins;
        if (lds)
            hipLaunchKernelGGL(k_level_hist_lds, grid_for(T, 256 * kLvlPer), dim3(256), 0, s, height, T,
                               (int32_t)H, cnt);
        else
            hipLaunchKernelGGL(k_level_hist, grid_for(T), dim3(256), 0, s, height, T, cnt);
        DCHK(hipGetLastError());
        hcnt.resize(H);
        DCHK(hipMemcpyAsync(hcnt.data(), cnt, sizeof(int32_t) * H, hipMemcpyDeviceToHost, s));
        DCHK(hipStreamSynchronize(s));
        std::vector<int32_t> start(H + 1, 0);
        for (int64_t h = 0; h < H; ++h) start[h + 1] = start[h] + hcnt[h];
        DCHK(hipMemcpyAsync(cnt, start.data(), sizeof(int32_t) * H, hipMemcpyHostToDevice, s));
        DCHK(pool.alloc((void **)&list, sizeof(int32_t) * T));
        if (lds)
            hipLaunchKernelGGL(k_level_scatter_lds, grid_for(T, 256 * kLvlPer), dim3(256), 0, s, height,
                               T, (int32_t)H, cnt, list);
        else
            hipLaunchKernelGGL(k_level_scatter, grid_for(T), dim3(256), 0, s, height, T, cnt, list);
        DCHK(hipGetLastError());
        DCHK(pool.alloc((void **)&canon, sizeof(int32_t) * T));
        DCHK(pool.alloc((void **)&table, sizeof(int32_t) * cap));
        DCHK(hipMemsetAsync(table, 0xff, sizeof(int32_t) * cap, s));
        for (int64_t h = 0; h < H; ++h) {
            const int32_t n = hcnt[h];
            if (!n) continue;
            const int32_t *lst = list + start[h];
            hipLaunchKernelGGL(k_hash_insert, grid_for(n), dim3(256), 0, s, lst, n, tok, kid, canon,
                               table, (uint64_t)(cap - 1), g_debug_hash_bits, commute, rewrite);
            hipLaunchKernelGGL(k_hash_resolve, grid_for(n), dim3(256), 0, s, lst, n, tok, kid,
                               canon, table, (uint64_t)(cap - 1), g_debug_hash_bits, commute, rewrite, st);
        }
        DCHK(hipGetLastError());
        hipLaunchKernelGGL(k_class_to_token, grid_for(T), dim3(256), 0, s, canon, T, table);
        DCHK(hipGetLastError());
        DCHK(pool.alloc((void **)&flag, sizeof(int32_t) * T));
        DCHK(pool.alloc((void **)&pos, sizeof(int32_t) * T));
        hipLaunchKernelGGL(k_flags, grid_for(T), dim3(256), 0, s, canon, T, flag);
        DCHK(exclusive_scan(flag, pos, T, s));
        int32_t last[2] = {0, 0};
        DCHK(hipMemcpyAsync(&last[0], pos + T - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        DCHK(hipMemcpyAsync(&last[1], flag + T - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        DCHK(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
        DCHK(hipStreamSynchronize(s));
        if (hs.lost_key) {
            res.status = TGP_EHIP;
            snprintf(err, errlen, "hash-consing found no table slot for a subtree (internal error)");
            goto done;
        }
        U = (int64_t)last[0] + last[1];
        res.U = U;
        dev->U = U;
        // One block, in the order of DagDevice::blob_bytes: op, value, kid[3],
        // height, mult, indeg (U each), roots (R).
        DCHK(pool.alloc((void **)&dev->blob, DagDevice::blob_bytes(U, R)));
        dev->node_op = dev->blob;
        dev->node_value = reinterpret_cast<float *>(dev->blob + U);
        dev->node_kid = dev->blob + 2 * U;
        dev->node_height = dev->blob + 5 * U;
        dev->mult = dev->blob + 6 * U;
        dev->indeg = dev->blob + 7 * U;
        dev->roots = dev->blob + 8 * U;
        DCHK(hipMemsetAsync(dev->mult, 0, sizeof(int32_t) * 2 * U, s));
        hipLaunchKernelGGL(k_emit_nodes, grid_for(T), dim3(256), 0, s, tok, canon, pos, height, T,
                           dev->node_op, dev->node_value, dev->node_height);
        hipLaunchKernelGGL(k_emit_edges, grid_for(T, kEmitBlock), dim3(kEmitBlock), 0, s, canon, pos, kid, T,
                           dev->node_kid, dev->indeg, dev->mult);
        hipLaunchKernelGGL(k_emit_roots, grid_for(R), dim3(256), 0, s, root_tok, canon, pos, R,
                           dev->roots);
        DCHK(hipGetLastError());
    }
done:
    hipStreamSynchronize(s);  // every kernel that used the scratch has finished
    pool.release(kid);
    pool.release(height);
    pool.release(stk);
    pool.release(root_tok);
    pool.release(st);
    pool.release(cnt);
    pool.release(list);
    pool.release(canon);
    pool.release(table);
    pool.release(flag);
    pool.release(pos);
    if (res.status != TGP_OK) dag_device_free(dev, pool);
    return res;
}

}  // namespace tgp
