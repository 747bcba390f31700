// k_breed.hip -- one generation of tree GP bred on the device: tournament
// selection, subtree crossover, subtree mutation and reproduction over
// postfix token arrays (the operators the paper runs on the host between
// evaluations, Sec. 4.2; their textbook form, Koza 1992).
//
// Four launches: the shape of every parent token (subtree size, height,
// depth from the root), the decisions of every offspring (one thread each,
// drawing from its own counter-based stream, writing one record and the
// length of each child tree), an exclusive scan of the lengths into the
// offspring offsets, and the copy of the child trees (one wave per child:
// coalesced copies of the kept parts of the first parent and of the second
// parent's subtree; a mutation's new subtree is regenerated from its
// recorded position in the stream by lane 0).
#include <hip/hip_runtime.h>

#include "tgp_internal.h"

namespace tgp {

namespace {

// SplitMix64 (Steele, Lea & Flood 2014) as a counter-based generator:
// output n of the generator started from `seed`.
__device__ inline uint64_t splitmix64(uint64_t seed, uint64_t n) {
    uint64_t z = seed + n * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// The draws of one offspring o: draw k is output o * 2^32 + k + 1.
struct Draws {
    uint64_t seed, base;
    uint32_t k;
    __device__ uint64_t next() { return splitmix64(seed, base + (uint64_t)k++ + 1); }
    // floor(x * m / 2^64): multiply-shift, no rejection
    __device__ uint32_t below(uint64_t m) { return (uint32_t)__umul64hi(next(), m); }
    __device__ double uniform() { return (double)(next() >> 11) * 0x1p-53; }
    // fl32(2u - 1), u = 24 random bits / 2^24 (exact in FP32)
    __device__ float constant() {
        const double u = (double)(next() >> 40) * 0x1p-24;
        return (float)(2.0 * u - 1.0);
    }
};

__device__ inline int tok_op(uint2 t) { return (int)(t.x & 0xffu); }

// A random tree of the given depth, full or grow: nodes chosen in
// pre-order, emitted in postfix.  Returns its token count; writes the tokens
// to out when out != nullptr.  The open function nodes are kept in a small
// stack (at most `depth` frames).
__device__ int32_t random_tree(Draws &dr, int depth, bool full, const BreedArgs &A, uint2 *out) {
    uint8_t st_op[kMaxMutationDepth + 1];
    uint8_t st_left[kMaxMutationDepth + 1];
    int sp = 0;
    int32_t n = 0;
    const uint32_t nf = (uint32_t)A.n_functions;
    const uint32_t nt = (uint32_t)A.ndim + (A.use_constants ? 1u : 0u);
    auto terminal = [&](uint32_t t) {
        uint2 tk;
        if (t < (uint32_t)A.ndim) {
            tk = uint2{(uint32_t)TGP_VAR | (t << 8), 0u};
        } else {
            const float v = dr.constant();
            tk = uint2{(uint32_t)TGP_CONST, __float_as_uint(v)};
        }
        if (out) out[n] = tk;
        ++n;
    };
    for (;;) {
        // choose the node at remaining depth depth - sp
        const int d = depth - sp;
        bool leaf = true;
        if (d == 0) {
            terminal(dr.below(nt));
        } else if (full) {
            st_op[sp] = A.functions[dr.below(nf)];
            leaf = false;
        } else {
            const uint32_t j = dr.below(nf + nt);
            if (j >= nf) {
                terminal(j - nf);
            } else {
                st_op[sp] = A.functions[j];
                leaf = false;
            }
        }
        if (!leaf) {
            st_left[sp] = (uint8_t)arity_of(st_op[sp]);
            ++sp;
            continue;
        }
        // a subtree is complete: close the function nodes whose operands are all there
        while (sp > 0) {
            if (--st_left[sp - 1] > 0) break;
            --sp;
            if (out) out[n] = uint2{(uint32_t)st_op[sp], 0u};
            ++n;
        }
        if (sp == 0) return n;
    }
}

// Fitness for selection: non-finite counts as +inf; no fitness: all equal.
__device__ inline double sel_fit(const double *fit, uint32_t i) {
    if (!fit) return 0.0;
    const double f = fit[i];
    return isfinite(f) ? f : __builtin_inf();
}

__device__ inline uint32_t tournament(Draws &dr, const BreedArgs &A) {
    uint32_t best = dr.below((uint64_t)A.n_parents);
    double fb = sel_fit(A.fitness, best);
    for (int t = 1; t < A.tournament; ++t) {
        const uint32_t c = dr.below((uint64_t)A.n_parents);
        const double fc = sel_fit(A.fitness, c);
        if (fc < fb) {
            best = c;
            fb = fc;
        }
    }
    return best;
}

// Shape of one tree in global memory (the fallback for trees whose operand
// stack outgrows the LDS stack): subtree size and height from the operands
// (the last operand ends just before its parent, each earlier one just
// before the next), then the depth from the root, parents before children.
// Returns 0, 1 (malformed) or 2 (unknown operator).
__device__ int shape_global(const uint2 *tok, int64_t o0, int64_t o1, int32_t *size, int32_t *height,
                            int32_t *depth) {
    for (int64_t i = o0; i < o1; ++i) {
        const int op = tok_op(tok[i]);
        if (op >= TGP_NUM_OPS) return 2;
        int32_t s = 1, h = 0;
        int64_t c = i - 1;
        for (int j = 0; j < arity_of(op); ++j) {
            if (c < o0) return 1;
            s += size[c];
            h = max(h, height[c] + 1);
            c -= size[c];
        }
        size[i] = s;
        height[i] = h;
    }
    if (size[o1 - 1] != (int32_t)(o1 - o0)) return 1;
    depth[o1 - 1] = 0;
    for (int64_t i = o1 - 1; i >= o0; --i) {
        const int32_t d = depth[i] + 1;
        int64_t c = i - 1;
        for (int j = 0; j < arity_of(tok_op(tok[i])); ++j) {
            depth[c] = d;
            c -= size[c];
        }
    }
    return 0;
}

constexpr int kShapeStack = 32;  // LDS operand-stack entries per thread

// Shape of every token, one thread per tree.  Forward, an operand stack of
// (size, height) pairs in LDS gives each token's subtree size and height
// from its operands' entries; backward from the root, a stack of (depth of
// the children, children still to come) frames gives each token's depth.
// Both stacks hold at most the tree's postfix stack depth; a tree that needs
// more than kShapeStack entries is redone with shape_global.  A tree that is
// not exactly one postfix tree, or holds an unknown operator, raises *bad
// (1 = malformed, 2 = operator).
__global__ __launch_bounds__(64) void k_shape(const uint2 *tok, const int64_t *off, int64_t R, int64_t T,
                                              int32_t *size, int32_t *height, int32_t *depth, int32_t *bad) {
    __shared__ int2 stk[kShapeStack][64];
    const int lane = threadIdx.x;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + lane;
    if (r >= R) return;
    const int64_t o0 = off[r], o1 = off[r + 1];
    if (o0 < 0 || o1 <= o0 || o1 > T) {
        atomicMax(bad, 1);
        return;
    }
    int sp = 0, verdict = 0;
    bool overflow = false;
    for_tokens<8, false>(tok, o0, o1, [&](int64_t i, uint2 w) {
        const int op = tok_op(w);
        if (op >= TGP_NUM_OPS) {
            verdict = 2;
            return false;
        }
        const int a = arity_of(op);
        if (sp < a) {
            verdict = 1;
            return false;
        }
        int32_t s = 1, h = 0;
        for (int j = 0; j < a; ++j) {
            const int2 e = stk[--sp][lane];
            s += e.x;
            h = max(h, e.y + 1);
        }
        size[i] = s;
        height[i] = h;
        if (sp == kShapeStack) {
            overflow = true;
            return false;
        }
        stk[sp++][lane] = int2{s, h};
        return true;
    });
    if (verdict) {
        atomicMax(bad, verdict);
        return;
    }
    if (overflow) {
        const int v = shape_global(tok, o0, o1, size, height, depth);
        if (v) atomicMax(bad, v);
        return;
    }
    if (sp != 1) {
        atomicMax(bad, 1);
        return;
    }
    // backward: frames (depth of the children, children still to come)
    sp = 0;
    for_tokens<8, true>(tok, o0, o1, [&](int64_t i, uint2 w) {
        const int a = arity_of(tok_op(w));
        int32_t d = 0;
        if (sp > 0) {
            int2 &f = stk[sp - 1][lane];
            d = f.x;
            if (--f.y == 0) --sp;
        }
        depth[i] = d;
        if (a > 0) stk[sp++][lane] = int2{d + 1, a};
        return true;
    });
}

// The decisions of one offspring (one thread each): operator, parents, and
// for each channel tree the parts of the child and its length.
__global__ void k_breed_plan(BreedArgs A, const int32_t *bad) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= A.n_offspring) return;
    const int nch = A.n_channels;
    if (*bad) {  // malformed parents: no offspring tokens; the host reports it
        for (int ch = 0; ch < nch; ++ch) A.lens[o * nch + ch] = 0;
        return;
    }
    Draws dr{A.seed, (uint64_t)o << 32, 0};
    const double u = dr.uniform();
    const uint32_t p1 = tournament(dr, A);
    const bool cross = u < A.p_crossover;
    const bool mutate = !cross && u < A.p_crossover + A.p_mutation;
    const uint32_t p2 = cross ? tournament(dr, A) : 0u;
    for (int ch = 0; ch < nch; ++ch) {
        const int64_t ra = (int64_t)p1 * nch + ch;
        const int64_t a0 = A.off[ra], a1 = A.off[ra + 1];
        const int64_t la = a1 - a0;
        BreedRec rec;
        rec.a0 = a0;
        rec.a1 = a1;
        rec.cut_lo = rec.cut_hi = a1;
        rec.b_lo = 0;
        rec.mid = 0;
        rec.kind = kBreedCopy;
        rec.sub_k = 0;
        rec.sub_depth = 0;
        rec.sub_full = 0;
        if (cross) {
            const int64_t rb = (int64_t)p2 * nch + ch;
            const int64_t b0 = A.off[rb], lb = A.off[rb + 1] - b0;
            for (int t = 0; t < A.tries; ++t) {
                const int64_t i = a0 + dr.below((uint64_t)la);
                const int64_t j = b0 + dr.below((uint64_t)lb);
                if (A.depth[i] + A.height[j] <= A.max_depth) {
                    rec.kind = kBreedSplice;
                    rec.cut_lo = i - A.size[i] + 1;
                    rec.cut_hi = i + 1;
                    rec.b_lo = j - A.size[j] + 1;
                    rec.mid = A.size[j];
                    break;
                }
            }
        } else if (mutate) {
            const int64_t i = a0 + dr.below((uint64_t)la);
            const int room = max(A.max_depth - A.depth[i], 0);
            const int d = (int)dr.below((uint64_t)(min(room, A.max_mutation_depth) + 1));
            const bool full = dr.below(2) == 0;
            rec.kind = kBreedMutate;
            rec.cut_lo = i - A.size[i] + 1;
            rec.cut_hi = i + 1;
            rec.sub_k = dr.k;
            rec.sub_depth = d;
            rec.sub_full = full ? 1 : 0;
            rec.mid = random_tree(dr, d, full, A, nullptr);
        }
        A.recs[o * nch + ch] = rec;
        A.lens[o * nch + ch] = (rec.cut_lo - a0) + rec.mid + (a1 - rec.cut_hi);
    }
}

// Exclusive scan of the child lengths into offsets (n + 1 entries): blocks
// of 1024 scanned in LDS, block totals scanned by one block, then added.
constexpr int kScanBlock = 1024;

__device__ inline int64_t block_scan(int64_t v, int64_t *lds) {
    // inclusive scan of one value per thread (256 threads)
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int64_t add = threadIdx.x >= (unsigned)o ? lds[threadIdx.x - o] : 0;
        __syncthreads();
        lds[threadIdx.x] += add;
        __syncthreads();
    }
    return lds[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_scan_lens(const int64_t *in, int64_t n, int64_t *out,
                                                   int64_t *block_sum) {
    __shared__ int64_t lds[256];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * 4;
    int64_t v[4], s = 0;
    for (int j = 0; j < 4; ++j) {
        v[j] = base + j < n ? in[base + j] : 0;
        s += v[j];
    }
    const int64_t incl = block_scan(s, lds);
    int64_t run = incl - s;
    for (int j = 0; j < 4; ++j) {
        if (base + j < n) out[base + j] = run;
        run += v[j];
    }
    if (threadIdx.x == 255) block_sum[blockIdx.x] = incl;
}

// One block: exclusive scan of the block totals in chunks of 1024, and the
// grand total into out[n].
__global__ __launch_bounds__(256) void k_scan_blocks(int64_t *block_sum, int64_t nb, int64_t *out, int64_t n) {
    __shared__ int64_t lds[256];
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += kScanBlock) {
        const int64_t base = c0 + threadIdx.x * 4;
        int64_t v[4], s = 0;
        for (int j = 0; j < 4; ++j) {
            v[j] = base + j < nb ? block_sum[base + j] : 0;
            s += v[j];
        }
        const int64_t incl = block_scan(s, lds);
        int64_t run = carry + incl - s;
        for (int j = 0; j < 4; ++j) {
            if (base + j < nb) block_sum[base + j] = run;
            run += v[j];
        }
        carry += lds[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[n] = carry;
}

__global__ void k_scan_add(int64_t *out, int64_t n, const int64_t *block_sum) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += block_sum[i / kScanBlock];
}

// One wave per child tree: the kept head of the first parent, the middle
// part (the second parent's subtree, or a new subtree regenerated by lane 0
// from the recorded draw), the kept tail.
__global__ __launch_bounds__(256) void k_breed_write(BreedArgs A, const int64_t *out_off, uint2 *out_tok) {
    const int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int lane = threadIdx.x & 63;
    const int64_t n_child = (int64_t)A.n_offspring * A.n_channels;
    if (c >= n_child) return;
    const BreedRec rec = A.recs[c];
    uint2 *dst = out_tok + out_off[c];
    const int64_t head = rec.cut_lo - rec.a0;
    for (int64_t t = lane; t < head; t += 64) dst[t] = A.tok[rec.a0 + t];
    if (rec.kind == kBreedSplice) {
        for (int64_t t = lane; t < rec.mid; t += 64) dst[head + t] = A.tok[rec.b_lo + t];
    } else if (rec.kind == kBreedMutate && lane == 0) {
        Draws dr{A.seed, (uint64_t)(c / A.n_channels) << 32, rec.sub_k};
        random_tree(dr, rec.sub_depth, rec.sub_full != 0, A, dst + head);
    }
    const int64_t tail = rec.a1 - rec.cut_hi;
    for (int64_t t = lane; t < tail; t += 64) dst[head + rec.mid + t] = A.tok[rec.cut_hi + t];
}

inline dim3 grid_of(int64_t n, int b) { return dim3((unsigned)((n + b - 1) / b)); }

}  // namespace

hipError_t launch_shape(const uint2 *tok, const int64_t *off, int64_t R, int64_t T, int32_t *size,
                        int32_t *height, int32_t *depth, int32_t *bad, hipStream_t s) {
    if (R <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_shape, grid_of(R, 64), dim3(64), 0, s, tok, off, R, T, size, height, depth, bad);
    return hipGetLastError();
}

hipError_t launch_breed(const BreedArgs &A, const int32_t *bad, int64_t *out_off, int64_t *block_sum,
                        hipStream_t s) {
    const int64_t n = (int64_t)A.n_offspring * A.n_channels;
    if (A.n_offspring > 0) hipLaunchKernelGGL(k_breed_plan, grid_of(A.n_offspring, 64), dim3(64), 0, s, A, bad);
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    if (n > 0) hipLaunchKernelGGL(k_scan_lens, dim3((unsigned)nb), dim3(256), 0, s, A.lens, n, out_off, block_sum);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(256), 0, s, block_sum, nb, out_off, n);
    if (n > 0) hipLaunchKernelGGL(k_scan_add, grid_of(n, 256), dim3(256), 0, s, out_off, n, block_sum);
    return hipGetLastError();
}

int64_t breed_scan_blocks(int64_t n) { return (n + kScanBlock - 1) / kScanBlock; }

hipError_t launch_breed_write(const BreedArgs &A, const int64_t *out_off, uint2 *out_tok, hipStream_t s) {
    const int64_t n = (int64_t)A.n_offspring * A.n_channels;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_breed_write, grid_of(n * 64, 256), dim3(256), 0, s, A, out_off, out_tok);
    return hipGetLastError();
}

}  // namespace tgp
