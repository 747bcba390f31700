// tgp_internal.h -- definitions shared by the host runtime and the HIP
// kernels of libtgp (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <unordered_map>
#include <vector>

#include "../../include/tgp.h"
#include "div_magic.h"

namespace tgp {

// Arity of each public opcode (Table 1), shared by the host tables and the
// device constant table of the DAG builder.
#define TGP_ARITY_LIST                                                 \
    0, 0,                         /* var const */                      \
        2, 2, 2, 2,               /* add sub mult div */               \
        1, 1, 1,                  /* sin cos tan */                    \
        1, 1, 2,                  /* exp log pow */                    \
        2, 2, 2, 1,               /* min max mdist neg */              \
        1, 1, 1, 3,               /* sqrt sign abs clip */             \
        2, 1, 3,                  /* mod frac if */                    \
        1, 1, 1, 2, 3,            /* step sstep sstepp len lerp */     \
        2, 2, 2,                  /* or xor and */                     \
        3                         /* warp */

constexpr int kArityList[] = {TGP_ARITY_LIST};
static_assert(sizeof(kArityList) / sizeof(int) == TGP_NUM_OPS, "one arity per opcode");
constexpr int kArity[TGP_NUM_OPS] = {TGP_ARITY_LIST};

// The same arities packed two bits per opcode into one 64-bit constant, so
// that device code looks an arity up with a shift instead of a memory load
// (a per-lane load from a constant table is a vector memory load, and its
// wait also waits for every vector load issued before it).
constexpr uint64_t pack_arities() {
    uint64_t r = 0;
    for (int i = 0; i < TGP_NUM_OPS; ++i) r |= (uint64_t)kArityList[i] << (2 * i);
    return r;
}
constexpr uint64_t kArityPacked = pack_arities();
static_assert(TGP_NUM_OPS <= 32, "two bits per opcode in 64 bits");
// Arity of a valid opcode (op < TGP_NUM_OPS).
__host__ __device__ constexpr int arity_of(uint32_t op) { return (int)((kArityPacked >> (2 * op)) & 3u); }

// Interpreter instructions.  An instruction is a uint2.  .x = (S << 8) |
// code, where S is the depth of the operand stack before the instruction
// (the emitter knows it; the register-stack interpreter dispatches on the
// whole word, the LDS-stack one on code alone).  .y = the FP32 bits of a
// constant (I_CONST, constant-operand fused forms), a cache row (I_CACHE,
// I_WARP, cache-operand fused forms: the row starts cache_stride floats
// times .y past the job's cache base), or the kind of a bitwise operator
// (0 or, 1 xor, 2 and; the three share the code of TGP_OR).  Function codes
// are the public opcode plus kFnBase.  Operators whose children were
// evaluated out of left-to-right order (to bound the stack, Sethi-Ullman
// order) use the permuted forms: kRevBase + op for a reversed
// non-commutative binary operator, kPermBase + 6 t + p for ternary operator
// t (clip, if, lerp) whose children were evaluated in the order kPerms[p].
// Fused forms (superinstructions): a binary operator whose last-evaluated
// operand is x, y, a constant or a cache row reads that operand itself,
// code kFuseBase + 16 * kind + v, with kind one of kFuseX .. kFuseCache and
// v the index of (operator, reversed) in kFuseOps / kFuseRev; reversed
// means the terminal is the operator's first operand.  A fused form at depth
// S reads slot S - 1 and writes it.
enum : uint32_t {
    I_X = 0, I_Y = 1, I_Z = 2, I_CONST = 3, I_CACHE = 4, I_END = 5,
    I_WARP = 6,  // pops t0, t1; pushes cache row .y at the point they name
    kFnBase = 8,
    kRevBase = 40,
    kPermBase = 72,
    kFuseBase = 96,
    kFuseX = 0, kFuseY = 1, kFuseConst = 2, kFuseCache = 3,
};
constexpr int kNumFused = 14;
constexpr int kFuseOps[kNumFused] = {TGP_ADD, TGP_SUB, TGP_MULT, TGP_DIV, TGP_POW, TGP_MIN,  TGP_MAX,
                                     TGP_MDIST, TGP_MOD, TGP_LEN, TGP_SUB, TGP_DIV, TGP_POW, TGP_MOD};
constexpr bool kFuseRev[kNumFused] = {false, false, false, false, false, false, false,
                                      false, false, false, true,  true,  true,  true};

// Index v of (op, reversed) in kFuseOps / kFuseRev, or -1 if it has no
// fused form.
inline int fused_index(int op, bool rev) {
    for (int v = 0; v < kNumFused; ++v)
        if (kFuseOps[v] == op && kFuseRev[v] == rev) return v;
    return -1;
}
// The code of an instruction word.
__host__ __device__ constexpr uint32_t ins_code(uint32_t x) { return x & 0xffu; }
// Whether the instruction's .y names a cache row.
inline bool reads_cache_row(uint32_t x) {
    const uint32_t c = ins_code(x);
    return c == I_CACHE || c == I_WARP || (c >= kFuseBase + 16 * kFuseCache && c < kFuseBase + 16 * (kFuseCache + 1));
}

constexpr uint8_t kPerms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

inline bool is_commutative(int op) {
    return op == TGP_ADD || op == TGP_MULT || op == TGP_MIN || op == TGP_MAX || op == TGP_MDIST ||
           op == TGP_LEN || op == TGP_OR || op == TGP_XOR || op == TGP_AND;
}
inline int ternary_index(int op) {
    return op == TGP_CLIP ? 0 : (op == TGP_IF ? 1 : (op == TGP_LERP ? 2 : -1));
}

// One program of the interpreter: a postfix instruction stream that leaves a
// single value per case.  dest is the cache slot (cache fill), the output row
// (evaluate) or the partial-sum row (fitness); chan is the target channel.
struct ProgDesc {
    uint32_t code_off;
    uint32_t len;
    int32_t dest;
    int32_t chan;
};

// Everything a work item needs to know about the domain and the buffers of
// the evaluation it belongs to.
// A job covers the n_cases consecutive cases of the domain that start at
// case case_base (all of it, or one slab of it); every per-case array below
// is indexed by the global case index case_base + i.
struct JobDesc {
    const uint2 *code;           // all instructions of the job, then one I_END
    int32_t n_stripes;           // work items per program
    int32_t tiles_per_stripe;    // tiles of 64*K cases per work item
    int32_t n_cases;             // cases of the job
    int32_t case_base;           // global index of its first case
    int32_t ndim;
    int32_t shape[3];
    int32_t stride[3];
    uint32_t div_m[2], div_s[2]; // multiply-shift division by stride[0], stride[1] (div_magic.h)
    const float *coord[3];       // per-axis coordinate tables of the whole domain
    const float *cache;          // I_CACHE row r: cache + r * cache_stride
    float *out;                  // STORE: row dest at out + dest * out_stride
    const float *target;         // REDUCE: channel chan at target + chan * target_stride
    float2 *partial;             // REDUCE: [dest][n_stripes] (sum, compensation)
    int64_t cache_stride, out_stride, target_stride;
    float warp_lo[2], warp_scale[2]; // warp: axis k position of t is (t - lo) * scale
};

// Launch arguments of the plain (one program set, one domain) interpreter:
// work item i is program i / n_stripes, stripe i % n_stripes.
struct InterpArgs {
    JobDesc job;
    const ProgDesc *progs;
    int32_t n_progs;
};

// Batched evaluation: a pair is one program of one job; its work items are
// item_first[p] .. item_first[p + 1] - 1 (one per stripe).  A group is a
// contiguous range of pairs evaluated by one launch.
struct PairDesc {
    int32_t job;
    uint32_t code_off;
    int32_t dest;
    int32_t chan;
};

struct GroupDesc {
    uint32_t pair_begin, pair_end;
    uint32_t item_begin, item_end;
};

// Finalize of one job in a batch.  Without acc the job covers the whole
// domain and out receives the loss.  With acc (one FP64 running sum per
// individual, a job over one slab of the domain) the slab's sum is added to
// acc, and on the last slab the loss of the total goes to out.
struct FinJob {
    const float2 *partial;
    const int32_t *ind_rows;
    double *out;
    double *acc;
    double n_terms;
    int32_t n_ch;
    int32_t n_stripes;
    int32_t loss;
    uint32_t ind_begin;          // first global individual index of the job
    int32_t first;               // acc holds nothing yet (first slab)
    int32_t last;
};

// Instantiated kernel variants (cases per lane K, stack registers D).
struct Variant {
    int K;
    int D;
};

// ext: the interpreter that also knows the bitwise operators and warp (only
// K = 4).
hipError_t launch_interp(int K, int D, bool store, const InterpArgs &a, hipStream_t s, bool bit);
// Batched interpreter kernels (for graph nodes): the persistent form takes
// (jobs, pairs, item_first, groups, g, counters[groups x batch_parts()]),
// the direct form (jobs, pairs, item_first, groups, g) with one wave per item.
const void *batch_kernel(int K, int D, bool store, bool persistent, bool bit);
int batch_grid(int K, int D, bool store, bool bit);  // resident waves of the persistent form
uint32_t batch_parts();
const void *reset_kernel();           // (uint32_t *counters, int32_t n)
const void *finalize_batch_kernel();  // (const FinJob *, const int32_t *n_jobs, const uint32_t *n_ind)
hipError_t launch_reset(uint32_t *counters, int32_t n, hipStream_t s);
// Constant folding over the DAGs of a batch: evaluates the n (DAG, node)
// entries of `list` (one height) into each DAG's val (indexed by node id).
struct FoldDesc {
    const int32_t *node_op;
    const float *node_value;
    const int32_t *node_kid;
    float *val;
};
hipError_t launch_fold_level(const FoldDesc *jobs, const int2 *list, int32_t n, hipStream_t s);
hipError_t launch_finalize_batch(const FinJob *jobs, const int32_t *n_jobs, const uint32_t *n_ind,
                                 int32_t grid, hipStream_t s);
#ifdef __HIPCC__
// Calls f(i, token i) for the tokens of [lo, hi) in order (REV: from hi - 1
// down to lo), reading them N at a time with the next N in flight, until f
// returns false; returns whether every token was visited.  Per-tree scans
// (one thread per tree) use it so that each token's load does not stall the
// scan's dependent steps.  Two buffers alternate (a copy from the in-flight
// buffer would wait for it), and every load is unconditional, at an index
// clamped into [lo, hi) (a branch around each load hides from the compiler
// which loads are outstanding, and it then waits for all of them).
template <int N, bool REV, typename F>
__device__ __forceinline__ bool for_tokens(const uint2 *tok, int64_t lo, int64_t hi, F &&f) {
    if (hi <= lo) return true;
    uint2 a[N], b[N];
    auto at = [&](int64_t base, int j) { return REV ? base - j : base + j; };
    auto ok = [&](int64_t i) { return i >= lo && i < hi; };
    auto load = [&](uint2 (&buf)[N], int64_t base) {
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const int64_t i = at(base, j);
            buf[j] = tok[i < lo ? lo : (i >= hi ? hi - 1 : i)];
        }
    };
    auto run = [&](const uint2 (&buf)[N], int64_t base) {
#pragma unroll
        for (int j = 0; j < N; ++j)
            if (ok(at(base, j)) && !f(at(base, j), buf[j])) return false;
        return true;
    };
    int64_t base = REV ? hi - 1 : lo;
    load(a, base);
    for (;;) {
        const int64_t nb = at(base, N);
        load(b, nb);
        if (!run(a, base)) return false;
        if (!ok(nb)) return true;
        const int64_t nb2 = at(nb, N);
        load(a, nb2);
        if (!run(b, nb)) return false;
        if (!ok(nb2)) return true;
        base = nb2;
    }
}
#endif

// Genetic operators (k_breed.hip).  A child tree is the first parent's
// tokens [a0, cut_lo) + a middle part of `mid` tokens + [cut_hi, a1); the
// middle is the second parent's tokens from b_lo (splice) or a new random
// subtree regenerated from draw sub_k of the offspring's stream (mutate).
constexpr int kMaxMutationDepth = 16;
enum { kBreedCopy = 0, kBreedSplice = 1, kBreedMutate = 2 };
struct BreedRec {
    int64_t a0, a1, cut_lo, cut_hi, b_lo;
    int32_t mid, kind;
    uint32_t sub_k;
    int32_t sub_depth, sub_full, pad;
};
struct BreedArgs {
    const uint2 *tok;          // parent tokens
    const int64_t *off;        // parent offsets
    const int32_t *size, *height, *depth;  // shape of every parent token
    const double *fitness;     // [n_parents] or nullptr
    const uint8_t *functions;  // [n_functions] operator codes (device)
    BreedRec *recs;            // [n_offspring * n_channels]
    int64_t *lens;             // [n_offspring * n_channels]
    uint64_t seed;
    double p_crossover, p_mutation;
    int32_t n_parents, n_channels, n_offspring, tournament, max_depth, max_mutation_depth, tries;
    int32_t ndim, use_constants, n_functions;
};
hipError_t launch_shape(const uint2 *tok, const int64_t *off, int64_t R, int64_t T, int32_t *size,
                        int32_t *height, int32_t *depth, int32_t *bad, hipStream_t s);
// Decisions, then the exclusive scan of the child lengths into out_off
// (n_offspring * n_channels + 1 entries; block_sum holds breed_scan_blocks
// entries, at least one).
hipError_t launch_breed(const BreedArgs &A, const int32_t *bad, int64_t *out_off, int64_t *block_sum,
                        hipStream_t s);
int64_t breed_scan_blocks(int64_t n);
hipError_t launch_breed_write(const BreedArgs &A, const int64_t *out_off, uint2 *out_tok, hipStream_t s);
bool interp_variant_exists(int K, int D, bool bit = false);
int interp_max_stack();   // register stack slots
int interp_lds_stack();   // LDS stack slots (the other stack form, K = 2)

// Finalize: per individual, FP64 sum of its channels' partial rows.
hipError_t launch_finalize(const float2 *partial, const int32_t *ind_rows, int32_t n_ind,
                           int32_t n_ch, int32_t n_stripes, double n_terms, int32_t loss,
                           double *out, hipStream_t s);

// A caching allocator of device memory: blocks are kept by power-of-two size
// class and handed out again instead of being freed, so that building DAGs
// and plans step after step does not pay hipMalloc/hipFree (hipFree also
// waits for the whole device).  Blocks are only released to the pool once
// the work that used them is known to be complete (the callers synchronise
// their stream first).  Owned by one context, used by one thread.
struct DevicePool {
    std::vector<std::vector<void *>> free_;
    std::unordered_map<void *, int> cls_;
    static int class_of(size_t bytes) {
        int c = 8;  // 256 bytes minimum
        while (((size_t)1 << c) < bytes) ++c;
        return c;
    }
    hipError_t alloc(void **p, size_t bytes) {
        const int c = class_of(bytes);
        if ((int)free_.size() <= c) free_.resize(c + 1);
        if (!free_[c].empty()) {
            *p = free_[c].back();
            free_[c].pop_back();
            return hipSuccess;
        }
        hipError_t e = hipMalloc(p, (size_t)1 << c);
        if (e == hipSuccess) cls_[*p] = c;
        return e;
    }
    void release(void *p) {
        if (!p) return;
        auto it = cls_.find(p);
        if (it == cls_.end()) return;
        free_[it->second].push_back(p);
    }
    // Frees every block ever handed out (the owner is going away).
    void drain() {
        for (auto &kv : cls_) hipFree(kv.first);
        cls_.clear();
        free_.clear();
    }
};

// DAG construction kernels (k_dag.hip).
struct DagDevice {
    int64_t T = 0, R = 0, U = 0;
    int32_t *blob = nullptr;         // one pool block holding every array below
    int32_t *node_op = nullptr;      // packed per node: op | var << 8
    float *node_value = nullptr;
    int32_t *node_kid = nullptr;     // [U][3]
    int32_t *node_height = nullptr;
    int32_t *roots = nullptr;        // [R]
    int32_t *mult = nullptr;         // [U]
    int32_t *indeg = nullptr;        // [U]
    static size_t blob_bytes(int64_t U, int64_t R) { return sizeof(int32_t) * (8 * U + R); }
};

struct DagBuildResult {
    int status;        // tgp_status
    int64_t bad_tree;  // offending tree for EPARSE/EOP/EINVAL
    int64_t T, U, max_height, max_stack, max_var, tree_internal;
};

// Builds the DAG of R trees given device tokens/offsets; allocates the dev
// arrays from the pool (returned with dag_device_free once the stream has
// passed every use).
// commute: identify nodes of operators whose operands commute by the
// unordered pair of their children; rewrite: apply the identity rewrites
// (tgp_ctx_set_rewrite).
DagBuildResult build_dag_device(const tgp_token *tok_dev, const int64_t *off_dev, int64_t R,
                                int64_t T, DagDevice *dev, DevicePool &pool, hipStream_t s,
                                char *err, size_t errlen, bool commute, bool rewrite);
void dag_device_free(DagDevice *dev, DevicePool &pool);

}  // namespace tgp
