/*
 * tgp.h -- C ABI of libtgp: whole-population genetic-programming fitness
 * evaluation on one AMD Instinct MI355X (gfx950).
 *
 * The method (TensorGP, Baeta et al.): every individual is an expression tree
 * over the primitive set of Table 1; the tree is evaluated over a fixed domain
 * of fitness cases held as an N-dimensional coordinate grid (Sec. 3.1), all
 * cases at once ("vectorisation", Sec. 1 and Sec. 2), with results of
 * intermediate subtrees cached so that code shared between individuals is not
 * executed again (Sec. 1, Sec. 3.1; the population DAG of Handley described
 * in Sec. 2), and each individual's error against a target tensor is reduced
 * to its root mean squared error (Sec. 4.1, Table 2).
 *
 * Conventions for every call:
 *   - every function returns tgp_status (TGP_OK = 0 on success) except the
 *     destroy functions and tgp_last_error; no C++ exception crosses the ABI;
 *   - arguments are validated on the host before any kernel is launched; the
 *     message of the last failure on a context is tgp_last_error(ctx);
 *   - "device pointer" means memory on the context's GPU (for instance a torch
 *     tensor's data_ptr()); it belongs to the caller and must be large enough;
 *   - host buffers passed in are only read during the call; handles belong to
 *     the library and are released by the matching *_destroy; the DAGs,
 *     domains, batches and offspring made on a context are destroyed before
 *     the context (destroying it releases their device memory; a server
 *     keeps contexts of its own and may outlive the one it was made from);
 *   - device work is ordered on the context's HIP stream and is asynchronous
 *     unless a function says it blocks;
 *   - a context is used by one host thread at a time.
 */
#ifndef TGP_H
#define TGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TGP_OK = 0,
    TGP_EINVAL = -1,  /* bad argument (null pointer, bad size, bad loss, ...) */
    TGP_EPARSE = -2,  /* a token range is not exactly one postfix tree */
    TGP_EDEPTH = -3,  /* a program cannot be fitted into the evaluator's stack */
    TGP_EOP = -4,     /* unknown opcode */
    TGP_ENOMEM = -5,  /* device or host allocation failed, or over budget */
    TGP_EHIP = -6,    /* a HIP runtime call failed (text in tgp_last_error) */
    TGP_ESHAPE = -7,  /* domain / channel / variable-axis mismatch */
    TGP_EBUSY = -8    /* timed out, or the request cannot be admitted yet */
} tgp_status;

/*
 * Opcodes: the pointwise operators of Table 1 in the paper's order, after the
 * two terminal kinds.  Arity in brackets.  Trigonometric arguments are in
 * half-turns (multiplied by pi, Sec. 3.2).  Protected forms follow Table 1;
 * where the table is silent the library uses the reading given here.
 */
enum tgp_opcode {
    TGP_VAR = 0,    /* [0] coordinate along axis `var` (0 = x, 1 = y, 2 = z) */
    TGP_CONST = 1,  /* [0] the FP32 constant `value` */
    TGP_ADD = 2,    /* [2] x + y */
    TGP_SUB = 3,    /* [2] x - y */
    TGP_MULT = 4,   /* [2] x * y */
    TGP_DIV = 5,    /* [2] x / y, 0 when y == 0 (either sign) */
    TGP_SIN = 6,    /* [1] sin(pi x) (Table 1 prints sin and cos swapped) */
    TGP_COS = 7,    /* [1] cos(pi x) */
    TGP_TAN = 8,    /* [1] sin(pi x) / cos(pi x), IEEE division at the poles */
    TGP_EXP = 9,    /* [1] e^x */
    TGP_LOG = 10,   /* [1] ln x, -1 when x < 0 (ln 0 = -inf) */
    TGP_POW = 11,   /* [2] x^y, 0 when x == y == 0, otherwise C99 pow */
    TGP_MIN = 12,   /* [2] IEEE minNum, -0 below +0 (either operand order) */
    TGP_MAX = 13,   /* [2] IEEE maxNum, +0 above -0 (either operand order) */
    TGP_MDIST = 14, /* [2] (x + y) / 2 */
    TGP_NEG = 15,   /* [1] -x */
    TGP_SQRT = 16,  /* [1] sqrt(x), 0 when x < 0 (arity 1; the table prints 2) */
    TGP_SIGN = 17,  /* [1] -1 / 0 / 1; NaN gives 0 */
    TGP_ABS = 18,   /* [1] |x| */
    TGP_CLIP = 19,  /* [3] max(min(x, z), y) */
    TGP_MOD = 20,   /* [2] floored remainder (sign of y), 0 when y == 0 */
    TGP_FRAC = 21,  /* [1] x - floor(x) */
    TGP_IF = 22,    /* [3] x != 0 ? y : z (NaN counts as true) */
    TGP_STEP = 23,  /* [1] -1 when x < 0, else 1 */
    TGP_SSTEP = 24, /* [1] x^2 (3 - 2x) */
    TGP_SSTEPP = 25,/* [1] x^3 (x (6x - 15) + 10) */
    TGP_LEN = 26,   /* [2] sqrt(x^2 + y^2) without intermediate overflow */
    TGP_LERP = 27,  /* [3] x + (y - x) frac(z) */
    /* The bitwise operators of Table 1 (listed there under Logic), appended
     * here.  Each operand is first converted to a 32-bit integer: NaN gives
     * 0, other values are truncated toward zero and saturated to
     * [-2^31, 2^31 - 1]; the integer result is rounded to FP32. */
    TGP_OR = 28,    /* [2] int(x) | int(y) */
    TGP_XOR = 29,   /* [2] int(x) ^ int(y) */
    TGP_AND = 30,   /* [2] int(x) & int(y) */
    /* [3] warp(v, t0, t1): the image transform of Table 1 and Sec. 3.2, read
     * as a gather: the value at a case is v at the grid point whose positions
     * along axes 0 and 1 are given by t0 and t1 (domain units; nearest point,
     * halves rounded up, clamped to the axis, NaN giving the first point); a
     * third axis keeps the case's own point and a 1-D domain ignores t1.  v
     * is materialised over the whole domain first (it is always a cached
     * subtree). */
    TGP_WARP = 31,
    TGP_NUM_OPS = 32
};

/* One tree node.  Trees are postfix (children before parent, left to right).
 * `var` is read only for TGP_VAR and `value` only for TGP_CONST; the other
 * fields of a node are ignored.  Two constants are the same node exactly when
 * their FP32 bit patterns are equal. */
typedef struct {
    uint8_t op;
    uint8_t var;
    uint16_t pad;
    float value;
} tgp_token;

enum { TGP_MEM_HOST = 0, TGP_MEM_DEVICE = 1 };

/* A population of n_individuals, each made of n_channels trees (one tree per
 * output channel, e.g. R, G, B of an image, Sec. 3.1).  Tree r = i * n_channels
 * + ch is tokens[offsets[r] .. offsets[r + 1]).  offsets has n_individuals *
 * n_channels + 1 entries, starts at 0 and never decreases.  `memory` says
 * whether offsets and tokens are host (TGP_MEM_HOST) or device pointers. */
typedef struct {
    int32_t n_individuals;
    int32_t n_channels;
    const int64_t *offsets;
    const tgp_token *tokens;
    int32_t memory;
} tgp_population;

typedef enum { TGP_RMSE = 0, TGP_MSE = 1 } tgp_loss;

/* Counts that describe a population DAG.  "internal" = function nodes. */
typedef struct {
    int64_t tree_nodes;      /* tokens in the population */
    int64_t tree_internal;   /* function tokens */
    int64_t dag_nodes;       /* distinct subtrees (nodes of the DAG) */
    int64_t dag_internal;    /* distinct function subtrees */
    int64_t shared_internal; /* distinct function subtrees occurring >= 2 times */
    int64_t max_stack;       /* deepest left-to-right postfix stack of any tree */
    int64_t max_height;      /* tallest tree (a lone terminal has height 0) */
    int64_t n_roots;         /* n_individuals * n_channels */
    int64_t max_var;         /* largest axis index used, -1 when none */
} tgp_dag_stats;

typedef struct tgp_ctx_s *tgp_ctx;
typedef struct tgp_domain_s *tgp_domain;
typedef struct tgp_dag_s *tgp_dag;

/* ------------------------------------------------------------ context */

/* Create a context on HIP device `device` that orders its work on
 * `hip_stream` (a hipStream_t; NULL = the device's null stream).  The device
 * must be a gfx950 GPU; the call fails with TGP_EHIP otherwise. */
tgp_status tgp_ctx_create(int device, void *hip_stream, tgp_ctx *out);
void tgp_ctx_destroy(tgp_ctx ctx);
/* Switch the stream later work is ordered on. */
tgp_status tgp_ctx_set_stream(tgp_ctx ctx, void *hip_stream);
/* Message of the last failed call on ctx ("" when none); valid until the
 * next call on ctx.  Accepts NULL (returns the last context-less failure). */
const char *tgp_last_error(tgp_ctx ctx);
/* Largest number of bytes the subtree-result cache of one evaluation may
 * occupy (default: 1/4 of the device memory).  Cached subtrees that would
 * exceed it are recomputed instead, except those needed to bound the
 * evaluator's stack, whose excess makes the evaluation fail with TGP_ENOMEM. */
tgp_status tgp_ctx_set_cache_budget(tgp_ctx ctx, size_t bytes);

/* Tuning of the evaluator (the autotuner sets these): cases_per_lane is K,
 * the number of fitness cases each lane of a wave owns per tile (2 or 4; 0 =
 * chosen from the domain size); tiles_per_item is how many consecutive tiles
 * of 64*K cases one wave evaluates for one program (0 = chosen so that a
 * launch has about 65536 work items).  Per-case values do not depend on
 * either; a fitness changes only through the order of its compensated sums. */
tgp_status tgp_ctx_set_tuning(tgp_ctx ctx, int32_t cases_per_lane, int32_t tiles_per_item);

/* Planning options.  reorder_children != 0 (default) evaluates the children
 * of every node in decreasing order of the stack they need (Sethi and
 * Ullman's order), which keeps programs within the register stack; 0 keeps
 * left-to-right order and spills more subtrees to cache rows.
 * cache_access_cost is the price, in VALU lane-slots per case, of one 4-byte
 * cache-row access (default 20); a shared subtree is cached when recomputing
 * it costs more than its accesses; a negative value caches only the
 * subtrees needed to bound the stack.  Values never depend on either. */
tgp_status tgp_ctx_set_plan(tgp_ctx ctx, int32_t reorder_children, double cache_access_cost);

/* Where the interpreter keeps a program's operand stack: lds = 0 (default)
 * in 8 register slots per case, with one dispatch loop over (stack depth,
 * instruction) and four cases per lane; lds != 0 in 16 LDS slots per case (the top of the
 * stack in registers, one dispatch loop, two cases per lane), which needs
 * fewer subtrees spilled to cache rows for deep programs.  Values never
 * depend on it; the autotuner chooses between the two. */
tgp_status tgp_ctx_set_stack(tgp_ctx ctx, int32_t lds);

/* Constant folding (default on): a subtree with no variable has the same
 * value at every case, so it is evaluated once, on the device with the
 * interpreter's own FP32 operators, and its programs use the value as a
 * constant.  Values are bitwise the same either way. */
tgp_status tgp_ctx_set_folding(tgp_ctx ctx, int32_t on);

/* Hash-consing identity of later tgp_build_dag calls: structural (0, the
 * default: op, payload and children in order, Handley's DAG of Sec. 2), or
 * also up to the operand order of the operators whose operands commute
 * bitwise in this library, NaN payloads aside (1: add, mult, min, max,
 * mdist, len, or, xor, and; min and max order -0 below +0 and give the
 * other operand for a NaN).  A node keeps the child order of its first
 * occurrence.  Values are the same
 * either way; the DAG (and the credited node count) can only shrink. */
tgp_status tgp_ctx_set_hashing(tgp_ctx ctx, int32_t commutative);

/* Identity rewrites while hash-consing later tgp_build_dag calls (on != 0;
 * default off): the algebraic-equivalence caching of Wong and Zhang (Sec. 2)
 * and the expression simplification the paper proposes (Sec. 5), kept to
 * rules that hold bit for bit under this library's readings (NaN payloads
 * aside) and map a node to one that already exists:
 *   neg(neg(x)) -> x, abs(abs(x)) -> abs(x), sign(sign(x)) -> sign(x),
 *   step(step(x)) -> step(x), min(x, x) -> x, max(x, x) -> x,
 *   if(c, y, y) -> y, sub(x, +0) -> x, add(x, -0) -> x, add(-0, x) -> x,
 *   mult(x, 1) -> x, mult(1, x) -> x, div(x, 1) -> x
 * (x, y, c any subtrees; the constants are literal tokens with exactly
 * these bits).  A rewritten token gets no node of its own: it stands for
 * the node it maps to, which counts it in its multiplicity.  Per-case values
 * are the same as without rewrites; the DAG can only shrink. */
tgp_status tgp_ctx_set_rewrite(tgp_ctx ctx, int32_t on);

/* Test hook: keep only the low `bits` bits of the DAG builder's 64-bit key
 * hash (0 = all bits), forcing collisions so that the full-key comparison is
 * exercised.  Process-wide; the DAG produced must not change. */
tgp_status tgp_debug_set_hash_bits(int32_t bits);

/* ------------------------------------------------------------- domain */

/* The grid of fitness cases (Sec. 3.1, Sec. 4.1): ndim in 1..3 axes of
 * shape[k] >= 1 points; point i of axis k has coordinate
 * fl32(lo[k] + (hi[k] - lo[k]) * i / (shape[k] - 1)) computed in FP64 (lo[k]
 * when shape[k] == 1).  lo/hi NULL mean -1 and 1 for every axis (the paper's
 * standard range).  Cases are numbered row-major, last axis fastest; at most
 * 2^30 cases (a row of one FP32 value per case then stays within 4 GiB, which
 * the interpreter addresses with 32-bit byte offsets).  The coordinate tables
 * are copied to the device. */
tgp_status tgp_domain_create(tgp_ctx ctx, int32_t ndim, const int64_t *shape, const double *lo,
                             const double *hi, tgp_domain *out);
void tgp_domain_destroy(tgp_domain dom);
int64_t tgp_domain_cases(tgp_domain dom);

/* ---------------------------------------------------------------- DAG */

/* Hash-cons a population into one DAG (Handley's population DAG, Sec. 2):
 * structurally identical subtrees (same opcode, same payload, identical
 * children) become one node.  Runs on the GPU (structure scan, level-by-level
 * hash-consing with a device hash table, compaction) and blocks until the DAG
 * is built.  Node ids follow the first occurrence of each subtree in a
 * postfix walk of the trees in population order, so children precede parents.
 * Errors: TGP_EPARSE (tree r malformed, r in the message), TGP_EOP,
 * TGP_EINVAL (bad offsets or sizes). */
tgp_status tgp_build_dag(tgp_ctx ctx, const tgp_population *pop, tgp_dag *out);
tgp_status tgp_dag_stats_get(tgp_dag dag, tgp_dag_stats *out);
/* Copy the DAG to host arrays of dag_nodes (nodes, multiplicity, indegree),
 * dag_nodes * 3 (children, -1 where a child slot is unused) and n_roots
 * (roots) entries.  multiplicity = number of tokens of the population that
 * map to the node; indegree = number of (parent, child slot) edges into it.
 * Any output pointer may be NULL.  Blocks. */
tgp_status tgp_dag_export(tgp_dag dag, tgp_token *nodes, int32_t *children, int32_t *roots,
                          int32_t *multiplicity, int32_t *indegree);
void tgp_dag_destroy(tgp_dag dag);

/* --------------------------------------------------------- evaluation */

/* Phenotypes (Sec. 3.1): the value of every tree at every case, FP32, written
 * to out_dev[r][case] with r = individual * n_channels + channel (device
 * pointer, n_roots * cases floats).  TGP_ESHAPE when a tree uses an axis the
 * domain does not have. */
tgp_status tgp_evaluate(tgp_ctx ctx, tgp_dag dag, tgp_domain dom, float *out_dev);

/* Fitness (Sec. 4.1): per individual, the RMSE (TGP_RMSE) or MSE (TGP_MSE)
 * over all channels and cases against target_dev[channel][case] (device,
 * n_channels * cases floats), written as FP64 to out[individual].  out is a
 * device pointer (the work is queued on the context's stream and the call
 * returns without waiting for it) or host memory, pageable or pinned (the
 * values go through a context-owned device buffer and the call blocks until
 * they are in out).  Squares are accumulated with compensated FP32 sums and
 * combined in FP64; any non-finite term makes the fitness +inf. */
tgp_status tgp_fitness(tgp_ctx ctx, tgp_dag dag, tgp_domain dom, const float *target_dev,
                       int32_t loss, double *out);

/* tgp_fitness without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same kernels, same arguments and the same result
 * bits as tgp_fitness, with these limits:
 *   - target_dev and out must be device memory (TGP_EINVAL otherwise);
 *   - dag must already hold its plan for a domain of dom's size under the
 *     context's current settings, i.e. it has been evaluated once by
 *     tgp_fitness or tgp_evaluate on such a domain (TGP_EINVAL otherwise);
 *   - the partial sums (8 bytes per root program per stripe) and the cached
 *     subtree rows (4 bytes per cached subtree per case) live in a fixed
 *     64 MiB device array per GPU, held until the process ends; a call that
 *     needs more returns TGP_ENOMEM without launching anything (lower the
 *     cache budget, tgp_ctx_set_cache_budget, before planning to fit).
 * Every call on a GPU shares that array, so calls that overlap on one GPU
 * (two streams, or two contexts on the same device) race: order them.
 * Queued on the context's stream; returns without waiting. */
tgp_status tgp_fitness_noalloc(tgp_ctx ctx, tgp_dag dag, tgp_domain dom, const float *target_dev,
                               int32_t loss, double *out);

/* Work counts of the last tgp_evaluate / tgp_fitness on ctx (for reports).
 * VALU figures are lane-slots: cases x the per-operator instruction counts of
 * the compiled interpreter (a cost model, documented with the library). */
typedef struct {
    int64_t credited_node_evals; /* DAG nodes x cases (each distinct subtree once) */
    int64_t executed_node_evals; /* interpreter instructions run x cases */
    int64_t cached_nodes;        /* subtrees materialised in the cache */
    int64_t stack_spills;        /* of which cached only to bound the register stack */
    int64_t cache_levels;        /* dependent cache-fill launches */
    int64_t programs;            /* root programs (distinct (root, channel) pairs) */
    int64_t instructions;        /* total program length */
    double algorithmic_valu;     /* every DAG node once, cost model x cases */
    double executed_valu_fill;   /* cache-fill launches, cost model x cases */
    double executed_valu_roots;  /* root-program launch, cost model x cases */
    int64_t cache_bytes_read;    /* HBM bytes of cache loads (algorithmic) */
    int64_t cache_bytes_written; /* HBM bytes of cache stores (algorithmic) */
    int64_t folded_nodes;        /* constant subtrees evaluated once and used as constants */
} tgp_work_stats;
tgp_status tgp_last_work(tgp_ctx ctx, tgp_work_stats *out);

/* Phase times of the last tgp_build_dag, tgp_fitness / tgp_evaluate and
 * tgp_breed on ctx.  Device times come from HIP events recorded on the context's stream
 * around the launches, and are only taken while timing is enabled
 * (tgp_ctx_set_timing); tgp_last_timing blocks until those events complete. */
typedef struct {
    double build_dag_ms;  /* host wall time of the blocking tgp_build_dag */
    double plan_ms;       /* host wall time of planning and program upload */
    double fill_ms;       /* device time of the cache-fill launches */
    double interp_ms;     /* device time of the root-program launch */
    double finalize_ms;   /* device time of the per-individual finalize */
    int64_t interp_items; /* work items (waves) of the root-program launch */
    int32_t cases_per_lane;
    int32_t tiles_per_item;
    /* parts of plan_ms: constant folding (with its device round trip), the
     * caching and stack decisions, program emission, the rest */
    double plan_fold_ms, plan_decide_ms, plan_emit_ms;
    /* device times of the last tgp_breed: the parents' shape launch, the
     * decisions and the offset scan, the copy of the child trees */
    double breed_shape_ms, breed_plan_ms, breed_write_ms;
} tgp_timing;
tgp_status tgp_ctx_set_timing(tgp_ctx ctx, int32_t enable);
tgp_status tgp_last_timing(tgp_ctx ctx, tgp_timing *out);

/* ----------------------------------------------------- batched fitness */

/* One fitness evaluation of a batch: the arguments of tgp_fitness. */
typedef struct {
    tgp_dag dag;
    tgp_domain domain;
    const float *target_dev; /* [n_channels][cases] on the device */
    int32_t loss;            /* TGP_RMSE or TGP_MSE */
    double *out_dev;         /* [n_individuals] on the device */
} tgp_job;

typedef struct tgp_batch_s *tgp_batch;

/* A batch evaluates many populations of uneven sizes and domain shapes (for
 * instance one generation of many GP runs) together: one persistent launch
 * per cache-fill level, one persistent launch for every job's root programs
 * fused with the error reduction, one finalize for every individual.  With
 * use_graph != 0 the launches of a step are captured once as a HIP graph
 * and replayed (recaptured only when the batch outgrows its buffers).
 * Results equal tgp_fitness on each job up to the order of the compensated
 * sums.  A batch belongs to its context and its thread. */
tgp_status tgp_batch_create(tgp_ctx ctx, int32_t use_graph, tgp_batch *out);
/* Evaluate n_jobs fitness jobs (asynchronous on the context stream; the host
 * arrays are read during the call).  Blocks until the previous step of this
 * batch has consumed its uploads. */
tgp_status tgp_batch_run(tgp_batch batch, int32_t n_jobs, const tgp_job *jobs);
void tgp_batch_destroy(tgp_batch batch);
/* Launch form of later batched steps: persistent != 0 runs resident waves
 * that draw work items from atomic counters (the default), 0 one wave per
 * work item. */
tgp_status tgp_ctx_set_batch_form(tgp_ctx ctx, int32_t persistent);
/* tgp_batch_run on a graph-replayed batch that the context keeps. */
tgp_status tgp_fitness_batch(tgp_ctx ctx, int32_t n_jobs, const tgp_job *jobs);

typedef struct {
    int64_t jobs, pairs, items, levels;  /* last step: jobs, programs, work items, fill levels */
    int64_t captures, replays;           /* graph captures and launches so far */
    int64_t credited_node_evals;         /* last step: sum of DAG nodes x cases */
    double pack_ms;                      /* last step: host planning and packing */
    int32_t tiles_per_item, cases_per_lane;
    int32_t persistent;                  /* launch form of the last step */
} tgp_batch_stats;
tgp_status tgp_batch_stats_get(tgp_batch batch, tgp_batch_stats *out);

/* Autotuner: times the stack form and cases per lane (registers with K in
 * {2, 4}, or LDS with K = 2) x the cap on tiles per work item in {4, 16} x
 * the batched launch form (persistent waves drawing items from partitioned
 * atomic counters, or one wave per item) on the given jobs
 * (a warm-up and a timed batched run each) and installs the fastest in ctx.
 * With cache_path != NULL the choice is appended to that file (one JSON
 * object per line, keyed by the workload's size class) and reused without
 * timing for a later workload of the same class. */
typedef struct {
    int32_t cases_per_lane, tiles_cap, persistent;
    int32_t candidates, from_cache;
    int32_t stack_lds;       /* chosen stack form (tgp_ctx_set_stack) */
    double best_ms;
} tgp_tune_result;
tgp_status tgp_autotune(tgp_ctx ctx, int32_t n_jobs, const tgp_job *jobs, const char *cache_path,
                        tgp_tune_result *out);

/* ------------------------------------------------------------- serving */

/* A server evaluates the per-generation populations of many concurrent GP
 * runs (TensorGP's evaluation step of Sec. 3.1, once per generation of each
 * run) with continuous batching: a request loop admits each submitted
 * population when a slot and device memory for its cached subtrees are free,
 * and every batched step on the GPU carries one slab of cases of every
 * admitted request, so a request that arrives while others run joins at the
 * next step instead of waiting for them to finish.  Subtree results are
 * kept in a device cache across requests, keyed by the subtree's structure
 * and the domain, and reused by later generations (the effect noted in
 * Sec. 4.2), with least-recently-used eviction when space is needed.
 *
 * A request's fitness values do not depend on what else is being served: its
 * slabs, work split and summation order are chosen from the request alone,
 * and a resident subtree holds the same FP32 values the request would
 * compute.  The server has threads of its own and its own HIP streams on
 * the context's device; submit, wait, ticket_info, stats and end_run may be
 * called from any thread.  The context passed in is only read at creation
 * (device, tuning) and stays free for its owner to use. */
typedef struct tgp_server_s *tgp_server;

/* cache_budget_bytes: device memory reserved for resident subtree results (0:
 * a quarter of the device's memory); max_active: requests evaluated at once
 * (0: 16).  Blocks while the cache memory is allocated. */
tgp_status tgp_server_create(tgp_ctx ctx, size_t cache_budget_bytes, int32_t max_active, tgp_server *out);
/* Waits for the admitted requests to finish; requests not admitted yet end
 * with TGP_EBUSY.  Domains and targets of finished requests are not touched
 * afterwards. */
void tgp_server_destroy(tgp_server server);
/* Work per slab, in DAG nodes x cases (default 2^33): a request with more
 * work than this is evaluated in slabs of consecutive cases, one per step. */
tgp_status tgp_server_set_slab_work(tgp_server server, double node_evals);
/* Launch shape of later steps: persistent waves (1) or one wave per work
 * item (0, the default), or unchanged (-1); tiles of 64 x cases-per-lane
 * cases per work item (0: chosen from each request's slab size; applies to
 * requests admitted afterwards). */
tgp_status tgp_server_set_launch(tgp_server server, int32_t persistent, int32_t tiles_per_item);

/* Queue one fitness evaluation (does not block on the GPU).  pop must be in
 * host memory (copied during the call); domain and target_dev (device,
 * [n_channels][cases]) must stay valid until the request ends; out (host,
 * [n_individuals] doubles) receives the fitness values before tgp_server_wait
 * returns TGP_OK.  run_id groups the requests of one GP run (for
 * tgp_server_end_run).  *ticket identifies the request. */
tgp_status tgp_server_submit(tgp_server server, int64_t run_id, const tgp_population *pop,
                             tgp_domain domain, const float *target_dev, int32_t loss, double *out,
                             int64_t *ticket);
/* Blocks until the request ends or timeout_us passes (timeout_us < 0: no
 * limit).  Returns TGP_OK (out written), TGP_EBUSY on time-out, or the
 * request's own error (TGP_EPARSE, TGP_EOP, TGP_ESHAPE, TGP_ENOMEM when its
 * cached subtrees can never fit the cache budget, TGP_EHIP). */
tgp_status tgp_server_wait(tgp_server server, int64_t ticket, int64_t timeout_us);
/* Frees the run's resident subtrees (those still in use are freed when the
 * requests using them end). */
tgp_status tgp_server_end_run(tgp_server server, int64_t run_id);
const char *tgp_server_last_error(tgp_server server);

typedef struct {
    int32_t status;        /* TGP_OK when done, TGP_EBUSY while queued or running, else its error */
    int32_t slabs;         /* slabs the request's cases were split into */
    double submit_ms, admit_ms, start_ms, done_ms; /* server clock (ms since creation) */
    double latency_ms;     /* done - submit */
    double prep_ms;        /* DAG build, cache look-up and planning */
    int64_t dag_nodes;     /* unique subtrees of the request's population */
    int64_t credited_node_evals; /* dag_nodes x cases */
    int32_t cache_hits;    /* cached subtrees read from earlier requests */
    int32_t cache_new;     /* cached subtrees computed and kept by this request */
} tgp_ticket_info;
tgp_status tgp_server_ticket_info(tgp_server server, int64_t ticket, tgp_ticket_info *out);

typedef struct {
    int64_t submitted, completed, failed;
    int64_t steps, slabs;          /* batched steps launched, request slabs they carried */
    int64_t cache_hits, cache_new, evictions, entries;
    int64_t bytes_in_use, bytes_peak, bytes_capacity;  /* resident subtree cache */
    int64_t credited_node_evals;   /* of completed requests */
    int32_t max_active_seen;       /* most requests evaluated together */
    int32_t pad;
    double step_ms;                /* GPU time of the steps (first launch to last) */
} tgp_server_stats;
tgp_status tgp_server_stats_get(tgp_server server, tgp_server_stats *out);


/* ------------------------------------------------- genetic operators */

/* One generation bred on the device from a population and its fitness, so
 * that a GP run can stay on the GPU between evaluations (the paper runs its
 * genetic operators on the host, Sec. 4.2, and names ramped half-and-half as
 * its generation method, Table 2; it does not fix selection or variation).
 * The operators are the textbook tree-GP ones (Koza 1992):
 *
 *   offspring o draws its decisions from a counter-based stream: draw k is
 *   output number o * 2^32 + k + 1 of SplitMix64 (Steele, Lea & Flood 2014)
 *   started from `seed`; below(m) = floor(x * m / 2^64), uniform() =
 *   (x >> 11) * 2^-53, a new constant = fl32(2u - 1) with u = (x >> 40) * 2^-24.
 *   Draws in order: u = uniform(); parent p1 by tournament; when
 *   u < p_crossover parent p2 by tournament.  A tournament draws
 *   `tournament` parents below(n_parents) with replacement and keeps the
 *   first of the lowest fitness (NaN and +-inf count as +inf; fitness NULL:
 *   the first draw).  Then, for each channel ch, with a = tree ch of p1:
 *     crossover: up to crossover_tries times draw i = below(len a) and
 *       j = below(len b), b = tree ch of p2, and accept when depth_a(i) +
 *       height_b(j) <= max_depth: the child is a with the subtree rooted at
 *       token i replaced by b's subtree rooted at token j; with no accepted
 *       draw the child is a copy of a;
 *     mutation (p_crossover <= u < p_crossover + p_mutation): i = below(len a),
 *       d = below(min(max(max_depth - depth_a(i), 0), max_mutation_depth) + 1),
 *       full = below(2) == 0, and the subtree at i is replaced by a new random
 *       tree of depth d, full or grow (nodes chosen in pre-order: at depth 0
 *       a terminal below(n_terminals); full: a function below(n_functions);
 *       grow: below(n_functions + n_terminals), a function when below
 *       n_functions, else that terminal; terminals are the variables
 *       0..ndim-1, then the constant when use_constants, which draws its
 *       value);
 *     reproduction (otherwise): a copy of a.
 *   depth_a(i) is token i's distance from the root of a, height_b(j) the
 *   height of the subtree at j (a leaf has height 0).
 *
 * Offspring are independent of each other (the first m of n offspring do not
 * depend on n), and the output is a pure function of the inputs and seed. */
typedef struct {
    uint64_t seed;
    int32_t n_offspring;        /* individuals bred (each of the parents' n_channels trees) */
    int32_t tournament;         /* >= 1 */
    double p_crossover;         /* in [0, 1] */
    double p_mutation;          /* in [0, 1 - p_crossover]; the rest is reproduction */
    int32_t max_depth;          /* >= 0 */
    int32_t max_mutation_depth; /* >= 0 */
    int32_t crossover_tries;    /* >= 1 */
    int32_t ndim;               /* variables 0..ndim-1 (1 to 3) */
    int32_t use_constants;      /* the ephemeral constant is a terminal */
    int32_t n_functions;        /* >= 1 */
    const uint8_t *functions;   /* host [n_functions] operator codes, each of arity >= 1 */
} tgp_breed_params;

typedef struct tgp_offspring_s *tgp_offspring;

/* Breeds params->n_offspring individuals from `parents` (device or host
 * memory; at least one individual when n_offspring > 0).  fitness_dev is a
 * device array of n_individuals doubles (e.g. the output of tgp_fitness) or
 * NULL.  Work is ordered on the context stream; the call blocks once, to
 * learn the offspring's size.  Errors: TGP_EINVAL for bad parameters,
 * TGP_EOP for an operator code that is not a function, TGP_EPARSE when a
 * parent tree is not one postfix tree, TGP_EHIP, TGP_ENOMEM. */
tgp_status tgp_breed(tgp_ctx ctx, const tgp_population *parents, const double *fitness_dev,
                     const tgp_breed_params *params, tgp_offspring *out);
/* A device view of the offspring (memory = TGP_MEM_DEVICE), valid until
 * tgp_offspring_destroy; it can be passed to tgp_build_dag or be the parents
 * of the next tgp_breed. */
tgp_status tgp_offspring_population(tgp_offspring offspring, tgp_population *view);
/* *n_tokens = the offspring's token count; when offsets_host and tokens_host
 * are not NULL, also copies the offsets (n_individuals * n_channels + 1) and
 * the tokens (*n_tokens) to host memory (blocks until they are written). */
tgp_status tgp_offspring_export(tgp_offspring offspring, int64_t *n_tokens, int64_t *offsets_host,
                                tgp_token *tokens_host);
void tgp_offspring_destroy(tgp_offspring offspring);

#ifdef __cplusplus
}
#endif
#endif /* TGP_H */
