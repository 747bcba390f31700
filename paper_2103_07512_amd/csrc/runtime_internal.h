// runtime_internal.h -- host objects of libtgp shared by the translation
// units of the runtime (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <functional>
#include <string>
#include <vector>

#include "tgp_internal.h"

using namespace tgp;

// ------------------------------------------------------------------ objects
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

struct tgp_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    size_t cache_budget = 0;
    std::string err;
    tgp_work_stats work{};
    int force_K = 0;  // 0 = automatic
    int force_tiles = 0;
    int tile_cap = 0;  // cap on automatic tiles per item (0 = 16)
    int batch_persistent = 1;  // batched launches: persistent waves (1) or one wave per item
    tgp_batch batch = nullptr;  // kept by tgp_fitness_batch
    int reorder = 1;                     // Sethi-Ullman child order
    bool plan_upload = true;             // plans also kept on the device
    int stack_lds = 0;                   // operand stack in LDS (1) or registers (0)
    int fold = 1;                        // constant folding
    int commute = 0;                     // hash-consing up to operand order of commuting operators
    int rewrite = 0;                     // identity rewrites while hash-consing
    double cache_access_cost = 20.0;     // < 0: no benefit-driven caching
    DevBuf partial, cache;
    DevBuf fit_out;  // device copy of fitness values bound for host memory
    DevicePool pool;             // DAG, plan and population blocks
    void *pin = nullptr;         // pinned staging for uploads and readbacks
    size_t pin_cap = 0;
    hipEvent_t pin_ev = nullptr; // recorded after the last copy out of `pin`
    bool pin_pending = false;
    bool timing = false;
    bool ev_ready = false;
    // fill begin/end, interp begin/end, finalize begin/end, then breeding:
    // shape begin, shape end = decisions begin, decisions end, copy begin/end
    hipEvent_t ev[11] = {};
    uint32_t recorded = 0;  // bit i: ev[i] has been recorded
    bool fill_recorded = false;
    tgp_timing times{};
};

inline double now_ms() {
    return std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

inline void record(tgp_ctx ctx, int i) {
    if (ctx->timing && ctx->ev_ready && hipEventRecord(ctx->ev[i], ctx->stream) == hipSuccess)
        ctx->recorded |= 1u << i;
}

struct tgp_domain_s {
    tgp_ctx ctx = nullptr;
    int32_t ndim = 0;
    int64_t shape[3] = {1, 1, 1};
    int64_t stride[3] = {1, 1, 1};
    int64_t cases = 0;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    float *coord[3] = {nullptr, nullptr, nullptr};
};

// A compiled evaluation plan of one DAG for one case count.
struct Plan {
    int64_t cases = -1;
    int D = 0;                          // stack slots the programs were planned for
    bool reorder = true;
    double access_cost = 0;
    int fold = -1;
    int64_t n_folded = 0;               // constant subtrees folded
    int32_t n_slots = 0;
    int64_t n_spills = 0;               // cached only to bound the register stack
    std::vector<int32_t> level_first;   // fill programs of level l: [level_first[l], level_first[l+1])
    int32_t n_fill = 0;
    int32_t n_reduce = 0;               // programs for (root, channel)
    int32_t n_store = 0;                // programs for distinct roots
    std::vector<int32_t> store_rows;    // for each root r: the store program's dest row, or -1
    std::vector<int32_t> dup_src;       // for each root r: row r copies row dup_src[r] (-1: none)
    // Device copies in two pool blocks, so that the fill can start before the
    // root programs are emitted: blob holds the fill programs' code and
    // descriptors, blob_roots the root programs' code (code_roots_dev), the
    // reduce and store descriptors (code offsets relative to code_roots_dev)
    // and the individual rows.
    void *blob = nullptr, *blob_roots = nullptr;
    uint2 *code_dev = nullptr, *code_roots_dev = nullptr;
    ProgDesc *fill_dev = nullptr, *reduce_dev = nullptr, *store_dev = nullptr;
    int32_t *ind_rows_dev = nullptr;
    int64_t root_code_at = 0;           // first root instruction in code_host
    // host copies (the batched path packs them into its own buffers); code
    // offsets in all three descriptor lists are into code_host
    std::vector<uint2> code_host;
    std::vector<ProgDesc> fill_host, reduce_host, store_host;
    std::vector<int32_t> ind_rows_host;
    std::vector<int32_t> slot_node;     // DAG node held by each cache slot
    std::vector<uint8_t> slot_pre;      // slot already resident (no fill program)
    bool ext = false;                   // uses the bitwise operators, warp or the third axis
    bool warp = false;                  // uses warp
    int64_t instructions = 0;
    double exec_per_case = 0;           // instructions run per case, fitness form
    double valu_dag_per_case = 0;       // cost-model slots of each DAG node once
    double valu_fill_per_case = 0;      // cost-model slots run by the fill programs
    double valu_roots_per_case = 0;     // cost-model slots run by the reduce programs
    int64_t cache_reads_per_case = 0;   // I_CACHE instructions executed, fitness form
    // The caller guarantees that no queued kernel still reads the block.
    void release(DevicePool &pool) {
        pool.release(blob);
        pool.release(blob_roots);
        blob = blob_roots = nullptr;
        code_dev = code_roots_dev = nullptr;
        fill_dev = reduce_dev = store_dev = nullptr;
        ind_rows_dev = nullptr;
        cases = -1;
    }
};

struct tgp_dag_s {
    tgp_ctx ctx = nullptr;
    int32_t n_ind = 0, n_ch = 0;
    tgp_dag_stats stats{};
    DagDevice dev;
    // host copies
    std::vector<int32_t> op;   // op | var << 8
    std::vector<float> value;
    std::vector<int32_t> kid;  // [U][3]
    std::vector<int32_t> roots, mult, indeg, height;
    std::vector<uint8_t> precached;  // nodes whose values are resident (empty: none)
    Plan plan;
};

// ------------------------------------------------------------------ errors
tgp_status fail(tgp_ctx ctx, tgp_status st, const char *fmt, ...);

#define HCHK(ctx, x)                                                                           \
    do {                                                                                       \
        hipError_t _e = (x);                                                                   \
        if (_e != hipSuccess)                                                                  \
            return fail(ctx, TGP_EHIP, "%s failed: %s", #x, hipGetErrorString(_e));            \
    } while (0)

inline hipError_t ensure(DevBuf &b, size_t bytes) {
    if (b.cap >= bytes && b.p) return hipSuccess;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        if (e != hipSuccess) return e;
        b.p = nullptr;
        b.cap = 0;
    }
    size_t want = std::max<size_t>(bytes, 256);
    hipError_t e = hipMalloc(&b.p, want);
    if (e == hipSuccess) b.cap = want;
    return e;
}


// Pinned staging of at least `bytes`, free to be overwritten (waits for the
// copy that last read it).
hipError_t ctx_pinned(tgp_ctx ctx, size_t bytes, void **out);
// Marks the staging as read by copies enqueued on the context stream.
hipError_t ctx_pinned_enqueued(tgp_ctx ctx);

// One job of a batched step: a plan's programs over the cases
// [case_base, case_base + n_cases) of a domain.
struct StepJob {
    const Plan *plan;             // host copies of the programs are used
    tgp_domain domain;
    int32_t n_ind = 0, n_ch = 0;
    int32_t case_base = 0, n_cases = 0;
    const float *target = nullptr;   // [n_ch][domain cases]
    // Cache rows: with cache == nullptr the step allocates [slots][domain
    // cases] rows itself (slot s is row s); otherwise the plan's slot numbers
    // are rows of `cache` with stride cache_stride.
    const float *cache = nullptr;
    int64_t cache_stride = 0;
    double *acc = nullptr;        // slab running sums (nullptr: whole domain)
    int32_t first = 1, last = 1;  // first / last slab of the domain
    double *out = nullptr;        // device, [n_ind]
    int32_t loss = TGP_RMSE;
    int32_t tiles_per_item = 0;   // 0: chosen from the whole step's work
    // Programs and individual rows already on the device (nullptr: the step
    // uploads the plan's host copies).
    const uint2 *code_dev = nullptr;
    const int32_t *rows_dev = nullptr;
};
tgp_status batch_step(tgp_batch b, int32_t n_jobs, const StepJob *jobs, int64_t credited);

// --------------------------------------------------------------- shared helpers
extern const double kOpCost[TGP_NUM_OPS];
// Plans d for domains of `cases` cases (a no-op when its plan is current) and
// uploads the programs when the context keeps plans on the device.  When a
// new plan is uploaded, after_fill (if given) is called once the fill
// programs are on the device and before the root programs are emitted, so
// that the caller can queue the cache fill while the host emits the rest.
tgp_status build_plan(tgp_ctx ctx, tgp_dag d, int64_t cases,
                      const std::function<tgp_status()> &after_fill = nullptr);
// Plans many DAGs at once (host threads, one device round trip for constant
// folding); programs stay on the host.  A DAG listed more than once is
// planned once, for its largest domain.
tgp_status build_plans(tgp_ctx ctx, int32_t n, const tgp_dag *dags, const int64_t *cases);
int choose_K(tgp_ctx ctx, int64_t cases, bool ext);
int ctx_stack_slots(tgp_ctx ctx);
void choose_split(tgp_ctx ctx, int64_t n_progs, int64_t cases, int K, int32_t *stripes,
                  int32_t *tiles_per);
void fill_job(JobDesc &j, tgp_domain dom, const uint2 *code, const float *cache);
tgp_status check_eval_args(tgp_ctx ctx, tgp_dag d, tgp_domain dom);
