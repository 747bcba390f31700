// runtime.cpp -- host side of libtgp: contexts, domains, the population DAG,
// the cache planner, the program emitter and the C ABI of include/tgp.h.
//
// Evaluation of a DAG over a domain (TensorGP Sec. 3.1, with the subtree
// caching of Sec. 1 / Sec. 2) is planned on the host:
//   * every distinct (root, channel) pair becomes one interpreter program;
//   * a shared subtree is materialised once in an HBM cache row when
//     re-computing it at each use costs more VALU work than writing the row
//     once and reading it at each use (HBM traffic priced in VALU slots);
//   * subtrees whose evaluation would need more stack slots than the
//     interpreter keeps in registers are materialised as well, so every
//     program fits the register stack;
//   * cached subtrees are filled level by level (a row's program may read
//     rows of lower levels), then the root programs run fused with the error
//     reduction (fitness) or with a store of their values (evaluate).
#include <hip/hip_runtime.h>

#include <sched.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "runtime_internal.h"

namespace tgp {
extern uint32_t g_debug_hash_bits;
}

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

hipError_t ctx_pinned(tgp_ctx ctx, size_t bytes, void **out) {
    if (ctx->pin_pending) {
        hipError_t e = hipEventSynchronize(ctx->pin_ev);
        if (e != hipSuccess) return e;
        ctx->pin_pending = false;
    }
    if (ctx->pin_cap < bytes) {
        if (ctx->pin) hipHostFree(ctx->pin);
        ctx->pin = nullptr;
        ctx->pin_cap = 0;
        size_t want = 1 << 20;
        while (want < bytes) want <<= 1;
        hipError_t e = hipHostMalloc(&ctx->pin, want, hipHostMallocDefault);
        if (e != hipSuccess) return e;
        ctx->pin_cap = want;
    }
    *out = ctx->pin;
    return hipSuccess;
}

hipError_t ctx_pinned_enqueued(tgp_ctx ctx) {
    if (!ctx->pin_ev) {
        hipError_t e = hipEventCreateWithFlags(&ctx->pin_ev, hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipEventRecord(ctx->pin_ev, ctx->stream);
    if (e == hipSuccess) ctx->pin_pending = true;
    return e;
}

tgp_status fail(tgp_ctx ctx, tgp_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    g_err = buf;
    return st;
}

// The device code looks arities up in a packed constant; it must agree with
// the table for every opcode.
constexpr bool packed_arities_match() {
    for (int i = 0; i < TGP_NUM_OPS; ++i)
        if (arity_of((uint32_t)i) != kArityList[i] || kArityList[i] > 3) return false;
    return true;
}
static_assert(packed_arities_match(), "every arity fits two bits and unpacks to the table's value");

// --------------------------------------------------------------- cost model
// The planner's estimate of each operator's cost in VALU instructions per
// case, first measured with one-operator kernels over random inputs in
// [-1, 1] (SQ_INSTS_VALU less loads, stores and indexing) on earlier
// implementations of the operators; pow, mod, exp, log and sqrt have fast
// paths since and cost less, which only makes the planner cache a little
// more of them than it would.  Terminals cost the register move that places
// them on the stack; warp is estimated (two axis points and a gathered
// read).  It steers caching and program order only; reported throughput
// does not use it.
const double kOpCost[TGP_NUM_OPS] = {
    1,  1,              // var const
    1,  1,  1, 13,      // add sub mult div
    38, 35, 55,         // sin cos tan
    14, 15, 83,         // exp log pow
    3,  3,  3,  1,      // min max mdist neg
    19, 4,  1,  5,      // sqrt sign abs clip
    42, 2,  2,          // mod frac if
    2,  6,  9, 27, 9,   // step sstep sstepp len lerp
    16, 16, 16,         // or xor and
    24                  // warp
};
// Writing a cache row once and reading it back, in VALU-slot equivalents per
// case: 4 bytes of HBM traffic at 8 TB/s against 256 CUs x 64 lanes x 2.4 GHz
// of VALU issue is about 20 slots per access (the default of
// tgp_ctx_set_plan's cache_access_cost).

// ------------------------------------------------- fixed device scratch
// tgp_fitness_noalloc keeps its partial sums and subtree cache rows in this
// array instead of allocated buffers, so it calls no allocator.  Each GPU
// the library runs on holds its own copy until the process ends.  In host
// code `scratch` only names the symbol: its device address is looked up once
// per device (hipGetSymbolAddress, at context creation, with the device
// current) and that address is what kernels and copies receive.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];
}  // namespace

// With `device` current: its scratch address, looked up on first use.
static void scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_ptr[device]) return;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_err[device] = e;
    if (e == hipSuccess) g_scratch_ptr[device] = p;
    else (void)hipGetLastError();  // leave no error behind for the next call
}

// --------------------------------------------------------------- contexts
extern "C" {

tgp_status tgp_ctx_create(int device, void *hip_stream, tgp_ctx *out) {
    if (!out) return fail(nullptr, TGP_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0)
        return fail(nullptr, TGP_EHIP, "no HIP device: %s", hipGetErrorString(e));
    if (device < 0 || device >= n) return fail(nullptr, TGP_EINVAL, "device %d out of range", device);
    e = hipSetDevice(device);
    if (e != hipSuccess) return fail(nullptr, TGP_EHIP, "hipSetDevice: %s", hipGetErrorString(e));
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess)
        return fail(nullptr, TGP_EHIP, "hipGetDeviceProperties: %s", hipGetErrorString(e));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, TGP_EHIP, "device %d is %s, libtgp is built for gfx950", device,
                    prop.gcnArchName);
    scratch_setup(device);
    tgp_ctx c = new tgp_ctx_s();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->cache_budget = prop.totalGlobalMem / 4;
    *out = c;
    return TGP_OK;
}

void tgp_ctx_destroy(tgp_ctx ctx) {
    if (!ctx) return;
    hipSetDevice(ctx->device);
    hipStreamSynchronize(ctx->stream);
    tgp_batch_destroy(ctx->batch);
    hipFree(ctx->partial.p);
    hipFree(ctx->cache.p);
    hipFree(ctx->fit_out.p);
    ctx->pool.drain();
    if (ctx->pin) hipHostFree(ctx->pin);
    if (ctx->pin_ev) hipEventDestroy(ctx->pin_ev);
    if (ctx->ev_ready)
        for (auto &e : ctx->ev) hipEventDestroy(e);
    delete ctx;
}

tgp_status tgp_ctx_set_stream(tgp_ctx ctx, void *hip_stream) {
    if (!ctx) return fail(nullptr, TGP_EINVAL, "ctx is NULL");
    ctx->stream = (hipStream_t)hip_stream;
    return TGP_OK;
}

const char *tgp_last_error(tgp_ctx ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

tgp_status tgp_ctx_set_cache_budget(tgp_ctx ctx, size_t bytes) {
    if (!ctx) return fail(nullptr, TGP_EINVAL, "ctx is NULL");
    ctx->cache_budget = bytes;
    return TGP_OK;
}

tgp_status tgp_ctx_set_timing(tgp_ctx ctx, int32_t enable) {
    if (!ctx) return fail(nullptr, TGP_EINVAL, "ctx is NULL");
    if (enable && !ctx->ev_ready) {
        HCHK(ctx, hipSetDevice(ctx->device));
        for (auto &e : ctx->ev) HCHK(ctx, hipEventCreate(&e));
        ctx->ev_ready = true;
    }
    ctx->timing = enable != 0;
    return TGP_OK;
}

tgp_status tgp_last_timing(tgp_ctx ctx, tgp_timing *out) {
    if (!ctx || !out) return fail(ctx, TGP_EINVAL, "NULL argument");
    tgp_timing t = ctx->times;
    t.fill_ms = t.interp_ms = t.finalize_ms = 0;
    t.breed_shape_ms = t.breed_plan_ms = t.breed_write_ms = 0;
    if (ctx->timing && ctx->ev_ready) {
        // device time between two recorded events (0 when one never was)
        auto span = [ctx](int a, int b, double *out) -> hipError_t {
            if (!(ctx->recorded >> a & 1u) || !(ctx->recorded >> b & 1u)) return hipSuccess;
            hipError_t e = hipEventSynchronize(ctx->ev[b]);
            float ms = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ctx->ev[a], ctx->ev[b]);
            if (e == hipSuccess) *out = ms;
            return e;
        };
        if (ctx->fill_recorded) HCHK(ctx, span(0, 1, &t.fill_ms));
        HCHK(ctx, span(2, 3, &t.interp_ms));
        HCHK(ctx, span(4, 5, &t.finalize_ms));
        HCHK(ctx, span(6, 7, &t.breed_shape_ms));
        HCHK(ctx, span(7, 8, &t.breed_plan_ms));
        HCHK(ctx, span(9, 10, &t.breed_write_ms));
    }
    *out = t;
    return TGP_OK;
}

// Tuning knobs (used by the autotuner and tests): cases per lane (2 or 4, 0 =
// automatic) and tiles per work item (0 = automatic).
tgp_status tgp_ctx_set_tuning(tgp_ctx ctx, int32_t cases_per_lane, int32_t tiles_per_item) {
    if (!ctx) return fail(nullptr, TGP_EINVAL, "ctx is NULL");
    if (cases_per_lane != 0 && !interp_variant_exists(cases_per_lane, interp_max_stack()))
        return fail(ctx, TGP_EINVAL, "no interpreter with %d cases per lane", cases_per_lane);
    if (tiles_per_item < 0) return fail(ctx, TGP_EINVAL, "tiles_per_item < 0");
    ctx->force_K = cases_per_lane;
    ctx->force_tiles = tiles_per_item;
    ctx->tile_cap = 0;
    return TGP_OK;
}

tgp_status tgp_ctx_set_hashing(tgp_ctx ctx, int32_t commutative) {
    if (!ctx) return fail(nullptr, TGP_EINVAL, "ctx is NULL");
    ctx->commute = commutative != 0;
    return TGP_OK;
}

tgp_status tgp_ctx_set_rewrite(tgp_ctx ctx, int32_t on) {
    if (!ctx) return fail(nullptr, TGP_EINVAL, "ctx is NULL");
    ctx->rewrite = on != 0;
    return TGP_OK;
}

tgp_status tgp_ctx_set_folding(tgp_ctx ctx, int32_t on) {
    if (!ctx) return fail(nullptr, TGP_EINVAL, "ctx is NULL");
    ctx->fold = on != 0;
    return TGP_OK;
}

tgp_status tgp_ctx_set_stack(tgp_ctx ctx, int32_t lds) {
    if (!ctx) return fail(nullptr, TGP_EINVAL, "ctx is NULL");
    ctx->stack_lds = lds != 0;
    return TGP_OK;
}

tgp_status tgp_ctx_set_plan(tgp_ctx ctx, int32_t reorder_children, double cache_access_cost) {
    if (!ctx) return fail(nullptr, TGP_EINVAL, "ctx is NULL");
    ctx->reorder = reorder_children != 0;
    ctx->cache_access_cost = cache_access_cost;
    return TGP_OK;
}

tgp_status tgp_debug_set_hash_bits(int32_t bits) {
    if (bits < 0 || bits > 32) return fail(nullptr, TGP_EINVAL, "bits must be 0..32");
    g_debug_hash_bits = (uint32_t)bits;
    return TGP_OK;
}

// ---------------------------------------------------------------- domains
tgp_status tgp_domain_create(tgp_ctx ctx, int32_t ndim, const int64_t *shape, const double *lo,
                             const double *hi, tgp_domain *out) {
    if (!ctx || !out || !shape) return fail(ctx, TGP_EINVAL, "NULL argument");
    *out = nullptr;
    if (ndim < 1 || ndim > 3) return fail(ctx, TGP_ESHAPE, "ndim must be 1..3, got %d", ndim);
    int64_t cases = 1;
    for (int k = 0; k < ndim; ++k) {
        if (shape[k] < 1) return fail(ctx, TGP_ESHAPE, "shape[%d] = %lld < 1", k, (long long)shape[k]);
        cases *= shape[k];
        if (cases > (1LL << 30)) return fail(ctx, TGP_ESHAPE, "more than 2^30 cases");
    }
    HCHK(ctx, hipSetDevice(ctx->device));
    tgp_domain d = new tgp_domain_s();
    d->ctx = ctx;
    d->ndim = ndim;
    d->cases = cases;
    int64_t st = 1;
    for (int k = ndim - 1; k >= 0; --k) {
        d->shape[k] = shape[k];
        d->stride[k] = st;
        st *= shape[k];
    }
    for (int k = 0; k < ndim; ++k) {
        const double l = lo ? lo[k] : -1.0, h = hi ? hi[k] : 1.0;
        d->lo[k] = l;
        d->hi[k] = h;
        std::vector<float> tab(shape[k]);
        for (int64_t i = 0; i < shape[k]; ++i) {
            const double v = shape[k] == 1 ? l : l + (h - l) * (double)i / (double)(shape[k] - 1);
            tab[i] = (float)v;
        }
        hipError_t e = hipMalloc((void **)&d->coord[k], sizeof(float) * shape[k]);
        if (e == hipSuccess)
            e = hipMemcpy(d->coord[k], tab.data(), sizeof(float) * shape[k], hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            tgp_domain_destroy(d);
            return fail(ctx, TGP_EHIP, "coordinate table: %s", hipGetErrorString(e));
        }
    }
    *out = d;
    return TGP_OK;
}

void tgp_domain_destroy(tgp_domain d) {
    if (!d) return;
    for (int k = 0; k < 3; ++k) hipFree(d->coord[k]);
    delete d;
}

int64_t tgp_domain_cases(tgp_domain d) { return d ? d->cases : -1; }

// -------------------------------------------------------------------- DAG
tgp_status tgp_build_dag(tgp_ctx ctx, const tgp_population *pop, tgp_dag *out) {
    if (!ctx || !pop || !out) return fail(ctx, TGP_EINVAL, "NULL argument");
    *out = nullptr;
    const double t0 = now_ms();
    if (pop->n_individuals < 0 || pop->n_channels < 1)
        return fail(ctx, TGP_EINVAL, "n_individuals < 0 or n_channels < 1");
    if (pop->memory != TGP_MEM_HOST && pop->memory != TGP_MEM_DEVICE)
        return fail(ctx, TGP_EINVAL, "memory must be TGP_MEM_HOST or TGP_MEM_DEVICE");
    const int64_t R = (int64_t)pop->n_individuals * pop->n_channels;
    if (R > 0 && (!pop->offsets || !pop->tokens)) return fail(ctx, TGP_EINVAL, "NULL offsets/tokens");
    HCHK(ctx, hipSetDevice(ctx->device));
    int64_t T = 0;
    const int64_t *off_dev = nullptr;
    const tgp_token *tok_dev = nullptr;
    int64_t *off_own = nullptr;
    tgp_token *tok_own = nullptr;
    if (R > 0) {
        if (pop->memory == TGP_MEM_HOST) {
            if (pop->offsets[0] != 0) return fail(ctx, TGP_EINVAL, "offsets[0] must be 0");
            for (int64_t r = 0; r < R; ++r)
                if (pop->offsets[r + 1] < pop->offsets[r])
                    return fail(ctx, TGP_EINVAL, "offsets decrease at tree %lld", (long long)r);
            T = pop->offsets[R];
            if (T > 0x7fffffffLL) return fail(ctx, TGP_EINVAL, "more than 2^31-1 tokens");
            // offsets and tokens in one block, through the pinned staging
            const size_t ob = sizeof(int64_t) * (R + 1), tb = sizeof(tgp_token) * T;
            void *stage = nullptr;
            HCHK(ctx, ctx->pool.alloc((void **)&off_own, ob + tb));
            tok_own = reinterpret_cast<tgp_token *>(off_own + R + 1);
            HCHK(ctx, ctx_pinned(ctx, ob + tb, &stage));
            memcpy(stage, pop->offsets, ob);
            if (T) memcpy((char *)stage + ob, pop->tokens, tb);
            HCHK(ctx, hipMemcpyAsync(off_own, stage, ob + tb, hipMemcpyHostToDevice, ctx->stream));
            HCHK(ctx, ctx_pinned_enqueued(ctx));
            off_dev = off_own;
            tok_dev = tok_own;
        } else {
            int64_t ends[2];
            HCHK(ctx, hipMemcpyAsync(&ends[0], pop->offsets, sizeof(int64_t), hipMemcpyDeviceToHost,
                                     ctx->stream));
            HCHK(ctx, hipMemcpyAsync(&ends[1], pop->offsets + R, sizeof(int64_t),
                                     hipMemcpyDeviceToHost, ctx->stream));
            HCHK(ctx, hipStreamSynchronize(ctx->stream));
            if (ends[0] != 0) return fail(ctx, TGP_EINVAL, "offsets[0] must be 0");
            T = ends[1];
            if (T < 0 || T > 0x7fffffffLL) return fail(ctx, TGP_EINVAL, "bad token count");
            off_dev = pop->offsets;
            tok_dev = pop->tokens;
        }
    }
    tgp_dag d = new tgp_dag_s();
    d->ctx = ctx;
    d->n_ind = pop->n_individuals;
    d->n_ch = pop->n_channels;
    d->stats.n_roots = R;
    d->stats.max_var = -1;
    if (R > 0) {
        char msg[256] = "";
        DagBuildResult br =
            build_dag_device(tok_dev, off_dev, R, T, &d->dev, ctx->pool, ctx->stream, msg, sizeof msg,
                             ctx->commute != 0, ctx->rewrite != 0);
        ctx->pool.release(off_own);  // build_dag_device has synchronised the stream
        if (br.status != TGP_OK) {
            delete d;
            return fail(ctx, (tgp_status)br.status, "build_dag: %s", msg);
        }
        const int64_t U = br.U;
        d->op.resize(U);
        d->value.resize(U);
        d->kid.resize(3 * U);
        d->height.resize(U);
        d->roots.resize(R);
        d->mult.resize(U);
        d->indeg.resize(U);
        // one readback of the whole DAG block through the pinned staging
        const size_t bytes = DagDevice::blob_bytes(U, R);
        void *stage = nullptr;
        hipError_t e = ctx_pinned(ctx, bytes, &stage);
        if (e == hipSuccess)
            e = hipMemcpyAsync(stage, d->dev.blob, bytes, hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e == hipSuccess) {
            const int32_t *h = static_cast<const int32_t *>(stage);
            memcpy(d->op.data(), h, sizeof(int32_t) * U);
            memcpy(d->value.data(), h + U, sizeof(float) * U);
            memcpy(d->kid.data(), h + 2 * U, sizeof(int32_t) * 3 * U);
            memcpy(d->height.data(), h + 5 * U, sizeof(int32_t) * U);
            memcpy(d->mult.data(), h + 6 * U, sizeof(int32_t) * U);
            memcpy(d->indeg.data(), h + 7 * U, sizeof(int32_t) * U);
            memcpy(d->roots.data(), h + 8 * U, sizeof(int32_t) * R);
        }
        if (e != hipSuccess) {
            tgp_dag_destroy(d);
            return fail(ctx, TGP_EHIP, "DAG readback: %s", hipGetErrorString(e));
        }
        d->stats.tree_nodes = T;
        d->stats.tree_internal = br.tree_internal;
        d->stats.dag_nodes = U;
        int64_t di = 0, sh = 0;
        for (int64_t i = 0; i < U; ++i) {
            const int op = d->op[i] & 0xff;
            if (kArity[op] > 0) {
                ++di;
                if (d->mult[i] >= 2) ++sh;
            }
        }
        d->stats.dag_internal = di;
        d->stats.shared_internal = sh;
        d->stats.max_stack = br.max_stack;
        d->stats.max_height = br.max_height;
        d->stats.max_var = br.max_var;
    }
    *out = d;
    ctx->times.build_dag_ms = now_ms() - t0;
    return TGP_OK;
}

tgp_status tgp_dag_stats_get(tgp_dag dag, tgp_dag_stats *out) {
    if (!dag || !out) return fail(nullptr, TGP_EINVAL, "NULL argument");
    *out = dag->stats;
    return TGP_OK;
}

tgp_status tgp_dag_export(tgp_dag dag, tgp_token *nodes, int32_t *children, int32_t *roots,
                          int32_t *multiplicity, int32_t *indegree) {
    if (!dag) return fail(nullptr, TGP_EINVAL, "dag is NULL");
    const int64_t U = dag->stats.dag_nodes;
    if (nodes)
        for (int64_t i = 0; i < U; ++i) {
            nodes[i].op = (uint8_t)(dag->op[i] & 0xff);
            nodes[i].var = (uint8_t)((dag->op[i] >> 8) & 0xff);
            nodes[i].pad = 0;
            nodes[i].value = dag->value[i];
        }
    if (children && U) memcpy(children, dag->kid.data(), sizeof(int32_t) * 3 * U);
    if (roots && dag->stats.n_roots) memcpy(roots, dag->roots.data(), sizeof(int32_t) * dag->stats.n_roots);
    if (multiplicity && U) memcpy(multiplicity, dag->mult.data(), sizeof(int32_t) * U);
    if (indegree && U) memcpy(indegree, dag->indeg.data(), sizeof(int32_t) * U);
    return TGP_OK;
}

void tgp_dag_destroy(tgp_dag dag) {
    if (!dag) return;
    tgp_ctx ctx = dag->ctx;
    hipSetDevice(ctx->device);
    hipStreamSynchronize(ctx->stream);  // no queued kernel reads the blocks any more
    dag->plan.release(ctx->pool);
    dag_device_free(&dag->dev, ctx->pool);
    delete dag;
}

}  // extern "C"

// ------------------------------------------------------------------ planner
namespace {

// Processors this process may use: its affinity mask (the machine's count
// when the mask cannot be read), capped by a CPU quota of its control group
// (cgroup v2 cpu.max, "quota period"), rounded up.  The planner's threads
// wait for each other level by level, so more threads than processors would
// only slow it down.
unsigned usable_cpus() {
    static const unsigned n = [] {
        unsigned c = std::max(1u, std::thread::hardware_concurrency());
        cpu_set_t set;
        if (sched_getaffinity(0, sizeof set, &set) == 0) c = (unsigned)std::max(1, CPU_COUNT(&set));
        if (FILE *f = fopen("/sys/fs/cgroup/cpu.max", "r")) {
            char quota[32] = "";
            long long period = 0;
            if (fscanf(f, "%31s %lld", quota, &period) == 2 && strcmp(quota, "max") != 0 && period > 0) {
                const long long q = atoll(quota);
                if (q > 0) c = std::min<unsigned>(c, (unsigned)std::max(1LL, (q + period - 1) / period));
            }
            fclose(f);
        }
        return c;
    }();
    return n;
}

// A spin-wait hint to the host processor.
inline void cpu_relax() {
#if defined(__x86_64__) || defined(__i386__)
    __builtin_ia32_pause();
#endif
}

// Runs fn(t, barrier) on T host threads (the caller's thread is t = 0);
// barrier() returns once all T threads have reached it.  A waiting thread
// spins for a few microseconds first (the threads of one level usually
// arrive close together), then yields its processor.
template <class F>
void run_team(int T, F &&fn) {
    std::atomic<int> arrived{0}, generation{0};
    auto barrier = [&]() {
        const int g = generation.load(std::memory_order_acquire);
        if (arrived.fetch_add(1, std::memory_order_acq_rel) + 1 == T) {
            arrived.store(0, std::memory_order_relaxed);
            generation.fetch_add(1, std::memory_order_acq_rel);
        } else {
            for (int i = 0; i < 2000 && generation.load(std::memory_order_acquire) == g; ++i)
                cpu_relax();
            while (generation.load(std::memory_order_acquire) == g) std::this_thread::yield();
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < T; ++t) th.emplace_back([&, t] { fn(t, barrier); });
    fn(0, barrier);
    for (auto &x : th) x.join();
}

// The nodes 0..U-1 ordered by height (id order within a height) on T
// threads: order[first[h] .. first[h+1]) are the nodes of height h.
void height_order(const int32_t *hgt, int64_t U, int T, std::vector<int32_t> &order,
                  std::vector<int64_t> &first) {
    std::vector<std::vector<int64_t>> hist(T);
    int32_t H = 0;
    order.resize(U);
    run_team(T, [&](int t, auto &barrier) {
        const int64_t b = U * t / T, e = U * (t + 1) / T;
        std::vector<int64_t> &c = hist[t];
        for (int64_t n = b; n < e; ++n) {
            if ((size_t)hgt[n] >= c.size()) c.resize(hgt[n] + 1, 0);
            ++c[hgt[n]];
        }
        barrier();
        if (t == 0) {
            for (int i = 0; i < T; ++i) H = std::max(H, (int32_t)hist[i].size() - 1);
            first.assign(H + 2, 0);
            int64_t at = 0;
            for (int32_t h = 0; h <= H; ++h) {
                first[h] = at;
                for (int i = 0; i < T; ++i) {
                    const int64_t k = (size_t)h < hist[i].size() ? hist[i][h] : 0;
                    if ((size_t)h < hist[i].size()) hist[i][h] = at;
                    at += k;
                }
            }
            first[H + 1] = at;
        }
        barrier();
        for (int64_t n = b; n < e; ++n) order[c[hgt[n]]++] = (int32_t)n;
    });
}

struct Planner {
    const tgp_dag_s &d;
    int D;
    size_t budget_slots;
    std::vector<uint8_t> cached;
    std::vector<uint8_t> pre;   // cached and already resident: read, never filled
    std::vector<uint8_t> perm;  // evaluation order of each node's children (index in kPerms)
    std::vector<int32_t> slot, level;
    std::vector<double> cost;
    int64_t spills = 0;

    bool reorder = true;
    double access_cost = 20.0;

    Planner(const tgp_dag_s &dag, int stack, size_t slots) : d(dag), D(stack), budget_slots(slots) {}

    // nodes by height (filled by the parallel preparation or decisions)
    std::vector<int32_t> lorder;
    std::vector<int64_t> lfirst;
    std::vector<uint8_t> folded;  // constant subtrees replaced by their value
    std::vector<float> fold_val;
    // Operator and arity of every node as the planner sees it (a folded node
    // is a constant leaf), filled at the start of decide.
    std::vector<uint8_t> opv, arv;
    double valu_dag = 0;  // cost-model slots of every DAG node once (unfolded)
    int op(int64_t n) const { return opv[n]; }
    int arity(int64_t n) const { return arv[n]; }

    // Whether child j of binary node n, evaluated last, is read by the
    // node's fused form (x, y, a constant or a cached row under an operator
    // with a fused form): it then never occupies a stack slot.  The emitter
    // fuses exactly these (cached only grows, so a later decision can only
    // fuse more).
    bool fuses_last(int64_t n, int j) const {
        const int o = opv[n];
        if (fused_index(o, j == 0 && !is_commutative(o)) < 0) return false;
        const int32_t c = d.kid[3 * n + j];
        if (cached[c]) return true;
        if (opv[c] == TGP_CONST) return true;
        return opv[c] == TGP_VAR && ((d.op[c] >> 8) & 0xff) <= 1;
    }
    // Stack slots a node needs with its children in order o: the i-th
    // child evaluated sits on i values; a fused last child takes none.
    int order_need(int64_t n, int a, const uint8_t *o, const int *r) const {
        if (a == 2 && fuses_last(n, o[1])) return r[o[0]];
        int v = 0;
        for (int q = 0; q < a; ++q) v = std::max(v, q + r[o[q]]);
        return v;
    }

    // The same decisions made level by level (DAG node heights) on T host
    // threads.  Within a level the nodes are independent: each reads only
    // what lower levels decided (bottom-up passes) or higher levels
    // contributed (the top-down use counts), so the outcome does not depend
    // on thread timing.  It can differ from the sequential form in one way:
    // two parents of one height that share a child do not see each other's
    // stack spills, so both may spill where the sequential pass spilled
    // once.  Cache-budget admissions are made in node order within a level.
    tgp_status decide_parallel(const std::vector<int32_t> &rootrefs, std::string &why, int T) {
        const int64_t U = (int64_t)d.op.size();
        const int32_t *kid = d.kid.data();
        const int32_t *hgt = d.height.data();
        opv.resize(U);
        arv.resize(U);
        cached.assign(U, 0);
        pre.assign(U, 0);
        cost.resize(U);
        perm.assign(U, 0);
        std::vector<uint8_t> need(U, 1);
        std::vector<int64_t> uses(U, 0);
        std::vector<int32_t> dep(U, 0);
        level.assign(U, -1);
        slot.assign(U, -1);
        const bool any_folded = !folded.empty();
        auto range = [U, T](int t, int64_t &b, int64_t &e) {
            b = U * t / T;
            e = U * (t + 1) / T;
        };
        if (lorder.size() != (size_t)U) height_order(hgt, U, T, lorder, lfirst);
        const std::vector<int32_t> &order = lorder;
        const std::vector<int64_t> &lvl_first = lfirst;
        const int32_t H = (int32_t)lvl_first.size() - 2;
        std::vector<double> valu_part(T, 0.0);
        std::vector<std::vector<int32_t>> spill(T), cand(T);
        std::vector<int64_t> slot_part(T + 1, 0);
        std::atomic<int64_t> used{0};
        tgp_status result = TGP_OK;
        auto level_nodes = [&](int32_t h, int t, int64_t &b, int64_t &e) {
            const int64_t n0 = lvl_first[h], n1 = lvl_first[h + 1];
            b = n0 + (n1 - n0) * t / T;
            e = n0 + (n1 - n0) * (t + 1) / T;
        };
        auto mark = [&](int32_t c) {  // returns whether c was not cached before
            return __atomic_exchange_n(&cached[c], (uint8_t)1, __ATOMIC_RELAXED) == 0;
        };
        run_team(T, [&](int t, auto &barrier) {
            int64_t b, e;
            range(t, b, e);
            // operators, arities, cost-model work
            double v = 0;
            for (int64_t n = b; n < e; ++n) {
                const int o = d.op[n] & 0xff;
                v += kOpCost[o];
                const int x = any_folded && folded[n] ? TGP_CONST : o;
                opv[n] = (uint8_t)x;
                arv[n] = (uint8_t)kArity[x];
            }
            valu_part[t] = v;
            barrier();
            // cost, bottom-up
            for (int32_t h = 0; h <= H; ++h) {
                int64_t lb, le;
                level_nodes(h, t, lb, le);
                for (int64_t i = lb; i < le; ++i) {
                    const int32_t n = order[i];
                    double c = kOpCost[opv[n]];
                    const int32_t *k = kid + 3 * (int64_t)n;
                    const int a = arv[n];
                    if (a > 0) c += cost[k[0]];
                    if (a > 1) c += cost[k[1]];
                    if (a > 2) c += cost[k[2]];
                    cost[n] = c;
                }
                barrier();
            }
            // resident subtrees and warp sources
            if (!d.precached.empty() && access_cost >= 0)
                for (int64_t n = b; n < e; ++n)
                    if (d.precached[n] && arv[n] > 0 && cost[n] > access_cost) cached[n] = pre[n] = 1;
            barrier();
            int64_t u = 0;
            for (int64_t n = b; n < e; ++n)
                if (opv[n] == TGP_WARP && mark(kid[3 * n])) ++u;
            used.fetch_add(u);
            barrier();
            // stack need, bottom-up; spills of one level applied after it
            for (int32_t h = 0; h <= H; ++h) {
                int64_t lb, le;
                level_nodes(h, t, lb, le);
                spill[t].clear();
                for (int64_t i = lb; i < le; ++i) {
                    const int32_t n = order[i];
                    const int a = arv[n];
                    if (a == 0) continue;
                    const int32_t *k = kid + 3 * (int64_t)n;
                    auto ref_need = [&](int32_t c) { return cached[c] ? 1 : (int)need[c]; };
                    if (opv[n] == TGP_WARP) {  // t0 then t1 on the stack, in that order
                        int r1 = ref_need(k[1]), r2 = ref_need(k[2]);
                        while (std::max(r1, 1 + r2) > D) {
                            const int32_t c = r1 >= r2 ? k[1] : k[2];
                            spill[t].push_back(c);
                            if (k[1] == c) r1 = 1;
                            if (k[2] == c) r2 = 1;
                        }
                        need[n] = (uint8_t)std::max(r1, 1 + r2);
                        continue;
                    }
                    if (a == 1) {
                        need[n] = (uint8_t)ref_need(k[0]);
                        continue;
                    }
                    int r[3] = {0, 0, 0};
                    for (int j = 0; j < a; ++j) r[j] = ref_need(k[j]);
                    for (;;) {
                        int best_p = 0, best = 1 << 30;
                        const int n_orders = reorder ? (a == 3 ? 6 : 2) : 1;
                        for (int p = 0; p < n_orders; ++p) {
                            const uint8_t *o = a == 2 ? (p ? kPerms[2] : kPerms[0]) : kPerms[p];
                            const int vv = order_need(n, a, o, r);
                            if (vv < best) {
                                best = vv;
                                best_p = a == 2 ? (p ? 2 : 0) : p;
                            }
                        }
                        if (best <= D) {
                            need[n] = (uint8_t)best;
                            perm[n] = (uint8_t)best_p;
                            break;
                        }
                        int wj = 0;
                        for (int j = 1; j < a; ++j)
                            if (r[j] > r[wj]) wj = j;
                        spill[t].push_back(k[wj]);
                        for (int j = 0; j < a; ++j)
                            if (k[j] == k[wj]) r[j] = 1;
                    }
                }
                barrier();
                int64_t su = 0;
                for (int32_t c : spill[t])
                    if (mark(c)) ++su;
                used.fetch_add(su);
                barrier();
            }
            if (t == 0) {
                spills = used.load();
                if ((size_t)spills > budget_slots) {
                    why = "the subtree cache needed to bound the evaluator stack exceeds the cache budget";
                    result = TGP_ENOMEM;
                }
            }
            barrier();
            if (result != TGP_OK) return;
            // use counts, top-down; caching where it pays for its HBM traffic
            for (int64_t n = b; n < e; ++n) uses[n] = rootrefs[n];
            barrier();
            for (int32_t h = H; h >= 0; --h) {
                int64_t lb, le;
                level_nodes(h, t, lb, le);
                cand[t].clear();
                for (int64_t i = lb; i < le; ++i) {
                    const int32_t n = order[i];
                    const double un = (double)uses[n];
                    if (!cached[n] && access_cost >= 0 && arv[n] > 0 && un >= 2 &&
                        cost[n] * (un - 1) > access_cost * (un + 1))
                        cand[t].push_back(n);
                }
                barrier();
                if (t == 0) {  // admissions in node order (within the budget)
                    for (int i = 0; i < T; ++i)
                        for (int32_t n : cand[i])
                            if ((size_t)used.load() < budget_slots) {
                                cached[n] = 1;
                                used.fetch_add(1);
                            }
                }
                barrier();
                // A count is at most the number of occurrences of the node in
                // the population's trees (each unit is one root-to-node path),
                // so it cannot overflow.  Leaves are skipped unless cached (a
                // warp source): nothing reads their counts, and they are the
                // most shared nodes, so their additions would contend most.
                for (int64_t i = lb; i < le; ++i) {
                    const int32_t n = order[i];
                    const int64_t contrib = pre[n] ? 0 : (cached[n] ? 1 : uses[n]);
                    if (contrib > 0)
                        for (int j = 0; j < arv[n]; ++j) {
                            const int32_t c = kid[3 * (int64_t)n + j];
                            if (arv[c] > 0 || cached[c]) __atomic_fetch_add(&uses[c], contrib, __ATOMIC_RELAXED);
                        }
                }
                barrier();
            }
            // spills below resident subtrees that nothing else reads
            for (int64_t n = b; n < e; ++n)
                if (cached[n] && !pre[n] && uses[n] == 0) cached[n] = 0;
            barrier();
            // levels of the cached nodes, bottom-up
            for (int32_t h = 0; h <= H; ++h) {
                int64_t lb, le;
                level_nodes(h, t, lb, le);
                for (int64_t i = lb; i < le; ++i) {
                    const int32_t n = order[i];
                    int32_t dp = 0;
                    for (int j = 0; j < arv[n]; ++j) {
                        const int32_t c = kid[3 * (int64_t)n + j];
                        dp = std::max(dp, cached[c] ? level[c] + 1 : dep[c]);
                    }
                    dep[n] = dp;
                    if (pre[n]) level[n] = -1;  // available before the first fill level
                    else if (cached[n]) level[n] = dp;
                }
                barrier();
            }
            // slots in node order
            int64_t cnt = 0;
            for (int64_t n = b; n < e; ++n) cnt += cached[n];
            slot_part[t + 1] = cnt;
            barrier();
            if (t == 0)
                for (int i = 0; i < T; ++i) slot_part[i + 1] += slot_part[i];
            barrier();
            int32_t ns = (int32_t)slot_part[t];
            for (int64_t n = b; n < e; ++n)
                if (cached[n]) slot[n] = ns++;
        });
        valu_dag = 0;
        for (double v : valu_part) valu_dag += v;
        return result;
    }

    // Decide the cached nodes; returns TGP_OK or an error.
    tgp_status decide(const std::vector<int32_t> &rootrefs, std::string &why) {
        const int64_t U = (int64_t)d.op.size();
        const int32_t *kid = d.kid.data();
        opv.resize(U);
        arv.resize(U);
        valu_dag = 0;
        const bool any_folded = !folded.empty();
        for (int64_t n = 0; n < U; ++n) {
            const int o = d.op[n] & 0xff;
            valu_dag += kOpCost[o];
            const int v = any_folded && folded[n] ? TGP_CONST : o;
            opv[n] = (uint8_t)v;
            arv[n] = (uint8_t)kArity[v];
        }
        cached.assign(U, 0);
        pre.assign(U, 0);
        cost.resize(U);
        for (int64_t n = 0; n < U; ++n) {
            double c = kOpCost[opv[n]];
            const int32_t *k = kid + 3 * n;
            const int a = arv[n];
            if (a > 0) c += cost[k[0]];
            if (a > 1) c += cost[k[1]];
            if (a > 2) c += cost[k[2]];
            cost[n] = c;
        }
        // Subtrees whose values over this domain are already resident (kept
        // from an earlier evaluation) are read instead of recomputed when
        // recomputing costs more than the read.
        if (!d.precached.empty() && access_cost >= 0)
            for (int64_t n = 0; n < U; ++n)
                if (d.precached[n] && arv[n] > 0 && cost[n] > access_cost) cached[n] = pre[n] = 1;
        // The value a warp gathers from is read at other cases than the one
        // being evaluated, so it is always materialised (a cached row).
        size_t used = 0;
        for (int64_t n = 0; n < U; ++n)
            if (opv[n] == TGP_WARP && !cached[kid[3 * n]]) {
                cached[kid[3 * n]] = 1;
                ++used;
            }
        // Bottom-up: bound the register stack of every program.  Children are
        // evaluated in decreasing order of the stack they need (Sethi-Ullman,
        // a fused last operand taking no slot); a node whose children still
        // cannot be evaluated within D slots gets its most demanding child's
        // subtree spilled to a cache row.
        std::vector<uint8_t> need(U, 1);
        perm.assign(U, 0);
        auto ref_need = [&](int32_t c) { return cached[c] ? 1 : (int)need[c]; };
        for (int64_t n = 0; n < U; ++n) {
            const int a = arv[n];
            if (a == 0) continue;
            const int32_t *k = kid + 3 * n;
            if (opv[n] == TGP_WARP) {  // t0 then t1 on the stack, in that order
                for (;;) {
                    const int32_t c1 = k[1], c2 = k[2];
                    const int r1 = ref_need(c1), r2 = ref_need(c2);
                    const int v = std::max(r1, 1 + r2);
                    if (v <= D) {
                        need[n] = (uint8_t)v;
                        break;
                    }
                    cached[r1 >= r2 ? c1 : c2] = 1;
                    ++used;
                }
                continue;
            }
            if (a == 1) {  // a unary node needs what its operand needs
                need[n] = (uint8_t)ref_need(k[0]);
                continue;
            }
            for (;;) {
                int r[3] = {0, 0, 0};
                for (int j = 0; j < a; ++j) r[j] = ref_need(k[j]);
                // stable sort of child positions by need, largest first
                int best_p = 0, best = 1 << 30;
                const int n_orders = reorder ? (a == 3 ? 6 : 2) : 1;
                for (int p = 0; p < n_orders; ++p) {
                    const uint8_t *o = a == 2 ? (p ? kPerms[2] : kPerms[0]) : kPerms[p];
                    const int v = order_need(n, a, o, r);
                    if (v < best) {
                        best = v;
                        best_p = a == 2 ? (p ? 2 : 0) : p;
                    }
                }
                if (best <= D) {
                    need[n] = (uint8_t)best;
                    perm[n] = (uint8_t)best_p;
                    break;
                }
                int wj = 0;
                for (int j = 1; j < a; ++j)
                    if (r[j] > r[wj]) wj = j;
                cached[k[wj]] = 1;
                ++used;
            }
        }
        spills = (int64_t)used;
        if (used > budget_slots) {
            why = "the subtree cache needed to bound the evaluator stack exceeds the cache budget";
            return TGP_ENOMEM;
        }
        // Top-down: how often each node would be evaluated, and whether
        // caching it pays for its HBM traffic (within the remaining budget).
        std::vector<double> uses(rootrefs.begin(), rootrefs.end());
        for (int64_t n = U - 1; n >= 0; --n) {
            const int a = arv[n];
            if (!cached[n] && access_cost >= 0 && a > 0 && uses[n] >= 2 && used < budget_slots) {
                const double save = cost[n] * (uses[n] - 1);
                const double pay = access_cost * (uses[n] + 1);
                if (save > pay) {
                    cached[n] = 1;
                    ++used;
                }
            }
            const double contrib = pre[n] ? 0.0 : (cached[n] ? 1.0 : uses[n]);
            if (contrib > 0)
                for (int j = 0; j < a; ++j) uses[kid[3 * n + j]] += contrib;
        }
        // A spill below a resident subtree that nothing else reads is dropped
        // (its fill would be wasted).  Then levels and slots.
        std::vector<int32_t> dep(U, 0);
        level.assign(U, -1);
        slot.assign(U, -1);
        int32_t ns = 0;
        for (int64_t n = 0; n < U; ++n) {
            if (cached[n] && !pre[n] && uses[n] == 0) {
                cached[n] = 0;
                --used;
            }
            int32_t dp = 0;
            const int32_t *k = kid + 3 * n;
            for (int j = 0; j < arv[n]; ++j) {
                const int32_t c = k[j];
                dp = std::max(dp, cached[c] ? level[c] + 1 : dep[c]);
            }
            dep[n] = dp;
            if (pre[n]) {
                level[n] = -1;  // available before the first fill level
                slot[n] = ns++;
            } else if (cached[n]) {
                level[n] = dp;
                slot[n] = ns++;
            }
        }
        return TGP_OK;
    }

    // The FP32 bits of constant (or folded) node n; every NaN becomes the
    // quiet NaN 0x7fc00000, so that no signalling NaN reaches the
    // interpreter's min and max (ops_device.h).
    uint32_t const_word(int64_t n) const {
        const float v = !folded.empty() && folded[n] ? fold_val[n] : d.value[n];
        uint32_t w;
        memcpy(&w, &v, 4);
        return v == v ? w : 0x7fc00000u;
    }

    // The fused-form kind and .y word of child c when c can be a fused
    // operand (x, y, a constant or a cached row), else -1.
    int fuse_operand(int32_t c, uint32_t &y) const {
        if (cached[c]) {
            y = (uint32_t)slot[c];
            return kFuseCache;
        }
        const int o = op(c);
        if (o == TGP_VAR) {
            const int v = (d.op[c] >> 8) & 0xff;
            return v == 0 ? kFuseX : (v == 1 ? kFuseY : -1);
        }
        if (o == TGP_CONST) {
            y = const_word(c);
            return kFuseConst;
        }
        return -1;
    }

    // Postfix program of node n (n itself is expanded even when cached).
    // Every instruction carries the stack depth before it (.x bits 8-15).
    // A binary operator whose last-evaluated child is a terminal takes its
    // fused form and reads that child itself.  Adds the cost-model slots of
    // its instructions to *valu; sets *ext when it emits a bitwise operator,
    // warp or the third axis, *warp_used for warp.
    void emit(int32_t root, std::vector<uint2> &code, int64_t &cache_reads, double *valu, bool *ext,
              bool *warp_used) const {
        struct Frame {
            int32_t n, done;  // node, children emitted
            int32_t fv;       // fused form index, or -1
        };
        std::vector<Frame> st;
        uint32_t S = 0;  // stack depth before the next instruction
        auto frame = [&](int32_t n) {
            Frame f{n, 0, -1};
            const int o = op(n);
            if (n == root || !cached[n]) {
                if (arity(n) == 2 && o != TGP_WARP) {
                    const int last = kPerms[perm[n]][1];
                    uint32_t y = 0;
                    if (fuse_operand(d.kid[3 * n + last], y) >= 0) {
                        const bool rev = last == 0 && !is_commutative(o);
                        f.fv = fused_index(o, rev);
                    }
                }
            }
            return f;
        };
        st.push_back(frame(root));
        while (!st.empty()) {
            Frame &top = st.back();
            const int32_t n = top.n;
            const bool leafish = arity(n) == 0 || (n != root && cached[n]);
            const bool warp = op(n) == TGP_WARP;  // stack children t0, t1 only
            const int stacked = leafish ? 0 : (warp ? 2 : arity(n)) - (top.fv >= 0 ? 1 : 0);
            if (top.done < stacked) {
                const int32_t c = warp ? d.kid[3 * n + 1 + top.done] : d.kid[3 * n + kPerms[perm[n]][top.done]];
                ++top.done;
                st.push_back(frame(c));
                continue;
            }
            uint2 ins{0, 0};
            uint32_t after = S + 1;
            if (n != root && cached[n]) {
                ins.x = I_CACHE;
                ins.y = (uint32_t)slot[n];
                ++cache_reads;
                *valu += 1.0;
            } else {
                const int o = op(n);
                *valu += kOpCost[o];
                if (o == TGP_VAR) {
                    const int v = (d.op[n] >> 8) & 0xff;
                    ins.x = v == 0 ? I_X : (v == 1 ? I_Y : I_Z);
                    if (v > 1) *ext = true;  // the third axis: extended interpreter only
                } else if (o == TGP_CONST) {
                    ins.x = I_CONST;
                    ins.y = const_word(n);
                } else if (top.fv >= 0) {
                    const int32_t c = d.kid[3 * n + kPerms[perm[n]][1]];
                    const int kind = fuse_operand(c, ins.y);
                    ins.x = kFuseBase + 16 * (uint32_t)kind + (uint32_t)top.fv;
                    if (kind == kFuseCache) {
                        ++cache_reads;
                        *valu += 1.0;
                    } else {
                        *valu += kOpCost[op(c)];
                    }
                    after = S;
                } else if (o == TGP_OR || o == TGP_XOR || o == TGP_AND) {
                    ins.x = kFnBase + TGP_OR;
                    ins.y = (uint32_t)(o - TGP_OR);
                    *ext = true;
                    after = S - 1;
                } else if (o == TGP_WARP) {
                    ins.x = I_WARP;
                    *ext = *warp_used = true;
                    ins.y = (uint32_t)slot[d.kid[3 * n]];
                    ++cache_reads;
                    after = S - 1;
                } else {
                    if (perm[n] == 0 || (kArity[o] == 2 && is_commutative(o)))
                        ins.x = kFnBase + o;
                    else if (kArity[o] == 2)
                        ins.x = kRevBase + o;
                    else
                        ins.x = kPermBase + 6 * ternary_index(o) + perm[n];
                    after = S + 1 - (uint32_t)kArity[o];
                }
            }
            ins.x |= S << 8;
            S = after;
            code.push_back(ins);
            st.pop_back();
        }
        code.push_back(uint2{(S << 8) | I_END, 0});
    }
};

// Programs of many nodes emitted by a few host threads (emission only reads
// the planner's decisions); each node's code stays contiguous, in order.
struct Emitted {
    uint32_t off, len;
    int64_t reads;
    double valu;
    bool ext, warp;  // uses the bitwise operators or warp
};

void emit_all(const Planner &pl, const std::vector<int32_t> &nodes, std::vector<uint2> &code,
              std::vector<Emitted> &out, int threads) {
    const size_t n = nodes.size();
    out.assign(n, Emitted{0, 0, 0, 0.0, false, false});
    const unsigned hw = usable_cpus();
    const int T = n < 512 ? 1 : (int)std::min<unsigned>((unsigned)std::max(threads, 1), hw);
    std::vector<std::vector<uint2>> local(T);
    auto work = [&](int t) {
        const size_t b = n * t / T, e = n * (t + 1) / T;
        for (size_t i = b; i < e; ++i) {
            Emitted &m = out[i];
            m.off = (uint32_t)local[t].size();
            pl.emit(nodes[i], local[t], m.reads, &m.valu, &m.ext, &m.warp);
            m.len = (uint32_t)(local[t].size() - m.off);
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < T; ++t) th.emplace_back(work, t);
    work(0);
    for (auto &x : th) x.join();
    for (int t = 0; t < T; ++t) {
        const uint32_t base = (uint32_t)code.size();
        code.insert(code.end(), local[t].begin(), local[t].end());
        for (size_t i = n * t / T; i < n * (t + 1) / T; ++i) out[i].off += base;
    }
}

}  // namespace

// ------------------------------------------------------------------ planning
// DAGs of at least this many nodes are planned level-parallel on host threads,
// at most kPlanThreads of them (fewer when the host has fewer processors).
constexpr int64_t kParallelDecideNodes = 1 << 15;
constexpr int kPlanThreads = 16;

//
// Planning one DAG runs in phases so that a batch of many DAGs can run each
// phase for all of them at once: host preparation (program lists, the
// variable-free subtrees), constant folding on the device (one round trip
// for the whole batch), the caching and stack decisions with program
// emission (host, one DAG per thread), and the upload of the programs (only
// for the single-DAG calls; a batch packs the host copies itself).
struct PlanJob {
    tgp_dag d;
    int64_t cases;
    Planner pl;
    std::vector<int32_t> rootrefs, ind_rows, store_of, store_list;
    std::vector<std::pair<int32_t, int32_t>> reduce_list;  // (root node, channel)
    // variable-free nodes by height (folding), this job's place in the batch
    std::vector<int32_t> fold_first, fold_list;
    size_t fold_list_at = 0, fold_val_at = 0;
    double t_decide = 0, t_emit = 0;
    // fill-program figures carried from the fill emission to the root one
    int64_t cache_reads_fill = 0;
    double valu_fill = 0;
    tgp_status st = TGP_OK;
    std::string err;
    PlanJob(tgp_dag dag, int64_t n_cases, int D, size_t budget)
        : d(dag), cases(n_cases), pl(*dag, D, budget) {}
};

static void plan_prepare(PlanJob &w, bool fold, int threads = 1) {
    tgp_dag d = w.d;
    Plan &P = d->plan;
    const int64_t U = d->stats.dag_nodes, R = d->stats.n_roots;
    const int n_ch = d->n_ch;
    // distinct programs
    std::unordered_map<int64_t, int32_t> reduce_of;  // (root id, ch) -> program
    w.rootrefs.assign(U, 0);
    w.ind_rows.resize(R);
    w.store_of.assign(U, -1);
    P.store_rows.assign(R, -1);
    P.dup_src.assign(R, -1);
    for (int64_t r = 0; r < R; ++r) {
        const int32_t n = d->roots[r];
        const int ch = (int)(r % n_ch);
        const int64_t key = (int64_t)n * n_ch + ch;
        auto it = reduce_of.find(key);
        if (it == reduce_of.end()) {
            it = reduce_of.emplace(key, (int32_t)w.reduce_list.size()).first;
            w.reduce_list.push_back({n, ch});
            w.rootrefs[n] += 1;
        }
        w.ind_rows[r] = it->second;
        if (w.store_of[n] < 0) {
            w.store_of[n] = (int32_t)r;
            w.store_list.push_back(n);
            P.store_rows[r] = (int32_t)r;
        } else {
            P.dup_src[r] = w.store_of[n];
        }
    }
    if (!fold) return;
    // Constant subtrees (no variable below) that some non-constant node or a
    // root uses are folded: marked in pl.folded, evaluated on the device.
    // novar: no variable below; 2 = also an operator (a foldable subtree)
    std::vector<uint8_t> novar(U, 0), use(U, 0);
    int64_t n_use = 0;
    auto mark = [&](int32_t c) {
        if (novar[c] == 2 && !use[c]) {
            use[c] = 1;
            ++n_use;
        }
    };
    const int32_t *kid = d->kid.data();
    const int32_t *height = d->height.data();
    const int T = (int)std::min<unsigned>((unsigned)std::max(threads, 1), usable_cpus());
    if (U >= kParallelDecideNodes && T > 1) {
        // level by level on T threads; the height order is kept for the
        // parallel decisions
        std::vector<int32_t> &order = w.pl.lorder;
        std::vector<int64_t> &first = w.pl.lfirst;
        height_order(height, U, T, order, first);
        const int32_t H = (int32_t)first.size() - 2;
        std::atomic<int64_t> marked{0};
        run_team(T, [&](int t, auto &barrier) {
            int64_t m = 0;
            for (int32_t h = 0; h <= H; ++h) {
                const int64_t n0 = first[h], n1 = first[h + 1];
                for (int64_t i = n0 + (n1 - n0) * t / T; i < n0 + (n1 - n0) * (t + 1) / T; ++i) {
                    const int32_t n = order[i];
                    const int o = d->op[n] & 0xff;
                    const int a = kArity[o];
                    bool nv = o != TGP_VAR;
                    for (int j = 0; j < a; ++j) nv = nv && novar[kid[3 * (int64_t)n + j]];
                    if (nv) {
                        novar[n] = a > 0 ? 2 : 1;
                    } else {
                        for (int j = 0; j < a; ++j) {
                            const int32_t c = kid[3 * (int64_t)n + j];
                            if (novar[c] == 2) {
                                __atomic_store_n(&use[c], (uint8_t)1, __ATOMIC_RELAXED);
                                ++m;
                            }
                        }
                    }
                }
                barrier();
            }
            marked.fetch_add(m);
        });
        n_use = marked.load();
        for (int32_t r : d->roots) mark(r);
        if (n_use == 0) return;
        w.fold_first.assign(1, 0);
        for (int32_t h = 0; h <= H; ++h) {
            for (int64_t i = first[h]; i < first[h + 1]; ++i)
                if (novar[order[i]] == 2) w.fold_list.push_back(order[i]);
            w.fold_first.push_back((int32_t)w.fold_list.size());
        }
        // up to the highest variable-free operator node
        while (w.fold_first.size() > 1 && w.fold_first[w.fold_first.size() - 2] == w.fold_first.back())
            w.fold_first.pop_back();
        w.pl.folded.swap(use);
        return;
    }
    // the variable-free operator nodes by height (constant leaves are read
    // from the node values by the fold kernel)
    std::vector<std::vector<int32_t>> by_h;
    for (int64_t n = 0; n < U; ++n) {  // children have smaller ids
        const int o = d->op[n] & 0xff;
        const int a = kArity[o];
        bool nv = o != TGP_VAR;
        for (int j = 0; j < a; ++j) nv = nv && novar[kid[3 * n + j]];
        if (nv) {
            novar[n] = a > 0 ? 2 : 1;
            if (a > 0) {
                const int32_t h = height[n];
                if ((int32_t)by_h.size() <= h) by_h.resize(h + 1);
                by_h[h].push_back((int32_t)n);
            }
        } else {
            for (int j = 0; j < a; ++j) mark(kid[3 * n + j]);
        }
    }
    for (int32_t r : d->roots) mark(r);
    if (n_use == 0) return;
    // children before parents: one list, cut at each height
    w.fold_first.assign(by_h.size() + 1, 0);
    for (size_t h = 0; h < by_h.size(); ++h) w.fold_first[h + 1] = w.fold_first[h] + (int32_t)by_h[h].size();
    w.fold_list.reserve(w.fold_first.back());
    for (const auto &v : by_h) w.fold_list.insert(w.fold_list.end(), v.begin(), v.end());
    w.pl.folded.swap(use);
}

// Folds the marked subtrees of every job: one upload of the node lists, one
// launch per height over all jobs, one read-back of the values.
static tgp_status fold_run(tgp_ctx ctx, const std::vector<PlanJob *> &jobs) {
    std::vector<PlanJob *> fj;
    size_t n_list = 0, n_val = 0;
    int32_t max_h = -1;
    for (PlanJob *w : jobs)
        if (!w->fold_list.empty()) {
            w->fold_list_at = n_list;
            w->fold_val_at = n_val;
            n_list += w->fold_list.size();
            n_val += (size_t)w->d->stats.dag_nodes;
            max_h = std::max(max_h, (int32_t)w->fold_first.size() - 2);
            fj.push_back(w);
        }
    if (fj.empty()) return TGP_OK;
    // the (job, node) lists of all jobs ordered by height, then job
    std::vector<int32_t> hfirst(max_h + 2, 0);
    for (PlanJob *w : fj)
        for (size_t h = 0; h + 1 < w->fold_first.size(); ++h)
            hfirst[h + 1] += w->fold_first[h + 1] - w->fold_first[h];
    for (int h = 0; h <= max_h; ++h) hfirst[h + 1] += hfirst[h];
    const size_t desc_bytes = sizeof(FoldDesc) * fj.size();
    const size_t list_off = (desc_bytes + 255) & ~(size_t)255;
    const size_t val_off = (list_off + sizeof(int2) * n_list + 255) & ~(size_t)255;
    const size_t up_bytes = list_off + sizeof(int2) * n_list;
    void *blk = nullptr, *stage = nullptr;
    hipError_t e = ctx->pool.alloc(&blk, val_off + sizeof(float) * n_val);
    if (e == hipSuccess) e = ctx_pinned(ctx, std::max(up_bytes, sizeof(float) * n_val), &stage);
    if (e == hipSuccess) {
        FoldDesc *desc = static_cast<FoldDesc *>(stage);
        int2 *list = reinterpret_cast<int2 *>(static_cast<char *>(stage) + list_off);
        float *val_dev = reinterpret_cast<float *>(static_cast<char *>(blk) + val_off);
        std::vector<int32_t> at(hfirst.begin(), hfirst.end() - 1);
        for (size_t j = 0; j < fj.size(); ++j) {
            const PlanJob &w = *fj[j];
            desc[j] = FoldDesc{w.d->dev.node_op, w.d->dev.node_value, w.d->dev.node_kid, val_dev + w.fold_val_at};
            for (size_t h = 0; h + 1 < w.fold_first.size(); ++h)
                for (int32_t q = w.fold_first[h]; q < w.fold_first[h + 1]; ++q)
                    list[at[h]++] = int2{(int32_t)j, w.fold_list[q]};
        }
        e = hipMemcpyAsync(blk, stage, up_bytes, hipMemcpyHostToDevice, ctx->stream);
    }
    if (e == hipSuccess) e = ctx_pinned_enqueued(ctx);
    const FoldDesc *desc_dev = static_cast<const FoldDesc *>(blk);
    const int2 *list_dev = reinterpret_cast<const int2 *>(static_cast<char *>(blk) + list_off);
    for (int h = 0; h <= max_h && e == hipSuccess; ++h)
        e = launch_fold_level(desc_dev, list_dev + hfirst[h], hfirst[h + 1] - hfirst[h], ctx->stream);
    if (e == hipSuccess) e = ctx_pinned(ctx, sizeof(float) * n_val, &stage);
    if (e == hipSuccess)
        e = hipMemcpyAsync(stage, static_cast<char *>(blk) + val_off, sizeof(float) * n_val,
                           hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess)
        for (PlanJob *w : fj) {
            const float *v = static_cast<const float *>(stage) + w->fold_val_at;
            w->pl.fold_val.assign(v, v + w->d->stats.dag_nodes);
        }
    hipStreamSynchronize(ctx->stream);
    ctx->pool.release(blk);
    if (e != hipSuccess) return fail(ctx, TGP_EHIP, "constant folding: %s", hipGetErrorString(e));
    return TGP_OK;
}

static void longest_first(std::vector<ProgDesc> &v) {
    std::stable_sort(v.begin(), v.end(), [](const ProgDesc &a, const ProgDesc &b) { return a.len > b.len; });
}

// Caching and stack decisions, then the fill programs by level (the first
// part of code_host).  Host only; emit_threads host threads emit.
static tgp_status plan_decide_emit_fill(PlanJob &w, int D, bool reorder, double access_cost, int fold,
                                        int emit_threads) {
    tgp_dag d = w.d;
    Plan &P = d->plan;
    Planner &pl = w.pl;
    const int64_t U = d->stats.dag_nodes;
    const double t0 = now_ms();
    P.n_folded = 0;
    for (uint8_t f : pl.folded) P.n_folded += f;
    pl.reorder = reorder;
    pl.access_cost = access_cost;
    const unsigned hw = usable_cpus();
    const int dt = (int)std::min<unsigned>((unsigned)std::max(emit_threads, 1), hw);
    tgp_status st = U >= kParallelDecideNodes && dt > 1 ? pl.decide_parallel(w.rootrefs, w.err, dt)
                                                        : pl.decide(w.rootrefs, w.err);
    if (st != TGP_OK) return st;
    const double t1 = now_ms();
    w.t_decide = t1 - t0;

    std::vector<uint2> code;
    std::vector<ProgDesc> fill;
    int32_t max_level = -1;
    std::vector<int32_t> cached_nodes;
    for (int64_t n = 0; n < U; ++n)
        if (pl.cached[n]) {
            cached_nodes.push_back((int32_t)n);
            max_level = std::max(max_level, pl.level[n]);
        }
    P.slot_node.assign(cached_nodes.size(), -1);
    P.slot_pre.assign(cached_nodes.size(), 0);
    for (int32_t n : cached_nodes) {
        P.slot_node[pl.slot[n]] = n;
        P.slot_pre[pl.slot[n]] = pl.pre[n];
    }
    P.level_first.assign(max_level + 2, 0);
    std::vector<std::vector<ProgDesc>> by_level(max_level + 1);
    int64_t cache_reads_fill = 0;
    double valu_fill = 0;
    std::vector<int32_t> fill_nodes;
    for (int32_t n : cached_nodes)
        if (!pl.pre[n]) fill_nodes.push_back(n);
    std::vector<Emitted> em;
    emit_all(pl, fill_nodes, code, em, emit_threads);
    for (size_t i = 0; i < fill_nodes.size(); ++i) {
        const int32_t n = fill_nodes[i];
        ProgDesc pd{em[i].off, em[i].len, pl.slot[n], 0};
        cache_reads_fill += em[i].reads;
        valu_fill += em[i].valu;
        by_level[pl.level[n]].push_back(pd);
    }
    for (int l = 0; l <= max_level; ++l) {
        longest_first(by_level[l]);
        P.level_first[l] = (int32_t)fill.size();
        fill.insert(fill.end(), by_level[l].begin(), by_level[l].end());
    }
    P.level_first[max_level + 1] = (int32_t)fill.size();
    code.push_back(uint2{I_END, 0});  // padding past the last program
    P.D = D;
    P.reorder = reorder;
    P.access_cost = access_cost;
    P.fold = fold;
    P.ext = P.warp = false;
    for (const Emitted &m : em) {
        P.ext = P.ext || m.ext;
        P.warp = P.warp || m.warp;
    }
    P.n_slots = (int32_t)cached_nodes.size();
    P.n_spills = pl.spills;
    P.n_fill = (int32_t)fill.size();
    P.code_host = std::move(code);
    P.fill_host = std::move(fill);
    P.root_code_at = (int64_t)P.code_host.size();
    w.cache_reads_fill = cache_reads_fill;
    w.valu_fill = valu_fill;
    w.t_emit = now_ms() - t1;
    return TGP_OK;
}

// The root programs, appended to code_host: one per distinct (root,
// channel) for the fitness form and one per distinct root for the evaluate
// form.  Completes the plan.
static void plan_emit_roots(PlanJob &w, int emit_threads) {
    const double t0 = now_ms();
    Plan &P = w.d->plan;
    const Planner &pl = w.pl;
    std::vector<uint2> &code = P.code_host;
    std::vector<ProgDesc> reduce, store;
    std::vector<Emitted> em;
    int64_t cache_reads_roots = 0;
    double exec_roots = 0;
    emit_all(pl, w.store_list, code, em, emit_threads);
    // program of each distinct root: store_list[i] <-> em[i]
    std::unordered_map<int32_t, int32_t> prog_of;
    prog_of.reserve(w.store_list.size() * 2);
    for (size_t i = 0; i < w.store_list.size(); ++i) prog_of.emplace(w.store_list[i], (int32_t)i);
    double valu_roots = 0;
    for (size_t p = 0; p < w.reduce_list.size(); ++p) {
        const Emitted &m = em[prog_of[w.reduce_list[p].first]];
        ProgDesc pd{m.off, m.len, (int32_t)p, w.reduce_list[p].second};
        reduce.push_back(pd);
        exec_roots += m.len - 1;
        cache_reads_roots += m.reads;
        valu_roots += m.valu;
    }
    for (size_t i = 0; i < w.store_list.size(); ++i) {
        ProgDesc pd{em[i].off, em[i].len, w.store_of[w.store_list[i]], 0};
        store.push_back(pd);
    }
    // reduce programs keep dest = their row; order them longest first
    longest_first(reduce);
    longest_first(store);
    code.push_back(uint2{I_END, 0});  // padding

    double exec_fill = 0;
    for (auto &pd : P.fill_host) exec_fill += pd.len - 1;
    P.exec_per_case = exec_fill + exec_roots;
    P.valu_dag_per_case = pl.valu_dag;
    P.valu_fill_per_case = w.valu_fill;
    P.valu_roots_per_case = valu_roots;
    P.cache_reads_per_case = w.cache_reads_fill + cache_reads_roots;
    P.instructions = (int64_t)code.size();
    for (const Emitted &m : em) {
        P.ext = P.ext || m.ext;
        P.warp = P.warp || m.warp;
    }
    P.n_reduce = (int32_t)reduce.size();
    P.n_store = (int32_t)store.size();
    P.reduce_host = std::move(reduce);
    P.store_host = std::move(store);
    P.ind_rows_host = std::move(w.ind_rows);
    P.cases = w.cases;
    w.t_emit += now_ms() - t0;
}

static tgp_status plan_decide_emit(PlanJob &w, int D, bool reorder, double access_cost, int fold,
                                   int emit_threads) {
    tgp_status st = plan_decide_emit_fill(w, D, reorder, access_cost, fold, emit_threads);
    if (st == TGP_OK) plan_emit_roots(w, emit_threads);
    return st;
}

// Copies n parts into one new pool block (256-byte aligned parts) by one copy
// from the pinned staging; later launches on the stream see it in order.
// A part's `rebase`, when nonzero, is subtracted from the code offset of
// each of its ProgDesc entries as it is staged.
struct UploadPart {
    const void *src;
    size_t bytes;
    uint32_t rebase;
};
static hipError_t upload_parts(tgp_ctx ctx, int n, const UploadPart *part, void **blob, char **base,
                               size_t *off) {
    size_t total = 0;
    for (int i = 0; i < n; ++i) {
        off[i] = total;
        total += (part[i].bytes + 255) & ~(size_t)255;
    }
    total = std::max<size_t>(total, 256);
    void *stage = nullptr;
    hipError_t e = ctx->pool.alloc(blob, total);
    if (e == hipSuccess) e = ctx_pinned(ctx, total, &stage);
    if (e != hipSuccess) return e;
    for (int i = 0; i < n; ++i) {
        if (!part[i].bytes) continue;
        char *dst = (char *)stage + off[i];
        memcpy(dst, part[i].src, part[i].bytes);
        if (part[i].rebase) {
            ProgDesc *pd = reinterpret_cast<ProgDesc *>(dst);
            for (size_t k = 0; k < part[i].bytes / sizeof(ProgDesc); ++k) pd[k].code_off -= part[i].rebase;
        }
    }
    e = hipMemcpyAsync(*blob, stage, total, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = ctx_pinned_enqueued(ctx);
    *base = static_cast<char *>(*blob);
    return e;
}

// The fill programs: code_host up to root_code_at and the fill descriptors.
static tgp_status plan_upload_fill(tgp_ctx ctx, Plan &P) {
    const UploadPart part[2] = {{P.code_host.data(), sizeof(uint2) * (size_t)P.root_code_at, 0},
                                {P.fill_host.data(), sizeof(ProgDesc) * P.fill_host.size(), 0}};
    size_t off[2];
    char *b = nullptr;
    hipError_t e = upload_parts(ctx, 2, part, &P.blob, &b, off);
    if (e != hipSuccess) {
        hipStreamSynchronize(ctx->stream);
        P.release(ctx->pool);
        return fail(ctx, TGP_EHIP, "plan upload: %s", hipGetErrorString(e));
    }
    P.code_dev = reinterpret_cast<uint2 *>(b + off[0]);
    P.fill_dev = reinterpret_cast<ProgDesc *>(b + off[1]);
    return TGP_OK;
}

// The root programs: the rest of code_host, the reduce and store descriptors
// (offsets rebased to the start of that code) and the individual rows.
static tgp_status plan_upload_roots(tgp_ctx ctx, Plan &P) {
    const uint32_t at = (uint32_t)P.root_code_at;
    const UploadPart part[4] = {
        {P.code_host.data() + at, sizeof(uint2) * (P.code_host.size() - at), 0},
        {P.reduce_host.data(), sizeof(ProgDesc) * P.reduce_host.size(), at},
        {P.store_host.data(), sizeof(ProgDesc) * P.store_host.size(), at},
        {P.ind_rows_host.data(), sizeof(int32_t) * P.ind_rows_host.size(), 0}};
    size_t off[4];
    char *b = nullptr;
    hipError_t e = upload_parts(ctx, 4, part, &P.blob_roots, &b, off);
    if (e != hipSuccess) {
        hipStreamSynchronize(ctx->stream);
        P.release(ctx->pool);
        return fail(ctx, TGP_EHIP, "plan upload: %s", hipGetErrorString(e));
    }
    P.code_roots_dev = reinterpret_cast<uint2 *>(b + off[0]);
    P.reduce_dev = reinterpret_cast<ProgDesc *>(b + off[1]);
    P.store_dev = reinterpret_cast<ProgDesc *>(b + off[2]);
    P.ind_rows_dev = reinterpret_cast<int32_t *>(b + off[3]);
    return TGP_OK;
}

static tgp_status plan_upload(tgp_ctx ctx, Plan &P) {
    tgp_status st = plan_upload_fill(ctx, P);
    return st == TGP_OK ? plan_upload_roots(ctx, P) : st;
}

int ctx_stack_slots(tgp_ctx ctx) { return ctx->stack_lds ? interp_lds_stack() : interp_max_stack(); }

static bool plan_current(tgp_ctx ctx, const Plan &P, int64_t cases) {
    return P.cases == cases && P.D == ctx_stack_slots(ctx) && P.reorder == (ctx->reorder != 0) &&
           P.access_cost == ctx->cache_access_cost && P.fold == ctx->fold;
}

static size_t budget_slots(tgp_ctx ctx, int64_t cases) {
    return (size_t)(ctx->cache_budget / (sizeof(float) * (size_t)std::max<int64_t>(cases, 1)));
}

tgp_status build_plan(tgp_ctx ctx, tgp_dag d, int64_t cases, const std::function<tgp_status()> &after_fill) {
    const double t0 = now_ms();
    Plan &P = d->plan;
    if (plan_current(ctx, P, cases)) {
        tgp_status st = ctx->plan_upload && !P.blob ? plan_upload(ctx, P) : TGP_OK;
        ctx->times.plan_ms = now_ms() - t0;
        return st;
    }
    if (P.blob) {
        HCHK(ctx, hipStreamSynchronize(ctx->stream));
        P.release(ctx->pool);
    }
    P.cases = -1;
    const int D = ctx_stack_slots(ctx);
    PlanJob w(d, cases, D, budget_slots(ctx, cases));
    plan_prepare(w, ctx->fold != 0, kPlanThreads);
    const double tf0 = now_ms();
    tgp_status st = fold_run(ctx, {&w});
    if (st != TGP_OK) return st;
    ctx->times.plan_fold_ms = now_ms() - tf0;
    st = plan_decide_emit_fill(w, D, ctx->reorder != 0, ctx->cache_access_cost, ctx->fold, kPlanThreads);
    if (st != TGP_OK) return fail(ctx, st, "%s", w.err.c_str());
    if (ctx->plan_upload) {
        // the fill goes to the device (and, through after_fill, to work)
        // while the root programs are emitted
        st = plan_upload_fill(ctx, P);
        if (st == TGP_OK && after_fill) st = after_fill();
        if (st != TGP_OK) return st;
    }
    plan_emit_roots(w, kPlanThreads);
    ctx->times.plan_decide_ms = w.t_decide;
    ctx->times.plan_emit_ms = w.t_emit;
    if (ctx->plan_upload) {
        st = plan_upload_roots(ctx, P);
        if (st != TGP_OK) return st;
    }
    ctx->times.plan_ms = now_ms() - t0;
    return TGP_OK;
}

tgp_status build_plans(tgp_ctx ctx, int32_t n, const tgp_dag *dags, const int64_t *cases) {
    const double t0 = now_ms();
    // one plan per distinct DAG, for the largest domain it is evaluated on
    // (the cache budget in rows is tightest there)
    std::unordered_map<tgp_dag, int64_t> want;
    std::vector<tgp_dag> order;
    for (int32_t i = 0; i < n; ++i) {
        auto it = want.find(dags[i]);
        if (it == want.end()) {
            want.emplace(dags[i], cases[i]);
            order.push_back(dags[i]);
        } else {
            it->second = std::max(it->second, cases[i]);
        }
    }
    const int D = ctx_stack_slots(ctx);
    std::vector<std::unique_ptr<PlanJob>> jobs;
    bool synced = false;
    for (tgp_dag d : order) {
        const int64_t c = want[d];
        if (plan_current(ctx, d->plan, c)) continue;
        if (d->plan.blob) {
            if (!synced) HCHK(ctx, hipStreamSynchronize(ctx->stream));
            synced = true;
            d->plan.release(ctx->pool);
        }
        d->plan.cases = -1;
        jobs.emplace_back(new PlanJob(d, c, D, budget_slots(ctx, c)));
    }
    if (jobs.empty()) {
        ctx->times.plan_ms = now_ms() - t0;
        return TGP_OK;
    }
    // largest first, taken by host threads in turn
    std::stable_sort(jobs.begin(), jobs.end(), [](const std::unique_ptr<PlanJob> &a, const std::unique_ptr<PlanJob> &b) {
        return a->d->stats.dag_nodes > b->d->stats.dag_nodes;
    });
    const unsigned hw = usable_cpus();
    const int T = (int)std::min<size_t>(std::min<unsigned>(16, hw), jobs.size());
    auto parallel = [&](auto &&fn) {
        std::atomic<size_t> next{0};
        auto run = [&]() {
            for (size_t i; (i = next.fetch_add(1)) < jobs.size();) fn(*jobs[i]);
        };
        std::vector<std::thread> th;
        for (int t = 1; t < T; ++t) th.emplace_back(run);
        run();
        for (auto &x : th) x.join();
    };
    const bool fold = ctx->fold != 0;
    parallel([&](PlanJob &w) { plan_prepare(w, fold); });
    const double tf0 = now_ms();
    std::vector<PlanJob *> ptrs;
    for (auto &w : jobs) ptrs.push_back(w.get());
    tgp_status st = fold_run(ctx, ptrs);
    if (st != TGP_OK) return st;
    const double tf1 = now_ms();
    const bool reorder = ctx->reorder != 0;
    const double access = ctx->cache_access_cost;
    const int fold_flag = ctx->fold;
    const int emit_threads = T > 1 ? 1 : 8;
    parallel([&](PlanJob &w) {
        w.st = plan_decide_emit(w, D, reorder, access, fold_flag, emit_threads);
        if (w.st != TGP_OK) w.d->plan.cases = -1;
    });
    for (auto &w : jobs)
        if (w->st != TGP_OK) return fail(ctx, w->st, "%s", w->err.c_str());
    const double tf2 = now_ms();
    ctx->times.plan_fold_ms = tf1 - tf0;
    ctx->times.plan_decide_ms = tf2 - tf1;
    ctx->times.plan_emit_ms = 0;
    ctx->times.plan_ms = tf2 - t0;
    return TGP_OK;
}

// Work split: each work item is one program over tiles_per_stripe tiles of
// 64*K cases.  Items are kept short (at most 16 tiles) so that a launch of
// programs of very different lengths balances over 256 CUs, but long enough
// that the per-item setup (program descriptor, partial-sum write) stays small.
void choose_split(tgp_ctx ctx, int64_t n_progs, int64_t cases, int K, int32_t *stripes,
                         int32_t *tiles_per) {
    const int64_t tile = 64 * (int64_t)K;
    const int64_t n_tiles = (cases + tile - 1) / tile;
    int64_t tps;
    if (ctx->force_tiles > 0) {
        tps = ctx->force_tiles;
    } else {
        const int64_t target_items = 1 << 19;
        const int64_t total = n_tiles * std::max<int64_t>(n_progs, 1);
        const int64_t cap = ctx->tile_cap > 0 ? ctx->tile_cap : 16;
        tps = std::max<int64_t>(1, std::min<int64_t>(cap, total / target_items));
    }
    tps = std::max<int64_t>(1, std::min(tps, n_tiles));
    *tiles_per = (int32_t)tps;
    *stripes = (int32_t)((n_tiles + tps - 1) / tps);
}

int choose_K(tgp_ctx ctx, int64_t cases, bool ext) {
    if (ctx->stack_lds) return 2;  // the LDS-stack interpreter
    if (ext) return 4;  // the register-stack interpreter built with the bitwise operators and warp
    if (ctx->force_K) return ctx->force_K;
    return cases >= 64 * 4 * 4 ? 4 : 2;
}

void fill_job(JobDesc &j, tgp_domain dom, const uint2 *code, const float *cache) {
    memset(&j, 0, sizeof j);
    j.code = code;
    j.n_cases = (int32_t)dom->cases;
    j.ndim = dom->ndim;
    for (int k = 0; k < 3; ++k) {
        j.shape[k] = (int32_t)dom->shape[k];
        j.stride[k] = (int32_t)dom->stride[k];
        j.coord[k] = dom->coord[k] ? dom->coord[k] : dom->coord[0];
    }
    for (int k = 0; k < 2; ++k) div_magic((uint32_t)dom->stride[k], &j.div_m[k], &j.div_s[k]);
    j.cache = cache;
    j.case_base = 0;
    j.cache_stride = j.out_stride = j.target_stride = dom->cases;
    for (int k = 0; k < 2; ++k) {
        j.warp_lo[k] = (float)dom->lo[k];
        j.warp_scale[k] = dom->shape[k] > 1 ? (float)((double)(dom->shape[k] - 1) / (dom->hi[k] - dom->lo[k])) : 0.0f;
    }
}

static void fill_args(InterpArgs &a, tgp_domain dom, const uint2 *code, const float *cache) {
    memset(&a, 0, sizeof a);
    fill_job(a.job, dom, code, cache);
}

// The cache-fill launches of d's plan, writing its cache rows to `cache`.
static tgp_status fill_into(tgp_ctx ctx, tgp_dag d, tgp_domain dom, int K, float *cache) {
    const Plan &P = d->plan;
    record(ctx, 0);
    ctx->fill_recorded = ctx->timing;
    for (size_t l = 0; l + 1 < P.level_first.size(); ++l) {
        const int32_t b = P.level_first[l], e = P.level_first[l + 1];
        if (e == b) continue;
        InterpArgs a;
        fill_args(a, dom, P.code_dev, cache);
        a.progs = P.fill_dev + b;
        a.n_progs = e - b;
        choose_split(ctx, a.n_progs, dom->cases, K, &a.job.n_stripes, &a.job.tiles_per_stripe);
        a.job.out = cache;
        HCHK(ctx, launch_interp(K, P.D, true, a, ctx->stream, P.ext));
    }
    record(ctx, 1);
    return TGP_OK;
}

static tgp_status run_fill(tgp_ctx ctx, tgp_dag d, tgp_domain dom, int K, float **cache_out) {
    const Plan &P = d->plan;
    *cache_out = nullptr;
    ctx->fill_recorded = false;
    if (P.n_slots == 0) return TGP_OK;
    const size_t bytes = sizeof(float) * (size_t)P.n_slots * (size_t)dom->cases;
    HCHK(ctx, ensure(ctx->cache, bytes));
    float *cache = (float *)ctx->cache.p;
    *cache_out = cache;
    return fill_into(ctx, d, dom, K, cache);
}

// The plan of d for dom with its cache filled (fill launches queued on the
// context's stream).  A new plan's fill is queued as soon as its programs
// are on the device, while the host still emits the root programs; the
// fill's operand stack form follows the fill programs alone (they may not
// need the bitwise operators or warp when the root programs do).
static tgp_status plan_and_fill(tgp_ctx ctx, tgp_dag d, tgp_domain dom, float **cache) {
    bool filled = false;
    tgp_status st = build_plan(ctx, d, dom->cases, [&]() {
        filled = true;
        return run_fill(ctx, d, dom, choose_K(ctx, dom->cases, d->plan.ext), cache);
    });
    if (st != TGP_OK || filled) return st;
    return run_fill(ctx, d, dom, choose_K(ctx, dom->cases, d->plan.ext), cache);
}

tgp_status check_eval_args(tgp_ctx ctx, tgp_dag d, tgp_domain dom) {
    if (!ctx || !d || !dom) return fail(ctx, TGP_EINVAL, "NULL argument");
    if (d->ctx != ctx || dom->ctx != ctx) return fail(ctx, TGP_EINVAL, "handles of another context");
    if (d->stats.max_var >= dom->ndim)
        return fail(ctx, TGP_ESHAPE, "a tree uses axis %lld but the domain has %d axes",
                    (long long)d->stats.max_var, dom->ndim);
    return TGP_OK;
}

static void record_work(tgp_ctx ctx, tgp_dag d, tgp_domain dom, bool fitness) {
    const Plan &P = d->plan;
    tgp_work_stats &w = ctx->work;
    const double cases = (double)dom->cases;
    w.credited_node_evals = d->stats.dag_nodes * dom->cases;
    w.executed_node_evals = (int64_t)(P.exec_per_case * cases);
    w.cached_nodes = P.n_slots;
    w.stack_spills = P.n_spills;
    w.cache_levels = (int64_t)P.level_first.size() - 1;
    w.programs = fitness ? P.n_reduce : P.n_store;
    w.instructions = P.instructions;
    w.algorithmic_valu = P.valu_dag_per_case * cases;
    w.executed_valu_fill = P.valu_fill_per_case * cases;
    w.executed_valu_roots = P.valu_roots_per_case * cases;
    w.cache_bytes_written = (int64_t)P.n_slots * dom->cases * 4;
    w.cache_bytes_read = P.cache_reads_per_case * dom->cases * 4;
    w.folded_nodes = P.n_folded;
}

extern "C" {

// Whether p is host memory (pageable or pinned) rather than device-resident.
static bool is_host_memory(const void *p) {
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();  // an unknown (pageable) pointer: clear the error it leaves
        return true;
    }
    return attr.type == hipMemoryTypeHost || attr.type == hipMemoryTypeUnregistered;
}

tgp_status tgp_fitness(tgp_ctx ctx, tgp_dag d, tgp_domain dom, const float *target_dev, int32_t loss,
                       double *out) {
    tgp_status st = check_eval_args(ctx, d, dom);
    if (st != TGP_OK) return st;
    if (loss != TGP_RMSE && loss != TGP_MSE) return fail(ctx, TGP_EINVAL, "loss must be TGP_RMSE or TGP_MSE");
    if (d->n_ind == 0) return TGP_OK;
    if (!target_dev || !out) return fail(ctx, TGP_EINVAL, "NULL target or output");
    HCHK(ctx, hipSetDevice(ctx->device));
    const bool host_out = is_host_memory(out);
    double *out_dev = out;
    if (host_out) {
        HCHK(ctx, ensure(ctx->fit_out, sizeof(double) * (size_t)d->n_ind));
        out_dev = static_cast<double *>(ctx->fit_out.p);
    }
    float *cache = nullptr;
    st = plan_and_fill(ctx, d, dom, &cache);
    if (st != TGP_OK) return st;
    const Plan &P = d->plan;
    const int K = choose_K(ctx, dom->cases, P.ext);
    InterpArgs a;
    fill_args(a, dom, P.code_roots_dev, cache);
    a.progs = P.reduce_dev;
    a.n_progs = P.n_reduce;
    choose_split(ctx, a.n_progs, dom->cases, K, &a.job.n_stripes, &a.job.tiles_per_stripe);
    a.job.target = target_dev;
    HCHK(ctx, ensure(ctx->partial, sizeof(float2) * (size_t)a.n_progs * (size_t)a.job.n_stripes));
    a.job.partial = (float2 *)ctx->partial.p;
    record(ctx, 2);
    HCHK(ctx, launch_interp(K, P.D, false, a, ctx->stream, P.ext));
    record(ctx, 3);
    record(ctx, 4);
    HCHK(ctx, launch_finalize(a.job.partial, P.ind_rows_dev, d->n_ind, d->n_ch, a.job.n_stripes,
                              (double)d->n_ch * (double)dom->cases, loss, out_dev, ctx->stream));
    record(ctx, 5);
    if (host_out) {
        HCHK(ctx, hipMemcpyAsync(out, out_dev, sizeof(double) * (size_t)d->n_ind, hipMemcpyDeviceToHost,
                                 ctx->stream));
        HCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    ctx->times.interp_items = (int64_t)a.n_progs * a.job.n_stripes;
    ctx->times.cases_per_lane = K;
    ctx->times.tiles_per_item = a.job.tiles_per_stripe;
    record_work(ctx, d, dom, true);
    return TGP_OK;
}

tgp_status tgp_fitness_noalloc(tgp_ctx ctx, tgp_dag d, tgp_domain dom, const float *target_dev,
                               int32_t loss, double *out_dev) {
    tgp_status st = check_eval_args(ctx, d, dom);
    if (st != TGP_OK) return st;
    if (loss != TGP_RMSE && loss != TGP_MSE) return fail(ctx, TGP_EINVAL, "loss must be TGP_RMSE or TGP_MSE");
    if (d->n_ind == 0) return TGP_OK;
    if (!target_dev || !out_dev) return fail(ctx, TGP_EINVAL, "NULL target or output");
    if (is_host_memory(out_dev) || is_host_memory(target_dev))
        return fail(ctx, TGP_EINVAL, "tgp_fitness_noalloc takes device-resident target and output");
    HCHK(ctx, hipSetDevice(ctx->device));
    if (ctx->device >= kMaxDevices || !g_scratch_ptr[ctx->device])
        return fail(ctx, TGP_EHIP, "no scratch address for device %d: %s", ctx->device,
                    ctx->device < kMaxDevices ? hipGetErrorString(g_scratch_err[ctx->device]) : "device index");
    const Plan &P = d->plan;
    if (!plan_current(ctx, P, dom->cases) || !P.blob || !P.code_roots_dev)
        return fail(ctx, TGP_EINVAL,
                    "the DAG has no plan for a domain of %lld cases under this context's settings "
                    "(evaluate it once with tgp_fitness or tgp_evaluate)", (long long)dom->cases);
    const int K = choose_K(ctx, dom->cases, P.ext);
    InterpArgs a;
    fill_args(a, dom, P.code_roots_dev, nullptr);
    a.progs = P.reduce_dev;
    a.n_progs = P.n_reduce;
    choose_split(ctx, a.n_progs, dom->cases, K, &a.job.n_stripes, &a.job.tiles_per_stripe);
    const size_t partial_bytes =
        (sizeof(float2) * (size_t)a.n_progs * (size_t)a.job.n_stripes + 255) & ~(size_t)255;
    const size_t cache_bytes = sizeof(float) * (size_t)P.n_slots * (size_t)dom->cases;
    if (partial_bytes + cache_bytes > kNoAllocScratchBytes)
        return fail(ctx, TGP_ENOMEM,
                    "needs %zu bytes of scratch (%zu of partial sums, %zu of cache rows); "
                    "tgp_fitness_noalloc has %zu", partial_bytes + cache_bytes, partial_bytes, cache_bytes,
                    kNoAllocScratchBytes);
    // Every (program, stripe) pair and every cache row is written before it
    // is read, so nothing in the scratch needs clearing between calls.
    char *base = static_cast<char *>(g_scratch_ptr[ctx->device]);
    float *cache = P.n_slots ? reinterpret_cast<float *>(base + partial_bytes) : nullptr;
    ctx->fill_recorded = false;
    if (P.n_slots) {
        st = fill_into(ctx, d, dom, K, cache);
        if (st != TGP_OK) return st;
    }
    a.job.cache = cache;
    a.job.target = target_dev;
    a.job.partial = reinterpret_cast<float2 *>(base);
    record(ctx, 2);
    HCHK(ctx, launch_interp(K, P.D, false, a, ctx->stream, P.ext));
    record(ctx, 3);
    record(ctx, 4);
    HCHK(ctx, launch_finalize(a.job.partial, P.ind_rows_dev, d->n_ind, d->n_ch, a.job.n_stripes,
                              (double)d->n_ch * (double)dom->cases, loss, out_dev, ctx->stream));
    record(ctx, 5);
    ctx->times.interp_items = (int64_t)a.n_progs * a.job.n_stripes;
    ctx->times.cases_per_lane = K;
    ctx->times.tiles_per_item = a.job.tiles_per_stripe;
    record_work(ctx, d, dom, true);
    return TGP_OK;
}

tgp_status tgp_evaluate(tgp_ctx ctx, tgp_dag d, tgp_domain dom, float *out_dev) {
    tgp_status st = check_eval_args(ctx, d, dom);
    if (st != TGP_OK) return st;
    if (d->stats.n_roots == 0) return TGP_OK;
    if (!out_dev) return fail(ctx, TGP_EINVAL, "NULL output");
    HCHK(ctx, hipSetDevice(ctx->device));
    float *cache = nullptr;
    st = plan_and_fill(ctx, d, dom, &cache);
    if (st != TGP_OK) return st;
    const Plan &P = d->plan;
    const int K = choose_K(ctx, dom->cases, P.ext);
    InterpArgs a;
    fill_args(a, dom, P.code_roots_dev, cache);
    a.progs = P.store_dev;
    a.n_progs = P.n_store;
    choose_split(ctx, a.n_progs, dom->cases, K, &a.job.n_stripes, &a.job.tiles_per_stripe);
    a.job.out = out_dev;
    record(ctx, 2);
    HCHK(ctx, launch_interp(K, P.D, true, a, ctx->stream, P.ext));
    record(ctx, 3);
    record(ctx, 4);
    record(ctx, 5);
    ctx->times.interp_items = (int64_t)a.n_progs * a.job.n_stripes;
    ctx->times.cases_per_lane = K;
    ctx->times.tiles_per_item = a.job.tiles_per_stripe;
    const size_t row = sizeof(float) * (size_t)dom->cases;
    for (int64_t r = 0; r < d->stats.n_roots; ++r)
        if (P.dup_src[r] >= 0)
            HCHK(ctx, hipMemcpyAsync((char *)out_dev + row * r, (char *)out_dev + row * P.dup_src[r], row,
                                     hipMemcpyDeviceToDevice, ctx->stream));
    record_work(ctx, d, dom, false);
    return TGP_OK;
}

tgp_status tgp_last_work(tgp_ctx ctx, tgp_work_stats *out) {
    if (!ctx || !out) return fail(ctx, TGP_EINVAL, "NULL argument");
    *out = ctx->work;
    return TGP_OK;
}

}  // extern "C"
