// batch.cpp -- batched fitness of many populations in one persistent launch
// per phase, replayed as a HIP graph, and the autotuner that picks its
// launch shape.
//
// A GP system evaluates one population per generation (TensorGP Sec. 3.1,
// Sec. 4.1); many independent runs, or many populations of uneven sizes and
// domain shapes, are evaluated together here.  Every job keeps its own plan
// (DAG, cached subtrees, programs); the batch packs the plans into one set of
// device buffers and runs
//   * one persistent launch per cache-fill level (level l of every job),
//   * one persistent launch for every job's root programs fused with the
//     error reduction,
//   * one finalize launch for every individual of every job.
// Resident waves draw work items from partitioned atomic counters, longest
// program first across all jobs, so small and large jobs share the GPU
// without a tail (or, in the direct form, one wave per work item in that
// order).  Launch arguments point at fixed device buffers whose contents
// change from step to step, so the step is built once as a HIP graph of
// kernel nodes and replayed; item counts are read on the device, and only the
// grids that follow the step's sizes (direct form, finalize) are updated in
// the instantiated graph between replays.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "runtime_internal.h"

namespace {

template <typename T>
struct Pinned {
    T *h = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t n) {
        if (n <= cap && h) return hipSuccess;
        if (h) hipHostFree(h);
        h = nullptr;
        cap = 0;
        size_t want = std::max<size_t>(n + n / 2, 64);
        hipError_t e = hipHostMalloc((void **)&h, want * sizeof(T), hipHostMallocDefault);
        if (e == hipSuccess) cap = want;
        return e;
    }
    void release() {
        if (h) hipHostFree(h);
        h = nullptr;
        cap = 0;
    }
};

template <typename T>
struct Dev {
    T *d = nullptr;
    size_t cap = 0;
    // Grows to at least n elements; returns true when the address changed.
    bool ensure(size_t n, hipError_t *err) {
        if (n <= cap && d) return false;
        if (d) hipFree(d);
        d = nullptr;
        cap = 0;
        size_t want = std::max<size_t>(n + n / 2, 64);
        *err = hipMalloc((void **)&d, want * sizeof(T));
        if (*err == hipSuccess) cap = want;
        return true;
    }
    void release() {
        if (d) hipFree(d);
        d = nullptr;
        cap = 0;
    }
};

}  // namespace

struct tgp_batch_s {
    tgp_ctx ctx = nullptr;
    bool use_graph = true;
    bool persistent = true;  // persistent kernels, or one wave per work item
    bool ext = false;        // interpreter with the bitwise operators and warp
    int D = 0;               // stack slots: the register form's or the LDS form's
    int K = 4;
    int levels_cap = 4;  // fill levels the graph has launches for
    int grid_store = 0, grid_reduce = 0;
    std::vector<uint32_t> group_items;  // items per group of the current step
    uint32_t n_ind = 0;
    // device buffers
    Dev<JobDesc> jobs;
    Dev<PairDesc> pairs;
    Dev<uint32_t> item_first;
    Dev<GroupDesc> groups;
    Dev<uint32_t> counters;
    Dev<FinJob> fin;
    Dev<int32_t> scalars;  // [0] = n_jobs, [1] = n_ind (as uint32)
    Dev<uint2> code;
    Dev<int32_t> rows;
    Dev<float> cache;
    Dev<float2> partial;
    // pinned staging
    Pinned<JobDesc> h_jobs;
    Pinned<PairDesc> h_pairs;
    Pinned<uint32_t> h_first;
    Pinned<GroupDesc> h_groups;
    Pinned<FinJob> h_fin;
    Pinned<int32_t> h_scalars;
    Pinned<uint2> h_code;
    Pinned<int32_t> h_rows;
    // graph: reset, levels_cap fill launches, the root launch, the finalize
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipGraphNode_t> nodes;
    bool stale = true;
    hipEvent_t staged_ev = nullptr;  // recorded after the uploads out of the staging buffers
    bool staged = false;
    tgp_batch_stats stats{};
    // kernel argument storage (launch i reads args[i])
    int32_t n_counters = 0;
    int32_t group_index[64] = {};
    uint32_t *n_ind_ptr = nullptr;
};

static void batch_release_graph(tgp_batch b) {
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->nodes.clear();
    b->stale = true;
}

// Kernel launch i of a step: 0 = counter reset, 1..levels_cap = fill level
// i - 1, levels_cap + 1 = root programs, levels_cap + 2 = finalize.
static int n_launches(tgp_batch b) { return b->levels_cap + 3; }

static hipKernelNodeParams launch_params(tgp_batch b, int i, void **args) {
    hipKernelNodeParams p{};
    const int L = b->levels_cap;
    p.blockDim = dim3(64);
    if (i == 0) {
        p.func = const_cast<void *>(reset_kernel());
        p.gridDim = dim3((b->n_counters + 255) / 256);
        p.blockDim = dim3(256);
        args[0] = &b->counters.d;
        args[1] = &b->n_counters;
    } else if (i <= L + 1) {
        const bool store = i <= L;
        const int g = i - 1;
        b->group_index[g] = g;
        p.func = const_cast<void *>(batch_kernel(b->K, b->D, store, b->persistent, b->ext));
        if (b->persistent) {
            p.gridDim = dim3(store ? b->grid_store : b->grid_reduce);
        } else {
            const uint32_t n = g < (int)b->group_items.size() ? b->group_items[g] : 0;
            p.gridDim = dim3(std::max<uint32_t>(1, n));
        }
        args[0] = &b->jobs.d;
        args[1] = &b->pairs.d;
        args[2] = &b->item_first.d;
        args[3] = &b->groups.d;
        args[4] = &b->group_index[g];
        args[5] = &b->counters.d;
    } else {
        p.func = const_cast<void *>(finalize_batch_kernel());
        p.gridDim = dim3(std::max<uint32_t>(1, b->n_ind));
        p.blockDim = dim3(256);
        static_assert(sizeof(uint32_t) == sizeof(int32_t), "scalars");
        args[0] = &b->fin.d;
        args[1] = &b->scalars.d;
        b->n_ind_ptr = reinterpret_cast<uint32_t *>(b->scalars.d + 1);
        args[2] = &b->n_ind_ptr;
    }
    p.sharedMemBytes = 0;
    p.kernelParams = args;
    p.extra = nullptr;
    return p;
}

static hipError_t enqueue_step(tgp_batch b, hipStream_t s) {
    void *args[8];
    hipError_t e = hipSuccess;
    for (int i = 0; i < n_launches(b) && e == hipSuccess; ++i) {
        hipKernelNodeParams p = launch_params(b, i, args);
        e = hipLaunchKernel(p.func, p.gridDim, p.blockDim, p.kernelParams, 0, s);
    }
    return e;
}

static hipError_t build_graph(tgp_batch b) {
    batch_release_graph(b);
    hipError_t e = hipGraphCreate(&b->graph, 0);
    hipGraphNode_t prev = nullptr;
    void *args[8];
    for (int i = 0; i < n_launches(b) && e == hipSuccess; ++i) {
        hipKernelNodeParams p = launch_params(b, i, args);
        hipGraphNode_t node;
        e = hipGraphAddKernelNode(&node, b->graph, prev ? &prev : nullptr, prev ? 1 : 0, &p);
        if (e == hipSuccess) {
            b->nodes.push_back(node);
            prev = node;
        }
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e == hipSuccess) {
        b->stale = false;
        b->stats.captures += 1;
    }
    return e;
}

// Grids that change with the step's sizes (direct form, finalize).
static hipError_t update_graph(tgp_batch b) {
    void *args[8];
    hipError_t e = hipSuccess;
    for (int i = 1; i < n_launches(b) && e == hipSuccess; ++i) {
        if (b->persistent && i != n_launches(b) - 1) continue;
        hipKernelNodeParams p = launch_params(b, i, args);
        e = hipGraphExecKernelNodeSetParams(b->exec, b->nodes[i], &p);
    }
    return e;
}

extern "C" {

tgp_status tgp_batch_create(tgp_ctx ctx, int32_t use_graph, tgp_batch *out) {
    if (!ctx || !out) return fail(ctx, TGP_EINVAL, "NULL argument");
    *out = nullptr;
    HCHK(ctx, hipSetDevice(ctx->device));
    tgp_batch b = new tgp_batch_s();
    b->ctx = ctx;
    b->use_graph = use_graph != 0;
    *out = b;
    return TGP_OK;
}

void tgp_batch_destroy(tgp_batch b) {
    if (!b) return;
    hipSetDevice(b->ctx->device);
    hipStreamSynchronize(b->ctx->stream);
    batch_release_graph(b);
    if (b->staged_ev) hipEventDestroy(b->staged_ev);
    b->jobs.release();
    b->pairs.release();
    b->item_first.release();
    b->groups.release();
    b->counters.release();
    b->fin.release();
    b->scalars.release();
    b->code.release();
    b->rows.release();
    b->cache.release();
    b->partial.release();
    b->h_jobs.release();
    b->h_pairs.release();
    b->h_first.release();
    b->h_groups.release();
    b->h_fin.release();
    b->h_scalars.release();
    b->h_code.release();
    b->h_rows.release();
    delete b;
}

tgp_status tgp_batch_stats_get(tgp_batch b, tgp_batch_stats *out) {
    if (!b || !out) return fail(nullptr, TGP_EINVAL, "NULL argument");
    *out = b->stats;
    return TGP_OK;
}

tgp_status tgp_batch_run(tgp_batch b, int32_t n_jobs, const tgp_job *jobs) {
    if (!b) return fail(nullptr, TGP_EINVAL, "batch is NULL");
    tgp_ctx ctx = b->ctx;
    if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return fail(ctx, TGP_EINVAL, "bad job list");
    HCHK(ctx, hipSetDevice(ctx->device));
    const double t0 = now_ms();
    std::vector<StepJob> sj(n_jobs);
    std::vector<tgp_dag> dags(n_jobs);
    std::vector<int64_t> cases(n_jobs);
    int64_t credited = 0;
    for (int32_t j = 0; j < n_jobs; ++j) {
        const tgp_job &J = jobs[j];
        tgp_status st = check_eval_args(ctx, J.dag, J.domain);
        if (st != TGP_OK) return fail(ctx, st, "job %d: %s", j, ctx->err.c_str());
        if (J.loss != TGP_RMSE && J.loss != TGP_MSE) return fail(ctx, TGP_EINVAL, "job %d: bad loss", j);
        if (J.dag->n_ind > 0 && (!J.target_dev || !J.out_dev))
            return fail(ctx, TGP_EINVAL, "job %d: NULL target or output", j);
        dags[j] = J.dag;
        cases[j] = J.domain->cases;
    }
    // every job's plan at once: host threads, one device round trip
    tgp_status pst = build_plans(ctx, n_jobs, dags.data(), cases.data());
    if (pst != TGP_OK) return pst;
    for (int32_t j = 0; j < n_jobs; ++j) {
        const tgp_job &J = jobs[j];
        StepJob &s = sj[j];
        s.plan = &J.dag->plan;
        s.domain = J.domain;
        s.n_ind = J.dag->n_ind;
        s.n_ch = J.dag->n_ch;
        s.case_base = 0;
        s.n_cases = (int32_t)J.domain->cases;
        s.target = J.target_dev;
        s.out = J.out_dev;
        s.loss = J.loss;
        credited += J.dag->stats.dag_nodes * J.domain->cases;
    }
    const double t_plan = now_ms() - t0;
    tgp_status st = batch_step(b, n_jobs, sj.data(), credited);
    b->stats.pack_ms += t_plan;
    return st;
}

}  // extern "C"

tgp_status batch_step(tgp_batch b, int32_t n_jobs, const StepJob *jobs, int64_t credited) {
    tgp_ctx ctx = b->ctx;
    const double t0 = now_ms();
    // The staging buffers are free once the copies of this batch's previous
    // step have run (later steps on other batches need not be waited for).
    if (b->staged) {
        HCHK(ctx, hipEventSynchronize(b->staged_ev));
        b->staged = false;
    }
    bool ext = false;
    const int D = ctx_stack_slots(ctx);
    for (int32_t j = 0; j < n_jobs; ++j) {
        ext = ext || jobs[j].plan->ext;
        if (jobs[j].plan->D != D) return fail(ctx, TGP_EINVAL, "job %d was planned for another stack form", j);
    }
    int K = ctx->force_K ? ctx->force_K : 4;
    if (ctx->stack_lds) K = 2;
    if (!interp_variant_exists(K, D, ext)) K = 4;
    if (K != b->K || ext != b->ext || D != b->D) {
        b->K = K;
        b->ext = ext;
        b->D = D;
        b->stale = true;
    }
    const bool persistent = ctx->batch_persistent != 0;
    if (persistent != b->persistent) {
        b->persistent = persistent;
        b->stale = true;
    }
    int max_levels = 0;
    for (int32_t j = 0; j < n_jobs; ++j)
        max_levels = std::max(max_levels, (int)jobs[j].plan->level_first.size() - 1);
    if (max_levels > b->levels_cap) {
        b->levels_cap = std::max(max_levels, 2 * b->levels_cap);
        if (b->levels_cap > 63) return fail(ctx, TGP_EINVAL, "more than 63 cache-fill levels");
        b->stale = true;
    }
    // ---- launch shape: tiles per item from the whole batch's work
    int64_t total_tiles = 0;
    std::vector<int64_t> ntiles(n_jobs), tps(n_jobs);
    for (int32_t j = 0; j < n_jobs; ++j) {
        ntiles[j] = (jobs[j].n_cases + 64 * K - 1) / (64 * K);
        total_tiles += ntiles[j] * std::max<int64_t>(jobs[j].plan->n_reduce, 0);
    }
    const int cap = ctx->tile_cap > 0 ? ctx->tile_cap : 16;
    int64_t tps_all = ctx->force_tiles > 0
                          ? ctx->force_tiles
                          : std::max<int64_t>(1, std::min<int64_t>(cap, total_tiles / (1 << 19)));
    // ---- sizes
    size_t n_code = 0, n_rows = 0, n_cache = 0, n_partial = 0, n_pairs = 0;
    uint32_t n_ind = 0;
    for (int32_t j = 0; j < n_jobs; ++j) {
        const Plan &P = *jobs[j].plan;
        const int64_t want = jobs[j].tiles_per_item > 0 ? jobs[j].tiles_per_item : tps_all;
        tps[j] = std::max<int64_t>(1, std::min<int64_t>(want, ntiles[j]));
        const int64_t stripes = (ntiles[j] + tps[j] - 1) / tps[j];
        if (!jobs[j].code_dev) n_code += P.code_host.size();
        if (!jobs[j].rows_dev) n_rows += P.ind_rows_host.size();
        if (!jobs[j].cache) n_cache += (size_t)P.n_slots * (size_t)jobs[j].domain->cases;
        n_partial += (size_t)P.n_reduce * (size_t)stripes;
        n_pairs += P.fill_host.size() + P.reduce_host.size();
        n_ind += (uint32_t)jobs[j].n_ind;
    }
    const int G = b->levels_cap + 1;
    hipError_t e = hipSuccess;
    bool moved = false;
    moved |= b->jobs.ensure(std::max<int32_t>(n_jobs, 1), &e);
    if (e == hipSuccess) moved |= b->pairs.ensure(std::max<size_t>(n_pairs, 1), &e);
    if (e == hipSuccess) moved |= b->item_first.ensure(n_pairs + 1, &e);
    if (e == hipSuccess) moved |= b->groups.ensure(G, &e);
    if (e == hipSuccess) moved |= b->counters.ensure((size_t)G * batch_parts(), &e);
    if (e == hipSuccess) moved |= b->fin.ensure(std::max<int32_t>(n_jobs, 1), &e);
    if (e == hipSuccess) moved |= b->scalars.ensure(2, &e);
    if (e == hipSuccess) moved |= b->code.ensure(n_code + 1, &e);
    if (e == hipSuccess) moved |= b->rows.ensure(std::max<size_t>(n_rows, 1), &e);
    if (e == hipSuccess) moved |= b->cache.ensure(std::max<size_t>(n_cache, 1), &e);
    if (e == hipSuccess) moved |= b->partial.ensure(std::max<size_t>(n_partial, 1), &e);
    if (e != hipSuccess) return fail(ctx, TGP_ENOMEM, "batch buffers: %s", hipGetErrorString(e));
    if (moved) b->stale = true;
    if (b->n_counters != G * (int32_t)batch_parts()) {
        b->n_counters = G * (int32_t)batch_parts();
        b->stale = true;
    }
    e = b->h_jobs.ensure(std::max<int32_t>(n_jobs, 1));
    if (e == hipSuccess) e = b->h_pairs.ensure(std::max<size_t>(n_pairs, 1));
    if (e == hipSuccess) e = b->h_first.ensure(n_pairs + 1);
    if (e == hipSuccess) e = b->h_groups.ensure(G);
    if (e == hipSuccess) e = b->h_fin.ensure(std::max<int32_t>(n_jobs, 1));
    if (e == hipSuccess) e = b->h_scalars.ensure(2);
    if (e == hipSuccess) e = b->h_code.ensure(n_code + 1);
    if (e == hipSuccess) e = b->h_rows.ensure(std::max<size_t>(n_rows, 1));
    if (e != hipSuccess) return fail(ctx, TGP_ENOMEM, "batch staging: %s", hipGetErrorString(e));

    // ---- pack
    struct PairSort {
        double work;
        PairDesc pd;
        uint32_t items;
    };
    std::vector<std::vector<PairSort>> groups(G);
    size_t code_at = 0, rows_at = 0, cache_at = 0, part_at = 0;
    uint32_t ind_at = 0;
    for (int32_t j = 0; j < n_jobs; ++j) {
        const StepJob &J = jobs[j];
        const Plan &P = *J.plan;
        const int64_t stripes = (ntiles[j] + tps[j] - 1) / tps[j];
        const int64_t dom_cases = J.domain->cases;
        JobDesc &jd = b->h_jobs.h[j];
        float *cache = J.cache ? const_cast<float *>(J.cache) : b->cache.d + cache_at;
        fill_job(jd, J.domain, J.code_dev ? J.code_dev : b->code.d + code_at, cache);
        jd.n_cases = J.n_cases;
        jd.case_base = J.case_base;
        jd.cache_stride = J.cache ? J.cache_stride : dom_cases;
        jd.out = cache;
        jd.out_stride = jd.cache_stride;
        jd.n_stripes = (int32_t)stripes;
        jd.tiles_per_stripe = (int32_t)tps[j];
        jd.target = J.target;
        jd.target_stride = dom_cases;
        jd.partial = b->partial.d + part_at;
        if (!J.code_dev)
            memcpy(b->h_code.h + code_at, P.code_host.data(), sizeof(uint2) * P.code_host.size());
        if (!J.rows_dev)
            memcpy(b->h_rows.h + rows_at, P.ind_rows_host.data(), sizeof(int32_t) * P.ind_rows_host.size());
        FinJob &f = b->h_fin.h[j];
        f.partial = jd.partial;
        f.ind_rows = J.rows_dev ? J.rows_dev : b->rows.d + rows_at;
        f.out = J.out;
        f.acc = J.acc;
        f.first = J.acc ? J.first : 1;
        f.last = J.acc ? J.last : 1;
        f.n_terms = (double)J.n_ch * (double)dom_cases;
        f.n_ch = J.n_ch;
        f.n_stripes = (int32_t)stripes;
        f.loss = J.loss;
        f.ind_begin = ind_at;
        for (size_t l = 0; l + 1 < P.level_first.size(); ++l)
            for (int32_t q = P.level_first[l]; q < P.level_first[l + 1]; ++q) {
                const ProgDesc &pd = P.fill_host[q];
                groups[l].push_back({(double)pd.len * tps[j], {j, pd.code_off, pd.dest, pd.chan},
                                     (uint32_t)stripes});
            }
        for (const ProgDesc &pd : P.reduce_host)
            groups[G - 1].push_back({(double)pd.len * tps[j], {j, pd.code_off, pd.dest, pd.chan},
                                     (uint32_t)stripes});
        if (!J.code_dev) code_at += P.code_host.size();
        if (!J.rows_dev) rows_at += P.ind_rows_host.size();
        if (!J.cache) cache_at += (size_t)P.n_slots * (size_t)dom_cases;
        part_at += (size_t)P.n_reduce * (size_t)stripes;
        ind_at += (uint32_t)J.n_ind;
    }
    b->h_code.h[code_at] = uint2{I_END, 0};
    size_t pi = 0;
    uint64_t item = 0;
    for (int g = 0; g < G; ++g) {
        auto &v = groups[g];
        std::stable_sort(v.begin(), v.end(), [](const PairSort &a, const PairSort &c) { return a.work > c.work; });
        GroupDesc &gd = b->h_groups.h[g];
        gd.pair_begin = (uint32_t)pi;
        gd.item_begin = (uint32_t)item;
        for (const PairSort &ps : v) {
            b->h_pairs.h[pi] = ps.pd;
            b->h_first.h[pi] = (uint32_t)item;
            item += ps.items;
            ++pi;
        }
        gd.pair_end = (uint32_t)pi;
        gd.item_end = (uint32_t)item;
    }
    b->h_first.h[pi] = (uint32_t)item;
    if (item > 0xffffffffull) return fail(ctx, TGP_EINVAL, "batch has more than 2^32 work items");
    b->group_items.resize(G);
    for (int g = 0; g < G; ++g) b->group_items[g] = b->h_groups.h[g].item_end - b->h_groups.h[g].item_begin;
    b->n_ind = n_ind;
    b->h_scalars.h[0] = n_jobs;
    b->h_scalars.h[1] = (int32_t)n_ind;

    // ---- upload and launch
    auto up = [&](void *dst, const void *src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, ctx->stream);
    };
    up(b->jobs.d, b->h_jobs.h, sizeof(JobDesc) * n_jobs);
    up(b->pairs.d, b->h_pairs.h, sizeof(PairDesc) * n_pairs);
    up(b->item_first.d, b->h_first.h, sizeof(uint32_t) * (n_pairs + 1));
    up(b->groups.d, b->h_groups.h, sizeof(GroupDesc) * G);
    up(b->fin.d, b->h_fin.h, sizeof(FinJob) * n_jobs);
    up(b->scalars.d, b->h_scalars.h, sizeof(int32_t) * 2);
    up(b->code.d, b->h_code.h, sizeof(uint2) * (n_code + 1));
    up(b->rows.d, b->h_rows.h, sizeof(int32_t) * n_rows);
    if (e == hipSuccess && !b->staged_ev) e = hipEventCreateWithFlags(&b->staged_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(b->staged_ev, ctx->stream);
    if (e != hipSuccess) return fail(ctx, TGP_EHIP, "batch upload: %s", hipGetErrorString(e));
    b->staged = true;
    const int gs = batch_grid(K, D, true, ext), gr = batch_grid(K, D, false, ext);
    if (gs != b->grid_store || gr != b->grid_reduce) {
        b->grid_store = gs;
        b->grid_reduce = gr;
        b->stale = true;
    }
    const double t1 = now_ms();
    record(ctx, 2);
    if (b->use_graph) {
        if (b->stale) {
            e = build_graph(b);
            if (e != hipSuccess) return fail(ctx, TGP_EHIP, "graph build: %s", hipGetErrorString(e));
        } else {
            e = update_graph(b);
            if (e != hipSuccess) return fail(ctx, TGP_EHIP, "graph update: %s", hipGetErrorString(e));
        }
        e = hipGraphLaunch(b->exec, ctx->stream);
        if (e != hipSuccess) return fail(ctx, TGP_EHIP, "hipGraphLaunch: %s", hipGetErrorString(e));
        b->stats.replays += 1;
    } else {
        e = enqueue_step(b, ctx->stream);
        if (e != hipSuccess) return fail(ctx, TGP_EHIP, "batch launch: %s", hipGetErrorString(e));
    }
    record(ctx, 3);
    record(ctx, 4);
    record(ctx, 5);
    ctx->fill_recorded = false;
    b->stats.jobs = n_jobs;
    b->stats.pairs = (int64_t)n_pairs;
    b->stats.items = (int64_t)item;
    b->stats.levels = max_levels;
    b->stats.tiles_per_item = (int32_t)tps_all;
    b->stats.cases_per_lane = K;
    b->stats.persistent = b->persistent ? 1 : 0;
    b->stats.pack_ms = t1 - t0;
    b->stats.credited_node_evals = credited;
    ctx->times.interp_items = (int64_t)item;
    ctx->times.cases_per_lane = K;
    ctx->times.tiles_per_item = (int32_t)tps_all;
    return TGP_OK;
}

extern "C" {

tgp_status tgp_ctx_set_batch_form(tgp_ctx ctx, int32_t persistent) {
    if (!ctx) return fail(nullptr, TGP_EINVAL, "ctx is NULL");
    ctx->batch_persistent = persistent != 0;
    return TGP_OK;
}

tgp_status tgp_fitness_batch(tgp_ctx ctx, int32_t n_jobs, const tgp_job *jobs) {
    if (!ctx) return fail(nullptr, TGP_EINVAL, "ctx is NULL");
    if (!ctx->batch) {
        tgp_status st = tgp_batch_create(ctx, 1, &ctx->batch);
        if (st != TGP_OK) return st;
    }
    return tgp_batch_run(ctx->batch, n_jobs, jobs);
}

// ------------------------------------------------------------------ autotune
//
// Candidates: the stack form with its cases per lane (registers with K in
// {4, 2}, LDS with K = 2) x the cap on tiles per work item in {4, 16} x the
// launch form (persistent waves or one wave per work item).  Each is timed
// (HIP events, after one warm-up run) on the caller's own jobs; the fastest
// is installed in the context and, with a
// cache path, recorded under a key made of the job count and the log2 sizes
// of the batch's cases and instructions, so a later call with a workload of
// the same class reuses it without timing.
static std::string tune_key(int32_t n_jobs, const tgp_job *jobs) {
    double cases = 0, instr = 0;
    for (int32_t j = 0; j < n_jobs; ++j) {
        cases += (double)jobs[j].domain->cases * std::max(1, jobs[j].dag->n_ind * jobs[j].dag->n_ch);
        instr += (double)jobs[j].dag->stats.tree_nodes;
    }
    char buf[96];
    snprintf(buf, sizeof buf, "jobs%d_cases2^%d_nodes2^%d", n_jobs, (int)std::lround(std::log2(cases + 1)),
             (int)std::lround(std::log2(instr + 1)));
    return buf;
}

static bool lookup(const char *path, const std::string &key, int *K, int *cap, int *pers, int *lds) {
    if (!path) return false;
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        // one JSON object per line: {"key": "...", "K": k, "tiles_cap": t, "persistent": p, "lds": l, "ms": m}
        const std::string tag = "\"key\": \"" + key + "\"";
        if (line.find(tag) == std::string::npos) continue;
        const size_t a = line.find("\"K\": "), c = line.find("\"tiles_cap\": "),
                     q = line.find("\"persistent\": "), l = line.find("\"lds\": ");
        if (a == std::string::npos || c == std::string::npos || q == std::string::npos) continue;
        *K = atoi(line.c_str() + a + 5);
        *cap = atoi(line.c_str() + c + 13);
        *pers = atoi(line.c_str() + q + 14);
        *lds = l == std::string::npos ? 0 : atoi(line.c_str() + l + 7);
        found = true;  // the last record of the key wins
    }
    return found;
}

tgp_status tgp_autotune(tgp_ctx ctx, int32_t n_jobs, const tgp_job *jobs, const char *cache_path,
                        tgp_tune_result *out) {
    if (!ctx || n_jobs <= 0 || !jobs) return fail(ctx, TGP_EINVAL, "bad arguments");
    const std::string key = tune_key(n_jobs, jobs);
    tgp_tune_result r{};
    int K = 0, cap = 0, pers = 1, lds = 0;
    if (lookup(cache_path, key, &K, &cap, &pers, &lds) &&
        interp_variant_exists(K, lds ? interp_lds_stack() : interp_max_stack(), lds != 0)) {
        ctx->force_K = K;
        ctx->tile_cap = cap;
        ctx->force_tiles = 0;
        ctx->batch_persistent = pers;
        ctx->stack_lds = lds;
        r.cases_per_lane = K;
        r.tiles_cap = cap;
        r.persistent = pers;
        r.stack_lds = lds;
        r.from_cache = 1;
        if (out) *out = r;
        return TGP_OK;
    }
    tgp_batch b = nullptr;
    tgp_status st = tgp_batch_create(ctx, 0, &b);
    if (st != TGP_OK) return st;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    // (stack form, cases per lane): registers with K = 4 or 2, LDS with K = 2
    const int forms[3][2] = {{0, 4}, {0, 2}, {1, 2}};
    const int caps[2] = {4, 16};
    double best = 1e300;
    int bestK = 4, bestCap = 16, bestP = 1, bestL = 0, tried = 0;
    const int oldK = ctx->force_K, oldCap = ctx->tile_cap, oldT = ctx->force_tiles,
              oldP = ctx->batch_persistent, oldL = ctx->stack_lds;
    for (const auto &f : forms) {
        const int lf = f[0], kk = f[1];
        if (!interp_variant_exists(kk, lf ? interp_lds_stack() : interp_max_stack(), lf != 0)) continue;
        for (int cp = 0; cp < 4; ++cp) {
            const int c = caps[cp % 2], pf = cp / 2 == 0 ? 1 : 0;
            ctx->force_K = kk;
            ctx->tile_cap = c;
            ctx->force_tiles = 0;
            ctx->batch_persistent = pf;
            ctx->stack_lds = lf;
            st = tgp_batch_run(b, n_jobs, jobs);  // warm-up (and planning for this stack form)
            if (st != TGP_OK) break;
            hipEventRecord(e0, ctx->stream);
            st = tgp_batch_run(b, n_jobs, jobs);
            hipEventRecord(e1, ctx->stream);
            if (st != TGP_OK) break;
            hipEventSynchronize(e1);
            float ms = 0;
            hipEventElapsedTime(&ms, e0, e1);
            ++tried;
            if (ms < best) {
                best = ms;
                bestK = kk;
                bestCap = c;
                bestP = pf;
                bestL = lf;
            }
        }
        if (st != TGP_OK) break;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    tgp_batch_destroy(b);
    if (st != TGP_OK) {
        ctx->force_K = oldK;
        ctx->tile_cap = oldCap;
        ctx->force_tiles = oldT;
        ctx->batch_persistent = oldP;
        ctx->stack_lds = oldL;
        return st;
    }
    ctx->force_K = bestK;
    ctx->tile_cap = bestCap;
    ctx->force_tiles = 0;
    ctx->batch_persistent = bestP;
    ctx->stack_lds = bestL;
    r.cases_per_lane = bestK;
    r.tiles_cap = bestCap;
    r.persistent = bestP;
    r.stack_lds = bestL;
    r.best_ms = best;
    r.candidates = tried;
    if (cache_path) {
        std::ofstream f(cache_path, std::ios::app);
        if (f) {
            f << "{\"key\": \"" << key << "\", \"K\": " << bestK << ", \"tiles_cap\": " << bestCap
              << ", \"persistent\": " << bestP << ", \"lds\": " << bestL << ", \"ms\": " << best << "}\n";
        }
    }
    if (out) *out = r;
    return TGP_OK;
}

}  // extern "C"
