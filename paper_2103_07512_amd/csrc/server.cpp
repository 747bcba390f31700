// server.cpp -- the serving form of libtgp: a request loop over the
// per-generation populations of many concurrent GP runs, with continuous
// batching, admission against device memory and a resident subtree cache.
//
// Threads of its own:
//   * four preparation threads take submitted requests in arrival order; each
//     builds the population's DAG on its own stream, looks the DAG's subtrees
//     up in the resident cache, plans the programs (a resident subtree
//     becomes a cache read), and admits the request once an evaluation slot
//     is free and the rows of the subtrees it will cache fit in the cache
//     arena (unpinned entries are evicted least recently used first);
//   * execution keeps up to two batched steps in flight on its stream.  A
//     step carries the next slab of cases of every admitted request: the
//     cache fill of the slab, the root programs fused with the error
//     reduction, and a finalize that adds the slab's FP64 sums to the
//     request's running sums (the last slab writes the loss).  Requests
//     admitted while a step runs join the next one.
// The slabs, tiles per work item and summation order of a request depend on
// the request alone, so its fitness values are the same whatever else is
// being served.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "runtime_internal.h"
#include "subtree_cache.h"

namespace {

constexpr int64_t kUnitFloats = 64;  // arena unit: 256 bytes
constexpr int64_t kSlabQuantum = 1 << 16;
constexpr int kPrepThreads = 4;

uint64_t mix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// 128-bit structural hash of every DAG node: opcode, axis, constant bits and
// the children's hashes in order (children have smaller ids than parents).
void subtree_hashes(const tgp_dag_s &d, std::vector<uint64_t> &h0, std::vector<uint64_t> &h1) {
    const size_t U = d.op.size();
    h0.resize(U);
    h1.resize(U);
    for (size_t n = 0; n < U; ++n) {
        const int op = d.op[n] & 0xff;
        uint32_t bits = 0;
        if (op == TGP_CONST) memcpy(&bits, &d.value[n], 4);
        uint64_t a = mix64(((uint64_t)(uint32_t)d.op[n] << 32) | bits);
        uint64_t b = mix64(a ^ 0x5851f42d4c957f2dull);
        for (int j = 0; j < kArity[op]; ++j) {
            const int32_t c = d.kid[3 * n + j];
            a = mix64(a ^ mix64(h0[c] + (uint64_t)(j + 1)));
            b = mix64(b + (h1[c] ^ (0xd1342543de82ef95ull * (uint64_t)(j + 1))));
        }
        h0[n] = a;
        h1[n] = b;
    }
}

uint64_t domain_hash(const tgp_domain_s &d) {
    uint64_t h = mix64(0x243f6a8885a308d3ull ^ (uint64_t)d.ndim);
    for (int k = 0; k < 3; ++k) {
        uint64_t lo, hi;
        memcpy(&lo, &d.lo[k], 8);
        memcpy(&hi, &d.hi[k], 8);
        h = mix64(h ^ (uint64_t)d.shape[k]);
        h = mix64(h ^ lo);
        h = mix64(h ^ hi);
    }
    return h;
}

struct Req {
    int64_t ticket = 0, run = 0;
    int32_t n_ind = 0, n_ch = 0;
    std::vector<int64_t> offsets;
    std::vector<tgp_token> tokens;
    tgp_domain dom = nullptr;
    const float *target = nullptr;
    int32_t loss = TGP_RMSE;
    double *out_host = nullptr;
    // prepared
    Plan plan;                         // host programs, cache slots mapped to arena rows
    std::vector<CacheEntry *> entry;   // per slot
    std::vector<uint8_t> writes;       // per slot: filled by this request
    int64_t dag_nodes = 0;
    int64_t slab = 0;
    int32_t n_slabs = 0, next_slab = 0, tps = 1;
    int32_t hits = 0, fresh = 0;
    // execution
    uint2 *code_dev = nullptr;
    int32_t *rows_dev = nullptr;
    double *acc = nullptr, *out_dev = nullptr;
    // outcome
    int status = TGP_EBUSY;
    bool finished = false;
    std::string err;
    double t_submit = 0, t_prep = 0, prep_ms = 0, t_admit = 0, t_start = 0, t_done = 0;
};
using ReqP = std::shared_ptr<Req>;

}  // namespace

struct tgp_server_s {
    int device = 0;
    hipStream_t prep_stream[kPrepThreads] = {}, exec_stream = nullptr, copy_stream = nullptr;
    tgp_ctx prep[kPrepThreads] = {}, exec = nullptr;
    tgp_batch batch[2] = {nullptr, nullptr};
    hipEvent_t done_ev[2] = {nullptr, nullptr};
    hipEvent_t begin_ev[2] = {nullptr, nullptr};  // before the step's first launch (timed)
    float *arena = nullptr;
    size_t arena_bytes = 0;
    std::unique_ptr<SubtreeCache> cache;
    int max_active = 16;
    double slab_work = 8589934592.0;  // 2^33 DAG nodes x cases
    int K = 4;
    int tiles = 0;                    // tiles per work item (0: from the slab size)
    std::atomic<int> persistent{0};   // launch form of the steps (one wave per item)

    std::mutex m;
    std::condition_variable cv_prep, cv_exec, cv_done;
    std::deque<ReqP> queued, ready;
    int n_admitted = 0;  // ready or being evaluated
    std::unordered_map<int64_t, ReqP> tickets;
    int64_t next_ticket = 1;
    bool stop = false, stop_exec = false;
    std::thread prep_thr[kPrepThreads], exec_thr;
    tgp_server_stats stats{};
    std::string err;
    std::chrono::steady_clock::time_point t0;

    // execution thread only
    double *pin_out = nullptr;
    size_t pin_cap = 0;

    double now() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

tgp_status srv_fail(tgp_server s, tgp_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (s) {
        std::lock_guard<std::mutex> lk(s->m);
        s->err = buf;
    }
    return st;
}

// Ends r with status st (called with the lock held).
void end_request_locked(tgp_server s, Req &r, int st, const std::string &msg) {
    r.status = st;
    r.err = msg;
    r.finished = true;
    r.t_done = s->now();
    if (st == TGP_OK) {
        s->stats.completed += 1;
        s->stats.credited_node_evals += r.dag_nodes * (r.dom ? r.dom->cases : 0);
    } else {
        s->stats.failed += 1;
    }
    r.tokens = std::vector<tgp_token>();
    r.offsets = std::vector<int64_t>();
    r.plan = Plan();
    r.entry.clear();
    r.writes.clear();
    s->cv_done.notify_all();
}

void end_request(tgp_server s, Req &r, int st, const std::string &msg) {
    std::lock_guard<std::mutex> lk(s->m);
    end_request_locked(s, r, st, msg);
}

// ------------------------------------------------------------ preparation
void prepare(tgp_server s, tgp_ctx pc, const ReqP &rp) {
    Req &r = *rp;
    r.t_prep = s->now();
    if (r.n_ind == 0) {
        end_request(s, r, TGP_OK, "");
        return;
    }
    tgp_population pop{r.n_ind, r.n_ch, r.offsets.data(), r.tokens.data(), TGP_MEM_HOST};
    tgp_dag d = nullptr;
    tgp_status st = tgp_build_dag(pc, &pop, &d);
    if (st != TGP_OK) {
        end_request(s, r, st, std::string("build_dag: ") + tgp_last_error(pc));
        return;
    }
    std::unique_ptr<tgp_dag_s, void (*)(tgp_dag)> guard(d, tgp_dag_destroy);
    if (d->stats.max_var >= r.dom->ndim) {
        end_request(s, r, TGP_ESHAPE, "a tree uses an axis the domain does not have");
        return;
    }
    const int64_t U = d->stats.dag_nodes;
    r.dag_nodes = U;
    std::vector<uint64_t> h0, h1;
    subtree_hashes(*d, h0, h1);
    const uint64_t dk = domain_hash(*r.dom);
    auto key_of = [&](int64_t n) {
        SubtreeKey k;
        k.h0 = h0[n];
        k.h1 = h1[n];
        k.dom = dk;
        return k;
    };
    // Resident subtrees (pinned while this request may read them).
    std::vector<CacheEntry *> hit(U, nullptr);
    {
        std::lock_guard<std::mutex> lk(s->m);
        for (int64_t n = 0; n < U; ++n)
            if (kArity[d->op[n] & 0xff] > 0) hit[n] = s->cache->find(key_of(n));
    }
    d->precached.assign(U, 0);
    for (int64_t n = 0; n < U; ++n) d->precached[n] = hit[n] != nullptr;
    auto unpin_hits = [&]() {
        std::lock_guard<std::mutex> lk(s->m);
        for (CacheEntry *e : hit)
            if (e) s->cache->unpin(e, false);
    };
    st = build_plan(pc, d, r.dom->cases);
    if (st != TGP_OK) {
        unpin_hits();
        end_request(s, r, st, std::string("plan: ") + tgp_last_error(pc));
        return;
    }
    const Plan &P = d->plan;
    const int32_t n_slots = P.n_slots;
    r.entry.assign(n_slots, nullptr);
    r.writes.assign(n_slots, 0);
    std::vector<uint8_t> read(U, 0);
    for (int32_t q = 0; q < n_slots; ++q)
        if (P.slot_pre[q]) {
            read[P.slot_node[q]] = 1;
            r.entry[q] = hit[P.slot_node[q]];
        } else {
            r.writes[q] = 1;
        }
    {
        std::lock_guard<std::mutex> lk(s->m);
        for (int64_t n = 0; n < U; ++n)
            if (hit[n] && !read[n]) s->cache->unpin(hit[n], false);
    }
    r.prep_ms = s->now() - r.t_prep;
    // Admission: a free slot, and arena rows for every subtree cached anew.
    const uint64_t len = (uint64_t)((r.dom->cases + kUnitFloats - 1) / kUnitFloats);
    {
        std::unique_lock<std::mutex> lk(s->m);
        for (;;) {
            if (s->stop) {
                for (int32_t q = 0; q < n_slots; ++q)
                    if (r.entry[q]) s->cache->unpin(r.entry[q], false);
                end_request_locked(s, r, TGP_EBUSY, "server shut down before admission");
                return;
            }
            if (s->n_admitted < s->max_active) {
                bool ok = true;
                for (int32_t q = 0; q < n_slots && ok; ++q) {
                    if (!r.writes[q]) continue;
                    const SubtreeKey k = key_of(P.slot_node[q]);
                    r.entry[q] = s->cache->create(&k, len, r.run);
                    ok = r.entry[q] != nullptr;
                }
                if (ok) break;
                for (int32_t q = 0; q < n_slots; ++q)
                    if (r.writes[q] && r.entry[q]) {
                        s->cache->unpin(r.entry[q], false);
                        r.entry[q] = nullptr;
                    }
                if (s->n_admitted == 0) {
                    // nothing else holds the arena: this request can never fit
                    for (int32_t q = 0; q < n_slots; ++q)
                        if (r.entry[q]) s->cache->unpin(r.entry[q], false);
                    char msg[160];
                    snprintf(msg, sizeof msg, "cached subtrees need %llu bytes, the cache holds %llu",
                             (unsigned long long)(len * kUnitFloats * 4 * (uint64_t)n_slots),
                             (unsigned long long)s->arena_bytes);
                    end_request_locked(s, r, TGP_ENOMEM, msg);
                    return;
                }
            }
            s->cv_done.wait(lk);
        }
        s->n_admitted += 1;
        r.t_admit = s->now();
        for (int32_t q = 0; q < n_slots; ++q) (r.writes[q] ? r.fresh : r.hits) += 1;
        s->stats.cache_hits += r.hits;
        s->stats.cache_new += r.fresh;
        s->stats.bytes_peak =
            std::max<int64_t>(s->stats.bytes_peak, (int64_t)(s->cache->used_units() * kUnitFloats * 4));
    }
    // Programs with slots mapped to arena rows (in arena units).
    r.plan = P;
    for (uint2 &ins : r.plan.code_host)
        if (reads_cache_row(ins.x)) ins.y = (uint32_t)r.entry[ins.y]->off;
    for (ProgDesc &pd : r.plan.fill_host) pd.dest = (int32_t)r.entry[pd.dest]->off;
    // Slabs and work split, from this request alone.
    const int64_t cases = r.dom->cases;
    // (from the DAG's size, not from the plan, which depends on what the
    // cache holds at the time)
    const double per_case = std::max<double>(1.0, (double)U);
    int64_t slab = (int64_t)(s->slab_work / per_case);
    slab = std::max<int64_t>(kSlabQuantum, slab / kSlabQuantum * kSlabQuantum);
    // warp reads its source at any case, so the source must be complete
    // before any warp runs: such a request is evaluated in one slab
    if (slab >= cases || P.warp) slab = cases;
    r.slab = slab;
    r.n_slabs = (int32_t)((cases + slab - 1) / slab);
    const int64_t tiles = (slab + 64 * s->K - 1) / (64 * s->K);
    r.tps = s->tiles > 0 ? s->tiles : (int32_t)std::max<int64_t>(1, std::min<int64_t>(16, tiles / 16));
    guard.reset();
    {
        std::lock_guard<std::mutex> lk(s->m);
        s->ready.push_back(rp);
    }
    s->cv_exec.notify_one();
}

void prep_loop(tgp_server s, int i) {
    hipSetDevice(s->device);
    for (;;) {
        ReqP r;
        {
            std::unique_lock<std::mutex> lk(s->m);
            s->cv_prep.wait(lk, [&] { return s->stop || !s->queued.empty(); });
            if (s->stop) {
                while (!s->queued.empty()) {
                    end_request_locked(s, *s->queued.front(), TGP_EBUSY, "server shut down before admission");
                    s->queued.pop_front();
                }
                return;
            }
            r = s->queued.front();
            s->queued.pop_front();
        }
        prepare(s, s->prep[i], r);
    }
}

// -------------------------------------------------------------- execution
template <typename T>
hipError_t pool_upload(tgp_server s, T **dst, const std::vector<T> &src) {
    hipError_t e = s->exec->pool.alloc((void **)dst, sizeof(T) * std::max<size_t>(src.size(), 1));
    if (e == hipSuccess && !src.empty())
        e = hipMemcpyAsync(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, s->exec_stream);
    return e;
}

void release_exec(tgp_server s, Req &r) {
    DevicePool &p = s->exec->pool;
    p.release(r.code_dev);
    p.release(r.rows_dev);
    p.release(r.acc);
    p.release(r.out_dev);
    r.code_dev = nullptr;
    r.rows_dev = nullptr;
    r.acc = r.out_dev = nullptr;
}

// Ends an admitted request after its last step (or a failure).
void retire(tgp_server s, Req &r, hipError_t e) {
    int st = TGP_OK;
    std::string msg;
    if (e == hipSuccess) {
        const size_t bytes = sizeof(double) * (size_t)r.n_ind;
        if (s->pin_cap < bytes) {
            if (s->pin_out) hipHostFree(s->pin_out);
            s->pin_out = nullptr;
            s->pin_cap = 0;
            e = hipHostMalloc((void **)&s->pin_out, std::max<size_t>(bytes, 4096), hipHostMallocDefault);
            if (e == hipSuccess) s->pin_cap = std::max<size_t>(bytes, 4096);
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->pin_out, r.out_dev, bytes, hipMemcpyDeviceToHost, s->copy_stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->copy_stream);
        if (e == hipSuccess) memcpy(r.out_host, s->pin_out, bytes);
    }
    if (e != hipSuccess) {
        st = TGP_EHIP;
        msg = std::string("evaluation: ") + hipGetErrorString(e);
    }
    release_exec(s, r);
    std::lock_guard<std::mutex> lk(s->m);
    for (size_t q = 0; q < r.entry.size(); ++q)
        if (r.entry[q]) s->cache->unpin(r.entry[q], st == TGP_OK && r.writes[q]);
    s->n_admitted -= 1;
    end_request_locked(s, r, st, msg);
}

void exec_loop(tgp_server s) {
    hipSetDevice(s->device);
    std::vector<ReqP> active;
    struct Flight {
        int b;
        std::vector<std::pair<ReqP, bool>> items;  // request, its last slab
    };
    std::deque<Flight> flights;
    int cur = 0;
    for (;;) {
        std::vector<ReqP> fresh;
        {
            std::unique_lock<std::mutex> lk(s->m);
            while (!s->ready.empty()) {
                fresh.push_back(s->ready.front());
                s->ready.pop_front();
            }
            if (fresh.empty() && active.empty() && flights.empty()) {
                if (s->stop_exec) return;
                s->cv_exec.wait(lk, [&] { return !s->ready.empty() || s->stop_exec; });
                continue;
            }
        }
        for (ReqP &r : fresh) {
            hipError_t e = pool_upload(s, &r->code_dev, r->plan.code_host);
            if (e == hipSuccess) e = pool_upload(s, &r->rows_dev, r->plan.ind_rows_host);
            if (e == hipSuccess) e = s->exec->pool.alloc((void **)&r->out_dev, sizeof(double) * r->n_ind);
            if (e == hipSuccess && r->n_slabs > 1)
                e = s->exec->pool.alloc((void **)&r->acc, sizeof(double) * r->n_ind);
            if (e != hipSuccess) {
                hipStreamSynchronize(s->exec_stream);
                retire(s, *r, e);
                continue;
            }
            r->t_start = s->now();
            active.push_back(r);
        }
        {
            std::lock_guard<std::mutex> lk(s->m);
            s->stats.max_active_seen = std::max<int32_t>(s->stats.max_active_seen, (int32_t)active.size());
        }
        if (flights.size() < 2) {
            std::vector<StepJob> jobs;
            Flight f;
            f.b = cur;
            int64_t credited = 0;
            for (ReqP &r : active) {
                if (r->next_slab >= r->n_slabs) continue;
                const int32_t k = r->next_slab++;
                StepJob j;
                j.plan = &r->plan;
                j.domain = r->dom;
                j.n_ind = r->n_ind;
                j.n_ch = r->n_ch;
                j.case_base = (int32_t)(k * r->slab);
                j.n_cases = (int32_t)std::min<int64_t>(r->slab, r->dom->cases - k * r->slab);
                j.target = r->target;
                j.cache = s->arena;
                j.cache_stride = kUnitFloats;
                j.acc = r->n_slabs > 1 ? r->acc : nullptr;
                j.first = k == 0;
                j.last = k == r->n_slabs - 1;
                j.out = r->out_dev;
                j.loss = r->loss;
                j.tiles_per_item = r->tps;
                j.code_dev = r->code_dev;
                j.rows_dev = r->rows_dev;
                jobs.push_back(j);
                f.items.push_back({r, k == r->n_slabs - 1});
                credited += r->dag_nodes * (int64_t)j.n_cases;
            }
            if (!jobs.empty()) {
                s->exec->batch_persistent = s->persistent.load();
                hipError_t e = hipEventRecord(s->begin_ev[cur], s->exec_stream);
                tgp_status st = batch_step(s->batch[cur], (int32_t)jobs.size(), jobs.data(), credited);
                if (e == hipSuccess)
                    e = st == TGP_OK ? hipEventRecord(s->done_ev[cur], s->exec_stream) : hipErrorUnknown;
                if (e != hipSuccess) {
                    // the step was not launched: its requests fail (after the
                    // steps in flight, which may use their buffers, are done)
                    hipStreamSynchronize(s->exec_stream);
                    for (auto &it : f.items)
                        if (!it.first->finished) retire(s, *it.first, hipErrorLaunchFailure);
                    active.erase(std::remove_if(active.begin(), active.end(),
                                                [](const ReqP &r) { return r->finished; }),
                                 active.end());
                    continue;
                }
                {
                    std::lock_guard<std::mutex> lk(s->m);
                    s->stats.steps += 1;
                    s->stats.slabs += (int64_t)jobs.size();
                }
                flights.push_back(std::move(f));
                cur ^= 1;
                continue;
            }
        }
        if (!flights.empty()) {
            Flight f = std::move(flights.front());
            flights.pop_front();
            const hipError_t e = hipEventSynchronize(s->done_ev[f.b]);
            if (e != hipSuccess) hipStreamSynchronize(s->exec_stream);
            float ms = 0;
            if (e == hipSuccess && hipEventElapsedTime(&ms, s->begin_ev[f.b], s->done_ev[f.b]) == hipSuccess) {
                std::lock_guard<std::mutex> lk(s->m);
                s->stats.step_ms += ms;
            }
            for (auto &it : f.items)
                if (it.second || e != hipSuccess) {
                    if (!it.first->finished) retire(s, *it.first, e);
                }
            active.erase(std::remove_if(active.begin(), active.end(), [](const ReqP &r) { return r->finished; }),
                         active.end());
        }
    }
}

}  // namespace

extern "C" {

tgp_status tgp_server_create(tgp_ctx ctx, size_t cache_budget_bytes, int32_t max_active, tgp_server *out) {
    if (!ctx || !out) return fail(ctx, TGP_EINVAL, "NULL argument");
    *out = nullptr;
    if (max_active < 0) return fail(ctx, TGP_EINVAL, "max_active < 0");
    HCHK(ctx, hipSetDevice(ctx->device));
    std::unique_ptr<tgp_server_s> s(new tgp_server_s());
    s->device = ctx->device;
    s->max_active = max_active ? max_active : 16;
    s->t0 = std::chrono::steady_clock::now();
    size_t free_b = 0, total_b = 0;
    HCHK(ctx, hipMemGetInfo(&free_b, &total_b));
    size_t budget = cache_budget_bytes ? cache_budget_bytes : total_b / 4;
    budget = budget / (kUnitFloats * 4) * (kUnitFloats * 4);
    if (budget / (kUnitFloats * 4) > 0x7fffffffull) return fail(ctx, TGP_EINVAL, "cache budget above 512 GiB");
    auto cleanup = [&](tgp_server_s *p) {
        for (auto &c : p->prep)
            if (c) tgp_ctx_destroy(c);
        for (auto &b : p->batch)
            if (b) tgp_batch_destroy(b);
        if (p->exec) tgp_ctx_destroy(p->exec);
        for (auto &e : p->done_ev)
            if (e) hipEventDestroy(e);
        for (auto &e : p->begin_ev)
            if (e) hipEventDestroy(e);
        for (auto &q : p->prep_stream)
            if (q) hipStreamDestroy(q);
        if (p->exec_stream) hipStreamDestroy(p->exec_stream);
        if (p->copy_stream) hipStreamDestroy(p->copy_stream);
        if (p->arena) hipFree(p->arena);
    };
    hipError_t e = hipStreamCreate(&s->exec_stream);
    for (int i = 0; i < kPrepThreads && e == hipSuccess; ++i) e = hipStreamCreate(&s->prep_stream[i]);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking);
    if (e == hipSuccess && budget) e = hipMalloc((void **)&s->arena, budget);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipEventCreate(&s->done_ev[i]);
        if (e == hipSuccess) e = hipEventCreate(&s->begin_ev[i]);
    }
    if (e != hipSuccess) {
        cleanup(s.get());
        return fail(ctx, e == hipErrorOutOfMemory ? TGP_ENOMEM : TGP_EHIP, "server setup: %s",
                    hipGetErrorString(e));
    }
    s->arena_bytes = budget;
    s->cache.reset(new SubtreeCache(budget / (kUnitFloats * 4)));
    tgp_status st = tgp_ctx_create(s->device, s->exec_stream, &s->exec);
    for (int i = 0; i < kPrepThreads && st == TGP_OK; ++i)
        st = tgp_ctx_create(s->device, s->prep_stream[i], &s->prep[i]);
    for (int i = 0; i < 2 && st == TGP_OK; ++i) st = tgp_batch_create(s->exec, 1, &s->batch[i]);
    if (st != TGP_OK) {
        cleanup(s.get());
        return fail(ctx, st, "server setup: %s", tgp_last_error(nullptr));
    }
    std::vector<tgp_ctx> all(s->prep, s->prep + kPrepThreads);
    all.push_back(s->exec);
    for (tgp_ctx c : all) {
        c->reorder = ctx->reorder;
        c->cache_access_cost = ctx->cache_access_cost;
        c->force_K = ctx->force_K;
        c->tile_cap = ctx->tile_cap;
        c->batch_persistent = ctx->batch_persistent;
    }
    // A request may plan new cache rows for at most half the arena, so that
    // it can be admitted beside the resident rows it reads (pinned while it
    // runs) even when the arena is fragmented; beyond that its plan
    // recomputes subtrees instead of caching them.
    for (tgp_ctx c : s->prep) {
        c->plan_upload = false;
        c->cache_budget = budget / 2;
    }
    // One case split for every step, whatever the requests in it: four cases
    // per lane (the split, and so the summation order, of a request must not
    // depend on its neighbours).
    s->K = 4;
    s->exec->force_K = 4;
    s->stats.bytes_capacity = (int64_t)budget;
    tgp_server raw = s.release();
    for (int i = 0; i < kPrepThreads; ++i) raw->prep_thr[i] = std::thread(prep_loop, raw, i);
    raw->exec_thr = std::thread(exec_loop, raw);
    *out = raw;
    return TGP_OK;
}

void tgp_server_destroy(tgp_server s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->m);
        s->stop = true;
    }
    s->cv_prep.notify_all();
    s->cv_done.notify_all();
    for (auto &t : s->prep_thr) t.join();
    {
        std::lock_guard<std::mutex> lk(s->m);
        s->stop_exec = true;
    }
    s->cv_exec.notify_all();
    s->exec_thr.join();
    hipSetDevice(s->device);
    for (auto &b : s->batch) tgp_batch_destroy(b);
    for (tgp_ctx c : s->prep) tgp_ctx_destroy(c);
    tgp_ctx_destroy(s->exec);
    for (auto &e : s->done_ev) hipEventDestroy(e);
    for (auto &e : s->begin_ev) hipEventDestroy(e);
    for (hipStream_t q : s->prep_stream) hipStreamDestroy(q);
    hipStreamDestroy(s->exec_stream);
    hipStreamDestroy(s->copy_stream);
    if (s->pin_out) hipHostFree(s->pin_out);
    s->cache.reset();
    hipFree(s->arena);
    delete s;
}

tgp_status tgp_server_set_slab_work(tgp_server s, double node_evals) {
    if (!s || !(node_evals >= 1.0)) return srv_fail(s, TGP_EINVAL, "bad slab work");
    std::lock_guard<std::mutex> lk(s->m);
    s->slab_work = node_evals;
    return TGP_OK;
}

tgp_status tgp_server_set_launch(tgp_server s, int32_t persistent, int32_t tiles_per_item) {
    if (!s || tiles_per_item < 0) return srv_fail(s, TGP_EINVAL, "bad launch shape");
    std::lock_guard<std::mutex> lk(s->m);
    if (persistent >= 0) s->persistent = persistent != 0;
    s->tiles = tiles_per_item;
    return TGP_OK;
}

tgp_status tgp_server_submit(tgp_server s, int64_t run_id, const tgp_population *pop, tgp_domain domain,
                             const float *target_dev, int32_t loss, double *out, int64_t *ticket) {
    if (!s || !pop || !domain || !ticket) return srv_fail(s, TGP_EINVAL, "NULL argument");
    if (pop->memory != TGP_MEM_HOST) return srv_fail(s, TGP_EINVAL, "a served population must be in host memory");
    if (pop->n_individuals < 0 || pop->n_channels < 1)
        return srv_fail(s, TGP_EINVAL, "n_individuals < 0 or n_channels < 1");
    if (loss != TGP_RMSE && loss != TGP_MSE) return srv_fail(s, TGP_EINVAL, "bad loss");
    if (domain->ctx->device != s->device) return srv_fail(s, TGP_EINVAL, "domain of another device");
    const int64_t R = (int64_t)pop->n_individuals * pop->n_channels;
    if (R > 0 && (!pop->offsets || !pop->tokens || !target_dev || !out))
        return srv_fail(s, TGP_EINVAL, "NULL offsets, tokens, target or output");
    auto r = std::make_shared<Req>();
    r->run = run_id;
    r->n_ind = pop->n_individuals;
    r->n_ch = pop->n_channels;
    r->dom = domain;
    r->target = target_dev;
    r->loss = loss;
    r->out_host = out;
    if (R > 0) {
        if (pop->offsets[0] != 0) return srv_fail(s, TGP_EINVAL, "offsets[0] must be 0");
        for (int64_t i = 0; i < R; ++i)
            if (pop->offsets[i + 1] < pop->offsets[i]) return srv_fail(s, TGP_EINVAL, "offsets decrease");
        r->offsets.assign(pop->offsets, pop->offsets + R + 1);
        r->tokens.assign(pop->tokens, pop->tokens + pop->offsets[R]);
    }
    {
        std::lock_guard<std::mutex> lk(s->m);
        if (s->stop) {
            s->err = "server is shutting down";
            return TGP_EBUSY;
        }
        r->ticket = s->next_ticket++;
        r->t_submit = s->now();
        s->tickets[r->ticket] = r;
        s->queued.push_back(r);
        s->stats.submitted += 1;
        *ticket = r->ticket;
    }
    s->cv_prep.notify_one();
    return TGP_OK;
}

tgp_status tgp_server_wait(tgp_server s, int64_t ticket, int64_t timeout_us) {
    if (!s) return TGP_EINVAL;
    std::unique_lock<std::mutex> lk(s->m);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) {
        s->err = "unknown ticket";
        return TGP_EINVAL;
    }
    ReqP r = it->second;
    auto done = [&] { return r->finished; };
    if (timeout_us < 0)
        s->cv_done.wait(lk, done);
    else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done))
        return TGP_EBUSY;
    if (r->status != TGP_OK) s->err = r->err;
    return (tgp_status)r->status;
}

tgp_status tgp_server_end_run(tgp_server s, int64_t run_id) {
    if (!s) return TGP_EINVAL;
    std::lock_guard<std::mutex> lk(s->m);
    s->cache->end_run(run_id);
    return TGP_OK;
}

const char *tgp_server_last_error(tgp_server s) {
    if (!s) return "server is NULL";
    std::lock_guard<std::mutex> lk(s->m);
    thread_local std::string copy;
    copy = s->err;
    return copy.c_str();
}

tgp_status tgp_server_ticket_info(tgp_server s, int64_t ticket, tgp_ticket_info *out) {
    if (!s || !out) return TGP_EINVAL;
    std::lock_guard<std::mutex> lk(s->m);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) {
        s->err = "unknown ticket";
        return TGP_EINVAL;
    }
    const Req &r = *it->second;
    tgp_ticket_info t{};
    t.status = r.finished ? r.status : TGP_EBUSY;
    t.slabs = r.n_slabs;
    t.submit_ms = r.t_submit;
    t.admit_ms = r.t_admit;
    t.start_ms = r.t_start;
    t.done_ms = r.t_done;
    t.latency_ms = r.finished ? r.t_done - r.t_submit : 0.0;
    t.prep_ms = r.prep_ms;
    t.dag_nodes = r.dag_nodes;
    t.credited_node_evals = r.dag_nodes * (r.dom ? r.dom->cases : 0);
    t.cache_hits = r.hits;
    t.cache_new = r.fresh;
    *out = t;
    return TGP_OK;
}

tgp_status tgp_server_stats_get(tgp_server s, tgp_server_stats *out) {
    if (!s || !out) return TGP_EINVAL;
    std::lock_guard<std::mutex> lk(s->m);
    tgp_server_stats st = s->stats;
    st.evictions = (int64_t)s->cache->evictions();
    st.entries = (int64_t)s->cache->entries();
    st.bytes_in_use = (int64_t)(s->cache->used_units() * kUnitFloats * 4);
    st.bytes_capacity = (int64_t)s->arena_bytes;
    *out = st;
    return TGP_OK;
}

}  // extern "C"
