// breed.cpp -- host side of the genetic operators (tgp_breed): argument
// checks, the parents' and functions' upload, the device launches of
// k_breed.hip, and the offspring handle that owns the new population.
#include <hip/hip_runtime.h>

#include <string.h>

#include <algorithm>
#include <vector>

#include "runtime_internal.h"

using namespace tgp;

struct tgp_offspring_s {
    tgp_ctx ctx = nullptr;
    int32_t n_ind = 0, n_ch = 0;
    int64_t n_tokens = 0;
    int64_t *offsets = nullptr;  // [n_ind * n_ch + 1], device
    tgp_token *tokens = nullptr; // [n_tokens], device
    // pool blocks: the output and the scratch the launches read (released
    // when the handle is destroyed, after the stream has drained)
    std::vector<void *> blocks;
};

static void offspring_free(tgp_offspring o) {
    if (!o) return;
    if (o->ctx) {
        hipSetDevice(o->ctx->device);
        hipStreamSynchronize(o->ctx->stream);
        for (void *b : o->blocks) o->ctx->pool.release(b);
    }
    delete o;
}

extern "C" {

tgp_status tgp_breed(tgp_ctx ctx, const tgp_population *par, const double *fitness_dev,
                     const tgp_breed_params *p, tgp_offspring *out) {
    if (!ctx || !par || !p || !out) return fail(ctx, TGP_EINVAL, "NULL argument");
    *out = nullptr;
    if (par->n_individuals < 0 || par->n_channels < 1)
        return fail(ctx, TGP_EINVAL, "parents: n_individuals < 0 or n_channels < 1");
    if (par->memory != TGP_MEM_HOST && par->memory != TGP_MEM_DEVICE)
        return fail(ctx, TGP_EINVAL, "parents: memory must be TGP_MEM_HOST or TGP_MEM_DEVICE");
    if (p->n_offspring < 0) return fail(ctx, TGP_EINVAL, "n_offspring < 0");
    if (p->n_offspring > 0 && par->n_individuals < 1) return fail(ctx, TGP_EINVAL, "no parents to breed from");
    if (p->tournament < 1) return fail(ctx, TGP_EINVAL, "tournament < 1");
    if (!(p->p_crossover >= 0.0 && p->p_mutation >= 0.0 && p->p_crossover + p->p_mutation <= 1.0))
        return fail(ctx, TGP_EINVAL, "p_crossover and p_mutation must be >= 0 with a sum <= 1");
    if (p->max_depth < 0) return fail(ctx, TGP_EINVAL, "max_depth < 0");
    if (p->max_mutation_depth < 0 || p->max_mutation_depth > kMaxMutationDepth)
        return fail(ctx, TGP_EINVAL, "max_mutation_depth must be in [0, %d]", kMaxMutationDepth);
    if (p->crossover_tries < 1) return fail(ctx, TGP_EINVAL, "crossover_tries < 1");
    if (p->ndim < 1 || p->ndim > 3) return fail(ctx, TGP_EINVAL, "ndim must be 1, 2 or 3");
    if (p->n_functions < 1 || !p->functions) return fail(ctx, TGP_EINVAL, "no functions");
    for (int32_t f = 0; f < p->n_functions; ++f)
        if (p->functions[f] >= TGP_NUM_OPS || kArity[p->functions[f]] < 1)
            return fail(ctx, TGP_EOP, "functions[%d] = %d is not a function", f, (int)p->functions[f]);
    const int64_t R = (int64_t)par->n_individuals * par->n_channels;
    if (R > 0 && (!par->offsets || !par->tokens)) return fail(ctx, TGP_EINVAL, "NULL offsets/tokens");
    const int64_t n_child = (int64_t)p->n_offspring * par->n_channels;
    if (n_child > 0x7fffffffLL) return fail(ctx, TGP_EINVAL, "too many offspring trees");
    HCHK(ctx, hipSetDevice(ctx->device));

    tgp_offspring o = new tgp_offspring_s();
    o->ctx = ctx;
    o->n_ind = p->n_offspring;
    o->n_ch = par->n_channels;
    auto give_up = [&](tgp_status st, const char *what, hipError_t e) {
        offspring_free(o);
        return fail(ctx, st, "%s: %s", what, hipGetErrorString(e));
    };
    auto alloc = [&](size_t bytes, void **ptr) {
        hipError_t e = ctx->pool.alloc(ptr, std::max<size_t>(bytes, 8));
        if (e == hipSuccess) o->blocks.push_back(*ptr);
        return e;
    };

    // ---- parents on the device, and the function codes
    int64_t T = 0;
    const int64_t *off_dev = par->offsets;
    const uint2 *tok_dev = reinterpret_cast<const uint2 *>(par->tokens);
    uint8_t *fn_dev = nullptr;
    hipError_t e = hipSuccess;
    void *stage = nullptr;
    if (par->memory == TGP_MEM_HOST) {
        if (R > 0) {
            if (par->offsets[0] != 0) {
                offspring_free(o);
                return fail(ctx, TGP_EINVAL, "offsets[0] must be 0");
            }
            for (int64_t r = 0; r < R; ++r)
                if (par->offsets[r + 1] < par->offsets[r]) {
                    offspring_free(o);
                    return fail(ctx, TGP_EINVAL, "offsets decrease at tree %lld", (long long)r);
                }
            T = par->offsets[R];
        }
        const size_t ob = sizeof(int64_t) * (R + 1), tb = sizeof(tgp_token) * T, fb = p->n_functions;
        void *blk = nullptr;
        e = alloc(ob + tb + fb, &blk);
        if (e == hipSuccess) e = ctx_pinned(ctx, ob + tb + fb, &stage);
        if (e != hipSuccess) return give_up(TGP_ENOMEM, "parent upload", e);
        if (R > 0) memcpy(stage, par->offsets, ob);
        else memset(stage, 0, ob);
        if (T) memcpy((char *)stage + ob, par->tokens, tb);
        memcpy((char *)stage + ob + tb, p->functions, fb);
        e = hipMemcpyAsync(blk, stage, ob + tb + fb, hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess) e = ctx_pinned_enqueued(ctx);
        if (e != hipSuccess) return give_up(TGP_EHIP, "parent upload", e);
        off_dev = static_cast<const int64_t *>(blk);
        tok_dev = reinterpret_cast<const uint2 *>((char *)blk + ob);
        fn_dev = reinterpret_cast<uint8_t *>((char *)blk + ob + tb);
    } else {
        if (R > 0) {
            int64_t ends[2];
            e = hipMemcpyAsync(&ends[0], par->offsets, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(&ends[1], par->offsets + R, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
            if (e != hipSuccess) return give_up(TGP_EHIP, "parent offsets", e);
            if (ends[0] != 0 || ends[1] < 0 || ends[1] > 0x7fffffffLL) {
                offspring_free(o);
                return fail(ctx, TGP_EINVAL, "bad parent offsets");
            }
            T = ends[1];
        }
        void *blk = nullptr;
        e = alloc(p->n_functions, &blk);
        if (e == hipSuccess) e = ctx_pinned(ctx, p->n_functions, &stage);
        if (e != hipSuccess) return give_up(TGP_ENOMEM, "function upload", e);
        memcpy(stage, p->functions, p->n_functions);
        e = hipMemcpyAsync(blk, stage, p->n_functions, hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess) e = ctx_pinned_enqueued(ctx);
        if (e != hipSuccess) return give_up(TGP_EHIP, "function upload", e);
        fn_dev = static_cast<uint8_t *>(blk);
    }

    // ---- scratch: token shapes, records, lengths, scan partials, the error flag
    const int64_t nb = std::max<int64_t>(breed_scan_blocks(n_child), 1);
    auto part = [](size_t bytes) { return (bytes + 255) & ~(size_t)255; };
    const size_t s_shape = part(sizeof(int32_t) * T), s_rec = part(sizeof(BreedRec) * n_child),
                 s_len = part(sizeof(int64_t) * n_child), s_blk = part(sizeof(int64_t) * nb);
    void *scr = nullptr, *offb = nullptr;
    e = alloc(3 * s_shape + s_rec + s_len + s_blk + 256, &scr);
    if (e == hipSuccess) e = alloc(sizeof(int64_t) * (n_child + 1), &offb);
    if (e != hipSuccess) return give_up(TGP_ENOMEM, "breeding scratch", e);
    char *q = static_cast<char *>(scr);
    int32_t *size = reinterpret_cast<int32_t *>(q);
    int32_t *height = reinterpret_cast<int32_t *>(q + s_shape);
    int32_t *depth = reinterpret_cast<int32_t *>(q + 2 * s_shape);
    BreedRec *recs = reinterpret_cast<BreedRec *>(q + 3 * s_shape);
    int64_t *lens = reinterpret_cast<int64_t *>(q + 3 * s_shape + s_rec);
    int64_t *bsum = reinterpret_cast<int64_t *>(q + 3 * s_shape + s_rec + s_len);
    int32_t *bad = reinterpret_cast<int32_t *>(q + 3 * s_shape + s_rec + s_len + s_blk);
    o->offsets = static_cast<int64_t *>(offb);

    BreedArgs A{};
    A.tok = tok_dev;
    A.off = off_dev;
    A.size = size;
    A.height = height;
    A.depth = depth;
    A.fitness = fitness_dev;
    A.functions = fn_dev;
    A.recs = recs;
    A.lens = lens;
    A.seed = p->seed;
    A.p_crossover = p->p_crossover;
    A.p_mutation = p->p_mutation;
    A.n_parents = par->n_individuals;
    A.n_channels = par->n_channels;
    A.n_offspring = p->n_offspring;
    A.tournament = p->tournament;
    A.max_depth = p->max_depth;
    A.max_mutation_depth = p->max_mutation_depth;
    A.tries = p->crossover_tries;
    A.ndim = p->ndim;
    A.use_constants = p->use_constants ? 1 : 0;
    A.n_functions = p->n_functions;

    e = hipMemsetAsync(bad, 0, sizeof(int32_t), ctx->stream);
    record(ctx, 6);
    if (e == hipSuccess) e = launch_shape(tok_dev, off_dev, R, T, size, height, depth, bad, ctx->stream);
    record(ctx, 7);
    if (e == hipSuccess) e = launch_breed(A, bad, o->offsets, bsum, ctx->stream);
    record(ctx, 8);
    // the offspring's token count and the parents' verdict
    int64_t total = 0;
    int32_t verdict = 0;
    if (e == hipSuccess) e = ctx_pinned(ctx, 16, &stage);
    if (e == hipSuccess)
        e = hipMemcpyAsync(stage, o->offsets + n_child, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync((char *)stage + 8, bad, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return give_up(TGP_EHIP, "breeding", e);
    memcpy(&total, stage, 8);
    memcpy(&verdict, (char *)stage + 8, 4);
    if (verdict) {
        offspring_free(o);
        return verdict == 2 ? fail(ctx, TGP_EOP, "parents hold an unknown operator")
                            : fail(ctx, TGP_EPARSE, "a parent tree is not one postfix tree");
    }
    if (total > 0x7fffffffLL) {
        offspring_free(o);
        return fail(ctx, TGP_EINVAL, "offspring of more than 2^31-1 tokens");
    }
    void *tb = nullptr;
    e = alloc(sizeof(tgp_token) * total, &tb);
    if (e != hipSuccess) return give_up(TGP_ENOMEM, "offspring tokens", e);
    o->tokens = static_cast<tgp_token *>(tb);
    o->n_tokens = total;
    record(ctx, 9);
    e = launch_breed_write(A, o->offsets, reinterpret_cast<uint2 *>(o->tokens), ctx->stream);
    record(ctx, 10);
    if (e != hipSuccess) return give_up(TGP_EHIP, "offspring write", e);
    *out = o;
    return TGP_OK;
}

tgp_status tgp_offspring_population(tgp_offspring o, tgp_population *view) {
    if (!o || !view) return fail(nullptr, TGP_EINVAL, "NULL argument");
    view->n_individuals = o->n_ind;
    view->n_channels = o->n_ch;
    view->offsets = o->offsets;
    view->tokens = o->tokens;
    view->memory = TGP_MEM_DEVICE;
    return TGP_OK;
}

tgp_status tgp_offspring_export(tgp_offspring o, int64_t *n_tokens, int64_t *offsets_host,
                                tgp_token *tokens_host) {
    if (!o || !n_tokens) return fail(nullptr, TGP_EINVAL, "NULL argument");
    *n_tokens = o->n_tokens;
    if (!offsets_host || !tokens_host) return TGP_OK;
    tgp_ctx ctx = o->ctx;
    HCHK(ctx, hipSetDevice(ctx->device));
    const size_t ob = sizeof(int64_t) * ((size_t)o->n_ind * o->n_ch + 1);
    HCHK(ctx, hipMemcpyAsync(offsets_host, o->offsets, ob, hipMemcpyDeviceToHost, ctx->stream));
    if (o->n_tokens)
        HCHK(ctx, hipMemcpyAsync(tokens_host, o->tokens, sizeof(tgp_token) * o->n_tokens, hipMemcpyDeviceToHost,
                                 ctx->stream));
    HCHK(ctx, hipStreamSynchronize(ctx->stream));
    return TGP_OK;
}

void tgp_offspring_destroy(tgp_offspring o) { offspring_free(o); }

}  // extern "C"
