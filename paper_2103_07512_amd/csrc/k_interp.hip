// k_interp.hip -- the fused postfix interpreter (fitness and evaluate forms)
// and the per-individual FP64 finalize.
//
// Vectorised evaluation (TensorGP Sec. 3.1): every program runs over all
// fitness cases of the domain.  Here one wave runs one program; each of its
// 64 lanes owns K cases of a tile of 64*K consecutive cases (case k of lane l
// is tile_base + 64*k + l, so every load and store is coalesced), and a wave
// walks tiles_per_stripe consecutive tiles.  Work items are numbered program
// by program (programs come longest first), so the longest work starts first
// and the tail of a launch is made of short items.  The operand stack lives in
// registers (see gen_interp.py), terminals come from per-axis coordinate
// tables, constants from the instruction stream, and cached subtree values
// from the HBM cache rows.
//
// Fitness form (Sec. 4.1, RMSE against a target): each lane accumulates
// (v - t)^2 over its cases with Kahan-compensated FP32, the wave merges its
// 64 (sum, compensation) pairs exactly-summed (TwoSum) through cross-lane
// shuffles, and lane 0 writes one pair per (program, stripe).  k_finalize
// adds an individual's pairs in FP64 in a fixed order and takes sqrt(sum/N)
// (RMSE) or sum/N (MSE); any non-finite term yields +inf.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "ops_device.h"
#include "tgp_internal.h"

namespace tgp {

// K cases of one lane, passed by value in registers.
template <int K>
struct FV {
    float v[K];
};

// What warp needs to know of the domain: the position scale of axes 0 and
// 1, their sizes and strides, and the number of axes.
struct WarpGeom {
    float lo0, lo1, sc0, sc1;
    int32_t n0, n1;
    uint32_t st0, st1;
    int32_t ndim;
};

// A row of FP32 values (one per case) read and written through a buffer
// resource: the row's base in scalar registers and each lane's 32-bit byte
// offset in one vector register, so no 64-bit address arithmetic is done per
// case.  The resource spans 4 GiB from the row's start (a row of at most
// 2^30 cases; the serving arena's rows are index * stride floats in, and
// longer than stride).  Word 3 is the 32-bit data format of the gfx9 family.
struct Row {
    __amdgpu_buffer_rsrc_t r;
};
__device__ __forceinline__ Row row_at(const float *base, int64_t stride, uint32_t index) {
    const float *p = base + (size_t)index * (size_t)stride;
    return Row{__builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(p), (short)0, -1, 0x00020000)};
}
__device__ __forceinline__ float row_load(const Row &row, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(row.r, off, 0, 0));
}
__device__ __forceinline__ void row_store(const Row &row, uint32_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), row.r, off, 0, 0);
}

// The case warp reads for a case c: the points named by t0 and t1 along
// axes 0 and 1, the case's own point along a third axis.
__device__ __forceinline__ int32_t warp_case(const WarpGeom &g, float t0, float t1, int32_t c) {
    uint32_t r = (uint32_t)warp_point(t0, g.lo0, g.sc0, g.n0) * g.st0;
    if (g.ndim > 1) {
        r += (uint32_t)warp_point(t1, g.lo1, g.sc1, g.n1) * g.st1;
        if (g.ndim > 2) r += (uint32_t)c % g.st1;
    }
    return (int32_t)r;
}

#include "interp_gen.inc"

enum { MODE_REDUCE = 0, MODE_STORE = 1 };

__device__ __forceinline__ void kahan_add(float &s, float &c, float x) {
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Exact sum s + e == a + b (Knuth's TwoSum).
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Merge two compensated pairs (value = s - c).
__device__ __forceinline__ void kahan_merge(float &s, float &c, float s2, float c2) {
    float t, e;
    two_sum(s, s2, t, e);
    c = (c + c2) - e;
    s = t;
}

// Stack forms: D = 8 register slots (depth-specialised dispatch), or
// D = kLdsSlots slots in LDS (one dispatch loop, top of stack in registers).
constexpr int kLdsSlots = 16;

template <int K, int D, bool EXT>
__device__ __forceinline__ void run_prog(const uint2 *ip, const FV<K> &xv, const FV<K> &yv,
                                         const FV<K> &zv, const float *cache, int64_t cache_stride,
                                         const uint32_t (&coff)[K], const WarpGeom &wg, float *sl,
                                         int lane, FV<K> &res) {
    static_assert(D == 8 || D == kLdsSlots, "compiled stack forms: 8 registers, 16 LDS slots");
    if constexpr (D == kLdsSlots)
        run_prog_lds<K>(ip, xv, yv, zv, cache, cache_stride, coff, wg, sl, lane, res);
    else
        run_prog_d8<K, EXT>(ip - 1, xv, yv, zv, cache, cache_stride, coff, wg, res);  // fetches pre-increment
}

// This wave's LDS stack rows (one wave per workgroup).
template <int K, int D>
__device__ __forceinline__ float *lds_stack() {
    __shared__ float rows[D == kLdsSlots ? kLdsSlots * K * 64 : 1];
    return rows;
}

// One work item: program `code` over tiles_per_stripe tiles of one stripe.
template <int K, int D, int MODE, bool EXT, typename Job>
__device__ __forceinline__ void run_item(const Job &a, const uint2 *code, int32_t dest, int32_t chan,
                                         uint32_t stripe, int lane) {
    const int32_t n = a.n_cases;
    const int64_t tile_cases = 64 * K;
    const int64_t first = (int64_t)stripe * a.tiles_per_stripe * tile_cases;
    const int32_t gb = a.case_base;

    float ks = 0.0f, kc = 0.0f;
    for (int t = 0; t < a.tiles_per_stripe; ++t) {
        const int64_t base = first + (int64_t)t * tile_cases;
        if (base >= n) break;
        int32_t cidx[K];
        bool valid[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int64_t c = base + 64 * k + lane;
            valid[k] = c < n;
            cidx[k] = gb + (valid[k] ? (int32_t)c : n - 1);  // global case index
        }
        FV<K> xv, yv, zv;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t c = (uint32_t)cidx[k];
            const uint32_t i0 = div_by_magic(c, a.div_m[0], a.div_s[0]);
            xv.v[k] = a.coord[0][i0];
            if (a.ndim > 1) {
                const uint32_t r = c - i0 * (uint32_t)a.stride[0];
                const uint32_t i1 = div_by_magic(r, a.div_m[1], a.div_s[1]);
                yv.v[k] = a.coord[1][i1];
                if (a.ndim > 2) {
                    const uint32_t i2 = r - i1 * (uint32_t)a.stride[1];
                    zv.v[k] = a.coord[2][i2];
                } else {
                    zv.v[k] = 0.0f;
                }
            } else {
                yv.v[k] = 0.0f;
                zv.v[k] = 0.0f;
            }
        }
        // byte offsets of the lane's cases in every row (cases < 2^30)
        uint32_t coff[K];
#pragma unroll
        for (int k = 0; k < K; ++k) coff[k] = (uint32_t)cidx[k] * 4u;
        // the target values are loaded before the program runs, so that
        // their latency overlaps its execution
        FV<K> tv;
        if constexpr (MODE != MODE_STORE) {
            const Row trow = row_at(a.target, a.target_stride, (uint32_t)chan);
#pragma unroll
            for (int k = 0; k < K; ++k) tv.v[k] = row_load(trow, coff[k]);
        }
        FV<K> res;
        WarpGeom wg{};
        if constexpr (EXT || D == kLdsSlots) {
            wg = WarpGeom{a.warp_lo[0], a.warp_lo[1], a.warp_scale[0], a.warp_scale[1], a.shape[0], a.shape[1],
                          (uint32_t)a.stride[0], (uint32_t)a.stride[1], a.ndim};
        }
        run_prog<K, D, EXT>(code, xv, yv, zv, a.cache, a.cache_stride, coff, wg, lds_stack<K, D>(), lane, res);
        if constexpr (MODE == MODE_STORE) {
            const Row row = row_at(a.out, a.out_stride, (uint32_t)dest);
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (valid[k]) row_store(row, coff[k], res.v[k]);
        } else {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float e = res.v[k] - tv.v[k];
                if (valid[k]) kahan_add(ks, kc, e * e);
            }
        }
    }
    if constexpr (MODE == MODE_REDUCE) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const float s2 = __shfl_xor(ks, off, 64);
            const float c2 = __shfl_xor(kc, off, 64);
            kahan_merge(ks, kc, s2, c2);
        }
        if (lane == 0)
            a.partial[(size_t)dest * (size_t)a.n_stripes + stripe] = make_float2(ks, kc);
    }
}

// Waves per SIMD the plain interpreter asks for.  The fitness form runs at
// seven (72 VGPRs): its dispatch chain waits on scalar loads and its cache
// rows on vector loads, and a seventh resident wave hides more of that than
// the few values that then live in scratch cost (only the z vector of 3-D
// domains is reloaded inside the dispatch loop; 1000 x 3 population on
// 1024^2: 66 ms against 69 ms at six).  The store form (cache fill) keeps
// six, where it spills less.  The batched kernels hold more descriptor state
// and spill far more at these counts (measured slower), so they keep the
// compiler's choice.
template <int MODE>
constexpr int min_waves() { return MODE == MODE_REDUCE ? 7 : 6; }

template <int K, int D, int MODE, bool EXT>
__global__ __launch_bounds__(64, min_waves<MODE>()) void k_interp(const InterpArgs a) {
    const uint32_t item = blockIdx.x;
    const uint32_t p = item / (uint32_t)a.job.n_stripes;
    const uint32_t stripe = item - p * (uint32_t)a.job.n_stripes;
    const ProgDesc pd = a.progs[p];
    run_item<K, D, MODE, EXT>(a.job, a.job.code + pd.code_off, pd.dest, pd.chan, stripe, threadIdx.x);
}

// Batched interpreter, two launch forms over the work items of group g
// (items ordered longest program first; pair p owns items item_first[p] ..
// item_first[p + 1] - 1, one per stripe).
//
// Persistent form: a fixed grid of resident waves.  The items are dealt into
// 8 interleaved partitions (item i belongs to partition i mod 8), each with
// its own atomic counter, so that claims from the chip's 8 XCDs rarely meet
// on one address; a wave starts on partition blockIdx mod 8, claims CH items
// per atomic, and when its partition is exhausted it helps the others.  The
// loops are bounded: every counter only grows, and a wave leaves a
// partition once its counter passes the partition's size.
// Descriptors are read through the constant address space: the loads are
// then known to be invariant, so the compiler keeps them scalar and may load
// them again instead of spilling them across the interpreter.
template <typename T>
__device__ __forceinline__ T load_const(const T *p) {
    T r;
    __builtin_memcpy(&r, (const __attribute__((address_space(4))) void *)(p), sizeof(T));
    return r;
}

// A job descriptor read in place through the constant address space: each
// field is a scalar load the compiler may repeat where it is used, so the
// descriptor does not occupy scalar registers for a whole work item.
typedef const __attribute__((address_space(4))) JobDesc CJobDesc;

__device__ __forceinline__ uint32_t load_const_u32(const uint32_t *p) {
    typedef const __attribute__((address_space(4))) uint32_t cword;
    return *(cword *)(p);
}

constexpr uint32_t kParts = 8;
constexpr uint32_t kChunk = 4;

__device__ __forceinline__ uint32_t find_pair(const uint32_t *__restrict__ item_first, uint32_t lo,
                                              uint32_t hi, uint32_t item) {
    // the last pair p in [lo, hi) with item_first[p] <= item
    while (hi - lo > 1) {
        const uint32_t m = (lo + hi) >> 1;
        if (load_const_u32(item_first + m) <= item) lo = m;
        else hi = m;
    }
    return lo;
}

template <int K, int D, int MODE, bool EXT>
__global__ __launch_bounds__(64, min_waves<MODE>()) void k_batch(const JobDesc *__restrict__ jobs,
                                              const PairDesc *__restrict__ pairs,
                                              const uint32_t *__restrict__ item_first,
                                              const GroupDesc *__restrict__ groups, int32_t g,
                                              uint32_t *__restrict__ counters) {
    const GroupDesc gd = load_const(groups + g);
    const uint32_t n_items = gd.item_end - gd.item_begin;
    const uint32_t first_part = blockIdx.x % kParts;
    for (uint32_t q = 0; q < kParts; ++q) {
        const uint32_t part = (first_part + q) % kParts;
        const uint32_t n_part = n_items > part ? (n_items - part + kParts - 1) / kParts : 0;
        uint32_t lo = gd.pair_begin;
        for (;;) {
            uint32_t k0 = 0;
            if (threadIdx.x == 0) k0 = atomicAdd(&counters[g * kParts + part], kChunk);
            k0 = __builtin_amdgcn_readfirstlane(k0);
            if (k0 >= n_part) break;
            const uint32_t k1 = k0 + kChunk < n_part ? k0 + kChunk : n_part;
            for (uint32_t k = k0; k < k1; ++k) {
                const uint32_t item = gd.item_begin + part + kParts * k;
                lo = find_pair(item_first, lo, gd.pair_end, item);
                const PairDesc pd = load_const(pairs + lo);
                const CJobDesc &jd = *(CJobDesc *)(jobs + pd.job);
                const uint32_t stripe = item - load_const_u32(item_first + lo);
                run_item<K, D, MODE, EXT>(jd, jd.code + pd.code_off, pd.dest, pd.chan, stripe, threadIdx.x);
            }
        }
    }
}

// Direct form: one wave per item (grid = the group's item count, or more);
// the hardware dispatcher hands out the waves in item order.
template <int K, int D, int MODE, bool EXT>
__global__ __launch_bounds__(64, min_waves<MODE>()) void k_batch_direct(const JobDesc *__restrict__ jobs,
                                                     const PairDesc *__restrict__ pairs,
                                                     const uint32_t *__restrict__ item_first,
                                                     const GroupDesc *__restrict__ groups, int32_t g) {
    const GroupDesc gd = load_const(groups + g);
    const uint32_t item = gd.item_begin + blockIdx.x;
    if (item >= gd.item_end) return;
    const uint32_t lo = find_pair(item_first, gd.pair_begin, gd.pair_end, item);
    const PairDesc pd = load_const(pairs + lo);
    const CJobDesc &jd = *(CJobDesc *)(jobs + pd.job);
    run_item<K, D, MODE, EXT>(jd, jd.code + pd.code_off, pd.dest, pd.chan, item - load_const_u32(item_first + lo),
                         threadIdx.x);
}

__global__ void k_reset(uint32_t *counters, int32_t n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) counters[i] = 0u;
}

// One block per individual: FP64 sum of the (sum - compensation) pairs of its
// channels' partial rows, stripes in order, then a fixed-shape tree in LDS.
__device__ __forceinline__ void finalize_one(const float2 *partial, const int32_t *ind_rows,
                                             int32_t n_ch, int32_t n_stripes, double n_terms,
                                             int32_t loss, double *out, double *acc_in, int first,
                                             int last, int i) {
    __shared__ double red[256];
    __shared__ int bad[256];
    const int tid = threadIdx.x;
    double acc = 0.0;
    int nonfinite = 0;
    const int64_t total = (int64_t)n_ch * n_stripes;
    for (int64_t j = tid; j < total; j += 256) {
        const int ch = (int)(j / n_stripes);
        const int st = (int)(j - (int64_t)ch * n_stripes);
        const int32_t row = ind_rows[(int64_t)i * n_ch + ch];
        const float2 v = partial[(size_t)row * (size_t)n_stripes + st];
        if (!isfinite(v.x) || !isfinite(v.y)) nonfinite = 1;
        acc += (double)v.x - (double)v.y;
    }
    red[tid] = acc;
    bad[tid] = nonfinite;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            red[tid] += red[tid + w];
            bad[tid] |= bad[tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        double s = red[0];
        if (bad[0]) s = INFINITY;
        if (acc_in) {  // one slab: running sum over the slabs in order
            if (!first) s = acc_in[i] + s;
            if (!last) {
                acc_in[i] = s;
                return;
            }
        }
        double f;
        if (!isfinite(s))
            f = INFINITY;
        else
            f = loss == TGP_RMSE ? sqrt(s / n_terms) : s / n_terms;
        out[i] = f;
    }
}

__global__ __launch_bounds__(256) void k_finalize(const float2 *partial, const int32_t *ind_rows,
                                                  int32_t n_ch, int32_t n_stripes, double n_terms,
                                                  int32_t loss, double *out) {
    finalize_one(partial, ind_rows, n_ch, n_stripes, n_terms, loss, out, nullptr, 1, 1, blockIdx.x);
}

// Batched finalize: block b is global individual b; blocks past the batch's
// individuals return at once (the grid is sized for the batch's capacity).
__global__ __launch_bounds__(256) void k_finalize_batch(const FinJob *jobs, const int32_t *n_jobs,
                                                        const uint32_t *n_ind) {
    const uint32_t b = blockIdx.x;
    if (b >= *n_ind) return;
    int32_t lo = 0, hi = *n_jobs;  // last job with ind_begin <= b
    while (hi - lo > 1) {
        const int32_t m = (lo + hi) >> 1;
        if (jobs[m].ind_begin <= b) lo = m;
        else hi = m;
    }
    const FinJob f = jobs[lo];
    finalize_one(f.partial, f.ind_rows, f.n_ch, f.n_stripes, f.n_terms, f.loss, f.out, f.acc, f.first, f.last,
                 (int)(b - f.ind_begin));
}

// ------------------------------------------------------------- launchers
template <int K, int D, bool EXT>
static hipError_t launch_kd(bool store, const InterpArgs &a, hipStream_t s) {
    const uint32_t items = (uint32_t)a.n_progs * (uint32_t)a.job.n_stripes;
    if (items == 0) return hipSuccess;
    if (store)
        hipLaunchKernelGGL((k_interp<K, D, MODE_STORE, EXT>), dim3(items), dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL((k_interp<K, D, MODE_REDUCE, EXT>), dim3(items), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <int K, int D, bool EXT>
static const void *batch_fn(bool store, bool persistent) {
    if (persistent)
        return store ? (const void *)k_batch<K, D, MODE_STORE, EXT> : (const void *)k_batch<K, D, MODE_REDUCE, EXT>;
    return store ? (const void *)k_batch_direct<K, D, MODE_STORE, EXT>
                 : (const void *)k_batch_direct<K, D, MODE_REDUCE, EXT>;
}

template <int K, int D, bool EXT>
static int grid_bd(bool store) {
    int per_cu = 0, dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (store)
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<K, D, MODE_STORE, EXT>, 64, 0);
    else
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<K, D, MODE_REDUCE, EXT>, 64, 0);
    return std::max(1, per_cu) * std::max(1, cus);
}

// Instantiated interpreters: (cases per lane, stack slots, bitwise operators
// and warp).  The LDS-stack form knows every operator.
#ifndef TGP_VARIANTS
#define TGP_VARIANTS(X) X(4, 8, false) X(2, 8, false) X(4, 8, true) X(2, 16, true)
#endif

bool interp_variant_exists(int K, int D, bool bit) {
    if (D == kLdsSlots) bit = true;
#define X(k, d, b) if (K == k && D == d && bit == b) return true;
    TGP_VARIANTS(X)
#undef X
    return false;
}

int interp_max_stack() { return 8; }
int interp_lds_stack() { return kLdsSlots; }

hipError_t launch_interp(int K, int D, bool store, const InterpArgs &a, hipStream_t s, bool bit) {
    if (D == kLdsSlots) bit = true;
#define X(k, d, b) if (K == k && D == d && bit == b) return launch_kd<k, d, b>(store, a, s);
    TGP_VARIANTS(X)
#undef X
    return hipErrorInvalidValue;
}

const void *batch_kernel(int K, int D, bool store, bool persistent, bool bit) {
    if (D == kLdsSlots) bit = true;
#define X(k, d, b) if (K == k && D == d && bit == b) return batch_fn<k, d, b>(store, persistent);
    TGP_VARIANTS(X)
#undef X
    return nullptr;
}

int batch_grid(int K, int D, bool store, bool bit) {
    if (D == kLdsSlots) bit = true;
#define X(k, d, b) if (K == k && D == d && bit == b) return grid_bd<k, d, b>(store);
    TGP_VARIANTS(X)
#undef X
    return 0;
}

hipError_t launch_reset(uint32_t *counters, int32_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_reset, dim3((n + 255) / 256), dim3(256), 0, s, counters, n);
    return hipGetLastError();
}

const void *reset_kernel() { return (const void *)k_reset; }
const void *finalize_batch_kernel() { return (const void *)k_finalize_batch; }
uint32_t batch_parts() { return kParts; }

hipError_t launch_finalize(const float2 *partial, const int32_t *ind_rows, int32_t n_ind,
                           int32_t n_ch, int32_t n_stripes, double n_terms, int32_t loss,
                           double *out, hipStream_t s) {
    if (n_ind == 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3(n_ind), dim3(256), 0, s, partial, ind_rows, n_ch, n_stripes,
                       n_terms, loss, out);
    return hipGetLastError();
}

hipError_t launch_finalize_batch(const FinJob *jobs, const int32_t *n_jobs, const uint32_t *n_ind,
                                 int32_t grid, hipStream_t s) {
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize_batch, dim3(grid), dim3(256), 0, s, jobs, n_jobs, n_ind);
    return hipGetLastError();
}

}  // namespace tgp
