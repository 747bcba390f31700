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

#include "ops_device.h"
#include "tgp_internal.h"

namespace tgp {

// K cases of one lane, passed by value in registers.
template <int K>
struct FV {
    float v[K];
};

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

template <int K, int D>
__device__ __forceinline__ void run_prog(const uint2 *ip, const FV<K> &xv, const FV<K> &yv,
                                         const FV<K> &zv, const float *cache, int32_t n_cases,
                                         const int32_t (&cidx)[K], FV<K> &res) {
    static_assert(D == 8, "compiled stack size: 8");
    run_prog_d8<K>(ip, xv, yv, zv, cache, n_cases, cidx, res);
}

template <int K, int D, int MODE>
__global__ __launch_bounds__(64) void k_interp(const InterpArgs a) {
    const int lane = threadIdx.x;
    const uint32_t item = blockIdx.x;
    const uint32_t p = item / (uint32_t)a.n_stripes;
    const uint32_t stripe = item - p * (uint32_t)a.n_stripes;
    const ProgDesc pd = a.progs[p];
    const uint2 *code = a.code + pd.code_off;
    const int32_t n = a.n_cases;
    const int64_t tile_cases = 64 * K;
    const int64_t first = (int64_t)stripe * a.tiles_per_stripe * tile_cases;

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
            cidx[k] = valid[k] ? (int32_t)c : n - 1;
        }
        FV<K> xv, yv, zv;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t c = (uint32_t)cidx[k];
            const uint32_t i0 = c / (uint32_t)a.stride[0];
            xv.v[k] = a.coord[0][i0];
            if (a.ndim > 1) {
                const uint32_t r = c - i0 * (uint32_t)a.stride[0];
                const uint32_t i1 = r / (uint32_t)a.stride[1];
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
        FV<K> res;
        run_prog<K, D>(code, xv, yv, zv, a.cache, n, cidx, res);
        if constexpr (MODE == MODE_STORE) {
            float *row = a.out + (size_t)pd.dest * (size_t)n;
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (valid[k]) row[cidx[k]] = res.v[k];
        } else {
            const float *trow = a.target + (size_t)pd.chan * (size_t)n;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float e = res.v[k] - trow[cidx[k]];
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
            a.partial[(size_t)pd.dest * (size_t)a.n_stripes + stripe] = make_float2(ks, kc);
    }
}

// One block per individual: FP64 sum of the (sum - compensation) pairs of its
// channels' partial rows, stripes in order, then a fixed-shape tree in LDS.
__global__ __launch_bounds__(256) void k_finalize(const float2 *partial, const int32_t *ind_rows,
                                                  int32_t n_ch, int32_t n_stripes, double n_terms,
                                                  int32_t loss, double *out) {
    __shared__ double red[256];
    __shared__ int bad[256];
    const int i = blockIdx.x;
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
        const double s = red[0];
        double f;
        if (bad[0] || !isfinite(s))
            f = INFINITY;
        else
            f = loss == TGP_RMSE ? sqrt(s / n_terms) : s / n_terms;
        out[i] = f;
    }
}

// ------------------------------------------------------------- launchers
template <int K, int D>
static hipError_t launch_kd(bool store, const InterpArgs &a, hipStream_t s) {
    const uint32_t items = (uint32_t)a.n_progs * (uint32_t)a.n_stripes;
    if (items == 0) return hipSuccess;
    if (store)
        hipLaunchKernelGGL((k_interp<K, D, MODE_STORE>), dim3(items), dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL((k_interp<K, D, MODE_REDUCE>), dim3(items), dim3(64), 0, s, a);
    return hipGetLastError();
}

#ifndef TGP_VARIANTS
#define TGP_VARIANTS(X) X(4, 8) X(2, 8)
#endif

bool interp_variant_exists(int K, int D) {
#define X(k, d) if (K == k && D == d) return true;
    TGP_VARIANTS(X)
#undef X
    return false;
}

int interp_max_stack() { return 8; }

hipError_t launch_interp(int K, int D, bool store, const InterpArgs &a, hipStream_t s) {
#define X(k, d) if (K == k && D == d) return launch_kd<k, d>(store, a, s);
    TGP_VARIANTS(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_finalize(const float2 *partial, const int32_t *ind_rows, int32_t n_ind,
                           int32_t n_ch, int32_t n_stripes, double n_terms, int32_t loss,
                           double *out, hipStream_t s) {
    if (n_ind == 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3(n_ind), dim3(256), 0, s, partial, ind_rows, n_ch, n_stripes,
                       n_terms, loss, out);
    return hipGetLastError();
}

}  // namespace tgp
