// k_fold.hip -- constant folding: every variable-free subtree that a
// variable-dependent node or a root uses is evaluated once on the device, one
// launch per subtree height, and enters the programs as a constant.
#include <hip/hip_runtime.h>
#include <math.h>

#include "ops_device.h"
#include "tgp_internal.h"

namespace tgp {

// The operator nodes of one height whose subtrees hold no variable, over the
// DAGs of a batch: entry i of list is (DAG, node).  Each node is evaluated
// once with the interpreter's own FP32 operators (ops_device.h, built with
// the same flags, so a folded value is bitwise the value every case
// computes); an operator child's value comes from the DAG's val, written by
// the launches of lower heights, a constant child's from the node values.
__global__ void k_fold_level(const FoldDesc *jobs, const int2 *list, int32_t n) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int2 e = list[i];
    const FoldDesc J = jobs[e.x];
    const int32_t u = e.y;
    const int32_t *node_kid = J.node_kid;
    const float *node_value = J.node_value;
    float *val = J.val;
    const int32_t *node_op = J.node_op;
    const int op = (int)((uint32_t)node_op[u] & 0xffu);
    const int32_t *k = node_kid + 3 * (int64_t)u;
    auto child = [&](int32_t c) {
        if (c < 0) return 0.0f;
        if (((uint32_t)node_op[c] & 0xffu) != TGP_CONST) return val[c];
        const float v = node_value[c];
        return v == v ? v : __builtin_nanf("");  // constants enter as quiet NaNs (ops_device.h, min/max)
    };
    const float a = child(k[0]);
    const float b = child(k[1]);
    const float c = child(k[2]);
    float r;
    switch (op) {
    case TGP_ADD: r = f_add(a, b); break;
    case TGP_SUB: r = f_sub(a, b); break;
    case TGP_MULT: r = f_mult(a, b); break;
    case TGP_DIV: r = f_div(a, b); break;
    case TGP_SIN: r = f_sin(a); break;
    case TGP_COS: r = f_cos(a); break;
    case TGP_TAN: r = f_tan(a); break;
    case TGP_EXP: r = f_exp(a); break;
    case TGP_LOG: r = f_log(a); break;
    case TGP_POW: r = f_pow(a, b); break;
    case TGP_MIN: r = f_min(a, b); break;
    case TGP_MAX: r = f_max(a, b); break;
    case TGP_MDIST: r = f_mdist(a, b); break;
    case TGP_NEG: r = f_neg(a); break;
    case TGP_SQRT: r = f_sqrt(a); break;
    case TGP_SIGN: r = f_sign(a); break;
    case TGP_ABS: r = f_abs(a); break;
    case TGP_CLIP: r = f_clip(a, b, c); break;
    case TGP_MOD: r = f_mod(a, b); break;
    case TGP_FRAC: r = f_frac(a); break;
    case TGP_IF: r = f_if(a, b, c); break;
    case TGP_STEP: r = f_step(a); break;
    case TGP_SSTEP: r = f_sstep(a); break;
    case TGP_SSTEPP: r = f_sstepp(a); break;
    case TGP_LEN: r = f_len(a, b); break;
    case TGP_LERP: r = f_lerp(a, b, c); break;
    case TGP_OR: r = f_bitop(a, b, 0); break;
    case TGP_XOR: r = f_bitop(a, b, 1); break;
    case TGP_AND: r = f_bitop(a, b, 2); break;
    case TGP_WARP: r = a; break;  // a constant source reads the same everywhere
    default: r = __builtin_nanf(""); break;
    }
    val[u] = r;
}

hipError_t launch_fold_level(const FoldDesc *jobs, const int2 *list, int32_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fold_level, dim3((n + 255) / 256), dim3(256), 0, s, jobs, list, n);
    return hipGetLastError();
}

}  // namespace tgp
