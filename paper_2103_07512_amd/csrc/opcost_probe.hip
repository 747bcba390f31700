// opcost_probe.hip -- measures the VALU cost model of the planner (kOpCost):
// one kernel per operator over N random
// inputs (uniform in [-1, 1], the GP domain); run under rocprofv3 --pmc
// SQ_INSTS_VALU SQ_WAVES, the VALU instructions per wave of a kernel less
// those of k_base (loads, stores, indexing) are its operator's cost per case
// (one extra for each further operand load).  Not part of the library.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "ops_device.h"
using namespace tgp;
#define KER(name, expr) __global__ void k_##name(const float *a, const float *b, const float *c, float *o, int n) { \
    const int i = blockIdx.x * blockDim.x + threadIdx.x; if (i >= n) return; \
    const float x = a[i], y = b[i], z = c[i]; (void)y; (void)z; o[i] = (expr); }
KER(base, x)
KER(add, f_add(x, y)) KER(div, f_div(x, y)) KER(sin, f_sin(x)) KER(cos, f_cos(x)) KER(tan, f_tan(x))
KER(exp, f_exp(x)) KER(log, f_log(x)) KER(pow, f_pow(x, y)) KER(min, f_min(x, y)) KER(mdist, f_mdist(x, y))
KER(sqrt, f_sqrt(x)) KER(sign, f_sign(x)) KER(clip, f_clip(x, y, z)) KER(mod, f_mod(x, y)) KER(frac, f_frac(x))
KER(iff, f_if(x, y, z)) KER(step, f_step(x)) KER(sstep, f_sstep(x)) KER(sstepp, f_sstepp(x)) KER(len, f_len(x, y))
KER(lerp, f_lerp(x, y, z)) KER(bitop, f_bitop(x, y, 1))
int main() {
    const int n = 1 << 24;
    std::vector<float> h(3 * (size_t)n);
    srand(1);
    for (auto &v : h) v = 2.0f * (float)rand() / (float)RAND_MAX - 1.0f;
    float *d, *o;
    if (hipMalloc(&d, sizeof(float) * 3 * (size_t)n) != hipSuccess || hipMalloc(&o, sizeof(float) * n) != hipSuccess) return 1;
    if (hipMemcpy(d, h.data(), sizeof(float) * 3 * (size_t)n, hipMemcpyHostToDevice) != hipSuccess) return 1;
    const float *a = d, *b = d + n, *c = d + 2 * (size_t)n;
    dim3 g(n / 256), bl(256);
#define RUN(name) hipLaunchKernelGGL(k_##name, g, bl, 0, 0, a, b, c, o, n);
    RUN(base) RUN(add) RUN(div) RUN(sin) RUN(cos) RUN(tan) RUN(exp) RUN(log) RUN(pow) RUN(min) RUN(mdist)
    RUN(sqrt) RUN(sign) RUN(clip) RUN(mod) RUN(frac) RUN(iff) RUN(step) RUN(sstep) RUN(sstepp) RUN(len) RUN(lerp) RUN(bitop)
    if (hipDeviceSynchronize() != hipSuccess) return 1;
    printf("done %d\n", n);
    return 0;
}
