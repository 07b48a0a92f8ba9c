// Issue-rate micro-kernels for the roofline of the pair kernel: each lane
// runs 8 independent dependency chains of one instruction, at full
// occupancy, so that the measured time is throughput- and not latency-bound.
#include "bem_internal.h"

namespace bem {

namespace {

constexpr int PR_CHAINS = 8;
constexpr int PR_ITERS = 2048;
constexpr int PR_THREADS = 256;
constexpr int PR_BLOCKS = 256 * 16;   // 16 workgroups per CU

enum { OP_FMA32 = 0, OP_SIN32, OP_COS32, OP_RSQ32, OP_FMA64, OP_COUNT };

template <int OP>
__global__ __launch_bounds__(PR_THREADS) void rate_kernel(float *__restrict__ out) {
    float a[PR_CHAINS];
    for (int c = 0; c < PR_CHAINS; c++) a[c] = 0.1f + 1e-3f * threadIdx.x + 0.01f * c;
    for (int i = 0; i < PR_ITERS; i++) {
#pragma unroll
        for (int c = 0; c < PR_CHAINS; c++) {
            if (OP == OP_FMA32) a[c] = __builtin_fmaf(a[c], 0.999f, 0.001f);
            if (OP == OP_SIN32) a[c] = __builtin_amdgcn_sinf(a[c]);    // stays in [-1, 1]
            if (OP == OP_COS32) a[c] = __builtin_amdgcn_cosf(a[c]);
            if (OP == OP_RSQ32) a[c] = __builtin_amdgcn_rsqf(a[c]);    // x -> x^(-1/2) > 0
        }
    }
    float s = 0;
    for (int c = 0; c < PR_CHAINS; c++) s += a[c];
    out[blockIdx.x * PR_THREADS + threadIdx.x] = s;
}

__global__ __launch_bounds__(PR_THREADS) void rate_kernel_f64(float *__restrict__ out) {
    double a[PR_CHAINS];
    for (int c = 0; c < PR_CHAINS; c++) a[c] = 0.1 + 1e-3 * threadIdx.x + 0.01 * c;
    for (int i = 0; i < PR_ITERS; i++) {
#pragma unroll
        for (int c = 0; c < PR_CHAINS; c++) a[c] = __builtin_fma(a[c], 0.999, 0.001);
    }
    double s = 0;
    for (int c = 0; c < PR_CHAINS; c++) s += a[c];
    out[blockIdx.x * PR_THREADS + threadIdx.x] = (float)s;
}

void launch_rate(int op, float *out, hipStream_t s) {
    const dim3 g(PR_BLOCKS), b(PR_THREADS);
    switch (op) {
    case OP_FMA32: hipLaunchKernelGGL(rate_kernel<OP_FMA32>, g, b, 0, s, out); break;
    case OP_SIN32: hipLaunchKernelGGL(rate_kernel<OP_SIN32>, g, b, 0, s, out); break;
    case OP_COS32: hipLaunchKernelGGL(rate_kernel<OP_COS32>, g, b, 0, s, out); break;
    case OP_RSQ32: hipLaunchKernelGGL(rate_kernel<OP_RSQ32>, g, b, 0, s, out); break;
    default: hipLaunchKernelGGL(rate_kernel_f64, g, b, 0, s, out); break;
    }
}

}   // namespace

void valu_rates(double *rates, hipStream_t s) {
    DevBuf<float> out((size_t)PR_BLOCKS * PR_THREADS);
    hipEvent_t a, b;
    BEM_HIP(hipEventCreate(&a));
    BEM_HIP(hipEventCreate(&b));
    const double lane_ops = (double)PR_BLOCKS * PR_THREADS * PR_ITERS * PR_CHAINS;
    hipError_t err = hipSuccess;
    for (int op = 0; op < OP_COUNT && err == hipSuccess; op++) {
        float best = 0;
        for (int rep = 0; rep < 3 && err == hipSuccess; rep++) {   // first launch warms up
            (void)hipEventRecord(a, s);
            launch_rate(op, out.p, s);
            err = hipGetLastError();
            (void)hipEventRecord(b, s);
            if (err == hipSuccess) err = hipEventSynchronize(b);
            float ms = 0;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, a, b);
            if (rep > 0 && (best == 0 || ms < best)) best = ms;
        }
        rates[op] = best > 0 ? lane_ops / (best * 1e-3) : 0.0;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    BEM_HIP(err);
}

}   // namespace bem
