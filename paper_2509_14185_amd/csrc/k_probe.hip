// k_probe.hip -- measured throughput of the FP64 matrix instructions (a
// practical ceiling reported beside the published peak; not part of the
// method).
#include "gn_internal.h"

namespace gn {

typedef double probe_acc_t __attribute__((ext_vector_type(4)));

// Throughput probe: independent MFMA chains, nothing read from memory; the
// sum of the accumulators is stored only under a condition that cannot hold
// for these inputs, so the chains stay live without a store per wave.
__device__ double mfma_probe_sink;

__global__ __launch_bounds__(256) void mfma_probe_kernel(int iters) {
    constexpr int CH = 8;
    probe_acc_t acc[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] = (probe_acc_t){0.0, 0.0, 0.0, 0.0};
    const double a = 1.0 + 1e-3 * (threadIdx.x & 63), b = 1.0 - 1e-7 * blockIdx.x;
    // iters is a multiple of 16; the unrolled body keeps the accumulators in
    // place (a rolled loop makes the compiler copy them every iteration)
    for (int i = 0; i < iters; i += 16) {
#pragma unroll
        for (int u = 0; u < 16; ++u)
#pragma unroll
            for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    }
    double sum = 0.0;
#pragma unroll
    for (int c = 0; c < CH; ++c) sum += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    if (sum < 0.0) mfma_probe_sink = sum;
}

hipError_t launch_mfma_probe(hipStream_t st, int cus, int iters, double *flops) {
    const unsigned grid = (unsigned)cus * 8u;
    hipLaunchKernelGGL(mfma_probe_kernel, dim3(grid), dim3(256), 0, st, iters);
    if (flops) *flops = (double)grid * 4.0 * (double)iters * 8.0 * 16.0 * 16.0 * 4.0 * 2.0;
    return hipGetLastError();
}

}  // namespace gn
