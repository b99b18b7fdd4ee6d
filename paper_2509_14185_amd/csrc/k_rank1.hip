// Kernels of the stochastic full-matrix Gauss-Newton step (Methods, "Second-
// order Optimizer"): the moving average of rank-1 curvature estimates, the
// products with J that give the exact quadratic model along two directions,
// and the update with the closed-form learning rate and momentum.  All of
// them are bound by HBM bandwidth: each reads (and the average also writes)
// its matrix once, rows contiguous along the thread index.
#include <hip/hip_runtime.h>

#include "gn_internal.h"

namespace gn {

// Lower triangle of G <- beta G + (1 - beta) u u^T.  blockIdx.y is the row,
// blockIdx.x a run of 1024 columns (4 per thread); runs right of the
// diagonal exit.
__global__ __launch_bounds__(256) void ema_rank1_kernel(double *G, int64_t p, int64_t ldg, double beta,
                                                        const double *__restrict__ u) {
    const int64_t i = blockIdx.y;
    const int64_t j0 = (int64_t)blockIdx.x * 1024;
    if (j0 > i) return;
    const double ci = (1.0 - beta) * u[i];
    double *row = G + i * ldg;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t j = j0 + k * 256 + threadIdx.x;
        if (j <= i) row[j] = fma(ci, u[j], beta * row[j]);
    }
}

hipError_t launch_ema_rank1(hipStream_t st, double *G, int64_t p, int64_t ldg, double beta, const double *u) {
    if (p <= 0) return hipSuccess;
    if (p > 65535) return hipErrorInvalidValue;  // one grid row per matrix row
    hipLaunchKernelGGL(ema_rank1_kernel, dim3((unsigned)((p + 1023) / 1024), (unsigned)p), dim3(256), 0, st, G, p,
                       ldg, beta, u);
    return hipGetLastError();
}

// Lower triangle (with the diagonal) of src into dst; same indexing.
__global__ __launch_bounds__(256) void copy_lower_kernel(const double *__restrict__ src, int64_t lds, double *dst,
                                                         int64_t ldd) {
    const int64_t i = blockIdx.y;
    const int64_t j0 = (int64_t)blockIdx.x * 1024;
    if (j0 > i) return;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t j = j0 + k * 256 + threadIdx.x;
        if (j <= i) dst[i * ldd + j] = src[i * lds + j];
    }
}

hipError_t launch_copy_lower(hipStream_t st, const double *src, int64_t lds, double *dst, int64_t ldd, int64_t n) {
    if (n <= 0) return hipSuccess;
    if (n > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(copy_lower_kernel, dim3((unsigned)((n + 1023) / 1024), (unsigned)n), dim3(256), 0, st, src, lds,
                       dst, ldd);
    return hipGetLastError();
}

// y1 = J x1, y2 = J x2 for a row-major m x p matrix (leading dimension ld):
// one wave per row, J read once for both products.
__global__ __launch_bounds__(256) void gemv_n2_kernel(const double *__restrict__ J, int64_t m, int64_t p, int64_t ld,
                                                      const double *__restrict__ x1, const double *__restrict__ x2,
                                                      double *__restrict__ y1, double *__restrict__ y2) {
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= m) return;
    const double *a = J + row * ld;
    double s1 = 0.0, s2 = 0.0;
    for (int64_t c = lane; c < p; c += 64) {
        const double v = a[c];
        s1 = fma(v, x1[c], s1);
        s2 = fma(v, x2[c], s2);
    }
    for (int o = 32; o > 0; o >>= 1) {
        s1 += __shfl_xor(s1, o, 64);
        s2 += __shfl_xor(s2, o, 64);
    }
    if (lane == 0) {
        y1[row] = s1;
        y2[row] = s2;
    }
}

hipError_t launch_gemv_n2(hipStream_t st, const double *J, int64_t m, int64_t p, int64_t ld, const double *x1,
                          const double *x2, double *y1, double *y2) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(gemv_n2_kernel, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st, J, m, p, ld, x1, x2, y1, y2);
    return hipGetLastError();
}

// Up to DOT_MAX dot products of equal-length vector pairs in two launches:
// block partials in a fixed order, then one sum per pair (deterministic).
constexpr int DOT_BLOCKS = 120;

__global__ __launch_bounds__(256) void dots_partial_kernel(DotPairs d, int64_t n, double *__restrict__ work) {
    __shared__ double red[DOT_MAX][4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double acc[DOT_MAX];
#pragma unroll
    for (int k = 0; k < DOT_MAX; ++k) acc[k] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < n; i += (int64_t)gridDim.x * 256) {
#pragma unroll
        for (int k = 0; k < DOT_MAX; ++k)
            if (k < d.count) acc[k] = fma(d.x[k][i], d.y[k][i], acc[k]);
    }
#pragma unroll
    for (int k = 0; k < DOT_MAX; ++k) {
        double v = acc[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) red[k][wave] = v;
    }
    __syncthreads();
    if (tid < d.count) work[tid * DOT_BLOCKS + blockIdx.x] = ((red[tid][0] + red[tid][1]) + red[tid][2]) + red[tid][3];
}

__global__ __launch_bounds__(64) void dots_final_kernel(int count, const double *__restrict__ work,
                                                        double *__restrict__ out) {
    const int k = threadIdx.x;
    if (k >= count) return;
    double s = 0.0;
    for (int b = 0; b < DOT_BLOCKS; ++b) s += work[k * DOT_BLOCKS + b];
    out[k] = s;
}

hipError_t launch_dots(hipStream_t st, const DotPairs &d, int64_t n, double *out, double *work) {
    if (d.count <= 0 || d.count > DOT_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(dots_partial_kernel, dim3(DOT_BLOCKS), dim3(256), 0, st, d, n, work);
    hipLaunchKernelGGL(dots_final_kernel, dim3(1), dim3(64), 0, st, d.count, work, out);
    return hipGetLastError();
}

int64_t dots_work_size() { return (int64_t)DOT_MAX * DOT_BLOCKS; }

// g1 = J^T r1 and g2 = J^T r2 (accumulate: added to g1, g2) in one pass over
// the row-major m x p matrix J: for each vector the partial sums over 64 row
// chunks and their final sum are those of launch_gemv_t (same chunks, same
// order), so the results are bitwise the same as two such calls.
constexpr int GEMV2_CHUNKS = 64;

int64_t gemv_t2_work_size(int64_t p) { return (int64_t)2 * GEMV2_CHUNKS * p; }

__global__ void gemv_t2_partial(const double *__restrict__ J, int64_t m, int64_t p, int64_t ldj,
                                const double *__restrict__ r1, const double *__restrict__ r2,
                                double *__restrict__ work) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= p) return;
    const int64_t per = (m + GEMV2_CHUNKS - 1) / GEMV2_CHUNKS;
    const int64_t i0 = blockIdx.y * per;
    const int64_t i1 = (i0 + per < m) ? i0 + per : m;
    double a1 = 0.0, a2 = 0.0;
    for (int64_t i = i0; i < i1; ++i) {
        const double v = J[i * ldj + c];
        a1 = fma(v, r1[i], a1);
        a2 = fma(v, r2[i], a2);
    }
    work[blockIdx.y * p + c] = a1;
    work[(GEMV2_CHUNKS + blockIdx.y) * p + c] = a2;
}

__global__ void gemv_t2_final(const double *__restrict__ work, int64_t p, double *g1, double *g2, int accumulate) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= p) return;
    double s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < GEMV2_CHUNKS; ++k) {
        s1 += work[k * p + c];
        s2 += work[(GEMV2_CHUNKS + k) * p + c];
    }
    g1[c] = accumulate ? g1[c] + s1 : s1;
    g2[c] = accumulate ? g2[c] + s2 : s2;
}

hipError_t launch_gemv_t2(hipStream_t st, const double *J, int64_t m, int64_t p, int64_t ldj, const double *r1,
                          const double *r2, double *g1, double *g2, double *work, int accumulate) {
    if (p <= 0) return hipSuccess;
    dim3 g((unsigned)((p + 255) / 256), GEMV2_CHUNKS);
    hipLaunchKernelGGL(gemv_t2_partial, g, dim3(256), 0, st, J, m, p, ldj, r1, r2, work);
    hipLaunchKernelGGL(gemv_t2_final, dim3((unsigned)((p + 255) / 256)), dim3(256), 0, st, work, p, g1, g2,
                       accumulate);
    return hipGetLastError();
}

// y_k = cs o x_k (accumulate = 0) or y_k += cs o x_k, k = 1, 2, over n
// entries: the row scale of the Hilbert coupling applied to two vectors.
__global__ void diag_scale2_kernel(int64_t n, const double *__restrict__ cs, const double *__restrict__ x1,
                                   const double *__restrict__ x2, double *y1, double *y2, int accumulate) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double c = cs[i];
    y1[i] = accumulate ? fma(c, x1[i], y1[i]) : c * x1[i];
    y2[i] = accumulate ? fma(c, x2[i], y2[i]) : c * x2[i];
}

hipError_t launch_diag_scale2(hipStream_t st, int64_t n, const double *cs, const double *x1, const double *x2,
                              double *y1, double *y2, int accumulate) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(diag_scale2_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, cs, x1, x2, y1, y2,
                       accumulate);
    return hipGetLastError();
}

// delta = alpha D + mu prev (written over prev), theta += delta.
__global__ void rank1_update_kernel(double *theta, double *prev, const double *__restrict__ D, double alpha,
                                    double mu, int64_t p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p) return;
    const double d = alpha * D[i] + mu * prev[i];
    prev[i] = d;
    theta[i] += d;
}

hipError_t launch_rank1_update(hipStream_t st, double *theta, double *prev, const double *D, double alpha, double mu,
                               int64_t p) {
    if (p <= 0) return hipSuccess;
    hipLaunchKernelGGL(rank1_update_kernel, dim3((unsigned)((p + 255) / 256)), dim3(256), 0, st, theta, prev, D, alpha,
                       mu, p);
    return hipGetLastError();
}

}  // namespace gn
