// Damped solve of the Gauss-Newton system on gfx950 (paper, Methods,
// "Second-order Optimizer": theta <- theta - (G + gamma I)^{-1} grad h).
//
// Right-looking blocked Cholesky with 64-wide panels:
//   1. diagonal block: one wave factors it in LDS and forms the inverse of
//      its triangular factor (forward substitution on the identity);
//   2. panel below: L21 = A21 L11^{-T} as an MFMA GEMM with the inverse;
//   3. trailing update: A22 -= L21 L21^T (lower) as an MFMA GEMM.
// A failed pivot records its 1-based global index and raises a device flag;
// every later kernel of the factorisation and solve sees the flag and exits.
//
// Border row: when the system is [[G, g], [g^T, r^T r]] (the gradient stored
// as an extra last row), the last row's diagonal is not square-rooted; it
// ends as the Schur complement r^T r - g^T (G + mu I)^{-1} g and the rest of
// that row as w = L^{-1} g, so the forward substitution comes for free.
//
// Triangular solves use the stored diagonal-block inverses: one launch per
// 64-row block computes the block's unknowns and applies them to the
// remaining right-hand side, row-parallel across workgroups.
#include "gn_internal.h"

namespace gn {

static constexpr int NB = 64;

int64_t chol_linv_size(int64_t n) { return ((n + NB - 1) / NB) * NB * NB; }

__global__ void add_diag_kernel(double *A, int64_t n, int64_t lda, double mu) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) A[i * lda + i] += mu;
}

// One wave.  at[c][r] holds A[k0+r][k0+c] so that "lane r owns row r" is a
// contiguous LDS access and column reads are broadcasts.
__global__ __launch_bounds__(64) void potrf_block_kernel(double *A, int64_t lda, int64_t k0, int kb, int kf,
                                                         double *linv, DevStatus *status) {
    if (status->flag) return;
    __shared__ double at[NB][NB];
    __shared__ double x[NB][NB];
    const int lane = threadIdx.x;
    for (int r = 0; r < NB; ++r) {
        double v = 0.0;
        if (r < kb && lane <= r) v = A[(k0 + r) * lda + k0 + lane];
        at[lane][r] = v;
    }
    __syncthreads();
    for (int j = 0; j < kf; ++j) {
        const double d = at[j][j];
        if (!(d > 0.0)) {  // uniform across the wave
            if (lane == 0) {
                status->chol_info = k0 + j + 1;
                status->flag = 1;
            }
            return;
        }
        const double ljj = sqrt(d);
        __syncthreads();
        if (lane == j) at[j][j] = ljj;
        if (lane > j && lane < kb) at[j][lane] /= ljj;
        __syncthreads();
        if (lane > j && lane < kb) {
            const double lij = at[j][lane];
            for (int c = j + 1; c <= lane; ++c) at[c][lane] -= lij * at[j][c];
        }
        __syncthreads();
    }
    // write the factor (lower triangle of the block)
    for (int r = 0; r < kb; ++r)
        if (lane <= r) A[(k0 + r) * lda + k0 + lane] = at[lane][r];
    // inverse of the leading kf x kf factor, row by row: lane c owns column c,
    // X[i][c] = (delta_ic - sum_{k<i} L[i][k] X[k][c]) / L[i][i]
    for (int i = 0; i < NB; ++i) {
        double v = 0.0;
        if (i < kf && lane <= i) {
            double s = (lane == i) ? 1.0 : 0.0;
            for (int k = lane; k < i; ++k) s -= at[k][i] * x[k][lane];
            v = s / at[i][i];
        }
        x[i][lane] = v;
        __syncthreads();
    }
    double *out = linv + (k0 / NB) * NB * NB;
    for (int r = 0; r < NB; ++r) out[r * NB + lane] = x[r][lane];
}

hipError_t launch_cholesky(hipStream_t st, double *A, int64_t n, int64_t lda, double mu, int border, double *linv,
                           DevStatus *status) {
    if (n <= 0) return hipSuccess;
    const int64_t nd = n - border;
    if (mu != 0.0 && nd > 0)
        hipLaunchKernelGGL(add_diag_kernel, dim3((unsigned)((nd + 255) / 256)), dim3(256), 0, st, A, nd, lda, mu);
    for (int64_t k0 = 0; k0 < n; k0 += NB) {
        const int kb = (int)((n - k0) < NB ? (n - k0) : NB);
        const int kf = (border && k0 + kb == n) ? kb - 1 : kb;
        hipLaunchKernelGGL(potrf_block_kernel, dim3(1), dim3(64), 0, st, A, lda, k0, kb, kf, linv, status);
        const int64_t rest = n - k0 - kb;
        if (rest <= 0) break;
        double *a21 = A + (k0 + kb) * lda + k0;
        GemmDesc t{};
        t.M = rest; t.N = kb; t.K = kb;
        t.A = a21; t.lda = lda; t.la = 0;
        t.B = linv + (k0 / NB) * NB * NB; t.ldb = NB; t.lb = 1;
        t.C = a21; t.ldc = lda;
        t.alpha = 1.0; t.beta = 0.0;
        t.stop_flag = &status->flag;
        hipError_t e = launch_dgemm(st, t);
        if (e != hipSuccess) return e;
        GemmDesc s{};
        s.M = rest; s.N = rest; s.K = kb;
        s.A = a21; s.lda = lda; s.la = 0;
        s.B = a21; s.ldb = lda; s.lb = 1;
        s.C = A + (k0 + kb) * lda + (k0 + kb); s.ldc = lda;
        s.alpha = -1.0; s.beta = 1.0;
        s.lower = 1;
        s.stop_flag = &status->flag;
        e = launch_dgemm(st, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

// ------------------------------------------------------- triangular solves
static constexpr int SOLVE_ROWS = 64;  // rows per workgroup in the forward update

__global__ __launch_bounds__(256) void fwd_step_kernel(const double *__restrict__ L, int64_t n, int64_t ldl,
                                                       const double *__restrict__ linv, double *b, double *z,
                                                       int64_t r0, int kb, const DevStatus *status) {
    if (status->flag) return;
    __shared__ double zi[NB];
    const int tid = threadIdx.x;
    const double *li = linv + (r0 / NB) * NB * NB;
    if (tid < NB) {
        double s = 0.0;
        if (tid < kb)
            for (int c = 0; c <= tid; ++c) s = fma(li[tid * NB + c], b[r0 + c], s);
        zi[tid] = s;
        if (blockIdx.x == 0 && tid < kb) z[r0 + tid] = s;
    }
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const int64_t base = r0 + kb + (int64_t)blockIdx.x * SOLVE_ROWS;
    for (int rr = wave; rr < SOLVE_ROWS; rr += 4) {
        const int64_t row = base + rr;
        if (row >= n) break;
        double v = (lane < kb) ? L[row * ldl + r0 + lane] * zi[lane] : 0.0;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) b[row] -= v;
    }
}

__global__ __launch_bounds__(256) void back_step_kernel(const double *__restrict__ L, int64_t ldl,
                                                        const double *__restrict__ linv, double *y, double *x,
                                                        int64_t r0, int kb, const DevStatus *status) {
    if (status->flag) return;
    __shared__ double xi[NB];
    const int tid = threadIdx.x;
    const double *li = linv + (r0 / NB) * NB * NB;
    if (tid < NB) {
        double s = 0.0;
        if (tid < kb)
            for (int c = tid; c < kb; ++c) s = fma(li[c * NB + tid], y[r0 + c], s);
        xi[tid] = s;
        if (blockIdx.x == 0 && tid < kb) x[r0 + tid] = s;
    }
    __syncthreads();
    const int64_t c = (int64_t)blockIdx.x * 256 + tid;
    if (c >= r0) return;
    double acc = 0.0;
    for (int i = 0; i < kb; ++i) acc = fma(L[(r0 + i) * ldl + c], xi[i], acc);
    y[c] -= acc;
}

hipError_t launch_solve_lower(hipStream_t st, const double *L, int64_t n, int64_t ldl, const double *linv,
                              double *b, double *z, DevStatus *status) {
    for (int64_t r0 = 0; r0 < n; r0 += NB) {
        const int kb = (int)((n - r0) < NB ? (n - r0) : NB);
        const int64_t rest = n - r0 - kb;
        const int64_t blocks = rest > 0 ? (rest + SOLVE_ROWS - 1) / SOLVE_ROWS : 1;
        hipLaunchKernelGGL(fwd_step_kernel, dim3((unsigned)blocks), dim3(256), 0, st, L, n, ldl, linv, b, z, r0, kb,
                           status);
    }
    return hipGetLastError();
}

hipError_t launch_solve_upper(hipStream_t st, const double *L, int64_t n, int64_t ldl, const double *linv,
                              double *y, double *x, DevStatus *status) {
    if (n <= 0) return hipSuccess;
    const int64_t nblk = (n + NB - 1) / NB;
    for (int64_t bI = nblk - 1; bI >= 0; --bI) {
        const int64_t r0 = bI * NB;
        const int kb = (int)((n - r0) < NB ? (n - r0) : NB);
        const int64_t blocks = r0 > 0 ? (r0 + 255) / 256 : 1;
        hipLaunchKernelGGL(back_step_kernel, dim3((unsigned)blocks), dim3(256), 0, st, L, ldl, linv, y, x, r0, kb,
                           status);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ small kernels
static constexpr int RED_BLOCKS = 256;

// Deterministic sum of squares: fixed per-block strided order, fixed tree.
__global__ __launch_bounds__(256) void sumsq_partial(const double *__restrict__ x, int64_t n, int64_t stride,
                                                     double *__restrict__ work) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)RED_BLOCKS * 256) {
        const double v = x[i * stride];
        acc = fma(v, v, acc);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) work[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void sum_final(const double *__restrict__ work, int count, double scale,
                                                 double *out) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < count; i += 256) acc += work[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = scale * sh[0];
}

hipError_t launch_sumsq(hipStream_t st, const double *x, int64_t n, int64_t stride, double *out, double *work) {
    hipLaunchKernelGGL(sumsq_partial, dim3(RED_BLOCKS), dim3(256), 0, st, x, n, stride, work);
    hipLaunchKernelGGL(sum_final, dim3(1), dim3(256), 0, st, work, RED_BLOCKS, 1.0, out);
    return hipGetLastError();
}

__global__ void check_finite_kernel(const double *__restrict__ x, int64_t n, DevStatus *status) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = x[i];
    if (!(v - v == 0.0)) atomicOr(&status->nonfinite, 1);
}

hipError_t launch_check_finite(hipStream_t st, const double *x, int64_t n, DevStatus *status) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n, status);
    return hipGetLastError();
}

// theta += delta when the residual is finite, the factorisation succeeded
// and delta is finite.
__global__ void apply_update_kernel(double *theta, const double *__restrict__ delta, int64_t p, DevStatus *status) {
    const double h = status->half_sq_norm;
    if (!(h - h == 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) status->nonfinite = 1;
        return;
    }
    if (status->flag || status->nonfinite) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < p) theta[i] += delta[i];
    if (i == 0) status->updated = 1;
}

hipError_t launch_finalize_step(hipStream_t st, double *theta, const double *delta, const double *, int64_t p,
                                int apply, DevStatus *status) {
    hipError_t e = launch_check_finite(st, delta, p, status);
    if (e != hipSuccess || !apply) return e;
    hipLaunchKernelGGL(apply_update_kernel, dim3((unsigned)((p + 255) / 256)), dim3(256), 0, st, theta, delta, p,
                       status);
    return hipGetLastError();
}

// out[c] (+)= sum_k partial[k][c] in order k = 0..count-1.
__global__ void reduce_partials_kernel(const double *__restrict__ partial, int64_t count, int64_t p,
                                       double *__restrict__ out, int accumulate) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= p) return;
    double acc = 0.0;
    for (int64_t k = 0; k < count; ++k) acc += partial[k * p + c];
    out[c] = accumulate ? out[c] + acc : acc;
}

hipError_t launch_reduce_partials(hipStream_t st, const double *partial, int64_t count, int64_t p, double *out,
                                  int accumulate) {
    if (p <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((p + 255) / 256)), dim3(256), 0, st, partial, count,
                       p, out, accumulate);
    return hipGetLastError();
}

__global__ void copy_strided_kernel(const double *__restrict__ src, int64_t n, int64_t ss, double *__restrict__ dst,
                                    int64_t ds, double scale) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i * ds] = scale * src[i * ss];
}

hipError_t launch_copy_strided(hipStream_t st, const double *src, int64_t n, int64_t src_stride, double *dst,
                               int64_t dst_stride, double scale) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_strided_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, n, src_stride,
                       dst, dst_stride, scale);
    return hipGetLastError();
}

__global__ void reset_status_kernel(DevStatus *s) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        s->max_R = 0;
        s->max_R_val = 0;
        s->chol_info = 0;
        s->flag = 0;
        s->nonfinite = 0;
        s->updated = 0;
        s->pad = 0;
        s->half_sq_norm = 0.0;
        s->grad_dot_delta = 0.0;
        s->model_sq_norm = 0.0;
    }
}

// Clears the step status with a kernel (no memset node, so the sequence can
// be captured in a graph and replayed).
hipError_t launch_reset_status(hipStream_t st, DevStatus *s) {
    hipLaunchKernelGGL(reset_status_kernel, dim3(1), dim3(64), 0, st, s);
    return hipGetLastError();
}

__global__ void mul_kernel(const double *__restrict__ a, const double *__restrict__ b, double *__restrict__ out,
                           int64_t n, double scale) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = scale * a[i] * b[i];
}

hipError_t launch_mul(hipStream_t st, const double *a, const double *b, double *out, int64_t n, double scale) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(mul_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, out, n, scale);
    return hipGetLastError();
}

}  // namespace gn
