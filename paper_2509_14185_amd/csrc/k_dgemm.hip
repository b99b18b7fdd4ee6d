// FP64 MFMA GEMM for gfx950 (v_mfma_f64_16x16x4_f64): the dense
// contractions of the damped Gauss-Newton step.
//   - Gram G = J^T J (lower triangle), the SYRK whose cost dominates the step
//     (paper, Methods, "Second-order Optimizer": full Gauss-Newton matrix).
//   - Hilbert coupling J[:N] += diag(sc Theta_y) Q B.
//   - Trailing update and triangular-inverse products of the blocked Cholesky.
//
// C[m][n] = beta C[m][n] + alpha * rowscale[m] * sum_k A(m,k) B(k,n)
//
// Tiling: a 256-thread workgroup (4 waves, 2 x 2) owns a BM x BN tile of C;
// each wave owns (BM/2) x (BN/2) as 16x16 MFMA blocks held in registers.
// K is consumed in chunks of BK staged through double-buffered LDS in a
// k-major layout ([k][m], [k][n]) so that an MFMA fragment (16 consecutive m
// or n for each of 4 k) is one contiguous LDS row segment.  Global loads for
// chunk c+1 are issued before the MFMAs of chunk c.  Both operand layouts
// (contiguous in m/n or contiguous in k) are read with unit-stride runs.
//
// Fragment layout of v_mfma_f64_16x16x4_f64 (wave64):
//   A (16x4):  lane l holds A[l%16][l/16]
//   B (4x16):  lane l holds B[l/16][l%16]
//   D (16x16): lane l, register r holds D[l/16 + 4*r][l%16]  (f64: one row per
//              register group, unlike the 4-row groups of the f32 variant)
#include "gn_internal.h"

namespace gn {

typedef double double4_t __attribute__((ext_vector_type(4)));

static constexpr int GEMM_THREADS = 256;

template <int BM, int BN, int BK, int LA, int LB>
__global__ __launch_bounds__(GEMM_THREADS) void dgemm_mfma_kernel(GemmDesc g, int tiles_m, int tiles_n) {
    if (g.stop_flag != nullptr && *g.stop_flag != 0) return;
    constexpr int WM = BM / 2, WN = BN / 2;
    constexpr int FM = WM / 16, FN = WN / 16;
    constexpr int A_PER = BM * BK / GEMM_THREADS;
    constexpr int B_PER = BN * BK / GEMM_THREADS;
    static_assert(A_PER * GEMM_THREADS == BM * BK, "A tile split");
    static_assert(B_PER * GEMM_THREADS == BN * BK, "B tile split");

    __shared__ double As[2][BK][BM];
    __shared__ double Bs[2][BK][BN];

    // tile coordinates (lower: enumerate tiles with tn <= tm, BM == BN)
    int tm, tn;
    if (g.lower) {
        const int64_t bid = blockIdx.x;
        int r = (int)((sqrt(8.0 * (double)bid + 1.0) - 1.0) * 0.5);
        while ((int64_t)(r + 1) * (r + 2) / 2 <= bid) ++r;
        while ((int64_t)r * (r + 1) / 2 > bid) --r;
        tm = r;
        tn = (int)(bid - (int64_t)r * (r + 1) / 2);
    } else {
        tm = blockIdx.x % tiles_m;
        tn = blockIdx.x / tiles_m;
    }
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    double4_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = (double4_t){0.0, 0.0, 0.0, 0.0};

    double ra[A_PER], rb[B_PER];

    auto load_chunk = [&](int64_t k0) {
#pragma unroll
        for (int e = 0; e < A_PER; ++e) {
            const int idx = tid + e * GEMM_THREADS;
            int mm, kk;
            if (LA == 1) { mm = idx % BM; kk = idx / BM; }   // contiguous in m
            else         { kk = idx % BK; mm = idx / BK; }   // contiguous in k
            const int64_t gm = m0 + mm, gk = k0 + kk;
            double v = 0.0;
            if (gm < g.M && gk < g.K) v = (LA == 1) ? g.A[gk * g.lda + gm] : g.A[gm * g.lda + gk];
            ra[e] = v;
        }
#pragma unroll
        for (int e = 0; e < B_PER; ++e) {
            const int idx = tid + e * GEMM_THREADS;
            int nn, kk;
            if (LB == 0) { nn = idx % BN; kk = idx / BN; }   // contiguous in n
            else         { kk = idx % BK; nn = idx / BK; }   // contiguous in k
            const int64_t gn_ = n0 + nn, gk = k0 + kk;
            double v = 0.0;
            if (gn_ < g.N && gk < g.K) v = (LB == 0) ? g.B[gk * g.ldb + gn_] : g.B[gn_ * g.ldb + gk];
            rb[e] = v;
        }
    };
    auto store_chunk = [&](int buf) {
#pragma unroll
        for (int e = 0; e < A_PER; ++e) {
            const int idx = tid + e * GEMM_THREADS;
            int mm, kk;
            if (LA == 1) { mm = idx % BM; kk = idx / BM; }
            else         { kk = idx % BK; mm = idx / BK; }
            As[buf][kk][mm] = ra[e];
        }
#pragma unroll
        for (int e = 0; e < B_PER; ++e) {
            const int idx = tid + e * GEMM_THREADS;
            int nn, kk;
            if (LB == 0) { nn = idx % BN; kk = idx / BN; }
            else         { kk = idx % BK; nn = idx / BK; }
            Bs[buf][kk][nn] = rb[e];
        }
    };

    const int64_t nk = (g.K + BK - 1) / BK;
    if (nk > 0) {
        load_chunk(0);
        store_chunk(0);
        __syncthreads();
    }
    const int fr = lane & 15, fk = lane >> 4;
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        if (kt + 1 < nk) load_chunk((kt + 1) * BK);
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
            double a[FM], b[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) a[i] = As[cur][ks + fk][wm * WM + i * 16 + fr];
#pragma unroll
            for (int j = 0; j < FN; ++j) b[j] = Bs[cur][ks + fk][wn * WN + j * 16 + fr];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (kt + 1 < nk) store_chunk(cur ^ 1);
        __syncthreads();
    }

    // epilogue
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int64_t gn_ = n0 + wn * WN + j * 16 + fr;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gm = m0 + wm * WM + i * 16 + fk + 4 * r;
                if (gm >= g.M || gn_ >= g.N) continue;
                if (g.lower && gn_ > gm) continue;
                double v = g.alpha * acc[i][j][r];
                if (g.rowscale) v *= g.rowscale[gm];
                double *c = g.C + gm * g.ldc + gn_;
                *c = (g.beta == 0.0) ? v : fma(g.beta, *c, v);
            }
        }
    }
}

template <int BM, int BN, int BK>
static hipError_t launch_tiles(hipStream_t st, const GemmDesc &g) {
    const int tiles_m = (int)((g.M + BM - 1) / BM);
    const int tiles_n = (int)((g.N + BN - 1) / BN);
    int64_t blocks;
    if (g.lower) {
        blocks = (int64_t)tiles_m * (tiles_m + 1) / 2;  // requires M == N and BM == BN
    } else {
        blocks = (int64_t)tiles_m * tiles_n;
    }
    if (blocks <= 0) return hipSuccess;
    dim3 grid((unsigned)blocks), block(GEMM_THREADS);
    if (g.la == 0 && g.lb == 0)
        hipLaunchKernelGGL((dgemm_mfma_kernel<BM, BN, BK, 0, 0>), grid, block, 0, st, g, tiles_m, tiles_n);
    else if (g.la == 0 && g.lb == 1)
        hipLaunchKernelGGL((dgemm_mfma_kernel<BM, BN, BK, 0, 1>), grid, block, 0, st, g, tiles_m, tiles_n);
    else if (g.la == 1 && g.lb == 0)
        hipLaunchKernelGGL((dgemm_mfma_kernel<BM, BN, BK, 1, 0>), grid, block, 0, st, g, tiles_m, tiles_n);
    else
        hipLaunchKernelGGL((dgemm_mfma_kernel<BM, BN, BK, 1, 1>), grid, block, 0, st, g, tiles_m, tiles_n);
    return hipGetLastError();
}

hipError_t launch_dgemm(hipStream_t st, const GemmDesc &g) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    if (g.lower && g.M != g.N) return hipErrorInvalidValue;
    if (!g.lower && g.N <= 64) return launch_tiles<128, 64, 16>(st, g);  // BN must equal BM when lower
    return launch_tiles<128, 128, 16>(st, g);
}

// ---------------------------------------------------------------- g = J^T r
// Pass 1: row chunks x column blocks; each thread owns one column and sums
// its chunk of rows in order.  Pass 2: fixed-order sum over chunks.
static constexpr int GEMV_CHUNKS = 64;

int64_t gemv_t_work_size(int64_t, int64_t p) { return (int64_t)GEMV_CHUNKS * p; }

__global__ void gemv_t_partial(const double *__restrict__ J, int64_t m, int64_t p, int64_t ldj,
                               const double *__restrict__ r, double *__restrict__ work) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= p) return;
    const int64_t per = (m + GEMV_CHUNKS - 1) / GEMV_CHUNKS;
    const int64_t i0 = blockIdx.y * per;
    const int64_t i1 = (i0 + per < m) ? i0 + per : m;
    double acc = 0.0;
    for (int64_t i = i0; i < i1; ++i) acc = fma(J[i * ldj + c], r[i], acc);
    work[blockIdx.y * p + c] = acc;
}

__global__ void gemv_t_final(const double *__restrict__ work, int64_t p, double *__restrict__ g) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= p) return;
    double acc = 0.0;
    for (int k = 0; k < GEMV_CHUNKS; ++k) acc += work[k * p + c];
    g[c] = acc;
}

hipError_t launch_gemv_t(hipStream_t st, const double *J, int64_t m, int64_t p, int64_t ldj, const double *r,
                         double *g, double *work) {
    if (p <= 0) return hipSuccess;
    dim3 g1((unsigned)((p + 255) / 256), GEMV_CHUNKS);
    hipLaunchKernelGGL(gemv_t_partial, g1, dim3(256), 0, st, J, m, p, ldj, r, work);
    hipLaunchKernelGGL(gemv_t_final, dim3((unsigned)((p + 255) / 256)), dim3(256), 0, st, work, p, g);
    return hipGetLastError();
}

}  // namespace gn
