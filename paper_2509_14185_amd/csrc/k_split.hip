// Split-precision Gram for gfx950: G = J^T J (lower) from FP32 hi/lo parts
// of the FP64 Jacobian, hi = fl32(x), lo = fl32(x - hi):
//   G ~= Jhi^T Jhi + Jhi^T Jlo + Jlo^T Jhi
// with v_mfma_f32_16x16x4f32.  The three products of one 32-row chunk are
// accumulated in FP32 and added into FP64 accumulators after every chunk, so
// FP32 accumulation never spans more than 32 rows.  The dropped term
// Jlo^T Jlo is below 2^-48 relative; the error is dominated by FP32 rounding
// of the products (about 1e-7 relative to |J|^T |J|).
//
// Tiling as in the FP64 GEMM: 512 threads (8 waves, 2 x 4), 128 x 128
// output tiles of the lower triangle in 4 x 8 super-tiles per XCD, K in
// chunks of 32 through double-buffered LDS ([k][m] layout; the four FP32
// tiles of a chunk take the same 128 KB as two FP64 tiles).
//
// Fragment layout of v_mfma_f32_16x16x4f32 (wave64):
//   A (16x4): lane l holds A[l%16][l/16];  B (4x16): lane l holds B[l/16][l%16]
//   D (16x16): lane l, register r holds D[4*(l/16) + r][l%16]
#include "gn_internal.h"

namespace gn {

typedef float float4_t __attribute__((ext_vector_type(4)));

static constexpr int ST = 512;  // threads
static constexpr int SBM = 128, SBK = 32;
static constexpr int S_SUP_M = 4, S_SUP_N = 8, S_SUP = 32, S_NXCD = 8;

__global__ void split_kernel(const double *__restrict__ J, int64_t m, int64_t p, int64_t ldj, float *__restrict__ hi,
                             float *__restrict__ lo) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = blockIdx.y;
    if (c >= p || i >= m) return;
    const double x = J[i * ldj + c];
    const float h = (float)x;
    hi[i * ldj + c] = h;
    lo[i * ldj + c] = (float)(x - (double)h);
}

hipError_t launch_split(hipStream_t st, const double *J, int64_t m, int64_t p, int64_t ldj, float *hi, float *lo) {
    if (m <= 0 || p <= 0) return hipSuccess;
    dim3 grid((unsigned)((p + 255) / 256), (unsigned)m);
    hipLaunchKernelGGL(split_kernel, grid, dim3(256), 0, st, J, m, p, ldj, hi, lo);
    return hipGetLastError();
}

__device__ __forceinline__ bool split_tile_of_block(int64_t b, int tiles, int &tm, int &tn) {
    const int64_t x = b % S_NXCD, pos = b / S_NXCD;
    const int64_t sidx = (pos / S_SUP) * S_NXCD + x;
    const int i = (int)(pos % S_SUP);
    const int64_t nsr = (tiles + S_SUP_M - 1) / S_SUP_M, nsc = (tiles + S_SUP_N - 1) / S_SUP_N;
    int64_t rem = sidx, a = 0;
    for (; a < nsr; ++a) {
        int64_t c = (S_SUP_M * a + S_SUP_M - 1) / S_SUP_N + 1;
        if (c > nsc) c = nsc;
        if (rem < c) break;
        rem -= c;
    }
    if (a >= nsr) return false;
    tm = (int)(a * S_SUP_M + i % S_SUP_M);
    tn = (int)(rem * S_SUP_N + i / S_SUP_M);
    return tm < tiles && tn < tiles && tn <= tm;
}

static int64_t split_super_count(int64_t tiles) {
    const int64_t nsr = (tiles + S_SUP_M - 1) / S_SUP_M, nsc = (tiles + S_SUP_N - 1) / S_SUP_N;
    int64_t n = 0;
    for (int64_t a = 0; a < nsr; ++a) {
        int64_t c = (S_SUP_M * a + S_SUP_M - 1) / S_SUP_N + 1;
        n += c < nsc ? c : nsc;
    }
    return n;
}

// C (lower, p x p, FP64) = Ahi^T Ahi + Ahi^T Alo + Alo^T Ahi, A m x p row-major (ld lda, floats).
__global__ __launch_bounds__(ST) void split_gram_kernel(const float *__restrict__ Ahi, const float *__restrict__ Alo,
                                                        int64_t m, int64_t p, int64_t lda, double *__restrict__ C,
                                                        int64_t ldc, int tiles, int accumulate) {
    constexpr int WAVES_N = 4, WM = SBM / 2, WN = SBM / 4;
    constexpr int FM = WM / 16, FN = WN / 16;
    extern __shared__ float fs[];
    // [buf][operand: 0 hi, 1 lo][k][m]
    auto lds = [&](int buf, int op) { return fs + ((buf * 2 + op) * SBK) * SBM; };

    int tm, tn;
    if (!split_tile_of_block(blockIdx.x, tiles, tm, tn)) return;
    const int64_t m0 = (int64_t)tm * SBM, n0 = (int64_t)tn * SBM;
    const bool diag = tm == tn;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WAVES_N, wn = wave % WAVES_N;
    const int fr = lane & 15, fk = lane >> 4;

    double acc[FM][FN][4];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;

    // operand tiles: rows k0..k0+31 of columns m0..m0+127 (A side) and n0.. (B side);
    // 128 x 32 floats = 1024 float4 per tile, 2 per thread
    float4 ra[2][2], rb[2][2];  // [op][e]
    const bool cols_in_a = m0 + SBM <= p, cols_in_b = n0 + SBM <= p;
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int idx = tid + e * ST;
            const int c4 = 4 * (idx % (SBM / 4)), kk = idx / (SBM / 4);
            const int64_t gk = k0 + kk;
#pragma unroll
            for (int op = 0; op < 2; ++op) {
                const float *src = op ? Alo : Ahi;
                float4 va = make_float4(0.f, 0.f, 0.f, 0.f), vb = va;
                if (gk < m) {
                    if (cols_in_a) {
                        va = *reinterpret_cast<const float4 *>(src + gk * lda + m0 + c4);
                    } else {
                        float t[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) t[q] = (m0 + c4 + q < p) ? src[gk * lda + m0 + c4 + q] : 0.f;
                        va = make_float4(t[0], t[1], t[2], t[3]);
                    }
                    if (!diag) {
                        if (cols_in_b) {
                            vb = *reinterpret_cast<const float4 *>(src + gk * lda + n0 + c4);
                        } else {
                            float t[4];
#pragma unroll
                            for (int q = 0; q < 4; ++q) t[q] = (n0 + c4 + q < p) ? src[gk * lda + n0 + c4 + q] : 0.f;
                            vb = make_float4(t[0], t[1], t[2], t[3]);
                        }
                    }
                }
                ra[op][e] = va;
                rb[op][e] = vb;
            }
        }
    };
    // LDS: A tiles at ops 0/1; B tiles follow at 2*2*SBK*SBM floats (unused when diag: B reads A)
    float *bbase = fs + 2 * 2 * SBK * SBM;
    auto ldsb = [&](int buf, int op) { return diag ? lds(buf, op) : bbase + ((buf * 2 + op) * SBK) * SBM; };
    auto store = [&](int buf) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int idx = tid + e * ST;
            const int c4 = 4 * (idx % (SBM / 4)), kk = idx / (SBM / 4);
#pragma unroll
            for (int op = 0; op < 2; ++op) {
                *reinterpret_cast<float4 *>(lds(buf, op) + kk * SBM + c4) = ra[op][e];
                if (!diag) *reinterpret_cast<float4 *>(ldsb(buf, op) + kk * SBM + c4) = rb[op][e];
            }
        }
    };

    const int64_t nk = (m + SBK - 1) / SBK;
    if (nk > 0) {
        load(0);
        store(0);
        __syncthreads();
    }
    for (int64_t kt = 0; kt < nk; ++kt) {
        const int cur = (int)(kt & 1);
        if (kt + 1 < nk) load((kt + 1) * SBK);
        float4_t hh[FM][FN], xx[FM][FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                hh[i][j] = (float4_t){0.f, 0.f, 0.f, 0.f};
                xx[i][j] = (float4_t){0.f, 0.f, 0.f, 0.f};
            }
        const float *ah = lds(cur, 0) + wm * WM + fr, *al = lds(cur, 1) + wm * WM + fr;
        const float *bh = ldsb(cur, 0) + wn * WN + fr, *bl = ldsb(cur, 1) + wn * WN + fr;
#pragma unroll
        for (int ks = 0; ks < SBK; ks += 4) {
            float a_h[FM], a_l[FM], b_h[FN], b_l[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                a_h[i] = ah[(ks + fk) * SBM + i * 16];
                a_l[i] = al[(ks + fk) * SBM + i * 16];
            }
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                b_h[j] = bh[(ks + fk) * SBM + j * 16];
                b_l[j] = bl[(ks + fk) * SBM + j * 16];
            }
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    hh[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_h[i], b_h[j], hh[i][j], 0, 0, 0);
                    xx[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_h[i], b_l[j], xx[i][j], 0, 0, 0);
                    xx[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_l[i], b_h[j], xx[i][j], 0, 0, 0);
                }
        }
        // promote the chunk's FP32 sums into FP64
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[i][j][r] += (double)hh[i][j][r] + (double)xx[i][j][r];
        if (kt + 1 < nk) store(cur ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int64_t gn_ = n0 + wn * WN + j * 16 + fr;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gm = m0 + wm * WM + i * 16 + 4 * fk + r;
                if (gm < p && gn_ < p && gn_ <= gm)
                    C[gm * ldc + gn_] = accumulate ? C[gm * ldc + gn_] + acc[i][j][r] : acc[i][j][r];
            }
        }
}

hipError_t launch_split_gram(hipStream_t st, const float *hi, const float *lo, int64_t m, int64_t p, int64_t lda,
                             double *C, int64_t ldc, int accumulate) {
    if (p <= 0) return hipSuccess;
    const int tiles = (int)((p + SBM - 1) / SBM);
    const int64_t supers = split_super_count(tiles);
    const int64_t blocks = (supers + S_NXCD - 1) / S_NXCD * S_NXCD * S_SUP;
    const size_t shm = sizeof(float) * 2 * 2 * 2 * SBK * SBM;  // [A,B] x [buf] x [hi,lo]
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)split_gram_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)shm);
        attr = true;
    }
    hipLaunchKernelGGL(split_gram_kernel, dim3((unsigned)blocks), dim3(ST), shm, st, hi, lo, m, p, lda, C, ldc, tiles,
                       accumulate);
    return hipGetLastError();
}

}  // namespace gn
