// Damped solve of the Gauss-Newton system on gfx950 (paper, Methods,
// "Second-order Optimizer": theta <- theta - (G + gamma I)^{-1} grad h).
//
// Right-looking blocked Cholesky, two levels (128-wide diagonal blocks inside
// 512-wide outer panels) with look-ahead:
//   1. diagonal block: one workgroup factors it in LDS (one-wave 32x32
//      register factorisations, the rest by all four waves) and forms the
//      inverse of its triangular factor;
//   2. panel below: L21 = A21 L11^{-T} as an MFMA GEMM with the inverse;
//   3. the remaining columns of the outer panel are updated (K = 128);
//   4. after an outer panel, the trailing matrix is updated with K = 512
//      (lower), split into the next outer panel's columns (main stream) and
//      the rest (a second stream, in two launches of K = 256), so the next
//      panel is factored while the bulk of the update runs.  A large K keeps
//      the update's C tiles (read and written once per launch) from
//      dominating its HBM traffic.
// A failed pivot records its 1-based global index and raises a device flag;
// every later kernel of the factorisation and solve sees the flag and exits.
//
// Border row: when the system is [[G, g], [g^T, r^T r]] (the gradient stored
// as an extra last row), the last row's diagonal is not square-rooted; it
// ends as the Schur complement r^T r - g^T (G + mu I)^{-1} g and the rest of
// that row as w = L^{-1} g, so the forward substitution comes for free.
//
// Triangular solves use the stored diagonal-block inverses: one launch per
// 128-row block applies the known block to the rest of the right-hand side,
// one workgroup per remaining block, and the workgroup of the next block
// then forms that block's unknowns.
#include <vector>

#include "gn_internal.h"

namespace gn {

static constexpr int CB = 128;         // diagonal block width of the blocked Cholesky
static constexpr int NB = 4 * CB;      // outer panel width (K of the trailing update)
static constexpr int LDS_LD = CB + 1;  // padded LDS row stride (doubles)

int64_t chol_linv_size(int64_t n) { return ((n + CB - 1) / CB) * CB * CB; }
int64_t chol_tmp_size() { return 64 * 64; }

__global__ void add_diag_kernel(double *A, int64_t n, int64_t lda, double mu) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) A[i * lda + i] += mu;
}

// ---- diagonal-block factorisation -------------------------------------
// The CB x CB block lives in LDS: L in the lower triangle (s[i*LDS_LD + c],
// c <= i) and X = L^{-1} stored transposed in the strict upper triangle plus
// the padding column (X(i,c) at s[c*LDS_LD + i + 1], i >= c), so both fit in
// one 128 x 129 tile.  Rows >= kb are identity padding.  Work is blocked by
// IB = 32: a one-wave register factorisation of each 32x32 diagonal block
// (inlined: the leaf loop is not unrolled, so the kernel holds one copy),
// then loops over the panel and trailing part with all 256 threads.
static constexpr int IB = 32;
#define LL(i, c) s[(i) * LDS_LD + (c)]
#define XX(i, c) s[(c) * LDS_LD + (i) + 1]

// 1/sqrt(d) for d > 0: hardware estimate refined by two Newton steps
// (y <- y (3 - d y^2) / 2), accurate to a few ulp; a short dependent chain
// where the IEEE sqrt plus division would take about thirty operations.
__device__ __forceinline__ double rsqrt_refined(double d) {
    double y = __builtin_amdgcn_rsq(d);
    double h = 0.5 * d;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}

__device__ __forceinline__ double readlane_d(double x, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}

typedef double double4_t __attribute__((ext_vector_type(4)));

// One 16x16 tile of an in-LDS product, acc += A(16 x KN) B(KN x 16) over
// k in [kbeg, kbeg + KN) (KN a multiple of 4, fully unrolled so that the
// fragment loads run ahead of the MFMAs), fragments read through accessors
// a_at(m, k), b_at(k, n) (unconditional LDS loads; masks are selects).
// FP64 MFMA layout: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// register r of the result is row l/16 + 4r, column l%16.
template <int KN, class FA, class FB>
__device__ __forceinline__ double4_t lds_mfma(double4_t acc, FA a_at, FB b_at, int kbeg) {
    const int lane = threadIdx.x & 63, fr = lane & 15, fk = lane >> 4;
    double a[KN / 4], b[KN / 4];
#pragma unroll
    for (int q = 0; q < KN / 4; ++q) {
        a[q] = a_at(fr, kbeg + 4 * q + fk);
        b[q] = b_at(kbeg + 4 * q + fk, fr);
    }
#pragma unroll
    for (int q = 0; q < KN / 4; ++q) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b[q], acc, 0, 0, 0);
    return acc;
}

__device__ __forceinline__ double sel(bool keep, double v) { return keep ? v : 0.0; }

// One wave, lanes 0..31: lane i holds row o+i of the 32x32 diagonal block in
// registers.  Columns are taken KS at a time: every lane reads the KS x KS
// diagonal block from its lanes (readlane, uniform values) and factors it
// redundantly (KS dependent reciprocal square roots), forms its own KS
// entries by a forward substitution with that factor, stores them to an LDS
// column buffer (two buffers by parity of the step) and reads the entries of
// the rows below back as broadcasts for its rank-KS update.  One LDS round
// trip per KS columns instead of one per column, and no branches: a failed
// pivot is recorded and the step carries on with NaNs.  Entries right of the
// diagonal are never read, so they are updated without masking.  Row bi
// (local, or -1) is a border row: its diagonal is not square-rooted (its
// reciprocal is taken as zero, so the column below it stays zero, as the rows
// below are identity padding) and it is excluded from X.
// Then X_oo = L_oo^{-1}: the two 16x16 diagonal blocks are inverted at once
// (lane c owns column c, rows of L read as LDS broadcasts; a 16-step chain
// instead of 32) and the off-diagonal block follows from two MFMA products,
// X21 = -X22 (L21 X11), with t (16 x 17 doubles of LDS) holding L21 X11.
// Returns -1 or the failing local pivot (uniform).
static constexpr int KS = 4;
__device__ __forceinline__ int potrf32_wave(double *s, int o, int bi, double *cb, double *t) {
    const int lane = threadIdx.x & 63;
    const bool act = lane < IB;
    // lanes 32..63 repeat lanes 0..31 (same row, same arithmetic), so loads and
    // stores need no exec mask
    const int ln = lane & (IB - 1);
    double row[IB];
#pragma unroll
    for (int c = 0; c < IB; ++c) {
        const double v = LL(o + ln, o + c);
        row[c] = c <= ln ? v : 0.0;
    }
    // rl[i]: 1 / l_ii of this lane's group of the inverse below (row g0 + i)
    constexpr int H = IB / 2;
    const int g0 = (lane & H);  // 0 or 16
    double rl[H];
#pragma unroll
    for (int i = 0; i < H; ++i) rl[i] = 0.0;
    int fail = -1;
#pragma unroll
    for (int j = 0; j < IB; j += KS) {
        // KS x KS diagonal block (lower part), uniform
        double a[KS][KS];
#pragma unroll
        for (int p = 0; p < KS; ++p)
#pragma unroll
            for (int q = 0; q <= p; ++q) a[p][q] = readlane_d(row[j + q], j + p);
        // its factor: ld[p][q] (q < p), rr[q] = 1 / sqrt of the q-th pivot
        double ld[KS][KS], rr[KS];
#pragma unroll
        for (int q = 0; q < KS; ++q) {
            double v = a[q][q];
#pragma unroll
            for (int k = 0; k < q; ++k) v = fma(-ld[q][k], ld[q][k], v);
            const bool border = (j + q == bi);
            fail = (fail < 0 && !border && !(v > 0.0)) ? j + q : fail;
            const double y = rsqrt_refined(border ? 1.0 : v);  // selects, not a branch
            rr[q] = border ? 0.0 : y;
#pragma unroll
            for (int p = q + 1; p < KS; ++p) {
                double w = a[p][q];
#pragma unroll
                for (int k = 0; k < q; ++k) w = fma(-ld[p][k], ld[q][k], w);
                ld[p][q] = w * rr[q];
            }
            if (g0 == ((j + q) & H)) rl[(j + q) & (H - 1)] = rr[q];
        }
        // this lane's entries of the KS columns (on lane j+q the substitution
        // repeats the factor's arithmetic, so v = d[q] there; the border row
        // keeps d[q] on its diagonal)
        double l[KS];
#pragma unroll
        for (int q = 0; q < KS; ++q) {
            double v = row[j + q];
#pragma unroll
            for (int k = 0; k < q; ++k) v = fma(-l[k], ld[q][k], v);
            l[q] = (j + q == bi && ln == bi) ? v : v * rr[q];
        }
        if (j + KS < IB) {
            // all 64 lanes store (lanes >= IB to their own slots), so no exec mask
            double *col = cb + ((j / KS) & 1) * KS * 64;
#pragma unroll
            for (int q = 0; q < KS; ++q) col[q * 64 + lane] = l[q];
            // row[c] -= sum_q l[q] l_c[q] for c >= j + KS, two columns c per LDS
            // read, in chunks of CH columns (the reads of a chunk in flight together)
            constexpr int CH = 8;
#pragma unroll
            for (int c0 = j + KS; c0 < IB; c0 += CH) {
                double2 w[CH / 2][KS];
#pragma unroll
                for (int cc = 0; cc < CH && c0 + cc < IB; cc += 2)
#pragma unroll
                    for (int q = 0; q < KS; ++q)
                        w[cc / 2][q] = *reinterpret_cast<const double2 *>(col + q * 64 + c0 + cc);
#pragma unroll
                for (int cc = 0; cc < CH && c0 + cc < IB; cc += 2)
#pragma unroll
                    for (int q = 0; q < KS; ++q) {
                        row[c0 + cc] = fma(-l[q], w[cc / 2][q].x, row[c0 + cc]);
                        row[c0 + cc + 1] = fma(-l[q], w[cc / 2][q].y, row[c0 + cc + 1]);
                    }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
#pragma unroll
        for (int q = 0; q < KS; ++q) row[j + q] = l[q];
    }
    if (fail >= 0) return fail;
    // the whole 32-wide row: right of the diagonal lies the storage of this
    // block's columns of X, written below
#pragma unroll
    for (int c = 0; c < IB; ++c) LL(o + ln, o + c) = row[c];
    // diagonal 16x16 blocks of X: lane c (group g = c / 16) forms column c of
    // X_gg, X[16g+i][c] = (delta - sum_{k<i} L[16g+i][16g+k] X[16g+k][c]) / L[16g+i][16g+i]
    const int cl = lane & (H - 1);
    double xc[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {
        if (i + g0 == bi) {
            xc[i] = 0.0;
        } else {
            double lr[H];
#pragma unroll
            for (int k = 0; k < i; ++k) lr[k] = LL(o + g0 + i, o + g0 + k);
            __builtin_amdgcn_sched_barrier(0);
            double a0 = (i == cl) ? 1.0 : 0.0, a1 = 0.0;
#pragma unroll
            for (int k = 0; k + 1 < i; k += 2) {
                a0 = fma(-lr[k], xc[k], a0);
                a1 = fma(-lr[k + 1], xc[k + 1], a1);
            }
            if (i & 1) a0 = fma(-lr[i - 1], xc[i - 1], a0);
            xc[i] = (a0 + a1) * rl[i];
        }
    }
    if (act && lane != bi) {
#pragma unroll
        for (int i = 0; i < H; ++i)
            if (i >= cl) XX(o + g0 + i, o + lane) = xc[i];
    }
    // X21 = -X22 (L21 X11)
    const int fr = lane & 15, fk = lane >> 4;
    double4_t acc = (double4_t){0.0, 0.0, 0.0, 0.0};
    acc = lds_mfma<H>(
        acc, [&](int m, int k) { return LL(o + H + m, o + k); },
        [&](int k, int n) { return sel(k >= n, XX(o + k, o + n)); }, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) t[(fk + 4 * r) * (H + 1) + fr] = acc[r];
    acc = (double4_t){0.0, 0.0, 0.0, 0.0};
    acc = lds_mfma<H>(
        acc, [&](int m, int k) { return sel(k <= m, XX(o + H + m, o + H + k)); },
        [&](int k, int n) { return t[k * (H + 1) + n]; }, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) XX(o + H + fk + 4 * r, o + fr) = -acc[r];
    return -1;
}

// Off-diagonal blocks X_rs of the inverse of the block's factor at distance
// D = r - s (in 32-blocks), from the blocks at smaller distances:
// W = sum_{k=s}^{r-1} L_rk X_ks, then X_rs = -X_rr W.  16x16 MFMA tiles
// spread over the four waves; W (three 32x33 buffers) holds the sums.
template <int D>
__device__ __forceinline__ void x_blocks_at_distance(double *s, double *W, int wave) {
    const int lane = threadIdx.x & 63, fr = lane & 15, fk = lane >> 4;
    constexpr int NBLK = CB / IB - D, NTILE = NBLK * 4;
    for (int t = wave; t < NTILE; t += 4) {
        const int q = t >> 2, ti = (t >> 1) & 1, tj = t & 1;
        const int ro = (q + D) * IB, so = q * IB;
        const int rm = ro + 16 * ti, cn = so + 16 * tj;
        double4_t acc = (double4_t){0.0, 0.0, 0.0, 0.0};
        acc = lds_mfma<IB * D>(
            acc, [&](int m, int k) { return LL(rm + m, k); },
            [&](int k, int n) { return sel(k >= cn + n, XX(k, cn + n)); }, so);
        double *Wq = W + q * IB * (IB + 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) Wq[(16 * ti + fk + 4 * r) * (IB + 1) + 16 * tj + fr] = acc[r];
    }
    __syncthreads();
    for (int t = wave; t < NTILE; t += 4) {
        const int q = t >> 2, ti = (t >> 1) & 1, tj = t & 1;
        const int ro = (q + D) * IB, so = q * IB;
        const double *Wq = W + q * IB * (IB + 1);
        double4_t acc = (double4_t){0.0, 0.0, 0.0, 0.0};
        acc = lds_mfma<IB>(
            acc, [&](int m, int k) { return sel(k <= 16 * ti + m, XX(ro + 16 * ti + m, ro + k)); },
            [&](int k, int n) { return Wq[k * (IB + 1) + 16 * tj + n]; }, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) XX(ro + 16 * ti + fk + 4 * r, so + 16 * tj + fr) = -acc[r];
    }
    __syncthreads();
}

// Factor one CB x CB diagonal block (rows/cols k0 .. k0+kb) of A and form X =
// L^{-1} of the block (row-major CB x CB, zero outside the factor and on the
// border row/column).  Right-looking over four 32-wide sub-blocks: a one-wave
// leaf factorisation, then the sub-panel solve and the trailing update as
// 16x16 FP64 MFMA tiles spread over the four waves; finally the off-diagonal
// blocks of X by distance, X_rs = -X_rr sum_{k=s}^{r-1} L_rk X_ks, as MFMA
// tiles as well.
__device__ __forceinline__ void potrf_block_body(double *A, int64_t lda, int64_t k0, int kb, int border_here, double *X,
                                                 DevStatus *status) {
    if (status->flag) return;
    extern __shared__ double s[];
    __shared__ int fail_sh;
    __shared__ __align__(16) double colbuf[2 * KS * 64];
    __shared__ double W[(CB / IB - 1) * IB * (IB + 1)];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: loops over tiles stay scalar
    const int fr = lane & 15, fk = lane >> 4;
    const int bi = border_here ? kb - 1 : -1;
    {
        // all 64 loads of a thread are issued before any LDS store: every lane
        // loads (indices clamped into the kb x kb block), selects afterwards,
        // so no load sits behind a branch and a wait for the one before it
        double v[CB * CB / 256];
#pragma unroll
        for (int e = 0; e < CB * CB / 256; ++e) {
            const int idx = tid + e * 256, r = idx / CB, c = idx % CB;
            const int rc = r < kb ? r : kb - 1, cc = c < kb ? c : kb - 1;
            v[e] = A[(k0 + rc) * lda + k0 + cc];
        }
#pragma unroll
        for (int e = 0; e < CB * CB / 256; ++e) {
            const int idx = tid + e * 256, r = idx / CB, c = idx % CB;
            v[e] = (r < kb && c <= r) ? v[e] : ((r >= kb && r == c) ? 1.0 : 0.0);
        }
#pragma unroll
        for (int e = 0; e < CB * CB / 256; ++e) {
            const int idx = tid + e * 256, r = idx / CB, c = idx % CB;
            s[r * LDS_LD + c] = v[e];
        }
        if (tid < CB) s[tid * LDS_LD + CB] = 0.0;
    }
    __syncthreads();
    // ---- blocked right-looking factorisation, inner blocks of IB
#pragma nounroll
    for (int sb = 0; sb < CB / IB; ++sb) {
        const int o = sb * IB;
        if (wave == 0) {
            const int lb = (bi >= o && bi < o + IB) ? bi - o : -1;
            const int f = potrf32_wave(s, o, lb, colbuf, W);
            if (lane == 0) fail_sh = f < 0 ? -1 : o + f;
        }
        __syncthreads();
        if (fail_sh >= 0) {
            if (tid == 0) {
                status->chol_info = k0 + fail_sh + 1;
                status->flag = 1;
            }
            return;
        }
        const int r0 = o + IB, nr = CB - r0;
        if (nr <= 0) break;
        // sub-panel: L[r][o+j] = sum_{k<=j} A[r][o+k] X[o+j][o+k]; (nr/16) x 2 tiles, at most 3 per wave
        {
            double4_t acc[3];
            const int ntile = (nr / 16) * 2;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                acc[q] = (double4_t){0.0, 0.0, 0.0, 0.0};
                const int t = wave + 4 * q;
                if (t < ntile) {
                    const int rm = r0 + 16 * (t >> 1), cn = o + 16 * (t & 1);
                    acc[q] = lds_mfma<IB>(
                        acc[q], [&](int m, int k) { return LL(rm + m, o + k); },
                        [&](int k, int n) { return sel(o + k <= cn + n, XX(cn + n, o + k)); }, 0);
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int t = wave + 4 * q;
                if (t < ntile) {
                    const int rm = r0 + 16 * (t >> 1), cn = o + 16 * (t & 1);
#pragma unroll
                    for (int r = 0; r < 4; ++r) LL(rm + fk + 4 * r, cn + fr) = acc[q][r];
                }
            }
        }
        __syncthreads();
        // trailing update (lower tiles): A[r][c] -= sum_k L[r][o+k] L[c][o+k]
        {
            const int nt = nr / 16, nlow = nt * (nt + 1) / 2;
            for (int t = wave; t < nlow; t += 4) {
                int ti = 0;
                while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
                const int tj = t - ti * (ti + 1) / 2;
                const int rm = r0 + 16 * ti, cn = r0 + 16 * tj;
                double4_t acc = (double4_t){0.0, 0.0, 0.0, 0.0};
                acc = lds_mfma<IB>(
                    acc, [&](int m, int k) { return LL(rm + m, o + k); },
                    [&](int k, int n) { return LL(cn + n, o + k); }, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = rm + fk + 4 * r, col = cn + fr;
                    if (col <= row) LL(row, col) -= acc[r];
                }
            }
        }
        __syncthreads();
    }
    // ---- off-diagonal blocks of X by distance d = r - s (all blocks of one
    //      distance together), 16x16 tiles:
    //      W = sum_{k=s}^{r-1} L_rk X_ks,  X_rs = -X_rr W
    x_blocks_at_distance<1>(s, W, wave);
    x_blocks_at_distance<2>(s, W, wave);
    x_blocks_at_distance<3>(s, W, wave);
    // ---- write L (rows < kb) and X (zero outside the factor) to global memory,
    //      16 elements a time: all LDS reads first, then the stores
    constexpr int SG = 16;
#pragma unroll 1
    for (int e0 = 0; e0 < CB * CB / 256; e0 += SG) {
        double lv[SG], xv[SG];
#pragma unroll
        for (int e = 0; e < SG; ++e) {
            const int idx = tid + (e0 + e) * 256, r = idx / CB, c = idx % CB;
            lv[e] = LL(r, c);
            xv[e] = XX(r, c);
        }
#pragma unroll
        for (int e = 0; e < SG; ++e) {
            const int idx = tid + (e0 + e) * 256, r = idx / CB, c = idx % CB;
            if (r < kb && c <= r) A[(k0 + r) * lda + k0 + c] = lv[e];
            const bool valid = c <= r && r < kb && r != bi && c != bi;
            X[idx] = valid ? xv[e] : 0.0;
        }
    }
}

__global__ __launch_bounds__(256) void potrf_block_kernel(double *A, int64_t lda, int64_t k0, int kb, int border_here,
                                                         double *X, double *, DevStatus *status) {
    potrf_block_body(A, lda, k0, kb, border_here, X, status);
}

// One diagonal block per instance of a batch (blockIdx.x = instance).
__global__ __launch_bounds__(256) void potrf_block_batched_kernel(const BatchChol *__restrict__ bc, int64_t k0, int kb,
                                                                 int border_here) {
    const BatchChol c = bc[blockIdx.x];
    potrf_block_body(c.A, c.lda, k0, kb, border_here, c.linv + (k0 / CB) * CB * CB, c.status);
}

#undef LL
#undef XX

// Row blocks of the side stream's trailing update per outer panel, and the K
// extent of each of its launches: the NB columns of the outer panel in two
// halves, so each tile holds its CU half as long and the critical chain's
// kernels find free CUs sooner.  Measured on the medium CCF step (ms per
// factorisation): K = 512 in one launch 10.03, two halves 9.76-9.84, four
// quarters 11.4; with halves, 3 row blocks 9.69-9.71, 4 blocks 9.80-9.84,
// 5 blocks 10.4.
static constexpr int SIDE_CHUNKS = 3;
static constexpr int64_t SIDE_K = NB / 2;

hipError_t launch_cholesky(hipStream_t st, hipStream_t side, hipEvent_t ev_panel, hipEvent_t ev_trail, double *A,
                           int64_t n, int64_t lda, double mu, int border, double *linv, double *tmp,
                           DevStatus *status) {
    if (n <= 0) return hipSuccess;
    static bool attr = false;
    const size_t shm = sizeof(double) * CB * LDS_LD;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)potrf_block_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)shm);
        attr = true;
    }
    // Without a distinct side stream (side == nullptr or st) every trailing
    // update goes to st in the same order and no events are used.
    const bool two = side != nullptr && side != st;
    if (!two) side = st;
    const int64_t nd = n - border;
    if (mu != 0.0 && nd > 0)
        hipLaunchKernelGGL(add_diag_kernel, dim3((unsigned)((nd + 255) / 256)), dim3(256), 0, st, A, nd, lda, mu);
    hipError_t e = hipSuccess;
    bool trail_pending = false;  // ev_trail marks a trailing update not yet waited for on st
    bool side_used = false;      // work was given to the side stream
    auto gemm = [&](hipStream_t s_, int64_t M, int64_t N, int64_t K, const double *a, const double *b, const double *bx,
                    double *c, double alpha, double beta, int lower, int mask) {
        GemmDesc g{};
        g.M = M; g.N = N; g.K = K;
        g.A = a; g.lda = lda; g.la = 0;
        g.B = b; g.ldb = bx ? CB : lda; g.lb = 1;
        if (bx) g.B = bx;
        g.C = c; g.ldc = lda;
        g.alpha = alpha; g.beta = beta;
        g.lower = lower; g.mask_lower = mask;
        g.stop_flag = &status->flag;
        if (s_ != side || K <= SIDE_K) return launch_dgemm(s_, g);
        // side stream: K in pieces of SIDE_K (shorter tiles free CUs for the chain sooner)
        for (int64_t k = 0; k < K; k += SIDE_K) {
            GemmDesc gk = g;
            gk.K = (K - k) < SIDE_K ? K - k : SIDE_K;
            gk.A = a + k;
            gk.B = b + k;
            const hipError_t e2 = launch_dgemm(s_, gk);
            if (e2 != hipSuccess) return e2;
        }
        return hipSuccess;
    };
    // Two-level right-looking blocking: outer panels of NB columns, factored
    // in CB-wide blocks (diagonal block, panel solve, update of the rest of the
    // outer panel); the trailing matrix is then updated once per outer panel
    // with K = NB, so each C tile is read and written once per NB columns.
    for (int64_t K0 = 0; K0 < n; K0 += NB) {
        const int64_t pe = (n - K0) < NB ? n : K0 + NB;  // end of the outer panel
        for (int64_t k0 = K0; k0 < pe; k0 += CB) {
            const int kb = (int)((n - k0) < CB ? (n - k0) : CB);
            const int bh = (border && k0 + kb == n) ? 1 : 0;
            double *Xb = linv + (k0 / CB) * CB * CB;
            hipLaunchKernelGGL(potrf_block_kernel, dim3(1), dim3(256), shm, st, A, lda, k0, kb, bh, Xb, tmp, status);
            const int64_t r1 = k0 + kb, rest = n - r1;
            if (rest <= 0) break;
            double *a21 = A + r1 * lda + k0;
            // L21 = A21 X^T in place: each output tile owns its rows over all kb columns
            if ((e = gemm(st, rest, kb, kb, a21, nullptr, Xb, a21, 1.0, 0.0, 0, 0)) != hipSuccess) return e;
            // remaining columns of this outer panel
            if (r1 < pe && (e = gemm(st, rest, pe - r1, kb, a21, a21, nullptr, A + r1 * lda + r1, -1.0, 1.0, 0, 1)) !=
                               hipSuccess)
                return e;
        }
        if (pe >= n) break;
        const int64_t rest = n - pe, kw = pe - K0;
        const double *lp = A + pe * lda + K0;  // L rows pe.. of the outer panel
        if (two && (e = hipEventRecord(ev_panel, st)) != hipSuccess) return e;
        // the next outer panel's columns first (main stream) ...
        const int64_t nb1 = rest < NB ? rest : NB;
        if (two && trail_pending) {
            if ((e = hipStreamWaitEvent(st, ev_trail, 0)) != hipSuccess) return e;
            trail_pending = false;
        }
        if ((e = gemm(st, rest, nb1, kw, lp, lp, nullptr, A + pe * lda + pe, -1.0, 1.0, 0, 1)) != hipSuccess) return e;
        // ... the rest of the trailing matrix on the side stream (look-ahead)
        const int64_t r2 = pe + nb1, rest2 = n - r2;
        if (rest2 > 0) {
            if (two && (e = hipStreamWaitEvent(side, ev_panel, 0)) != hipSuccess) return e;
            const double *l2 = A + r2 * lda + K0;
            // first the columns of the panel after next (rows r2.., lower part of its
            // diagonal block): the main stream's next update of them waits for this part only
            const int64_t nb2 = rest2 < NB ? rest2 : NB;
            if ((e = gemm(side, rest2, nb2, kw, l2, l2, nullptr, A + r2 * lda + r2, -1.0, 1.0, 0, 1)) != hipSuccess)
                return e;
            if (two && (e = hipEventRecord(ev_trail, side)) != hipSuccess) return e;
            trail_pending = two;
            side_used = two;
            // then the rest in SIDE_CHUNKS row blocks (a rectangle left of the diagonal
            // block, then the block's lower triangle): the main stream's panel kernels
            // queued meanwhile are dispatched between the side launches
            const int64_t r3 = r2 + nb2, rest3 = n - r3;
            const double *l3 = A + r3 * lda + K0;
            const int64_t rc = ((rest3 + SIDE_CHUNKS - 1) / SIDE_CHUNKS + CB - 1) / CB * CB;
            for (int64_t rs = 0; rs < rest3; rs += rc) {
                const int64_t rows = (rest3 - rs) < rc ? rest3 - rs : rc;
                if (rs > 0 && (e = gemm(side, rows, rs, kw, l3 + rs * lda, l3, nullptr, A + (r3 + rs) * lda + r3,
                                        -1.0, 1.0, 0, 0)) != hipSuccess)
                    return e;
                if ((e = gemm(side, rows, rows, kw, l3 + rs * lda, l3 + rs * lda, nullptr,
                              A + (r3 + rs) * lda + r3 + rs, -1.0, 1.0, 1, 0)) != hipSuccess)
                    return e;
            }
        }
    }
    // join: everything the side stream was given (ev_panel's last wait is already enqueued)
    if (side_used) {
        if ((e = hipEventRecord(ev_panel, side)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(st, ev_panel, 0)) != hipSuccess) return e;
    }
    return hipGetLastError();
}

// ------------------------------------------------------- triangular solves
// Blocks of CB rows; X_I is the inverse of the I-th diagonal block.
// Forward L z = b: z_0 = X_0 b_0; launch I updates b_w -= L_wI z_I for every
// block w > I (one workgroup per block) and the workgroup of block I+1 then
// forms z_{I+1} = X_{I+1} b_{I+1}.  Back L^T x = y mirrors it column-wise.

__device__ void block_lower_apply(const double *__restrict__ Xb, const double *bs, double *out, int kb) {
    // out[t] = sum_{c <= t} X[t][c] bs[c]: X staged through LDS in chunks of
    // 32 columns (coalesced row segments), two threads per row
    constexpr int KC = 32;
    __shared__ double xt[CB][KC + 1];
    __shared__ double part2[256];
    const int tid = threadIdx.x, row = tid & (CB - 1), half = tid >> 7;
    double acc = 0.0;
    for (int k0 = 0; k0 < kb; k0 += KC) {
        double v[CB * KC / 256];
#pragma unroll
        for (int e = 0; e < CB * KC / 256; ++e) {
            const int idx = tid + e * 256, rr = idx / KC, kk = idx % KC;
            v[e] = (rr < kb && k0 + kk < kb) ? Xb[rr * CB + k0 + kk] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < CB * KC / 256; ++e) {
            const int idx = tid + e * 256;
            xt[idx / KC][idx % KC] = v[e];
        }
        __syncthreads();
        const int kend = (kb - k0) < KC ? kb - k0 : KC;
        for (int kk = half; kk < kend; kk += 2) acc = fma(xt[row][kk], bs[k0 + kk], acc);
    }
    part2[tid] = acc;
    __syncthreads();
    if (half == 0 && row < kb) out[row] = part2[row] + part2[row + CB];
}

__device__ void block_upper_apply(const double *__restrict__ Xb, const double *ys, double *out, int kb) {
    // out[t] = sum_{c >= t} X[c][t] ys[c]; thread pairs per t (CB x 2 = 256 threads)
    __shared__ double part[256];
    const int tid = threadIdx.x, t = tid & (CB - 1), h = tid >> 7;
    double v0 = 0.0, v1 = 0.0;
    if (t < kb) {
        int c = t + h;
#pragma unroll 8
        for (; c + 2 < kb; c += 4) {
            v0 = fma(Xb[c * CB + t], ys[c], v0);
            v1 = fma(Xb[(c + 2) * CB + t], ys[c + 2], v1);
        }
        for (; c < kb; c += 2) v0 = fma(Xb[c * CB + t], ys[c], v0);
    }
    part[tid] = v0 + v1;
    __syncthreads();
    if (h == 0 && t < kb) out[t] = part[t] + part[t + CB];
}

__global__ __launch_bounds__(256) void fwd_init_kernel(const double *linv, const double *b, double *z, int kb,
                                                       const DevStatus *status) {
    if (status->flag) return;
    __shared__ double bs[CB];
    if (threadIdx.x < kb) bs[threadIdx.x] = b[threadIdx.x];
    __syncthreads();
    block_lower_apply(linv, bs, z, kb);
}

// Rows of block w = I + 1 + blockIdx.x: b_w -= L_wI z_I.  The 128 x kbI tile
// L_wI is staged through LDS in chunks of 32 columns (coalesced row
// segments, all loads of a thread issued before its stores); two threads
// per row each sum half of a chunk's columns.  The workgroup of block I + 1
// then forms z_{I+1} = X_{I+1} b_{I+1}.
__global__ __launch_bounds__(256) void fwd_update_kernel(const double *__restrict__ L, int64_t n, int64_t ldl,
                                                         const double *__restrict__ linv, double *b, double *z,
                                                         int64_t I, const DevStatus *status) {
    if (status->flag) return;
    constexpr int KC = 32;
    __shared__ double zs[CB];
    __shared__ double bs[CB];
    __shared__ double tile[CB][KC + 1];
    __shared__ double part[256];
    const int tid = threadIdx.x;
    const int64_t r0 = I * CB;
    const int kbI = (int)((n - r0) < CB ? (n - r0) : CB);
    const int64_t w = I + 1 + blockIdx.x;
    const int64_t w0 = w * CB;
    const int kbw = (int)((n - w0) < CB ? (n - w0) : CB);
    if (tid < kbI) zs[tid] = z[r0 + tid];
    const int row = tid & (CB - 1), half = tid >> 7;  // row of the tile, half of a chunk's columns
    double acc = 0.0;
    for (int k0 = 0; k0 < kbI; k0 += KC) {
        double v[CB * KC / 256];
#pragma unroll
        for (int e = 0; e < CB * KC / 256; ++e) {
            const int idx = tid + e * 256, rr = idx / KC, kk = idx % KC;
            v[e] = (rr < kbw && k0 + kk < kbI) ? L[(w0 + rr) * ldl + r0 + k0 + kk] : 0.0;
        }
        __syncthreads();  // previous chunk consumed (and zs written, first pass)
#pragma unroll
        for (int e = 0; e < CB * KC / 256; ++e) {
            const int idx = tid + e * 256;
            tile[idx / KC][idx % KC] = v[e];
        }
        __syncthreads();
        const int kend = (kbI - k0) < KC ? kbI - k0 : KC;
        for (int kk = half; kk < kend; kk += 2) acc = fma(tile[row][kk], zs[k0 + kk], acc);
    }
    part[tid] = acc;
    __syncthreads();
    if (half == 0 && row < kbw) {
        const double nb = b[w0 + row] - (part[row] + part[row + CB]);
        b[w0 + row] = nb;
        bs[row] = nb;
    }
    if (w != I + 1) return;
    __syncthreads();
    block_lower_apply(linv + w * CB * CB, bs, z + w0, kbw);
}

__global__ __launch_bounds__(256) void back_init_kernel(const double *linv, const double *y, double *x, int kb,
                                                        const DevStatus *status) {
    if (status->flag) return;
    __shared__ double ys[CB];
    if (threadIdx.x < kb) ys[threadIdx.x] = y[threadIdx.x];
    __syncthreads();
    block_upper_apply(linv, ys, x, kb);
}

__device__ __forceinline__ void back_update_body(const double *__restrict__ L, int64_t n, int64_t ldl,
                                                 const double *__restrict__ linv, double *y, double *x, int64_t I,
                                                 const DevStatus *status) {
    if (status->flag) return;
    __shared__ double xs[CB];
    __shared__ double part[256];
    __shared__ double ys[CB];
    const int tid = threadIdx.x, c = tid & (CB - 1), h = tid >> 7;
    const int64_t r0 = I * CB;
    const int kbI = (int)((n - r0) < CB ? (n - r0) : CB);
    const int64_t w = blockIdx.x;  // column block w < I (full CB columns)
    const int64_t col = w * CB + c;
    if (tid < kbI) xs[tid] = x[r0 + tid];
    __syncthreads();
    double v0 = 0.0, v1 = 0.0;
    if (kbI == CB) {
        // 64 independent loads per thread, issued together
        double lv[CB / 2];
#pragma unroll
        for (int e = 0; e < CB / 2; ++e) lv[e] = L[(r0 + 2 * e + h) * ldl + col];
#pragma unroll
        for (int e = 0; e < CB / 2; e += 2) {
            v0 = fma(lv[e], xs[2 * e + h], v0);
            v1 = fma(lv[e + 1], xs[2 * e + 2 + h], v1);
        }
    } else {
        for (int i = h; i < kbI; i += 2) v0 = fma(L[(r0 + i) * ldl + col], xs[i], v0);
    }
    part[tid] = v0 + v1;
    __syncthreads();
    if (h == 0) {
        const double ny = y[col] - (part[c] + part[c + CB]);
        y[col] = ny;
        ys[c] = ny;
    }
    if (w != I - 1) return;
    __syncthreads();
    block_upper_apply(linv + w * CB * CB, ys, x + w * CB, CB);
}

__global__ __launch_bounds__(256) void back_update_kernel(const double *__restrict__ L, int64_t n, int64_t ldl,
                                                          const double *__restrict__ linv, double *y, double *x,
                                                          int64_t I, const DevStatus *status) {
    back_update_body(L, n, ldl, linv, y, x, I, status);
}

// blockIdx.y = instance
__global__ __launch_bounds__(256) void back_init_batched_kernel(const BatchChol *__restrict__ bc, int64_t n) {
    const BatchChol c = bc[blockIdx.y];
    if (c.status->flag) return;
    const int64_t nblk = (n + CB - 1) / CB, rl = (nblk - 1) * CB;
    const int kb = (int)(n - rl);
    __shared__ double ys[CB];
    if (threadIdx.x < kb) ys[threadIdx.x] = c.y[rl + threadIdx.x];
    __syncthreads();
    block_upper_apply(c.linv + (nblk - 1) * CB * CB, ys, c.x + rl, kb);
}

__global__ __launch_bounds__(256) void back_update_batched_kernel(const BatchChol *__restrict__ bc, int64_t n, int64_t I) {
    const BatchChol c = bc[blockIdx.y];
    back_update_body(c.A, n, c.lda, c.linv, c.y, c.x, I, c.status);
}

// Border row of the bordered factor (row n of A): y = -w, |w|^2, corner value.
__global__ __launch_bounds__(256) void border_extract_batched_kernel(const BatchChol *__restrict__ bc, int64_t n) {
    const BatchChol c = bc[blockIdx.y];
    __shared__ double sh[256];
    const double *w = c.A + n * c.lda;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double v = w[i];
        c.y[i] = -v;
        acc = fma(v, v, acc);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        c.status->grad_dot_delta = sh[0];
        c.status->model_sq_norm = w[n];
    }
}

// theta += delta when the residual is finite, the factorisation succeeded and
// delta is finite (one workgroup per instance).
__global__ __launch_bounds__(256) void update_batched_kernel(const BatchChol *__restrict__ bc, int64_t p) {
    const BatchChol c = bc[blockIdx.y];
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < p; i += 256) {
        const double v = c.x[i];
        if (!(v - v == 0.0)) bad = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0 && bad) c.status->nonfinite = 1;
    const double h = c.status->half_sq_norm;
    if (!(h - h == 0.0) || c.status->flag || bad) {
        if (threadIdx.x == 0 && !(h - h == 0.0)) c.status->nonfinite = 1;
        return;
    }
    for (int64_t i = threadIdx.x; i < p; i += 256) c.theta[i] += c.x[i];
    if (threadIdx.x == 0) c.status->updated = 1;
}

hipError_t launch_cholesky_batched(hipStream_t st, const BatchChol *h_bc, const BatchChol *d_bc,
                                   const std::vector<BatchedGemmPlan> &plans, int nb, int64_t n, double mu,
                                   int border) {
    if (nb <= 0 || n <= 0) return hipSuccess;
    static bool attr = false;
    const size_t shm = sizeof(double) * CB * LDS_LD;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)potrf_block_batched_kernel,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        attr = true;
    }
    const int64_t nd = n - border;
    if (mu != 0.0 && nd > 0)
        for (int i = 0; i < nb; ++i)
            hipLaunchKernelGGL(add_diag_kernel, dim3((unsigned)((nd + 255) / 256)), dim3(256), 0, st, h_bc[i].A, nd,
                               h_bc[i].lda, mu);
    hipError_t e;
    size_t panel = 0;
    for (int64_t k0 = 0; k0 < n; k0 += CB, ++panel) {
        const int kb = (int)((n - k0) < CB ? (n - k0) : CB);
        const int bh = (border && k0 + kb == n) ? 1 : 0;
        hipLaunchKernelGGL(potrf_block_batched_kernel, dim3((unsigned)nb), dim3(256), shm, st, d_bc, k0, kb, bh);
        if (n - k0 - kb <= 0) break;
        if (2 * panel + 1 >= plans.size()) return hipErrorInvalidValue;
        if ((e = launch_batched_plan(st, plans[2 * panel])) != hipSuccess) return e;
        if ((e = launch_batched_plan(st, plans[2 * panel + 1])) != hipSuccess) return e;
    }
    return hipGetLastError();
}

void cholesky_batched_plans(const BatchChol *bc, int nb, int64_t n, std::vector<BatchedGemmPlan> &out) {
    out.clear();
    for (int64_t k0 = 0; k0 < n; k0 += CB) {
        const int kb = (int)((n - k0) < CB ? (n - k0) : CB);
        const int64_t r1 = k0 + kb, rest = n - r1;
        if (rest <= 0) break;
        for (int pass = 0; pass < 2; ++pass) {
            BatchedGemmPlan p;
            for (int i = 0; i < nb; ++i) {
                double *A = bc[i].A;
                const int64_t lda = bc[i].lda;
                double *a21 = A + r1 * lda + k0;
                GemmDesc g{};
                if (pass == 0) {
                    g.M = rest; g.N = kb; g.K = kb;
                    g.A = a21; g.lda = lda; g.la = 0;
                    g.B = bc[i].linv + (k0 / CB) * CB * CB; g.ldb = CB; g.lb = 1;
                    g.C = a21; g.ldc = lda;
                    g.alpha = 1.0; g.beta = 0.0;
                } else {
                    g.M = rest; g.N = rest; g.K = kb;
                    g.A = a21; g.lda = lda; g.la = 0;
                    g.B = a21; g.ldb = lda; g.lb = 1;
                    g.C = A + r1 * lda + r1; g.ldc = lda;
                    g.alpha = -1.0; g.beta = 1.0;
                    g.lower = 1;
                }
                g.stop_flag = &bc[i].status->flag;
                p.h_descs.push_back(g);
            }
            out.push_back(std::move(p));
        }
    }
}

hipError_t launch_solve_upper_batched(hipStream_t st, const BatchChol *d_bc, int nb, int64_t n) {
    if (n <= 0 || nb <= 0) return hipSuccess;
    const int64_t nblk = (n + CB - 1) / CB;
    hipLaunchKernelGGL(border_extract_batched_kernel, dim3(1, (unsigned)nb), dim3(256), 0, st, d_bc, n);
    hipLaunchKernelGGL(back_init_batched_kernel, dim3(1, (unsigned)nb), dim3(256), 0, st, d_bc, n);
    for (int64_t I = nblk - 1; I >= 1; --I)
        hipLaunchKernelGGL(back_update_batched_kernel, dim3((unsigned)I, (unsigned)nb), dim3(256), 0, st, d_bc, n, I);
    hipLaunchKernelGGL(update_batched_kernel, dim3(1, (unsigned)nb), dim3(256), 0, st, d_bc, n);
    return hipGetLastError();
}

hipError_t launch_solve_lower(hipStream_t st, const double *L, int64_t n, int64_t ldl, const double *linv,
                              double *b, double *z, DevStatus *status) {
    if (n <= 0) return hipSuccess;
    const int64_t nblk = (n + CB - 1) / CB;
    hipLaunchKernelGGL(fwd_init_kernel, dim3(1), dim3(256), 0, st, linv, b, z, (int)(n < CB ? n : CB), status);
    for (int64_t I = 0; I + 1 < nblk; ++I)
        hipLaunchKernelGGL(fwd_update_kernel, dim3((unsigned)(nblk - 1 - I)), dim3(256), 0, st, L, n, ldl, linv, b, z,
                           I, status);
    return hipGetLastError();
}

hipError_t launch_solve_upper(hipStream_t st, const double *L, int64_t n, int64_t ldl, const double *linv,
                              double *y, double *x, DevStatus *status) {
    if (n <= 0) return hipSuccess;
    const int64_t nblk = (n + CB - 1) / CB;
    const int64_t rl = (nblk - 1) * CB;
    hipLaunchKernelGGL(back_init_kernel, dim3(1), dim3(256), 0, st, linv + (nblk - 1) * CB * CB, y + rl, x + rl,
                       (int)(n - rl), status);
    for (int64_t I = nblk - 1; I >= 1; --I)
        hipLaunchKernelGGL(back_update_kernel, dim3((unsigned)I), dim3(256), 0, st, L, n, ldl, linv, y, x, I, status);
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
        s->delta_sq_norm = 0.0;
        s->half_sq_trial = 0.0;
        s->max_d1_val = 0;
        s->max_d2_val = 0;
    }
}

// Clears the factorisation and update fields of the status before another
// solve of the same system (the statistics of the residual are kept).
__global__ void reset_solve_status_kernel(DevStatus *s) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        s->chol_info = 0;
        s->flag = 0;
        s->nonfinite = 0;
        s->updated = 0;
        s->grad_dot_delta = 0.0;
        s->model_sq_norm = 0.0;
        s->delta_sq_norm = 0.0;
        s->half_sq_trial = 0.0;
    }
}

hipError_t launch_reset_solve_status(hipStream_t st, DevStatus *s) {
    hipLaunchKernelGGL(reset_solve_status_kernel, dim3(1), dim3(64), 0, st, s);
    return hipGetLastError();
}

// Keeps a copy of a symmetric matrix's lower triangle in its strictly upper
// triangle (transposed) and the diagonal in diag (SAVE), or writes it back
// (restore).  Nothing the Gram and the Cholesky write lies above the
// diagonal, so the copy survives a factorisation.  One 64 x 64 tile of the
// lower triangle per workgroup (tile row blockIdx.y, tile column blockIdx.x,
// upper tiles exit), transposed through LDS so that every global access runs
// along a row.  Reads and writes of a tile pair are disjoint (strictly lower
// versus strictly upper positions), so tiles need no ordering.
template <bool SAVE>
__global__ __launch_bounds__(256) void tri_mirror_kernel(double *A, int64_t n, int64_t lda, double *diag) {
    __shared__ double t[64][65];
    const int bi = blockIdx.y, bj = blockIdx.x;
    if (bj > bi) return;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)bi * 64, c0 = (int64_t)bj * 64;
    if (SAVE) {
        // t[i][j] = A[r0 + i][c0 + j] on and below the diagonal
        for (int k = ty; k < 64; k += 4) {
            const int64_t r = r0 + k, c = c0 + tx;
            t[k][tx] = (r < n && c <= r) ? A[r * lda + c] : 0.0;
        }
        __syncthreads();
        // A[c][r] = A[r][c] for c < r: destination row c0 + k, column r0 + tx
        for (int k = ty; k < 64; k += 4) {
            const int64_t c = c0 + k, r = r0 + tx;
            if (r < n && c < r) A[c * lda + r] = t[tx][k];
            if (bi == bj && r < n && c == r) diag[r] = t[tx][k];
        }
    } else {
        // t[i][j] = A[c0 + i][r0 + j] strictly above the diagonal
        for (int k = ty; k < 64; k += 4) {
            const int64_t c = c0 + k, r = r0 + tx;
            t[k][tx] = (r < n && c < r) ? A[c * lda + r] : 0.0;
        }
        __syncthreads();
        // A[r][c] = A[c][r] for c < r, diagonal from diag: row r0 + k, column c0 + tx
        for (int k = ty; k < 64; k += 4) {
            const int64_t r = r0 + k, c = c0 + tx;
            if (r < n && c < r) A[r * lda + c] = t[tx][k];
            else if (r < n && c == r) A[r * lda + c] = diag[r];
        }
    }
}

hipError_t launch_tri_save(hipStream_t st, double *A, int64_t n, int64_t lda, double *diag) {
    if (n <= 0) return hipSuccess;
    const unsigned T = (unsigned)((n + 63) / 64);
    hipLaunchKernelGGL(tri_mirror_kernel<true>, dim3(T, T), dim3(256), 0, st, A, n, lda, diag);
    return hipGetLastError();
}

hipError_t launch_tri_restore(hipStream_t st, double *A, int64_t n, int64_t lda, const double *diag) {
    if (n <= 0) return hipSuccess;
    const unsigned T = (unsigned)((n + 63) / 64);
    hipLaunchKernelGGL(tri_mirror_kernel<false>, dim3(T, T), dim3(256), 0, st, A, n, lda, (double *)diag);
    return hipGetLastError();
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
