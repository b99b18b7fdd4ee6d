// Damped solve of the Gauss-Newton system on gfx950 (paper, Methods,
// "Second-order Optimizer": theta <- theta - (G + gamma I)^{-1} grad h).
//
// Right-looking blocked Cholesky, two levels (128-wide diagonal blocks inside
// 384-wide outer panels) with look-ahead:
//   1. diagonal block: one workgroup factors it in LDS (one-wave 32x32
//      register factorisations, the rest by all four waves) and forms the
//      inverse of its triangular factor;
//   2. panel below: L21 = A21 L11^{-T} as an MFMA GEMM with the inverse;
//   3. the remaining columns of the outer panel are updated (K = 128);
//   4. after an outer panel, the trailing matrix is updated with K = 384
//      (lower), split into the next outer panel's columns (main stream) and
//      the rest (a second stream, in two row blocks), so the next panel is
//      factored while the bulk of the update runs.  A large K keeps
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
// Triangular solves use the stored diagonal-block inverses.  The handle's
// solves run in one launch each (fwd_sync_kernel, back_sync_kernel: one
// workgroup per 128-row block, each waiting for the blocks it depends on to
// be published); the launch-per-block versions (one launch per block applies
// the known block to the rest of the right-hand side, one workgroup per
// remaining block, and the workgroup of the next block then forms that
// block's unknowns) serve the solve without allocation and the batched step.
#include <vector>

#include "gn_internal.h"
#include "chol_block.h"

namespace gn {

// Outer panel width (K of the trailing update).  Measured at n = 8514 (ms per
// factorisation, two streams): 256 columns 8.83-9.27, 384 columns 8.71-8.83,
// 512 columns 8.87-8.93, 768 columns 8.97-9.21.  Narrower panels shorten the
// chain's own products (its update of the next outer panel is rest x NB x NB);
// wider ones give the side stream longer K.
static constexpr int NB = 3 * CB;

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
__global__ __launch_bounds__(256) void potrf_block_kernel(double *A, int64_t lda, int64_t k0, int kb, int border_here,
                                                         double *X, double *, DevStatus *status) {
    extern __shared__ double s[];
    __shared__ int fail_sh;
    __shared__ __align__(16) double colbuf[POTRF_COLBUF];
    __shared__ double W[POTRF_W];
    potrf_block_body<256>(A, lda, k0, kb, border_here, X, status, s, colbuf, W, fail_sh);
}

// One diagonal block per instance of a batch (blockIdx.x = instance).
__global__ __launch_bounds__(256) void potrf_block_batched_kernel(const BatchChol *__restrict__ bc, int64_t k0, int kb,
                                                                 int border_here) {
    const BatchChol c = bc[blockIdx.x];
    extern __shared__ double s[];
    __shared__ int fail_sh;
    __shared__ __align__(16) double colbuf[POTRF_COLBUF];
    __shared__ double W[POTRF_W];
    potrf_block_body<256>(c.A, c.lda, k0, kb, border_here, c.linv + (k0 / CB) * CB * CB, c.status, s, colbuf, W,
                          fail_sh);
}

// Row blocks of the side stream's trailing update per outer panel, and the K
// extent of each of its launches (a longer K is cut into pieces, so each tile
// holds its CU for a shorter time and the critical chain's kernels find free
// CUs sooner).  Measured at n = 8514 (ms per factorisation): with 512-column
// panels, K = 512 in one launch 10.03, two halves of 256 9.76-9.84, four
// quarters 11.4, and 3 row blocks 9.69-9.71 against 4 blocks 9.80-9.84 and 5
// blocks 10.4 (before the later diagonal-block and panel-solve changes); with
// 384-column panels (one piece of 384), 2 row blocks 8.71-8.73, 1 block
// 8.85, 3 blocks 8.78-8.83, 4 blocks 8.80, and pieces of 192 9.34.
static constexpr int SIDE_CHUNKS = 2;
static constexpr int64_t SIDE_K = NB;

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

// Back substitution L^T x = y in one launch.  Workgroup b owns column block
// w = nblk - 1 - b and keeps y_w in LDS.  For I = nblk - 1 down to w + 1 it
// issues the loads of L_Iw, waits until x_I is published, and subtracts
// L_Iw^T x_I with the per-thread sums and the pairing of back_update_body;
// then x_w = X_w^T y_w in the order of block_upper_apply (X_w staged in LDS
// before the first wait).  The result is bitwise that of the launch per
// block row.  A workgroup waits only on lower-numbered ones, which are
// dispatched first, so the lowest unfinished workgroup can always run.
//
// sync[0] is an epoch that the one-thread kernel before the solve advances;
// sync[1 + I] == epoch marks x_I as published.  Publishing: each storing
// thread waits until its stores of x_w have completed (they are in its XCD's
// L2), the workgroup barrier follows, then thread 0's release store of the
// marker (an agent-scope release: the L2 is written back before the marker is
// stored).  Waiting: thread 0 polls the marker with relaxed device-coherent
// loads and, once it is seen, issues one agent-scope acquire fence (the
// caches are invalidated once, not on every poll); the workgroup barrier after
// it orders every thread's reads of x_I.  A chain of 67 such hops measured
// 1.14 us per hop against 2.57 us with an acquire on every poll and a full
// fence in every storing thread.  Every wait is bounded:
// past SOLVE_SPIN_LIMIT polls the workgroup records wait_fail and the stop
// flag in the status and exits; waiting workgroups poll the stop flag too
// and leave as soon as it is set.
static constexpr long long SOLVE_SPIN_LIMIT = 1ll << 18;  // polls of about 0.1-1 us each

int64_t solve_sync_size(int64_t n) { return 1 + (n + CB - 1) / CB; }

__global__ void solve_epoch_kernel(unsigned *sync) {
    if (threadIdx.x == 0) {
        unsigned e = sync[0] + 1u;
        if (e == 0u) e = 1u;  // 0 is the value of a marker never written
        sync[0] = e;
    }
}

__global__ __launch_bounds__(256) void back_sync_kernel(const double *__restrict__ L, int64_t n, int64_t ldl,
                                                        const double *__restrict__ linv, const double *__restrict__ y,
                                                        double *x, DevStatus *status, unsigned *sync) {
    if (status->flag) return;
    extern __shared__ double Xs[];  // X_w, CB x CB
    __shared__ double ys[CB];
    __shared__ double xs[CB];
    __shared__ double part[256];
    __shared__ int ok_s;
    const int tid = threadIdx.x, c = tid & (CB - 1), h = tid >> 7;
    const unsigned epoch = sync[0];
    const int64_t nblk = (n + CB - 1) / CB;
    const int64_t w = nblk - 1 - (int64_t)blockIdx.x;
    const int64_t w0 = w * CB;
    const int kbw = (int)((n - w0) < CB ? (n - w0) : CB);
    {
        const double2 *src = reinterpret_cast<const double2 *>(linv + w * CB * CB);
        double2 *dst = reinterpret_cast<double2 *>(Xs);
#pragma unroll 8
        for (int e = tid; e < CB * CB / 2; e += 256) dst[e] = src[e];
    }
    if (tid < kbw) ys[tid] = y[w0 + tid];
    const int64_t col = w0 + c;
    for (int64_t I = nblk - 1; I > w; --I) {
        const int64_t r0 = I * CB;
        const int kbI = (int)((n - r0) < CB ? (n - r0) : CB);
        double lv[CB / 2];
        if (kbI == CB) {
#pragma unroll
            for (int e = 0; e < CB / 2; ++e) lv[e] = L[(r0 + 2 * e + h) * ldl + col];
        }
        if (tid == 0) {
            int ok = 1;
            long long spins = 0;
            while (__hip_atomic_load(sync + 1 + I, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
                if (__hip_atomic_load(&status->flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                    ok = -1;  // another workgroup gave up: leave without waiting out the bound
                    break;
                }
                if (++spins > SOLVE_SPIN_LIMIT) {
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            if (ok == 1) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the published block is visible from here
            if (ok == 0) {
                __hip_atomic_store(&status->wait_fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&status->flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            ok_s = ok;
        }
        __syncthreads();  // also: Xs and ys staged (first pass), part and xs consumed (later passes)
        if (ok_s != 1) return;
        if (tid < kbI) xs[tid] = x[r0 + tid];
        __syncthreads();
        double v0 = 0.0, v1 = 0.0;
        if (kbI == CB) {
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
        if (h == 0) ys[c] = ys[c] - (part[c] + part[c + CB]);
    }
    __syncthreads();
    // x_w = X_w^T y_w
    double v0 = 0.0, v1 = 0.0;
    if (c < kbw) {
        int cc = c + h;
#pragma unroll 8
        for (; cc + 2 < kbw; cc += 4) {
            v0 = fma(Xs[cc * CB + c], ys[cc], v0);
            v1 = fma(Xs[(cc + 2) * CB + c], ys[cc + 2], v1);
        }
        for (; cc < kbw; cc += 2) v0 = fma(Xs[cc * CB + c], ys[cc], v0);
    }
    part[tid] = v0 + v1;
    __syncthreads();
    if (h == 0 && c < kbw) {
        x[w0 + c] = part[c] + part[c + CB];
        __builtin_amdgcn_s_waitcnt(0);  // the store has completed before the barrier and the release
    }
    __syncthreads();
    if (tid == 0) __hip_atomic_store(sync + 1 + w, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Forward substitution L z = b in one launch.  Workgroup w owns row block w:
// thread (row, half) keeps the entries X_w[row][half + 2j] in registers, the
// ones its final sum needs, and, for I = 0 .. w-1, loads L_wI and puts it into an LDS tile before it
// waits for z_I to be published, then subtracts L_wI z_I with the per-thread
// sums of fwd_update_kernel (two threads per row, each summing every other
// column in order) and finally forms z_w = X_w b_w in the order of
// block_lower_apply, so the result is bitwise that of the launch per block
// column.  The whole 128 x 128 tile sits in LDS (132 KB), so each block takes
// three barriers instead of the ten of 32-column chunks.  Publication, epochs
// and bounded waits as in back_sync_kernel; b is not modified.
__global__ __launch_bounds__(256) void fwd_sync_kernel(const double *__restrict__ L, int64_t n, int64_t ldl,
                                                       const double *__restrict__ linv, const double *__restrict__ b,
                                                       double *z, DevStatus *status, unsigned *sync) {
    if (status->flag) return;
    constexpr int KC = 32, NE = CB * KC / 256;  // loads per thread per 32-column chunk
    constexpr int LD = CB + 1;
    extern __shared__ double tile[];             // CB x LD
    __shared__ double zs[CB];
    __shared__ double bs[CB];
    __shared__ double part[256];
    __shared__ int ok_s;
    const int tid = threadIdx.x, row = tid & (CB - 1), half = tid >> 7;
    const unsigned epoch = sync[0];
    const int64_t w = blockIdx.x;
    const int64_t w0 = w * CB;
    const int kbw = (int)((n - w0) < CB ? (n - w0) : CB);
    const double *Xb = linv + w * CB * CB;
    double xr[CB / 2];  // X_w[row][half + 2 j]
#pragma unroll
    for (int j = 0; j < CB / 2; ++j) xr[j] = (row < kbw && half + 2 * j < kbw) ? Xb[row * CB + half + 2 * j] : 0.0;
    if (tid < kbw) bs[tid] = b[w0 + tid];
    for (int64_t I = 0; I < w; ++I) {
        const int64_t r0 = I * CB;  // block I < w is full
        {
            double lv[CB / KC][NE];
#pragma unroll
            for (int ch = 0; ch < CB / KC; ++ch)
#pragma unroll
                for (int e = 0; e < NE; ++e) {
                    const int idx = tid + e * 256, rr = idx / KC, kk = idx % KC;
                    lv[ch][e] = rr < kbw ? L[(w0 + rr) * ldl + r0 + ch * KC + kk] : 0.0;
                }
            // the previous block's reads of the tile ended before its partial-sum barrier
#pragma unroll
            for (int ch = 0; ch < CB / KC; ++ch)
#pragma unroll
                for (int e = 0; e < NE; ++e) {
                    const int idx = tid + e * 256, rr = idx / KC, kk = idx % KC;
                    tile[rr * LD + ch * KC + kk] = lv[ch][e];
                }
        }
        if (tid == 0) {
            int ok = 1;
            long long spins = 0;
            while (__hip_atomic_load(sync + 1 + I, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
                if (__hip_atomic_load(&status->flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                    ok = -1;
                    break;
                }
                if (++spins > SOLVE_SPIN_LIMIT) {
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            if (ok == 1) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the published block is visible from here
            if (ok == 0) {
                __hip_atomic_store(&status->wait_fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&status->flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            ok_s = ok;
        }
        __syncthreads();  // the tile stored; bs staged (first block), bs updates of the previous block done
        if (ok_s != 1) return;
        if (tid < CB) zs[tid] = z[r0 + tid];
        __syncthreads();
        double acc = 0.0;
        for (int kk = half; kk < CB; kk += 2) acc = fma(tile[row * LD + kk], zs[kk], acc);
        part[tid] = acc;
        __syncthreads();
        if (half == 0 && row < kbw) bs[row] = bs[row] - (part[row] + part[row + CB]);
    }
    // z_w = X_w b_w from the registers, the sums in the order of block_lower_apply
    __syncthreads();  // bs final
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < CB / 2; ++j)
        if (half + 2 * j < kbw) acc = fma(xr[j], bs[half + 2 * j], acc);
    part[tid] = acc;
    __syncthreads();
    if (half == 0 && row < kbw) {
        z[w0 + row] = part[row] + part[row + CB];
        __builtin_amdgcn_s_waitcnt(0);  // the store has completed before the barrier and the release
    }
    __syncthreads();
    if (tid == 0) __hip_atomic_store(sync + 1 + w, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
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

hipError_t launch_solve_upper_sync(hipStream_t st, const double *L, int64_t n, int64_t ldl, const double *linv,
                                   const double *y, double *x, DevStatus *status, unsigned *sync) {
    if (n <= 0) return hipSuccess;
    static bool attr = false;
    const size_t shm = sizeof(double) * CB * CB;
    if (!attr) {
        const hipError_t e = hipFuncSetAttribute((const void *)back_sync_kernel,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int64_t nblk = (n + CB - 1) / CB;
    hipLaunchKernelGGL(solve_epoch_kernel, dim3(1), dim3(64), 0, st, sync);
    hipLaunchKernelGGL(back_sync_kernel, dim3((unsigned)nblk), dim3(256), shm, st, L, n, ldl, linv, y, x, status,
                       sync);
    return hipGetLastError();
}

hipError_t launch_solve_lower_sync(hipStream_t st, const double *L, int64_t n, int64_t ldl, const double *linv,
                                   const double *b, double *z, DevStatus *status, unsigned *sync) {
    if (n <= 0) return hipSuccess;
    const int64_t nblk = (n + CB - 1) / CB;
    hipLaunchKernelGGL(solve_epoch_kernel, dim3(1), dim3(64), 0, st, sync);
    static bool attr = false;
    const size_t shm = sizeof(double) * CB * (CB + 1);
    if (!attr) {
        // the kernel's static LDS (z_I, b_w, the partial sums) comes on top
        const hipError_t e = hipFuncSetAttribute((const void *)fwd_sync_kernel,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(fwd_sync_kernel, dim3((unsigned)nblk), dim3(256), shm, st, L, n, ldl, linv, b, z, status,
                       sync);
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
        s->wait_fail = 0;
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
        s->wait_fail = 0;
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
