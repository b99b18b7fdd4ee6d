// FP64 MFMA GEMM for gfx950 (v_mfma_f64_16x16x4_f64): the dense
// contractions of the damped Gauss-Newton step.
//   - Gram G = J^T J (lower triangle), the SYRK whose cost dominates the step
//     (paper, Methods, "Second-order Optimizer": full Gauss-Newton matrix).
//   - Hilbert coupling J[:N] += diag(sc Theta_y) Q B.
//   - Trailing update and triangular-inverse products of the blocked Cholesky.
//
// C[m][n] = beta C[m][n] + alpha * rowscale[m] * sum_k A(m,k) B(k,n)
//
// Tiling: a 512-thread workgroup (8 waves, 2 x 4, two per SIMD so one wave's
// memory waits overlap the other's MFMAs) owns a BM x BN tile of C; each wave
// owns (BM/2) x (BN/4) as 16x16 MFMA blocks held in registers.
// K is consumed in chunks of BK = 32 staged through double-buffered LDS.
// A second configuration uses 256-thread workgroups (2 x 2 waves of 64 x 64)
// with BK = 16, so that two workgroups (64 KB of LDS each) share a CU and one
// workgroup's barrier waits overlap the other's MFMAs.
// Each operand keeps its global orientation in LDS ([k][m] when contiguous
// along m, else [m][k] with a padded row), so staging is a straight 16-byte
// copy without bank conflicts and an MFMA fragment read (16 consecutive m or
// n for each of 4 k) touches distinct banks.  Global loads for chunk c+1
// (16-byte pairs along the operand's contiguous direction, no bounds checks
// for interior tiles) are issued before the MFMAs of chunk c.
// Tiles are grouped in 4 x 8 super-tiles, one per XCD at a time (L2 reuse).
// The Gram and the Hilbert coupling run on work plans built once per shape
// (plan_gram, plan_rect): the super-tiles dealt so that every XCD holds the
// same number of tiles, and the tiles of each XCD's last, partly filled round
// split into K ranges whose partial products gram_sum_kernel adds in a fixed
// order.  Workgroup b runs on XCD b % 8 and each XCD takes its share in order.
//
// Fragment layout of v_mfma_f64_16x16x4_f64 (wave64):
//   A (16x4):  lane l holds A[l%16][l/16]
//   B (4x16):  lane l holds B[l/16][l%16]
//   D (16x16): lane l, register r holds D[l/16 + 4*r][l%16]  (f64: one row per
//              register group, unlike the 4-row groups of the f32 variant)
#include "gn_internal.h"
#include "tile_loader.h"

#include <algorithm>

namespace gn {

static constexpr int GEMM_THREADS = 512;  // 8 waves: two per SIMD
static constexpr int SUP_M = 4, SUP_N = 8;   // tiles per super-tile (one XCD round)
static constexpr int SUP = SUP_M * SUP_N;
static constexpr int NXCD = 8;

// Tile order.  Workgroups are dispatched round-robin over the 8 XCDs and each
// XCD runs its share in order, 32 at a time (one per CU).  Block b is sent to
// super-tile s = (pos / 32) * 8 + xcd (pos = b / 8, xcd = b % 8), tile
// i = pos % 32 of it, so each XCD works on one compact 4 x 8 block of tiles at
// a time and its L2 serves 12 operand panels instead of up to 33.
// Lower-triangular GEMMs enumerate only super-tiles that touch the lower
// triangle (row a of super-tiles holds b = 0 .. (4a+3)/8).
// Narrow products (fewer than 8 tile columns: the panel solves and panel
// updates of the Cholesky) use super-tiles of all their tile columns and
// ceil(tiles_m / 8k) tile rows (k the smallest that fits 32 tiles), so that
// the grid holds little padding and every XCD gets a share: a padding block
// costs a dispatch slot, and while the look-ahead update holds the CUs,
// slots are what the factorisation's critical chain waits for.
__host__ __device__ inline int64_t lower_super_count(int64_t tiles) {
    const int64_t nsr = (tiles + SUP_M - 1) / SUP_M, nsc = (tiles + SUP_N - 1) / SUP_N;
    int64_t n = 0;
    for (int64_t a = 0; a < nsr; ++a) {
        int64_t c = (SUP_M * a + SUP_M - 1) / SUP_N + 1;
        n += c < nsc ? c : nsc;
    }
    return n;
}

// Super-tile shape of a product: SUP_M x SUP_N, or (rows, cols) for a narrow
// one, packed as rows | cols << 8.
static inline int super_shape(int lower, int tiles_m, int tiles_n) {
    if (lower || tiles_n >= SUP_N) return SUP_M | (SUP_N << 8);
    // rows per super-tile: the fewest that give a multiple of 8 super-tiles
    // within the SUP tiles of one round
    const int sn = tiles_n < 1 ? 1 : tiles_n;
    int sm = 1;
    for (int k = 1;; ++k) {
        sm = (tiles_m + NXCD * k - 1) / (NXCD * k);
        if (sm < 1) sm = 1;
        if (sm * sn <= SUP) break;
    }
    return sm | (sn << 8);
}

// Returns false for padding blocks and tiles outside the (lower) tile set.
__device__ __forceinline__ bool tile_of_block(int64_t b, int lower, int tiles_m, int tiles_n, int sup, int &tm,
                                              int &tn) {
    const int sup_m = sup & 0xff, sup_n = sup >> 8, per = sup_m * sup_n;
    const int64_t x = b % NXCD, pos = b / NXCD;
    const int64_t sidx = (pos / per) * NXCD + x;
    const int i = (int)(pos % per);
    int64_t sm, sn;
    if (lower) {
        const int64_t nsr = (tiles_m + SUP_M - 1) / SUP_M, nsc = (tiles_m + SUP_N - 1) / SUP_N;
        int64_t rem = sidx, a = 0;
        for (; a < nsr; ++a) {
            int64_t c = (SUP_M * a + SUP_M - 1) / SUP_N + 1;
            if (c > nsc) c = nsc;
            if (rem < c) break;
            rem -= c;
        }
        if (a >= nsr) return false;
        sm = a;
        sn = rem;
    } else {
        const int64_t nsm = (tiles_m + sup_m - 1) / sup_m, nsn = (tiles_n + sup_n - 1) / sup_n;
        if (sidx >= nsm * nsn) return false;
        sm = sidx % nsm;
        sn = sidx / nsm;
    }
    tm = (int)(sm * sup_m + i % sup_m);
    tn = (int)(sn * sup_n + i / sup_m);
    if (tm >= tiles_m || tn >= tiles_n) return false;
    if (lower && tn > tm) return false;
    return true;
}

// K extent of each piece of a split tile: K / pieces rounded up to whole chunks
__host__ __device__ inline int64_t gram_piece_k(int64_t K, int pieces, int bk) {
    const int64_t q = pieces > 1 ? (K + pieces - 1) / pieces : K;
    return (q + bk - 1) / bk * bk;
}

// PLAN: a planned product (launch_planned); a compile-time switch, so that the
// other instances carry none of its code.
template <int BM, int BN, int BK, int LA, int LB, bool BATCH, int NT, bool PLAN = false>
__global__ __launch_bounds__(NT, 512 / NT) void dgemm_mfma_kernel(GemmDesc g0, int tiles_m0, int tiles_n0, int sup0,
                                                                 const GemmDesc *__restrict__ batch,
                                                                 const int4 *__restrict__ work) {
    static_assert(!(BATCH && PLAN), "one table kind per instance");
    // batched launches read (problem, tile row, tile column) from a work table
    // laid out in dispatch order (entry b runs on XCD b % 8); a planned product
    // reads (unit, tile row, tile column, piece)
    int4 wi = make_int4(0, 0, 0, 0);
    if (BATCH || PLAN) {
        wi = work[blockIdx.x];
        if (BATCH ? wi.x < 0 : wi.y < 0) return;
    }
    const GemmDesc g = BATCH ? batch[wi.x] : g0;
    if (g.M <= 0 || g.N <= 0) return;
    if (g.stop_flag != nullptr && *g.stop_flag != 0) return;
    constexpr int WAVES_M = 2, WAVES_N = NT / 128;
    constexpr int WM = BM / WAVES_M, WN = BN / WAVES_N;
    constexpr int FM = WM / 16, FN = WN / 16;
    static_assert(FM >= 1 && FN >= 1, "wave tile");
    using LoaderA = TileLoader<BM, BK, LA == 1, NT>;
    using LoaderB = TileLoader<BN, BK, LB == 0, NT>;
    extern __shared__ double smem[];
    double *As = smem;                       // two buffers of LoaderA::SIZE
    double *Bs = smem + 2 * LoaderA::SIZE;   // two buffers of LoaderB::SIZE

    int tm = wi.y, tn = wi.z;
    if (!BATCH && !PLAN && !tile_of_block(blockIdx.x, g.lower, tiles_m0, tiles_n0, sup0, tm, tn)) return;
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const bool lower_mask = g.lower || g.mask_lower;
    if (lower_mask && n0 > m0 + BM - 1 + g.mask_shift) return;  // tile entirely above the diagonal

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WAVES_N, wn = wave % WAVES_N;

    double4_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = (double4_t){0.0, 0.0, 0.0, 0.0};

    LoaderA la;
    LoaderB lb;
    const bool a_aligned = ((g.lda & 1) == 0) && ((reinterpret_cast<uintptr_t>(g.A) & 15) == 0);
    const bool b_aligned = ((g.ldb & 1) == 0) && ((reinterpret_cast<uintptr_t>(g.B) & 15) == 0);
    const bool a_rows_in = m0 + BM <= g.M, b_rows_in = n0 + BN <= g.N;

    // K range [kb, ke): all of K, or one piece of a split tile
    const bool piece = PLAN && wi.x >= 0;
    int64_t kb = 0, ke = g.K;
    if constexpr (PLAN) {
        if (piece) {
            const int64_t kp = gram_piece_k(g.K, g.split_pieces, BK);
            kb = wi.w * kp;
            ke = kb + kp < g.K ? kb + kp : g.K;
            if (kb > ke) kb = ke;
        }
    }
    const int64_t nk = (ke - kb + BK - 1) / BK;
    auto load_chunk = [&](int64_t k0) {
        const bool kin = k0 + BK <= ke;
        la.load(g.A, g.lda, m0, k0, g.M, ke, kin && a_rows_in && a_aligned);
        lb.load(g.B, g.ldb, n0, k0, g.N, ke, kin && b_rows_in && b_aligned);
    };
    auto store_chunk = [&](int buf) {
        la.store(As + buf * LoaderA::SIZE);
        lb.store(Bs + buf * LoaderB::SIZE);
    };
    const int fr = lane & 15, fk = lane >> 4;
    // MFMAs of one staged chunk (a macro so the accumulators stay registers)
#define GEMM_COMPUTE(buf)                                                                          \
    do {                                                                                           \
        const double *as_ = As + (buf) * LoaderA::SIZE;                                            \
        const double *bs_ = Bs + (buf) * LoaderB::SIZE;                                            \
        _Pragma("unroll") for (int ks = 0; ks < BK; ks += 4) {                                     \
            double a_[FM], b_[FN];                                                                 \
            _Pragma("unroll") for (int i = 0; i < FM; ++i) a_[i] =                                 \
                as_[LoaderA::at(wm * WM + i * 16 + fr, ks + fk)];                                  \
            _Pragma("unroll") for (int j = 0; j < FN; ++j) b_[j] =                                 \
                bs_[LoaderB::at(wn * WN + j * 16 + fr, ks + fk)];                                  \
            _Pragma("unroll") for (int i = 0; i < FM; ++i)                                         \
                _Pragma("unroll") for (int j = 0; j < FN; ++j) acc[i][j] =                         \
                    __builtin_amdgcn_mfma_f64_16x16x4f64(a_[i], b_[j], acc[i][j], 0, 0, 0);        \
        }                                                                                          \
    } while (0)

    bool direct_done = false;
    if constexpr (LA == 1 && LB == 0) {
        // both operands contiguous: interior tiles copy full chunks global ->
        // LDS directly (no staging registers); a ragged last chunk of K is
        // staged through registers on its own after the loop
        if (a_rows_in && b_rows_in && a_aligned && b_aligned) {
            direct_done = true;
            const int64_t nkf = (ke - kb) / BK;
            if (nkf > 0) {
                LoaderA::direct(g.A, g.lda, m0, kb, As, wave);
                LoaderB::direct(g.B, g.ldb, n0, kb, Bs, wave);
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
            }
            for (int64_t kt = 0; kt < nkf; ++kt) {
                const int cur = (int)(kt & 1);
                if (kt + 1 < nkf) {
                    LoaderA::direct(g.A, g.lda, m0, kb + (kt + 1) * BK, As + (cur ^ 1) * LoaderA::SIZE, wave);
                    LoaderB::direct(g.B, g.ldb, n0, kb + (kt + 1) * BK, Bs + (cur ^ 1) * LoaderB::SIZE, wave);
                }
                GEMM_COMPUTE(cur);
                __builtin_amdgcn_s_waitcnt(0);  // this wave's copies of the next chunk have landed
                __syncthreads();
            }
            if (nkf < nk) {
                const int buf = (int)(nkf & 1);
                load_chunk(kb + nkf * BK);
                store_chunk(buf);
                __syncthreads();
                GEMM_COMPUTE(buf);
            }
        }
    }
    if (!direct_done) {
        if (nk > 0) {
            load_chunk(kb);
            store_chunk(0);
            __syncthreads();
        }
        for (int64_t kt = 0; kt < nk; ++kt) {
            const int cur = (int)(kt & 1);
            if (kt + 1 < nk) load_chunk(kb + (kt + 1) * BK);
            GEMM_COMPUTE(cur);
            if (kt + 1 < nk) store_chunk(cur ^ 1);
            __syncthreads();
        }
    }

#undef GEMM_COMPUTE
    if (PLAN && piece) {
        // a piece of a split tile: alpha * rowscale * (its partial sum) for the
        // whole BM x BN tile (zeros outside C), summed by gram_sum_kernel
        double *W = g.split_ws + (int64_t)wi.x * (BM * BN);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int lr = wm * WM + i * 16 + fk + 4 * r;
                const int64_t gm = m0 + lr;
                const double rs = (g.rowscale && gm < g.M) ? g.rowscale[gm] : 1.0;
#pragma unroll
                for (int j = 0; j < FN; ++j) W[lr * BN + wn * WN + j * 16 + fr] = g.alpha * acc[i][j][r] * rs;
            }
        return;
    }
    // epilogue: lane l, register r holds row fk + 4 r, column fr of each
    // 16x16 block.  The loads of C and the row scales of EI block rows are
    // issued before their stores so they overlap (all rows at once unless
    // that would hold more than 8 blocks of C in registers).
    constexpr int EI = FM * FN > 8 ? 1 : FM;
#pragma unroll
    for (int i0 = 0; i0 < FM; i0 += EI) {
        double cold[EI][FN][4], rs[EI][4];
#pragma unroll
        for (int ii = 0; ii < EI; ++ii)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gm = m0 + wm * WM + (i0 + ii) * 16 + fk + 4 * r;
                rs[ii][r] = (g.rowscale && gm < g.M) ? g.rowscale[gm] : 1.0;
            }
#pragma unroll
        for (int ii = 0; ii < EI; ++ii)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int64_t gn_ = n0 + wn * WN + j * 16 + fr;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t gm = m0 + wm * WM + (i0 + ii) * 16 + fk + 4 * r;
                    const bool ok = gm < g.M && gn_ < g.N && !(lower_mask && gn_ > gm + g.mask_shift);
                    cold[ii][j][r] = (ok && g.beta != 0.0) ? g.C[gm * g.ldc + gn_] : 0.0;
                }
            }
#pragma unroll
        for (int ii = 0; ii < EI; ++ii) {
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int64_t gn_ = n0 + wn * WN + j * 16 + fr;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t gm = m0 + wm * WM + (i0 + ii) * 16 + fk + 4 * r;
                    if (gm >= g.M || gn_ >= g.N) continue;
                    if (lower_mask && gn_ > gm + g.mask_shift) continue;
                    const double v = g.alpha * acc[i0 + ii][j][r] * rs[ii][r];
                    g.C[gm * g.ldc + gn_] = (g.beta == 0.0) ? v : fma(g.beta, cold[ii][j][r], v);
                }
            }
        }
    }
}

template <int BM, int BN, int BK, int LA, int LB, bool BATCH, int NT, bool PLAN = false>
static hipError_t launch_one(hipStream_t st, const GemmDesc &g, int tiles_m, int tiles_n, int64_t blocks,
                             const GemmDesc *batch, const int4 *work) {
    constexpr size_t shm =
        sizeof(double) * 2 * (TileLoader<BM, BK, LA == 1, NT>::SIZE + TileLoader<BN, BK, LB == 0, NT>::SIZE);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)dgemm_mfma_kernel<BM, BN, BK, LA, LB, BATCH, NT, PLAN>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        attr = true;
    }
    hipLaunchKernelGGL((dgemm_mfma_kernel<BM, BN, BK, LA, LB, BATCH, NT, PLAN>), dim3((unsigned)blocks), dim3(NT),
                       shm, st, g, tiles_m, tiles_n, super_shape(g.lower, tiles_m, tiles_n), batch, work);
    return hipGetLastError();
}

template <int BM, int BN, int BK>
static int64_t blocks_for(const GemmDesc &g, int &tiles_m, int &tiles_n) {
    tiles_m = (int)((g.M + BM - 1) / BM);
    tiles_n = (int)((g.N + BN - 1) / BN);
    if (g.M <= 0 || g.N <= 0) return 0;
    const int sup = super_shape(g.lower, tiles_m, tiles_n), sup_m = sup & 0xff, sup_n = sup >> 8;
    const int64_t supers = g.lower ? lower_super_count(tiles_m)
                                   : (int64_t)((tiles_m + sup_m - 1) / sup_m) * ((tiles_n + sup_n - 1) / sup_n);
    return (supers + NXCD - 1) / NXCD * NXCD * (sup_m * sup_n);
}

template <int BM, int BN, int BK, bool BATCH, int NT = GEMM_THREADS>
static hipError_t launch_tiles(hipStream_t st, const GemmDesc &g, int64_t blocks, int tiles_m, int tiles_n,
                               const GemmDesc *batch, const int4 *work) {
    if (blocks <= 0) return hipSuccess;
    if (g.la == 0 && g.lb == 0)
        return launch_one<BM, BN, BK, 0, 0, BATCH, NT>(st, g, tiles_m, tiles_n, blocks, batch, work);
    if (g.la == 0 && g.lb == 1)
        return launch_one<BM, BN, BK, 0, 1, BATCH, NT>(st, g, tiles_m, tiles_n, blocks, batch, work);
    if (g.la == 1 && g.lb == 0)
        return launch_one<BM, BN, BK, 1, 0, BATCH, NT>(st, g, tiles_m, tiles_n, blocks, batch, work);
    return launch_one<BM, BN, BK, 1, 1, BATCH, NT>(st, g, tiles_m, tiles_n, blocks, batch, work);
}

// Tile configuration.  128 x 128 tiles when there are enough of them to
// fill the chip twice; otherwise smaller tiles (64 x 64, or 64 x 128 for an
// in-place product) so that short, latency-bound products (the panel solves
// and updates of the Cholesky) spread over more CUs.  A lower product needs
// square tiles; an in-place product (C aliasing A, the panel solve
// L21 = A21 X^T) needs one tile column spanning all of N.
hipError_t launch_dgemm(hipStream_t st, const GemmDesc &g) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    if (g.lower && g.M != g.N) return hipErrorInvalidValue;
    const bool inplace = g.C == g.A;
    if (inplace && (g.lower || g.N > 128)) return hipErrorInvalidValue;
    constexpr int64_t FILL = 2 * 256;
    auto ntiles = [&](int bm, int bn) {
        const int64_t a = (g.M + bm - 1) / bm, b = (g.N + bn - 1) / bn;
        return g.lower ? a * (a + 1) / 2 : a * b;
    };
    int tm, tn;
    if (g.lower) {
        if (ntiles(128, 128) >= FILL) {
            const int64_t b = blocks_for<128, 128, 32>(g, tm, tn);
            // the Gram (both operands J, contiguous along m / n): four-wave
            // workgroups, two per CU, so one workgroup's K-chunk barrier is
            // covered by the other's products (medium Gram 10.52 -> 10.35 ms;
            // eight waves with K chunks of 16, 10.79 ms)
            if (g.la == 1 && g.lb == 0)
                return launch_one<128, 128, 16, 1, 0, false, 256>(st, g, tm, tn, b, nullptr, nullptr);
            return launch_tiles<128, 128, 32, false>(st, g, b, tm, tn, nullptr, nullptr);
        }
        const int64_t b = blocks_for<64, 64, 32>(g, tm, tn);
        return launch_tiles<64, 64, 32, false>(st, g, b, tm, tn, nullptr, nullptr);
    }
    if (g.N <= 64) {
        if (ntiles(128, 64) >= FILL) {
            const int64_t b = blocks_for<128, 64, 32>(g, tm, tn);
            return launch_tiles<128, 64, 32, false>(st, g, b, tm, tn, nullptr, nullptr);
        }
        const int64_t b = blocks_for<64, 64, 32>(g, tm, tn);
        return launch_tiles<64, 64, 32, false>(st, g, b, tm, tn, nullptr, nullptr);
    }
    if (ntiles(128, 128) >= FILL) {
        const int64_t b = blocks_for<128, 128, 32>(g, tm, tn);
        // both operands contiguous along m / n (the Hilbert coupling product):
        // four-wave workgroups, two per CU (measured 5% faster there)
        if (g.la == 1 && g.lb == 0)
            return launch_one<128, 128, 16, 1, 0, false, 256>(st, g, tm, tn, b, nullptr, nullptr);
        return launch_tiles<128, 128, 32, false>(st, g, b, tm, tn, nullptr, nullptr);
    }
    if (inplace) {
        // 32-row tiles while they fit one round on the CUs: the panel solve is
        // bound by each CU's own MFMA rate, so halving the rows per tile halves it
        if (ntiles(32, 128) <= 256) {
            const int64_t b = blocks_for<32, 128, 32>(g, tm, tn);
            return launch_tiles<32, 128, 32, false>(st, g, b, tm, tn, nullptr, nullptr);
        }
        const int64_t b = blocks_for<64, 128, 32>(g, tm, tn);
        return launch_tiles<64, 128, 32, false>(st, g, b, tm, tn, nullptr, nullptr);
    }
    const int64_t b = blocks_for<64, 64, 32>(g, tm, tn);
    return launch_tiles<64, 64, 32, false>(st, g, b, tm, tn, nullptr, nullptr);
}

// ------------------------------------------------------ planned products
// Two tile configurations take plans: 128 x 128 tiles on four-wave
// workgroups (K chunks of 16) for the products launch_dgemm gives 128 x 128
// tiles, and 64 x 64 tiles on eight-wave workgroups (K chunks of 32) for the
// smaller ones it gives 64 x 64 tiles.  Both hold two workgroups per CU.
static constexpr int GRAM_T = 128;
static constexpr int GRAM_BK = 16;
static constexpr int SMALL_T = 64;
static constexpr int SMALL_BK = 32;
static constexpr int GRAM_MAX_PIECES = 4;

int plan_tile_size(int64_t M, int64_t N, bool lower) {
    const int64_t a = (M + GRAM_T - 1) / GRAM_T, b = lower ? a : (N + GRAM_T - 1) / GRAM_T;
    return (lower ? a * (a + 1) / 2 : a * b) >= 2 * 256 ? GRAM_T : SMALL_T;
}

int64_t gram_plan_ws_doubles(int nsplit, int pieces, int tile) { return (int64_t)nsplit * pieces * tile * tile; }

static bool plan_tiles(int64_t M, int64_t N, bool lower, int cus, std::vector<int4> &table, int64_t &nwork,
                       int &nsplit, int &pieces, int &tile) {
    table.clear();
    nwork = 0;
    nsplit = 0;
    pieces = 1;
    tile = plan_tile_size(M, N, lower);
    const int T = tile;
    const int64_t tiles_m = (M + T - 1) / T, tiles_n = lower ? tiles_m : (N + T - 1) / T;
    if (M <= 0 || N <= 0 || (lower && M != N) || tiles_m > (1 << 30) || tiles_n > (1 << 30)) return false;
    // the products launch_dgemm gives to these tile shapes: lower products, or
    // rectangular ones wider than 64 columns; the smallest ones take no plan
    const int64_t ntiles = lower ? tiles_m * (tiles_m + 1) / 2 : tiles_m * tiles_n;
    if ((!lower && N <= 64) || ntiles < 64) return false;
    if (cus <= 0 || cus % NXCD != 0) return false;
    const int64_t slots = 2 * (int64_t)(cus / NXCD);  // resident workgroups per XCD
    // 4 x 8 super-tiles in the order of tile_of_block (rows of super-tiles,
    // tiles column by column inside one), each dealt whole to the XCD with
    // the fewest tiles so far
    std::vector<std::vector<int4>> per(NXCD);
    const int64_t nsr = (tiles_m + SUP_M - 1) / SUP_M, nsc = (tiles_n + SUP_N - 1) / SUP_N;
    for (int64_t a = 0; a < nsr; ++a) {
        const int64_t c = lower ? std::min((SUP_M * a + SUP_M - 1) / SUP_N + 1, nsc) : nsc;
        for (int64_t b = 0; b < c; ++b) {
            int x = 0;
            for (int k = 1; k < NXCD; ++k)
                if (per[k].size() < per[x].size()) x = k;
            for (int i = 0; i < SUP; ++i) {
                const int64_t tm = a * SUP_M + i % SUP_M, tn = b * SUP_N + i / SUP_M;
                if (tm < tiles_m && tn < tiles_n && (!lower || tn <= tm))
                    per[x].push_back(make_int4(-1, (int)tm, (int)tn, 0));
            }
        }
    }
    // even out the counts (they differ by at most one super-tile): tiles move
    // from the ends of the longest lists to the ends of the shortest
    for (;;) {
        int lo = 0, hi = 0;
        for (int k = 1; k < NXCD; ++k) {
            if (per[k].size() < per[lo].size()) lo = k;
            if (per[k].size() > per[hi].size()) hi = k;
        }
        if (per[hi].size() <= per[lo].size() + 1) break;
        per[lo].push_back(per[hi].back());
        per[hi].pop_back();
    }
    // pieces: the count (1 to 4) that makes the slowest XCD's last round
    // shortest, that round's r tiles becoming r * pieces units of 1 / pieces
    // of a tile's time on the XCD's slots (the fewest pieces among equals)
    int pc = 1;
    bool any = false;
    double best = 0.0;
    for (int q = 1; q <= GRAM_MAX_PIECES; ++q) {
        double worst = 0.0;
        for (int x = 0; x < NXCD; ++x) {
            const int64_t r = (int64_t)per[x].size() % slots;
            if (r == 0) continue;
            any = true;
            worst = std::max(worst, (double)((r * q + slots - 1) / slots) / q);
        }
        if (q == 1 || worst < best - 1e-9) {
            best = worst;
            pc = q;
        }
    }
    std::vector<int4> fix;
    if (any && pc >= 2) {
        pieces = pc;
        for (int x = 0; x < NXCD; ++x) {
            const int64_t n = (int64_t)per[x].size(), r = n % slots;
            per[x].reserve((size_t)(n + r * (pieces - 1)));
            for (int64_t i = n - r; i < n; ++i) {
                // copies: the appends below may move the list
                const int unit = nsplit * pieces, tm = per[x][i].y, tn = per[x][i].z;
                per[x][i].x = unit;
                fix.push_back(make_int4(unit, tm, tn, 0));
                for (int q = 1; q < pieces; ++q) per[x].push_back(make_int4(unit + q, tm, tn, q));
                ++nsplit;
            }
        }
    }
    size_t len = 0;
    for (auto &v : per) len = std::max(len, v.size());
    table.assign(len * NXCD, make_int4(-1, -1, 0, 0));
    for (int x = 0; x < NXCD; ++x)
        for (size_t q = 0; q < per[x].size(); ++q) table[q * NXCD + x] = per[x][q];
    nwork = (int64_t)table.size();
    table.insert(table.end(), fix.begin(), fix.end());
    return true;
}

bool plan_gram(int64_t M, int cus, std::vector<int4> &table, int64_t &nwork, int &nsplit, int &pieces, int &tile) {
    return plan_tiles(M, M, true, cus, table, nwork, nsplit, pieces, tile);
}

bool plan_rect(int64_t M, int64_t N, int cus, std::vector<int4> &table, int64_t &nwork, int &nsplit, int &pieces,
               int &tile) {
    return plan_tiles(M, N, false, cus, table, nwork, nsplit, pieces, tile);
}

// C = beta C + (sum of the pieces of each split tile, in piece order), the
// lower part only for a lower product.  Each split tile is summed by
// T / SUM_ROWS workgroups of SUM_ROWS rows, every thread issuing the
// loads of all its entries of a piece before adding them.
static constexpr int SUM_ROWS = 16;
template <int T>
__global__ __launch_bounds__(256) void gram_sum_kernel(GemmDesc g, const int4 *__restrict__ tiles) {
    if (g.stop_flag != nullptr && *g.stop_flag != 0) return;
    constexpr int PARTS = T / SUM_ROWS, PER = SUM_ROWS * T / 256;
    const int4 t = tiles[blockIdx.x / PARTS];
    const int base = (blockIdx.x % PARTS) * SUM_ROWS * T + threadIdx.x;  // entry of the tile, row-major
    const double *W = g.split_ws + (int64_t)t.x * (T * T);
    double v[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) v[e] = W[base + e * 256];
    for (int q = 1; q < g.split_pieces; ++q) {
        double w[PER];
#pragma unroll
        for (int e = 0; e < PER; ++e) w[e] = W[(int64_t)q * (T * T) + base + e * 256];
#pragma unroll
        for (int e = 0; e < PER; ++e) v[e] += w[e];
    }
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int idx = base + e * 256;
        const int64_t gm = (int64_t)t.y * T + idx / T, gn_ = (int64_t)t.z * T + idx % T;
        if (gm >= g.M || gn_ >= g.N || (g.lower && gn_ > gm)) continue;
        double *c = g.C + gm * g.ldc + gn_;
        *c = g.beta == 0.0 ? v[e] : fma(g.beta, *c, v[e]);
    }
}

hipError_t launch_planned(hipStream_t st, const GemmDesc &g, const TilePlan &p) {
    if (p.M <= 0 || p.d_work == nullptr || p.nwork <= 0 || g.M != p.M || g.N != p.N || (g.lower != 0) != p.lower ||
        g.la != 1 || g.lb != 0 || g.mask_lower || g.mask_shift != 0 || g.C == g.A || g.C == g.B)
        return launch_dgemm(st, g);
    if (p.nsplit > 0 && (p.ws == nullptr || p.pieces < 2)) return hipErrorInvalidValue;
    if (p.tile != GRAM_T && p.tile != SMALL_T) return hipErrorInvalidValue;
    GemmDesc q = g;
    q.split_ws = p.ws;
    q.split_pieces = p.pieces;
    const bool big = p.tile == GRAM_T;
    hipError_t e = big ? launch_one<GRAM_T, GRAM_T, GRAM_BK, 1, 0, false, 256, true>(st, q, 0, 0, p.nwork, nullptr,
                                                                                      p.d_work)
                       : launch_one<SMALL_T, SMALL_T, SMALL_BK, 1, 0, false, GEMM_THREADS, true>(st, q, 0, 0, p.nwork,
                                                                                                 nullptr, p.d_work);
    if (e != hipSuccess || p.nsplit == 0) return e;
    if (big)
        hipLaunchKernelGGL(gram_sum_kernel<GRAM_T>, dim3((unsigned)(p.nsplit * (GRAM_T / SUM_ROWS))), dim3(256), 0, st,
                           q, p.d_work + p.nwork);
    else
        hipLaunchKernelGGL(gram_sum_kernel<SMALL_T>, dim3((unsigned)(p.nsplit * (SMALL_T / SUM_ROWS))), dim3(256), 0,
                           st, q, p.d_work + p.nwork);
    return hipGetLastError();
}

// Batched tile configuration: 128 x 64 tiles for narrow rectangular products
// (in-place triangular solves need one tile column), 32 x 128 for products of
// at most 32 rows (the few last rows of bordered Grams), else 128 x 128.
enum BatchedShape { BS_SQUARE = 0, BS_SMALL_N = 1, BS_THIN = 2 };
static int batched_shape(const GemmDesc &f) {
    if (f.lower) return BS_SQUARE;
    if (f.N <= 64) return BS_SMALL_N;
    return f.M <= 32 ? BS_THIN : BS_SQUARE;
}

int64_t plan_dgemm_batched(const GemmDesc *descs, int n, std::vector<int4> &table) {
    table.clear();
    if (n <= 0) return 0;
    const GemmDesc &f = descs[0];
    const int shape = batched_shape(f);
    const int BM = shape == BS_THIN ? 32 : 128, BN = shape == BS_SMALL_N ? 64 : 128;
    for (int i = 0; i < n; ++i) {
        const GemmDesc &g = descs[i];
        if (g.la != f.la || g.lb != f.lb || g.lower != f.lower || batched_shape(g) != shape) return -1;
        if (g.lower && g.M != g.N) return -1;
    }
    // chunks: a block of tiles of one problem that share operand panels, 4 x 8
    // tiles, or smaller when that leaves fewer than 8 chunks per XCD
    struct Chunk { double cost; int inst; std::vector<int4> tiles; };
    std::vector<Chunk> chunks;
    static const int shapes[3][2] = {{SUP_M, SUP_N}, {2, 4}, {1, 1}};
    for (const auto &sh : shapes) {
        const int cm = sh[0], cn = sh[1];
        chunks.clear();
        for (int i = 0; i < n; ++i) {
            const GemmDesc &g = descs[i];
            if (g.M <= 0 || g.N <= 0) continue;
            const int tm_n = (int)((g.M + BM - 1) / BM), tn_n = (int)((g.N + BN - 1) / BN);
            const double per_tile = (double)(g.K > 0 ? g.K : 0) + 64.0;  // K loop plus epilogue
            for (int sm = 0; sm * cm < tm_n; ++sm)
                for (int sn = 0; sn * cn < tn_n; ++sn) {
                    Chunk c{0.0, i, {}};
                    for (int t = 0; t < cm * cn; ++t) {
                        const int tm = sm * cm + t % cm, tn = sn * cn + t / cm;
                        if (tm >= tm_n || tn >= tn_n) continue;
                        if ((g.lower || g.mask_lower) && (int64_t)tn * BN > (int64_t)tm * BM + BM - 1 + g.mask_shift)
                            continue;
                        c.tiles.push_back(make_int4(i, tm, tn, 0));
                    }
                    if (c.tiles.empty()) continue;
                    c.cost = per_tile * (double)c.tiles.size();
                    chunks.push_back(std::move(c));
                }
        }
        if (chunks.size() >= 8 * NXCD) break;
    }
    // longest-processing-time assignment of chunks to XCDs; inside an XCD the
    // hardware hands tiles to free CUs in table order, costliest chunks first
    std::stable_sort(chunks.begin(), chunks.end(), [](const Chunk &a, const Chunk &b) { return a.cost > b.cost; });
    std::vector<std::vector<int4>> per(NXCD);
    double load[NXCD] = {0};
    for (const Chunk &c : chunks) {
        int x = 0;
        for (int k = 1; k < NXCD; ++k)
            if (load[k] < load[x]) x = k;
        load[x] += c.cost;
        per[x].insert(per[x].end(), c.tiles.begin(), c.tiles.end());
    }
    size_t len = 0;
    for (auto &v : per) len = v.size() > len ? v.size() : len;
    table.assign(len * NXCD, make_int4(-1, 0, 0, 0));
    for (int x = 0; x < NXCD; ++x)
        for (size_t p = 0; p < per[x].size(); ++p) table[p * NXCD + x] = per[x][p];
    return (int64_t)table.size();
}

hipError_t launch_dgemm_batched(hipStream_t st, const GemmDesc *h_descs, const GemmDesc *d_descs, int n,
                                const int4 *d_work, int64_t nwork) {
    if (n <= 0 || nwork <= 0) return hipSuccess;
    const GemmDesc &f = h_descs[0];
    const int shape = batched_shape(f);
    if (shape == BS_SMALL_N) return launch_tiles<128, 64, 32, true>(st, f, nwork, 0, 0, d_descs, d_work);
    if (shape == BS_THIN) return launch_tiles<32, 128, 32, true>(st, f, nwork, 0, 0, d_descs, d_work);
    // coupling products (both operands contiguous along m / n): the four-wave
    // configuration, two workgroups per CU (64 instances of the small CCF
    // workload: 27.8 -> 26.1 ms per batch step); the batched Grams keep eight
    // waves (21.5 ms against 21.9 ms with four)
    if (f.la == 1 && f.lb == 0 && !f.lower)
        return launch_one<128, 128, 16, 1, 0, true, 256>(st, f, 0, 0, nwork, d_descs, d_work);
    return launch_tiles<128, 128, 32, true>(st, f, nwork, 0, 0, d_descs, d_work);
}

hipError_t batched_plan_upload(BatchedGemmPlan &p) {
    batched_plan_free(p);
    const int n = (int)p.h_descs.size();
    if (plan_dgemm_batched(p.h_descs.data(), n, p.h_work) < 0) return hipErrorInvalidValue;
    if (n == 0 || p.h_work.empty()) return hipSuccess;
    hipError_t e = hipMalloc((void **)&p.d_descs, sizeof(GemmDesc) * n);
    if (e == hipSuccess) e = hipMalloc((void **)&p.d_work, sizeof(int4) * p.h_work.size());
    if (e == hipSuccess) e = hipMemcpy(p.d_descs, p.h_descs.data(), sizeof(GemmDesc) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p.d_work, p.h_work.data(), sizeof(int4) * p.h_work.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) batched_plan_free(p);
    return e;
}

void batched_plan_free(BatchedGemmPlan &p) {
    if (p.d_descs) (void)hipFree(p.d_descs);
    if (p.d_work) (void)hipFree(p.d_work);
    p.d_descs = nullptr;
    p.d_work = nullptr;
}

hipError_t launch_batched_plan(hipStream_t st, const BatchedGemmPlan &p) {
    if (p.h_descs.empty() || p.h_work.empty()) return hipSuccess;
    if (!p.d_descs || !p.d_work) return hipErrorInvalidValue;
    return launch_dgemm_batched(st, p.h_descs.data(), p.d_descs, (int)p.h_descs.size(), p.d_work,
                                (int64_t)p.h_work.size());
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

__global__ void gemv_t_final(const double *__restrict__ work, int64_t p, double *__restrict__ g, int accumulate) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= p) return;
    double acc = 0.0;
    for (int k = 0; k < GEMV_CHUNKS; ++k) acc += work[k * p + c];
    g[c] = accumulate ? g[c] + acc : acc;
}

hipError_t launch_gemv_t(hipStream_t st, const double *J, int64_t m, int64_t p, int64_t ldj, const double *r,
                         double *g, double *work, int accumulate) {
    if (p <= 0) return hipSuccess;
    dim3 g1((unsigned)((p + 255) / 256), GEMV_CHUNKS);
    hipLaunchKernelGGL(gemv_t_partial, g1, dim3(256), 0, st, J, m, p, ldj, r, work);
    hipLaunchKernelGGL(gemv_t_final, dim3((unsigned)((p + 255) / 256)), dim3(256), 0, st, work, p, g, accumulate);
    return hipGetLastError();
}

}  // namespace gn
