// chol_block.h -- factorisation of one 128 x 128 diagonal block of the
// blocked Cholesky in LDS, with the inverse of its triangular factor, by one
// workgroup of four or eight waves (k_solve.hip: the single and batched
// diagonal-block kernels).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "gn_internal.h"

namespace gn {

static constexpr int CB = 128;         // diagonal block width of the blocked Cholesky
static constexpr int LDS_LD = CB + 1;  // padded LDS row stride (doubles)
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
__device__ __forceinline__ double4_t lds_mfma(double4_t acc, FA a_at, FB b_at, int kbeg, int lane = threadIdx.x & 63) {
    const int fr = lane & 15, fk = lane >> 4;
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

// The lane index through an opaque copy: the work that waves 1-3 do between
// the leaves computes its LDS and global addresses where it runs instead of
// having them hoisted to the kernel's start and kept live (spilled) across
// the leaves.
__device__ __forceinline__ int opaque_lane() {
    int l = threadIdx.x & 63;
    asm volatile("" : "+v"(l));
    return l;
}

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

// Wave-local ordering of LDS traffic: the wave's LDS writes have landed
// before its next LDS reads (other lanes of the same wave read them).
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
}

// Rows [R0, R0 + ROWS) of the kb x kb diagonal block into LDS by NT threads
// (thread index t in [0, NT)): every thread issues all of its loads before
// any LDS store (indices clamped into the block, values selected after), so
// no load waits behind a branch; rows >= kb become identity padding.
template <int R0, int ROWS, int NT>
__device__ __forceinline__ void load_block_rows(const double *A, int64_t lda, int64_t k0, int kb, double *s, int t) {
    constexpr int E = ROWS * CB / NT;
    static_assert(E * NT == ROWS * CB, "rows split evenly over the threads");
    double v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int idx = t + e * NT, r = R0 + idx / CB, c = idx % CB;
        const int rc = r < kb ? r : kb - 1, cc = c < kb ? c : kb - 1;
        v[e] = A[(k0 + rc) * lda + k0 + cc];
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int idx = t + e * NT, r = R0 + idx / CB, c = idx % CB;
        v[e] = (r < kb && c <= r) ? v[e] : ((r >= kb && r == c) ? 1.0 : 0.0);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int idx = t + e * NT, r = R0 + idx / CB, c = idx % CB;
        s[r * LDS_LD + c] = v[e];
    }
}

// One 16x16 lower tile of the trailing update by the 32 columns [o, o + IB):
// A[r][c] -= sum_k L[r][o+k] L[c][o+k] over the region [o + IB, CB)^2, tile t
// of its lower tiles in row order (t = 0, 1, 2 are the next diagonal block).
__device__ __forceinline__ void trail_tile(double *s, int o, int t) {
    const int lane = opaque_lane(), fr = lane & 15, fk = lane >> 4;
    const int r0 = o + IB;
    int ti = 0;
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    const int tj = t - ti * (ti + 1) / 2;
    const int rm = r0 + 16 * ti, cn = r0 + 16 * tj;
    double4_t acc = (double4_t){0.0, 0.0, 0.0, 0.0};
    acc = lds_mfma<IB>(
        acc, [&](int m, int k) { return LL(rm + m, o + k); }, [&](int k, int n) { return LL(cn + n, o + k); }, 0, lane);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = rm + fk + 4 * r, col = cn + fr;
        if (col <= row) LL(row, col) -= acc[r];
    }
}

// A 32x32 block product in LDS, acc[2 ti + tj] (its four 16x16 tiles) +=
// A(32 x KN) B(KN x 32) over k in [kbeg, kbeg + KN): per k-step the two A and
// two B fragments feed four independent MFMAs; all fragments are loaded
// before the first MFMA.
template <int KN, class FA, class FB>
__device__ __forceinline__ void lds_mfma_32x32(double4_t (&acc)[4], FA a_at, FB b_at, int kbeg, int lane) {
    const int fr = lane & 15, fk = lane >> 4;
    constexpr int NQ = KN / 4;
    double a0[NQ], a1[NQ], b0[NQ], b1[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int k = kbeg + 4 * q + fk;
        a0[q] = a_at(fr, k);
        a1[q] = a_at(16 + fr, k);
        b0[q] = b_at(k, fr);
        b1[q] = b_at(k, 16 + fr);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[q], b0[q], acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[q], b1[q], acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[q], b0[q], acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[q], b1[q], acc[3], 0, 0, 0);
    }
}

// Off-diagonal blocks X_rs (r > s, 32x32) of the inverse of the block's
// factor, from the blocks of earlier rows: X_rs = -X_rr W with
// W = sum_{k=s}^{r-1} L_rk X_ks, by one wave.
// w_sum_wave forms the part of W over the 32-wide k-blocks [kb0, kb1), into
// a 32 x 33 slot Wq, or (Wq null) into the storage of X_rs itself, which is
// free until X_rs is written.
__device__ __forceinline__ void w_sum_wave(double *s, double *Wq, int r, int sblk, int kb0, int kb1) {
    const int lane = opaque_lane(), fr = lane & 15, fk = lane >> 4;
    const int ro = r * IB, so = sblk * IB;
    double4_t acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = (double4_t){0.0, 0.0, 0.0, 0.0};
    for (int kk = kb0 * IB; kk < kb1 * IB; kk += IB)
        lds_mfma_32x32<IB>(
            acc, [&](int m, int k) { return LL(ro + m, k); },
            [&](int k, int n) { return sel(k >= so + n, XX(k, so + n)); }, kk, lane);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int m = 16 * (t >> 1) + fk + 4 * q, n = 16 * (t & 1) + fr;
            if (Wq)
                Wq[m * (IB + 1) + n] = acc[t][q];
            else
                XX(ro + m, so + n) = acc[t][q];
        }
    wave_lds_fence();
}

// X_rs = -X_rr W with W the sum of the slot Wq (if not null) and, if
// in_place, of the partial sum held in X_rs's own storage (read in full
// before X_rs is written).
__device__ __forceinline__ void x_from_w_wave(double *s, const double *Wq, bool in_place, int r, int sblk) {
    const int lane = opaque_lane(), fr = lane & 15, fk = lane >> 4;
    const int ro = r * IB, so = sblk * IB;
    double4_t acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = (double4_t){0.0, 0.0, 0.0, 0.0};
    lds_mfma_32x32<IB>(
        acc, [&](int m, int k) { return sel(k <= m, XX(ro + m, ro + k)); },
        [&](int k, int n) {
            const double w = Wq ? Wq[k * (IB + 1) + n] : 0.0;
            return in_place ? w + XX(ro + k, so + n) : w;
        },
        0, lane);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) XX(ro + 16 * (t >> 1) + fk + 4 * q, so + 16 * (t & 1) + fr) = -acc[t][q];
    wave_lds_fence();
}

// Block (rb, cb) of X = L^{-1} (32x32, row-major CB x CB in global memory;
// zero outside the factor and on the border row/column) by one wave.
__device__ __forceinline__ void store_x_block(double *X, const double *s, int rb, int cb, int kb, int bi) {
    const int lane = opaque_lane();
    if (cb > rb) {  // above the diagonal: zeros
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int e = lane + 64 * q;
            X[(rb * IB + e / IB) * CB + cb * IB + e % IB] = 0.0;
        }
        return;
    }
    double xv[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = lane + 64 * q, i = rb * IB + e / IB, c = cb * IB + e % IB;
        xv[q] = XX(i, c);
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = lane + 64 * q, i = rb * IB + e / IB, c = cb * IB + e % IB;
        const bool valid = c <= i && i < kb && i != bi && c != bi;
        X[i * CB + c] = valid ? xv[q] : 0.0;
    }
}

// Block column cb of L (rows 32 cb .. kb - 1, lower part) to A by nt threads
// (thread index t), 16 elements a time: LDS reads first, then the stores.
__device__ __forceinline__ void store_l_column(double *A, int64_t lda, int64_t k0, int kb, const double *s, int cb,
                                               int t, int nt) {
    const int n = (CB - cb * IB) * IB;
    constexpr int SG = 16;
    for (int e0 = t; e0 < n; e0 += SG * nt) {
        double lv[SG];
#pragma unroll
        for (int e = 0; e < SG; ++e) {
            const int idx = e0 + e * nt, r = cb * IB + idx / IB, c = cb * IB + idx % IB;
            lv[e] = idx < n ? LL(r, c) : 0.0;
        }
#pragma unroll
        for (int e = 0; e < SG; ++e) {
            const int idx = e0 + e * nt, r = cb * IB + idx / IB, c = cb * IB + idx % IB;
            if (idx < n && r < kb && c <= r) A[(k0 + r) * lda + k0 + c] = lv[e];
        }
    }
}

// Factor one CB x CB diagonal block (rows/cols k0 .. k0+kb) of A and form X =
// L^{-1} of the block (row-major CB x CB, zero outside the factor and on the
// border row/column).  Right-looking over four 32-wide sub-blocks: wave 0
// runs the leaf factorisation of sub-block b (with the inverse of its
// diagonal block) while waves 1-3 do the work that waits on nothing newer:
// the first leaf overlaps the load of rows 32-127; the later ones overlap the
// previous sub-block's trailing update below the next diagonal block, the
// off-diagonal blocks of X in row b - 1 (X_rs = -X_rr sum_{k=s}^{r-1} L_rk X_ks,
// one wave per block) and the stores of L's block column b - 1 and of X's
// block row b - 1; the last leaf also overlaps the sums of X's last block
// row, which leaves one 32 x 32 x 32 product per wave after it.  Between the leaves all four waves solve the sub-panel
// below the leaf and update the next 32 x 32 diagonal block, as 16x16 FP64
// MFMA tiles from LDS.
// LDS: s holds CB x LDS_LD doubles, colbuf 2 KS 64 (16-byte aligned; also
// the leaf's 16 x 17 coupling buffer), W (CB/IB - 1) IB (IB + 1) (one 32 x 33
// slot per wave that forms an X block), fail_sh one int.  Four waves.
static constexpr int POTRF_COLBUF = 2 * KS * 64;
static constexpr int POTRF_W = (CB / IB - 1) * IB * (IB + 1);
template <int NTH>
__device__ __forceinline__ void potrf_block_body(double *A, int64_t lda, int64_t k0, int kb, int border_here, double *X,
                                                 DevStatus *status, double *s, double *colbuf, double *W,
                                                 int &fail_sh) {
    static_assert(NTH == 256, "four waves: the leaves on wave 0, the deferred work on waves 1-3");
    constexpr int NW = NTH / 64, NB = CB / IB, WSLOT = IB * (IB + 1);
    if (status->flag) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: loops over tiles stay scalar
    const int fr = lane & 15, fk = lane >> 4;
    const int bi = border_here ? kb - 1 : -1;
    // rows of the first sub-block (the rest is loaded during the first leaf)
    load_block_rows<0, IB, NTH>(A, lda, k0, kb, s, tid);
    if (tid < CB) s[tid * LDS_LD + CB] = 0.0;
    __syncthreads();
#pragma nounroll
    for (int sb = 0; sb < NB; ++sb) {
        const int o = sb * IB;
        if (wave == 0) {
            const int lb = (bi >= o && bi < o + IB) ? bi - o : -1;
            const int f = potrf32_wave(s, o, lb, colbuf, colbuf);
            if (lane == 0) fail_sh = f < 0 ? -1 : o + f;
        } else {
            // opaque copies: keeps the compiler from hoisting this branch's
            // per-thread address arithmetic out of the loop (it would stay live
            // across the leaves and spill)
            int wt = tid - 64;
            double *Ab = A, *Xb = X;
            int64_t k0b = k0, ldab = lda;
            asm volatile("" : "+v"(wt), "+s"(Ab), "+s"(Xb), "+s"(k0b), "+s"(ldab));
            const int w1 = wave - 1;
            constexpr int WN = NTH - 64;
            if (sb == 0) {
                load_block_rows<IB, CB - IB, WN>(Ab, ldab, k0b, kb, s, wt);
            } else {
                const int ob = o - IB, r = sb - 1;
                // trailing update by block column ob below the diagonal block sb, on
                // the waves that form no X block of row r
                const int nt = (CB - o) / 16, nlow = nt * (nt + 1) / 2;
                if (w1 >= r)
                    for (int t = 3 + w1 - r; t < nlow; t += NW - 1 - r) trail_tile(s, ob, t);
                double *Wq = W + w1 * WSLOT;
                if (sb < NB - 1) {
                    // block row r of X: X_{r,w1} (w1 < r) by wave w1 + 1, then the rest of
                    // the row (X_rr and the zero blocks) and L's block column r
                    if (w1 < r) {
                        w_sum_wave(s, Wq, r, w1, w1, r);
                        x_from_w_wave(s, Wq, false, r, w1);
                        store_x_block(Xb, s, r, w1, kb, bi);
                    }
                    for (int c = r + w1; c < NB; c += NW - 1) store_x_block(Xb, s, r, c, kb, bi);
                    store_l_column(Ab, ldab, k0b, kb, s, r, wt, WN);
                } else if (w1 < r) {
                    // during the last leaf (r = 2), the sums behind X's last block row
                    // X_3s = -X_33 W_3s, W_3s = sum_{k=s}^{2} L_3k X_ks, spread so that
                    // each wave does 96-128 MFMAs: wave 1 forms X_20 and the k = 2 term
                    // of W_30 (slot 0); wave 2 forms X_21 and all of W_31 (slot 1)
                    w_sum_wave(s, Wq, r, w1, w1, r);
                    x_from_w_wave(s, Wq, false, r, w1);
                    store_x_block(Xb, s, r, w1, kb, bi);
                    w_sum_wave(s, Wq, r + 1, w1, w1 == 0 ? r : w1, r + 1);
                } else {
                    // wave 3: the k < 2 part of W_30 and all of W_32, each in the storage
                    // of its block, then the rest of X's row r and L's column r
                    w_sum_wave(s, nullptr, r + 1, 0, 0, r);
                    w_sum_wave(s, nullptr, r + 1, r, r, r + 1);
                    for (int c = r; c < NB; ++c) store_x_block(Xb, s, r, c, kb, bi);
                    store_l_column(Ab, ldab, k0b, kb, s, r, lane, 64);
                }
            }
        }
        __syncthreads();
        if (fail_sh >= 0) {
            if (tid == 0) {
                status->chol_info = k0 + fail_sh + 1;
                status->flag = 1;
            }
            return;
        }
        if (sb == NB - 1) break;
        const int r0 = o + IB, nr = CB - r0;
        // sub-panel: L[r][o+j] = sum_{k<=j} A[r][o+k] X[o+j][o+k]; (nr/16) x 2 tiles, at most 12 / NW per wave
        {
            constexpr int QT = (12 + NW - 1) / NW;
            double4_t acc[QT];
            const int ntile = (nr / 16) * 2;
#pragma unroll
            for (int q = 0; q < QT; ++q) {
                acc[q] = (double4_t){0.0, 0.0, 0.0, 0.0};
                const int t = wave + NW * q;
                if (t < ntile) {
                    const int rm = r0 + 16 * (t >> 1), cn = o + 16 * (t & 1);
                    acc[q] = lds_mfma<IB>(
                        acc[q], [&](int m, int k) { return LL(rm + m, o + k); },
                        [&](int k, int n) { return sel(o + k <= cn + n, XX(cn + n, o + k)); }, 0);
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < QT; ++q) {
                const int t = wave + NW * q;
                if (t < ntile) {
                    const int rm = r0 + 16 * (t >> 1), cn = o + 16 * (t & 1);
#pragma unroll
                    for (int r = 0; r < 4; ++r) LL(rm + fk + 4 * r, cn + fr) = acc[q][r];
                }
            }
        }
        __syncthreads();
        // the next diagonal block's part of the trailing update (the rest
        // runs on waves 1-3 during the next leaf)
        if (wave < 3) trail_tile(s, o, wave);
        __syncthreads();
    }
    // block row NB - 1 of X from the sums formed during the last leaf (one
    // block per wave) and the last block column of L
    const int r = NB - 1;
    double *Af = A, *Xf = X;
    asm volatile("" : "+s"(Af), "+s"(Xf));  // computed here, not kept live from the start
    if (wave < r) {
        // X_30: slot 0 plus its own storage; X_31: slot 1; X_32: its own storage
        x_from_w_wave(s, wave < 2 ? W + wave * WSLOT : nullptr, wave != 1, r, wave);
        store_x_block(Xf, s, r, wave, kb, bi);
    } else {
        store_x_block(Xf, s, r, r, kb, bi);
        store_l_column(Af, lda, k0, kb, s, r, lane, 64);
    }
}


#undef LL
#undef XX

}  // namespace gn
