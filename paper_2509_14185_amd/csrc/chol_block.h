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
template <int D, int NW>
__device__ __forceinline__ void x_blocks_at_distance(double *s, double *W, int wave) {
    const int lane = threadIdx.x & 63, fr = lane & 15, fk = lane >> 4;
    constexpr int NBLK = CB / IB - D, NTILE = NBLK * 4;
    for (int t = wave; t < NTILE; t += NW) {
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
    for (int t = wave; t < NTILE; t += NW) {
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
// LDS: s holds CB x LDS_LD doubles, colbuf 2 KS 64 (16-byte aligned), W
// (CB/IB - 1) IB (IB + 1), fail_sh one int; NTH threads (4 or 8 waves; the
// leaf factorisations run on wave 0, every wave takes part in the barriers).
static constexpr int POTRF_COLBUF = 2 * KS * 64;
static constexpr int POTRF_W = (CB / IB - 1) * IB * (IB + 1);
template <int NTH>
__device__ __forceinline__ void potrf_block_body(double *A, int64_t lda, int64_t k0, int kb, int border_here, double *X,
                                                 DevStatus *status, double *s, double *colbuf, double *W,
                                                 int &fail_sh) {
    static_assert(NTH == 256 || NTH == 512, "four or eight waves");
    constexpr int NW = NTH / 64;
    if (status->flag) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: loops over tiles stay scalar
    const int fr = lane & 15, fk = lane >> 4;
    const int bi = border_here ? kb - 1 : -1;
    {
        // all 64 loads of a thread are issued before any LDS store: every lane
        // loads (indices clamped into the kb x kb block), selects afterwards,
        // so no load sits behind a branch and a wait for the one before it
        double v[CB * CB / NTH];
#pragma unroll
        for (int e = 0; e < CB * CB / NTH; ++e) {
            const int idx = tid + e * NTH, r = idx / CB, c = idx % CB;
            const int rc = r < kb ? r : kb - 1, cc = c < kb ? c : kb - 1;
            v[e] = A[(k0 + rc) * lda + k0 + cc];
        }
#pragma unroll
        for (int e = 0; e < CB * CB / NTH; ++e) {
            const int idx = tid + e * NTH, r = idx / CB, c = idx % CB;
            v[e] = (r < kb && c <= r) ? v[e] : ((r >= kb && r == c) ? 1.0 : 0.0);
        }
#pragma unroll
        for (int e = 0; e < CB * CB / NTH; ++e) {
            const int idx = tid + e * NTH, r = idx / CB, c = idx % CB;
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
        // trailing update (lower tiles): A[r][c] -= sum_k L[r][o+k] L[c][o+k]
        {
            const int nt = nr / 16, nlow = nt * (nt + 1) / 2;
            for (int t = wave; t < nlow; t += NW) {
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
    x_blocks_at_distance<1, NW>(s, W, wave);
    x_blocks_at_distance<2, NW>(s, W, wave);
    x_blocks_at_distance<3, NW>(s, W, wave);
    // ---- write L (rows < kb) and X (zero outside the factor) to global memory,
    //      16 elements a time: all LDS reads first, then the stores
    constexpr int SG = 16;
#pragma unroll 1
    for (int e0 = 0; e0 < CB * CB / NTH; e0 += SG) {
        double lv[SG], xv[SG];
#pragma unroll
        for (int e = 0; e < SG; ++e) {
            const int idx = tid + (e0 + e) * NTH, r = idx / CB, c = idx % CB;
            lv[e] = LL(r, c);
            xv[e] = XX(r, c);
        }
#pragma unroll
        for (int e = 0; e < SG; ++e) {
            const int idx = tid + (e0 + e) * NTH, r = idx / CB, c = idx % CB;
            if (r < kb && c <= r) A[(k0 + r) * lda + k0 + c] = lv[e];
            const bool valid = c <= r && r < kb && r != bi && c != bi;
            X[idx] = valid ? xv[e] : 0.0;
        }
    }
}


#undef LL
#undef XX

}  // namespace gn
