// Gram G = J^T J (lower triangle) to FP64 accuracy from int8 matrix products,
// by exact modular arithmetic (the Ozaki scheme II of Ozaki, Uchino and
// Imamura, 2025, specialised to a symmetric product).
//
// Why: the Gram is the dominant contraction of the full Gauss-Newton step
// (paper, Methods, "Second-order Optimizer").  On gfx950 the int8 matrix
// cores run 64 times as many operations per cycle as the FP64 ones.
//
// Steps (J is m x p, row-major, FP64):
//   1. Column exponents.  E_j = ilogb(max_i |J_ij|) + 1, so that
//      max_i |J_ij| 2^-E_j lies in [1/2, 1).
//   2. Integers.  x_ij = rint(J_ij 2^(b - E_j)), |x_ij| <= 2^b, with b chosen
//      so that m 2^(2b) < M / 4, M = prod_t m_t.  This rounding is the only
//      inexact step: each entry keeps b bits below its column's maximum.
//   3. Residues.  For each of the T pairwise coprime moduli m_t <= 256,
//      r_t = x mod m_t in the balanced range [-128, 127], stored as int8 with
//      the row index i contiguous (R_t[j][i]).
//   4. Products.  C_t = R_t R_t^T with v_mfma_i32_16x16x64_i8: |r r'| <= 2^14
//      and K <= 130944 keep the int32 sums exact; y_t = C_t mod m_t in [0, m_t).
//   5. Reconstruction (Chinese remainder theorem).  v = sum_i x_ij x_ik is the
//      unique integer with |v| < M/2 and v = y_t (mod m_t):
//        v = sum_t y_t W_t - Q M,  W_t = (M/m_t) ((M/m_t)^-1 mod m_t),
//      Q = rint(sum_t y_t W_t / M) from FP64 fractions f_t = W_t / M (its
//      error is far below the margin 1/2 - |v|/M >= 1/4), and the difference
//      evaluated exactly in four 40-bit limbs held in FP64, normalised by
//      exact carries.  G_jk = v 2^(E_j + E_k - 2b), summed from the limbs in
//      FP64 (within 2 ulp of the exact value).
//
// A column whose maximum is not finite gives NaN in every entry of its row
// and column of G.
//
// Fragment layout of v_mfma_i32_16x16x64_i8 (wave64): lane l holds 16 bytes
// of row l%16 of A and of column l%16 of B, at the same 16 positions of the
// 64-deep k range for both (which positions does not matter: the product
// pairs A and B byte for byte); D (16x16): lane l, register r holds
// D[4*(l/16) + r][l%16].
#include "gn_internal.h"

#include <cmath>

namespace gn {

typedef int int4v __attribute__((ext_vector_type(4)));

// 16 pairwise coprime moduli (2^8, 3*5*17, 11*23, 13*19 and primes);
// M = 2^125.19.
static constexpr int MODS = 16;
static constexpr int MODULI[MODS] = {256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 211, 199, 197, 193, 191};

static constexpr int MG_BM = 256;        // output tile (rows and columns)
static constexpr int MG_BK = 128;        // k bytes per LDS stage (two MFMA depths of 64)
static constexpr int MG_STAGES = 2;      // LDS ring: copies run one stage ahead
static constexpr int MG_WM = 2, MG_WN = 4;     // 8 waves, 128 x 64 each
static constexpr int MG_NT = MG_WM * MG_WN * 64;
static constexpr int MG_LDS_BYTES = MG_STAGES * 2 * MG_BM * MG_BK;  // [stage][A, B]
// s_waitcnt immediate (gfx9 encoding) that waits for vmcnt <= n and leaves
// expcnt and lgkmcnt unconstrained
#define MG_VMCNT(n) ((((n) & 0xf) | (((n) >> 4) << 14)) | (0x7 << 4) | (0xf << 8))
static constexpr int MG_NXCD = 8;
static constexpr int64_t MG_K_LIMIT = GN_INT8_CRT_MAX_ROWS;  // int32 sums of 2^14-bounded products stay exact

struct ModConsts {
    int m[MODS];
    double inv[MODS];  // fl(1 / m_t)
};

// W_t and M as four 40-bit limbs held exactly in FP64 (W = sum_k w[k] 2^(40k))
struct CrtConsts {
    double w[4][MODS];
    double f[MODS];  // fl(W_t / M)
    double mlimb[4];
};

int64_t modgram_kpad(int64_t m) { return (m + MG_BK - 1) / MG_BK * MG_BK; }
int64_t modgram_ppad(int64_t p) { return (p + MG_BM - 1) / MG_BM * MG_BM; }
int64_t modgram_r_bytes(int64_t m, int64_t p) { return (int64_t)MODS * modgram_ppad(p) * modgram_kpad(m); }
// product residues: per modulus the lower MG_BM x MG_BM tiles only, packed
// tile (tm, tn <= tm) at index tm (tm + 1) / 2 + tn, each row-major
static inline int64_t mg_ytiles(int64_t p) {
    const int64_t t = modgram_ppad(p) / MG_BM;
    return t * (t + 1) / 2;
}
int64_t modgram_y_bytes(int64_t p) { return (int64_t)MODS * mg_ytiles(p) * MG_BM * MG_BM; }
__host__ __device__ inline int64_t mg_yoff(int64_t row, int64_t col) {
    const int64_t tm = row / MG_BM, tn = col / MG_BM;
    return ((tm * (tm + 1) / 2 + tn) * MG_BM + row % MG_BM) * MG_BM + col % MG_BM;
}
int modgram_moduli() { return MODS; }
void modgram_list(int32_t *out) {
    for (int t = 0; t < MODS; ++t) out[t] = MODULI[t];
}

// log2 M, summed in FP64
static double log2_modulus() {
    double s = 0.0;
    for (int t = 0; t < MODS; ++t) s += std::log2((double)MODULI[t]);
    return s;
}

// Bits kept per column: the largest b with m 2^(2b) < M / 4 (one bit of
// margin for the FP64 log2 on top of the factor 4 the quotient estimate
// needs), at most 58 so that the FP64 quotient x / m_t of the residue step
// (|x| <= 2^b, m_t >= 191) is within one of its floor.
int modgram_bits(int64_t m) {
    if (m < 1) m = 1;
    const int b = (int)std::floor((log2_modulus() - 3.0 - std::log2((double)m)) / 2.0);
    return b < 58 ? b : 58;
}

static ModConsts mod_consts() {
    ModConsts c{};
    for (int t = 0; t < MODS; ++t) {
        c.m[t] = MODULI[t];
        c.inv[t] = 1.0 / (double)MODULI[t];
    }
    return c;
}

static CrtConsts crt_consts() {
    typedef unsigned __int128 u128;
    const u128 LIMB_MASK = ((u128)1 << 40) - 1;
    u128 M = 1;
    for (int t = 0; t < MODS; ++t) M *= (u128)MODULI[t];
    CrtConsts c{};
    for (int t = 0; t < MODS; ++t) {
        const int mt = MODULI[t];
        const u128 Mt = M / (u128)mt;
        const int r = (int)(Mt % (u128)mt);
        int inv = 0;
        for (int v = 1; v < mt; ++v)
            if ((r * v) % mt == 1) { inv = v; break; }
        const u128 W = Mt * (u128)inv;  // < M: no reduction needed
        for (int k = 0; k < 4; ++k) c.w[k][t] = (double)(unsigned long long)((W >> (40 * k)) & LIMB_MASK);
        c.f[t] = (double)W / (double)M;
    }
    for (int k = 0; k < 4; ++k) c.mlimb[k] = (double)(unsigned long long)((M >> (40 * k)) & LIMB_MASK);
    return c;
}

static constexpr unsigned long long ABS_MASK = 0x7fffffffffffffffull;
static constexpr unsigned long long INF_BITS = 0x7ff0000000000000ull;

__global__ void mg_zero_kernel(unsigned long long *__restrict__ x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0ull;
}

// cmax[j] = bits of max_i |J_ij| (ordered like the magnitudes; NaN above Inf)
static constexpr int MG_COLMAX_ROWS = 64;
__global__ void mg_colmax_kernel(const double *__restrict__ J, int64_t m, int64_t p, int64_t ldj,
                                 unsigned long long *__restrict__ cmax) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= p) return;
    const int64_t i0 = (int64_t)blockIdx.y * MG_COLMAX_ROWS;
    const int64_t i1 = i0 + MG_COLMAX_ROWS < m ? i0 + MG_COLMAX_ROWS : m;
    unsigned long long mx = 0;
#pragma unroll 8
    for (int64_t i = i0; i < i1; ++i) {
        const unsigned long long bits = (unsigned long long)__double_as_longlong(J[i * ldj + j]) & ABS_MASK;
        mx = bits > mx ? bits : mx;
    }
    if (mx) atomicMax(&cmax[j], mx);
}

// Exponent shift of column j: x = rint(J 2^(b - E)); false for a column
// that is zero or not finite (its integers are all zero).
__device__ __forceinline__ bool column_shift(unsigned long long bits, int b, int &e) {
    if (bits == 0ull || bits >= INF_BITS) { e = 0; return false; }
    e = b - (ilogb(__longlong_as_double((long long)bits)) + 1);
    return true;
}

// Residues: a 64 (i) x 64 (j) block of J becomes MODS int8 tiles R_t[j][i],
// transposed through LDS four moduli at a time.  Each thread holds the
// integers of 4 runs of 4 consecutive rows of one column and packs their
// residues into one 32-bit LDS word per run (odd row stride: the 64 columns
// of a wave hit distinct banks); the tiles leave as 64-byte row segments.
// Covers i < kpad and j < ppad; entries outside J (i >= m, j >= p) are zero.
//
// |x| <= 2^58 is split exactly into four 15-bit parts carrying the sign of
// x, x = p3 2^45 + p2 2^30 + p1 2^15 + p0 with |p_k| < 2^15.  With the balanced
// constants c_k = 2^(15k) mod m_t in [-m_t/2, m_t/2], t = sum_k p_k c_k is
// congruent to x and |t| < 4 2^15 2^7 = 2^24, so the FP32 sums are exact
// integers; r = t - rint(t / m_t) m_t is then exact as well, and one
// correction each way brings it into the balanced range.
static constexpr int MG_CV_I = 64, MG_CV_J = 64, MG_CV_G = 4;
static constexpr int MG_CV_LD = MG_CV_I / 4 + 1;  // 32-bit words per LDS row
static constexpr int MG_CV_S = MG_CV_I / 16;       // runs of 4 rows per thread
__host__ __device__ constexpr int mg_modulus(int t) {
    constexpr int m[MODS] = {256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 211, 199, 197, 193, 191};
    return m[t];
}
__host__ __device__ constexpr int mg_pow2_bal(int e, int m) {  // 2^e mod m in [-m/2, m/2]
    int r = 1;
    for (int i = 0; i < e; ++i) r = (r * 2) % m;
    return r > m / 2 ? r - m : r;
}
static_assert(mg_modulus(0) == MODULI[0] && mg_modulus(MODS - 1) == MODULI[MODS - 1], "modulus table");

template <int T>
__device__ __forceinline__ uint32_t mg_residue8(const float (&pk)[4]) {
    constexpr int M = mg_modulus(T);
    constexpr float C1 = (float)mg_pow2_bal(15, M), C2 = (float)mg_pow2_bal(30, M), C3 = (float)mg_pow2_bal(45, M);
    constexpr float FM = (float)M, INV = 1.0f / (float)M;
    constexpr float HI = (float)((M - 1) / 2), LO = -(float)(M / 2);  // balanced range [LO, HI]
    const float t = fmaf(pk[3], C3, fmaf(pk[2], C2, fmaf(pk[1], C1, pk[0])));
    float r = fmaf(-rintf(t * INV), FM, t);
    r = r > HI ? r - FM : r;
    r = r < LO ? r + FM : r;
    return (uint32_t)(int)r & 0xffu;
}

template <int G>
__device__ __forceinline__ void mg_residue_group(const float (&pk)[4 * MG_CV_S][4], uint32_t *res, int tx, int ty) {
#pragma unroll
    for (int tt = 0; tt < MG_CV_G; ++tt) {
#pragma unroll
        for (int s = 0; s < MG_CV_S; ++s) {
            uint32_t w = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = 4 * s + q;
                uint32_t r;
                switch (G * MG_CV_G + tt) {  // resolved at compile time
                    case 0: r = mg_residue8<0>(pk[e]); break;
                    case 1: r = mg_residue8<1>(pk[e]); break;
                    case 2: r = mg_residue8<2>(pk[e]); break;
                    case 3: r = mg_residue8<3>(pk[e]); break;
                    case 4: r = mg_residue8<4>(pk[e]); break;
                    case 5: r = mg_residue8<5>(pk[e]); break;
                    case 6: r = mg_residue8<6>(pk[e]); break;
                    case 7: r = mg_residue8<7>(pk[e]); break;
                    case 8: r = mg_residue8<8>(pk[e]); break;
                    case 9: r = mg_residue8<9>(pk[e]); break;
                    case 10: r = mg_residue8<10>(pk[e]); break;
                    case 11: r = mg_residue8<11>(pk[e]); break;
                    case 12: r = mg_residue8<12>(pk[e]); break;
                    case 13: r = mg_residue8<13>(pk[e]); break;
                    case 14: r = mg_residue8<14>(pk[e]); break;
                    default: r = mg_residue8<15>(pk[e]); break;
                }
                w |= r << (8 * q);
            }
            res[(tt * MG_CV_J + tx) * MG_CV_LD + 4 * s + ty] = w;
        }
    }
}

__global__ __launch_bounds__(256) void mg_residue_kernel(const double *__restrict__ J, int64_t m, int64_t p, int64_t ldj,
                                                         const unsigned long long *__restrict__ cmax, int b,
                                                         int8_t *__restrict__ R, int64_t ldr, int64_t rplane) {
    __shared__ uint32_t res[MG_CV_G * MG_CV_J * MG_CV_LD];
    const int tx = threadIdx.x % MG_CV_J, ty = threadIdx.x / MG_CV_J;
    const int64_t j0 = (int64_t)blockIdx.x * MG_CV_J, i0 = (int64_t)blockIdx.y * MG_CV_I;
    const int64_t j = j0 + tx;
    int e = 0;
    const bool live = j < p && column_shift(cmax[j < p ? j : 0], b, e);
    float pk[4 * MG_CV_S][4];  // element 4 s + q: row i0 + 16 s + 4 ty + q
#pragma unroll
    for (int s = 0; s < MG_CV_S; ++s)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t i = i0 + 16 * s + 4 * ty + q;
            const double v = (live && i < m) ? J[i * ldj + j] : 0.0;
            const double x = rint(ldexp(v, e));
            // exact 15-bit parts of |x|, signed like x
            const double xa = fabs(x), sg = x < 0.0 ? -1.0 : 1.0;
            const double d3 = floor(xa * 0x1p-45), r3 = fma(-d3, 0x1p45, xa);
            const double d2 = floor(r3 * 0x1p-30), r2 = fma(-d2, 0x1p30, r3);
            const double d1 = floor(r2 * 0x1p-15), d0 = fma(-d1, 0x1p15, r2);
            const int k = 4 * s + q;
            pk[k][0] = (float)(sg * d0);
            pk[k][1] = (float)(sg * d1);
            pk[k][2] = (float)(sg * d2);
            pk[k][3] = (float)(sg * d3);
        }
    constexpr int WPR = MG_CV_I / 4, RPP = 256 / WPR;  // words per row, rows per pass
    const int wc = threadIdx.x % WPR, wr = threadIdx.x / WPR;
    const bool wlive = i0 + 4 * wc < ldr;
    auto flush = [&](int g) {
        __syncthreads();
#pragma unroll
        for (int tt = 0; tt < MG_CV_G; ++tt)
#pragma unroll
            for (int hh = 0; hh < MG_CV_J / RPP; ++hh) {
                const int row = wr + RPP * hh;
                if (wlive)
                    *reinterpret_cast<uint32_t *>(R + (g * MG_CV_G + tt) * rplane + (j0 + row) * ldr + i0 + 4 * wc) =
                        res[(tt * MG_CV_J + row) * MG_CV_LD + wc];
            }
        __syncthreads();
    };
    static_assert(MODS == 4 * MG_CV_G, "four groups of moduli");
    mg_residue_group<0>(pk, res, tx, ty);
    flush(0);
    mg_residue_group<1>(pk, res, tx, ty);
    flush(1);
    mg_residue_group<2>(pk, res, tx, ty);
    flush(2);
    mg_residue_group<3>(pk, res, tx, ty);
    flush(3);
}

// Work of block b.  Blocks are dealt round-robin over the 8 XCDs and each XCD
// runs its share in order, 32 at a time (one per CU).  Block b goes to
// super-tile (b / 8 / 32) * 8 + b % 8 and tile (b / 8) % 32 of it: each XCD
// works on one 4 x 8 block of output tiles of one modulus at a time, so a
// k-chunk of an operand panel is fetched once for 4 or 8 tiles.  Super-tiles
// are numbered modulus by modulus; in a modulus, row a of super-tiles holds
// the super-columns 0 .. (4a + 3) / 8 that touch the lower triangle.
static constexpr int MG_SUP_M = 4, MG_SUP_N = 8, MG_SUP = MG_SUP_M * MG_SUP_N;
__host__ __device__ inline int64_t mg_lower_supers(int64_t tiles) {
    const int64_t nsr = (tiles + MG_SUP_M - 1) / MG_SUP_M, nsc = (tiles + MG_SUP_N - 1) / MG_SUP_N;
    int64_t n = 0;
    for (int64_t a = 0; a < nsr; ++a) {
        const int64_t c = (MG_SUP_M * a + MG_SUP_M - 1) / MG_SUP_N + 1;
        n += c < nsc ? c : nsc;
    }
    return n;
}

__device__ __forceinline__ bool mg_work(int64_t b, int tiles, int64_t supers, int &t, int &tm, int &tn) {
    const int64_t sidx = (b / MG_NXCD / MG_SUP) * MG_NXCD + b % MG_NXCD;
    const int i = (int)((b / MG_NXCD) % MG_SUP);
    if (sidx >= supers * MODS) return false;
    t = (int)(sidx / supers);
    int64_t rem = sidx % supers, a = 0;
    const int64_t nsr = (tiles + MG_SUP_M - 1) / MG_SUP_M, nsc = (tiles + MG_SUP_N - 1) / MG_SUP_N;
    for (; a < nsr; ++a) {
        int64_t c = (MG_SUP_M * a + MG_SUP_M - 1) / MG_SUP_N + 1;
        if (c > nsc) c = nsc;
        if (rem < c) break;
        rem -= c;
    }
    tm = (int)(a * MG_SUP_M + i % MG_SUP_M);
    tn = (int)(rem * MG_SUP_N + i / MG_SUP_M);
    return tm < tiles && tn <= tm;
}

// C_t = R_t R_t^T mod m_t on the lower MG_BM x MG_BM tiles, MG_WM x MG_WN waves.
// R rows are kpad bytes long (kpad a multiple of MG_BK); all tiles are
// interior (the rows and k range are padded with zeros).
//
// Operand tiles move from global memory straight into LDS
// (global_load_lds, 16 bytes per lane, no registers), through a ring of
// MG_STAGES stages so that the copies of a stage are issued MG_STAGES - 1
// stages before it is used.  Each copy instruction fills 1 KB of LDS in lane
// order, i.e. 1024 / MG_BK whole tile rows; lane l takes the global chunk
// c = (l % CPR) ^ swz(row) of its row, so LDS chunk position c' of row r holds
// global chunk c' ^ swz(r).  swz spreads the 16 rows of a fragment read over
// all 64 banks: rows 256 / MG_BK apart share banks, and swz gives them
// distinct chunk positions.
__device__ __forceinline__ int mg_swz(int row) { return (row / (256 / MG_BK)) % (MG_BK / 16); }

template <bool ACC>
__global__ __launch_bounds__(MG_NT) void mg_gemm_kernel(const int8_t *__restrict__ R, int64_t ldr, int64_t rplane,
                                                        int kchunks, int tiles, int64_t supers, ModConsts mc,
                                                        uint8_t *__restrict__ Y, int64_t yplane) {
    constexpr int WTM = MG_BM / MG_WM, WTN = MG_BM / MG_WN;
    constexpr int FM = WTM / 16, FN = WTN / 16;
    constexpr int CPR = MG_BK / 16;                   // 16-byte chunks per tile row
    constexpr int ROWS_PER_COPY = 64 / CPR;           // tile rows per copy instruction
    constexpr int COPIES = MG_BM / ROWS_PER_COPY / (MG_NT / 64);  // per wave, per operand, per stage
    static_assert(COPIES * ROWS_PER_COPY * (MG_NT / 64) == MG_BM, "tile split");
    constexpr int TILE = MG_BM * MG_BK;               // bytes of one operand tile
    extern __shared__ __attribute__((aligned(16))) int8_t mg_lds[];

    int t, tm, tn;
    if (!mg_work(blockIdx.x, tiles, supers, t, tm, tn)) return;
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int wm = wave / MG_WN, wn = wave % MG_WN;
    const int8_t *Ag = R + t * rplane + (int64_t)tm * MG_BM * ldr;
    const int8_t *Bg = R + t * rplane + (int64_t)tn * MG_BM * ldr;

    // copies of stage kc into ring slot kc % MG_STAGES
    const int crow = lane / CPR, cpos = lane % CPR;
    auto issue = [&](int kc) {
        int8_t *la = mg_lds + (kc % MG_STAGES) * 2 * TILE, *lb = la + TILE;
        const int64_t k0 = (int64_t)kc * MG_BK;
#pragma unroll
        for (int q = 0; q < COPIES; ++q) {
            const int row0 = (wave * COPIES + q) * ROWS_PER_COPY, row = row0 + crow;
            const int64_t off = (int64_t)row * ldr + k0 + 16 * (cpos ^ mg_swz(row));
            __builtin_amdgcn_global_load_lds(Ag + off, la + row0 * MG_BK, 16, 0, 0);
            __builtin_amdgcn_global_load_lds(Bg + off, lb + row0 * MG_BK, 16, 0, 0);
        }
    };

    int4v acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int jj = 0; jj < FN; ++jj) acc[i][jj] = int4v{0, 0, 0, 0};

    for (int s = 0; s < MG_STAGES - 1 && s < kchunks; ++s) issue(s);
    const int frow = lane % 16, fchunk = lane / 16;
    for (int kc = 0; kc < kchunks; ++kc) {
        // this wave's copies of stage kc have landed once at most the copies
        // of the later stages already issued are outstanding
        const int later = (kchunks - 1 - kc) < (MG_STAGES - 2) ? (kchunks - 1 - kc) : (MG_STAGES - 2);
        if (later >= 2) __builtin_amdgcn_s_waitcnt(MG_VMCNT(2 * 2 * COPIES));
        else if (later == 1) __builtin_amdgcn_s_waitcnt(MG_VMCNT(2 * COPIES));
        else __builtin_amdgcn_s_waitcnt(MG_VMCNT(0));
        // Every wave's copies of stage kc have landed and every wave is done
        // reading slot (kc - 1) % MG_STAGES (its LDS reads completed before
        // its MFMAs).  A plain s_barrier: __syncthreads() would also wait for
        // the copies of the later stages still in flight.
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        if (kc + MG_STAGES - 1 < kchunks) issue(kc + MG_STAGES - 1);
        const int8_t *la = mg_lds + (kc % MG_STAGES) * 2 * TILE, *lb = la + TILE;
#pragma unroll
        for (int kk = 0; kk < MG_BK / 64; ++kk) {
            int4v a[FM], bb[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                const int r = wm * WTM + i * 16 + frow;
                a[i] = *reinterpret_cast<const int4v *>(la + r * MG_BK + 16 * ((kk * 4 + fchunk) ^ mg_swz(r)));
            }
#pragma unroll
            for (int jj = 0; jj < FN; ++jj) {
                const int r = wn * WTN + jj * 16 + frow;
                bb[jj] = *reinterpret_cast<const int4v *>(lb + r * MG_BK + 16 * ((kk * 4 + fchunk) ^ mg_swz(r)));
            }
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int jj = 0; jj < FN; ++jj)
                    acc[i][jj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i], bb[jj], acc[i][jj], 0, 0, 0);
        }
    }

    // y = C mod m_t in [0, m_t): the quotient from FP64 is within one of the
    // floor and corrected in integers
    const int md = mc.m[t];
    const double inv = mc.inv[t];
    uint8_t *Yt = Y + t * yplane;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int jj = 0; jj < FN; ++jj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = acc[i][jj][r];
                int y = c - (int)floor((double)c * inv) * md;
                y = y < 0 ? y + md : y;
                y = y >= md ? y - md : y;
                const int64_t row = (int64_t)tm * MG_BM + wm * WTM + i * 16 + (lane / 16) * 4 + r;
                const int64_t col = (int64_t)tn * MG_BM + wn * WTN + jj * 16 + lane % 16;
                const int64_t at = mg_yoff(row, col);
                if (ACC) {  // earlier row chunks: residues add modulo m_t
                    y += Yt[at];
                    y = y >= md ? y - md : y;
                }
                Yt[at] = (uint8_t)y;
            }
}

// G_jk (k <= j < p) from the residues y_t: one row j per blockIdx.y.
__global__ __launch_bounds__(256) void mg_crt_kernel(const uint8_t *__restrict__ Y, int64_t yplane,
                                                     int64_t p, const unsigned long long *__restrict__ cmax, int b,
                                                     CrtConsts cc, double *__restrict__ G, int64_t ldg) {
    const int64_t j = blockIdx.y;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= p || k > j) return;
    const unsigned long long bj = cmax[j], bk = cmax[k];
    if (bj >= INF_BITS || bk >= INF_BITS) {
        G[j * ldg + k] = __longlong_as_double(0x7ff8000000000000ll);
        return;
    }
    int ej = 0, ek = 0;
    const bool lj = column_shift(bj, b, ej), lk = column_shift(bk, b, ek);
    if (!lj || !lk) {
        G[j * ldg + k] = 0.0;
        return;
    }
    // v = sum_t y_t W_t - Q M limb by limb: every product y w < 2^48 and
    // every limb sum < 2^52, so the FP64 sums are exact integers
    double S[4] = {0.0, 0.0, 0.0, 0.0}, qs = 0.0;
#pragma unroll
    for (int t = 0; t < MODS; ++t) {
        const double y = (double)Y[t * yplane + mg_yoff(j, k)];
        qs = fma(y, cc.f[t], qs);
#pragma unroll
        for (int l = 0; l < 4; ++l) S[l] = fma(y, cc.w[l][t], S[l]);
    }
    const double Q = rint(qs);
#pragma unroll
    for (int l = 0; l < 4; ++l) S[l] = fma(-Q, cc.mlimb[l], S[l]);  // |S| < 2^53, exact
    // carries: limbs 0-2 into [0, 2^40), the sign into limb 3
    auto normalise = [&]() {
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const double c = floor(S[l] * 0x1p-40);
            S[l] = fma(-c, 0x1p40, S[l]);
            S[l + 1] += c;
        }
    };
    normalise();
    const bool neg = S[3] < 0.0;
    if (neg) {
#pragma unroll
        for (int l = 0; l < 4; ++l) S[l] = -S[l];
        normalise();
    }
    // |v| from non-negative limbs, largest first (within 2 ulp)
    double v = fma(S[2], 0x1p80, S[3] * 0x1p120);
    v = fma(S[1], 0x1p40, v);
    v += S[0];
    v = neg ? -v : v;
    // G = v 2^(E_j - b) 2^(E_k - b) = v 2^(-(e_j + e_k))
    G[j * ldg + k] = ldexp(v, -(ej + ek));
}

// The Gram in phases, for J formed in row chunks: begin (column maxima
// cleared), colmax over every chunk, then per chunk the residues and their
// products (accumulated modulo m_t after the first chunk), and finish (the
// reconstruction).  b comes from the total row count.
hipError_t launch_modgram_begin(hipStream_t st, int64_t p, const ModgramWork &w) {
    const int64_t ppad = modgram_ppad(p);
    if (p <= 0) return hipSuccess;
    if (ppad > w.cmax_len) return hipErrorInvalidValue;
    hipLaunchKernelGGL(mg_zero_kernel, dim3((unsigned)((ppad + 255) / 256)), dim3(256), 0, st, w.cmax, ppad);
    return hipGetLastError();
}

hipError_t launch_modgram_colmax(hipStream_t st, const double *J, int64_t m, int64_t p, int64_t ldj,
                                 const ModgramWork &w) {
    if (p <= 0 || m <= 0) return hipSuccess;
    if (modgram_ppad(p) > w.cmax_len) return hipErrorInvalidValue;
    hipLaunchKernelGGL(mg_colmax_kernel,
                       dim3((unsigned)((p + 255) / 256), (unsigned)((m + MG_COLMAX_ROWS - 1) / MG_COLMAX_ROWS)),
                       dim3(256), 0, st, J, m, p, ldj, w.cmax);
    return hipGetLastError();
}

hipError_t launch_modgram_chunk(hipStream_t st, const double *J, int64_t m, int64_t p, int64_t ldj, int b,
                                const ModgramWork &w, int accumulate) {
    if (p <= 0) return hipSuccess;
    if (m > MG_K_LIMIT) return hipErrorInvalidValue;
    const int64_t kpad = modgram_kpad(m < 1 ? 1 : m), ppad = modgram_ppad(p);
    if (modgram_r_bytes(m < 1 ? 1 : m, p) > w.r_bytes || modgram_y_bytes(p) > w.y_bytes || ppad > w.cmax_len)
        return hipErrorInvalidValue;
    const int64_t rplane = ppad * kpad, yplane = mg_ytiles(p) * MG_BM * MG_BM;
    const ModConsts mc = mod_consts();
    hipLaunchKernelGGL(mg_residue_kernel, dim3((unsigned)(ppad / MG_CV_J), (unsigned)((kpad + MG_CV_I - 1) / MG_CV_I)),
                       dim3(256), 0, st, J, m, p, ldj, w.cmax, b, w.R, kpad, rplane);
    const int tiles = (int)(ppad / MG_BM);
    const int64_t supers = mg_lower_supers(tiles);
    const int64_t blocks = (supers * MODS + MG_NXCD - 1) / MG_NXCD * MG_NXCD * MG_SUP;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)mg_gemm_kernel<false>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, MG_LDS_BYTES);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)mg_gemm_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    MG_LDS_BYTES);
        if (e != hipSuccess) return e;
        attr = true;
    }
    if (accumulate)
        hipLaunchKernelGGL(mg_gemm_kernel<true>, dim3((unsigned)blocks), dim3(MG_NT), MG_LDS_BYTES, st, w.R, kpad,
                           rplane, (int)(kpad / MG_BK), tiles, supers, mc, w.Y, yplane);
    else
        hipLaunchKernelGGL(mg_gemm_kernel<false>, dim3((unsigned)blocks), dim3(MG_NT), MG_LDS_BYTES, st, w.R, kpad,
                           rplane, (int)(kpad / MG_BK), tiles, supers, mc, w.Y, yplane);
    return hipGetLastError();
}

hipError_t launch_modgram_finish(hipStream_t st, int64_t p, int b, double *G, int64_t ldg, const ModgramWork &w) {
    if (p <= 0) return hipSuccess;
    const int64_t ppad = modgram_ppad(p);
    if (modgram_y_bytes(p) > w.y_bytes || ppad > w.cmax_len) return hipErrorInvalidValue;
    const CrtConsts cc = crt_consts();
    hipLaunchKernelGGL(mg_crt_kernel, dim3((unsigned)((p + 255) / 256), (unsigned)p), dim3(256), 0, st, w.Y,
                       mg_ytiles(p) * MG_BM * MG_BM, p, w.cmax, b, cc, G, ldg);
    return hipGetLastError();
}

hipError_t launch_modgram(hipStream_t st, const double *J, int64_t m, int64_t p, int64_t ldj, double *G, int64_t ldg,
                          const ModgramWork &w) {
    if (p <= 0) return hipSuccess;
    if (m > MG_K_LIMIT) return hipErrorInvalidValue;
    const int b = modgram_bits(m);
    hipError_t e = launch_modgram_begin(st, p, w);
    if (e == hipSuccess) e = launch_modgram_colmax(st, J, m, p, ldj, w);
    if (e == hipSuccess) e = launch_modgram_chunk(st, J, m, p, ldj, b, w, 0);
    if (e == hipSuccess) e = launch_modgram_finish(st, p, b, G, ldg, w);
    return e;
}

}  // namespace gn
