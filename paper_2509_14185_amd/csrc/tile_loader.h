// tile_loader.h -- staging of one GEMM operand tile (FP64) through LDS,
// shared by the GEMM kernels and the persistent factorisation kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace gn {

typedef double double4_t __attribute__((ext_vector_type(4)));

// One operand tile (rows x cols of the tile in (m or n, k) space) is loaded
// as 16-byte pairs along the operand's contiguous direction.
//   CONTIG_MN: element (r, k) at base[k*ld + r] (pairs along r)
//   else:      element (r, k) at base[r*ld + k] (pairs along k)
template <int R, int BK, bool CONTIG_MN, int NT>
struct TileLoader {
    static constexpr int PAIRS = R * BK / 2;
    static constexpr int PER = PAIRS / NT;
    static_assert(PER * NT == PAIRS, "tile split");
    double2 v[PER];

    __device__ __forceinline__ static void coords(int e, int &r, int &k) {
        const int idx = threadIdx.x + e * NT;
        if (CONTIG_MN) { r = 2 * (idx % (R / 2)); k = idx / (R / 2); }
        else           { k = 2 * (idx % (BK / 2)); r = idx / (BK / 2); }
    }
    // full: the whole tile lies inside [0,rmax) x [0,kmax) and pairs are aligned
    __device__ __forceinline__ void load(const double *base, int64_t ld, int64_t r0, int64_t k0, int64_t rmax,
                                         int64_t kmax, bool full) {
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            int r, k;
            coords(e, r, k);
            const int64_t gr = r0 + r, gk = k0 + k;
            if (full) {
                const double *p = CONTIG_MN ? base + gk * ld + gr : base + gr * ld + gk;
                v[e] = *reinterpret_cast<const double2 *>(p);
            } else {
                double a = 0.0, b = 0.0;
                if (CONTIG_MN) {
                    if (gk < kmax) {
                        if (gr < rmax) a = base[gk * ld + gr];
                        if (gr + 1 < rmax) b = base[gk * ld + gr + 1];
                    }
                } else {
                    if (gr < rmax) {
                        if (gk < kmax) a = base[gr * ld + gk];
                        if (gk + 1 < kmax) b = base[gr * ld + gk + 1];
                    }
                }
                v[e] = make_double2(a, b);
            }
        }
    }
    // LDS keeps the operand's global orientation, so every store is a plain
    // 16-byte copy: [k][r] (stride R) when contiguous along r, else [r][k]
    // with stride LDK = BK + 2 (even, so pairs stay 16-byte aligned; the pad
    // spreads the 16 rows of an MFMA fragment read over distinct banks).
    static constexpr int LDK = BK + 2;
    static constexpr int SIZE = CONTIG_MN ? BK * R : R * LDK;  // doubles per buffer
    __device__ __forceinline__ static int at(int r, int k) { return CONTIG_MN ? k * R + r : r * LDK + k; }
    // Direct global -> LDS copy of one chunk (operands contiguous along r,
    // whole chunk in bounds, 16-byte aligned): each wave instruction moves 64
    // x 16 bytes = 128 doubles, i.e. 128 / R consecutive k-rows of the tile,
    // which are also consecutive in the [k][r] LDS layout.  No registers are
    // involved; completion is waited for with vmcnt before the barrier.
    __device__ __forceinline__ static void direct(const double *base, int64_t ld, int64_t r0, int64_t k0, double *lds,
                                                  int wave) {
        static_assert(CONTIG_MN, "direct copies need the [k][r] layout");
        constexpr int ROWS = 128 / R;                          // k-rows per wave instruction
        constexpr int PERW = BK / ROWS / (NT / 64);  // instructions per wave
        static_assert(PERW * ROWS * (NT / 64) == BK, "chunk split");
        const int lane = threadIdx.x & 63;
        const int kin = (2 * lane) / R, r = (2 * lane) % R;
#pragma unroll
        for (int q = 0; q < PERW; ++q) {
            const int kk = (wave * PERW + q) * ROWS;
            __builtin_amdgcn_global_load_lds(base + (k0 + kk + kin) * ld + r0 + r, lds + kk * R, 16, 0, 0);
        }
    }
    __device__ __forceinline__ void store(double *lds) const {
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            int r, k;
            coords(e, r, k);
            *reinterpret_cast<double2 *>(lds + at(r, k)) = v[e];
        }
    }
};

}  // namespace gn
