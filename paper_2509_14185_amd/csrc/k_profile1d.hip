// 1D self-similar profile kernels for gfx950: geometry of the compactified
// coordinate, the half-line Hilbert quadrature, tanh-MLP sweeps (forward
// jets, Jacobian rows, vector-Jacobian product) and the residual rows.
//
// Paper (arXiv 2509.14185), Methods:
//  - "Solution Modeling and Equation Factorisation": q = (1+|y|^2)^{-1/(2(1+l))}
//    as network input; the field is an envelope times the network output;
//    tanh MLP.
//  - "Self-similar Solutions": static profile equation in y.
//  - "Training Loss": rows weighted by sqrt(rho/(N N_E)).
//
// Equation (CCF under the self-similar ansatz):
//   R = -lam Theta + ((1+lam) y + U) Theta_y,  U = H Theta,
//   Theta = E(y) NN(q),  Theta_y = E_y NN + E q_y NN_q.
// In terms of q = 1 - s (1 + y^2 = q^{-2(1+lam)}):
//   y^2 = expm1(-2(1+lam) log1p(-s)),  q_y = -y q^{3+2 lam}/(1+lam),
//   CCF envelope E = y^2/(1+y^2) q^{-lam} = y^2 q^{2+lam},
//       E_y = y/(1+lam) (lam q^{2+lam} + (2+lam) q^{4+3 lam}),
//   local (Burgers) envelope E = y/sqrt(1+y^2) q^{-lam} = y q,
//       E_y = q + y q_y.
// Hilbert term on the half line for an even field:
//   U_i = sum_j Q_ij (Theta(t_j) - Theta(y_i)),
//   Q_ij = wh_j 2 y_i / ((y_i - t_j)(y_i + t_j)),  wh_j = ws_j (dt/ds)_j / pi,
//   dt/ds = (1+lam)(1+t^2)/(q t).
#include "gn_internal.h"

namespace gn {

static constexpr int SWEEP_THREADS = 256;
static constexpr int SWEEP_TILE = 8;  // points per workgroup

__device__ __forceinline__ double hilbert_q(double yi, double tj, double whj) {
    return whj * (2.0 * yi) / ((yi - tj) * (yi + tj));
}

// ------------------------------------------------------------------ geometry
__global__ void geometry_kernel(int equation, double lam, int64_t n, const double *__restrict__ s,
                                const double *__restrict__ ws, Geo1D g) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double si = s[i];
    const double q = 1.0 - si;
    const double y2 = expm1(-2.0 * (1.0 + lam) * log1p(-si));
    const double y = sqrt(y2);
    const double qy = -y * pow(q, 3.0 + 2.0 * lam) / (1.0 + lam);
    double E, Ey;
    if (equation == GN_EQ_CCF1D) {
        const double a = pow(q, 2.0 + lam);
        E = y2 * a;
        Ey = y / (1.0 + lam) * (lam * a + (2.0 + lam) * pow(q, 4.0 + 3.0 * lam));
    } else {
        E = y * q;
        Ey = q + y * qy;
    }
    g.y[i] = y;
    g.q[i] = q;
    g.E[i] = E;
    g.Ey[i] = Ey;
    g.qy[i] = qy;
    if (ws != nullptr && g.wh != nullptr) {
        const double dtds = (1.0 + lam) * (1.0 + y2) / (q * y);
        g.wh[i] = ws[i] * dtds / M_PI;
    }
}

hipError_t launch_geometry(hipStream_t st, int equation, double lam, int64_t n, const double *s,
                           const double *ws, Geo1D g) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(geometry_kernel, dim3((unsigned)blocks), dim3(256), 0, st, equation, lam, n, s,
                       ws, g);
    return hipGetLastError();
}

// Q^T: row j (node), column i (point), so the coupling product reads it
// contiguously along i (the output rows) and the adjoint along i as well.
__global__ void hilbert_matrix_kernel(int64_t n, int64_t m, const double *__restrict__ y,
                                      const double *__restrict__ t, const double *__restrict__ wh,
                                      double *__restrict__ QT, int64_t ld) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t j = blockIdx.y;
    if (i >= n || j >= m) return;
    QT[j * ld + i] = hilbert_q(y[i], t[j], wh[j]);
}

hipError_t launch_hilbert_matrix(hipStream_t st, int64_t n, int64_t m, const double *y, const double *t,
                                 const double *wh, double *QT, int64_t ld) {
    if (n <= 0 || m <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)m);
    hipLaunchKernelGGL(hilbert_matrix_kernel, grid, dim3(256), 0, st, n, m, y, t, wh, QT, ld);
    return hipGetLastError();
}

// ------------------------------------------------------------ network sweeps
// LDS layout per workgroup (T = SWEEP_TILE points):
//   act: for each hidden layer input l = 1..L-1: Tl[T][w_l] (tanh values)
//        then ZXl[T][w_l] (input-derivative pre-activations);
//   cur: h/hx of the layer being computed in the forward pass (aliases act);
//   zb0/zbx0, zb1/zbx1: adjoint buffers, T x maxw each.
// Weights are read from global memory: row-major W for the adjoint (lanes
// over the input index are contiguous) and the transposed copy Wt for the
// forward pass (lanes over the output index are contiguous).
enum SweepMode { SWEEP_FORWARD = 0, SWEEP_ROWS = 1, SWEEP_VJP = 2 };

struct SweepLds {
    int act_off[GN_MAX_LAYERS + 1];  // offset of T^l (l >= 1); ZX^l follows at + T*w_l
    int zb_off;                       // start of the adjoint buffers
    int maxw;
    int total;                        // doubles
};

static SweepLds sweep_lds_layout(const MlpDesc &d) {
    SweepLds s{};
    int o = 0, maxw = 1;
    for (int l = 1; l < d.L; ++l) {
        s.act_off[l] = o;
        o += 2 * SWEEP_TILE * d.w[l];
        if (d.w[l] > maxw) maxw = d.w[l];
    }
    s.zb_off = o;
    s.maxw = maxw;
    s.total = o + 4 * SWEEP_TILE * maxw;
    return s;
}

template <int MODE>
__global__ __launch_bounds__(SWEEP_THREADS) void mlp_sweep_kernel(MlpDesc d, SweepLds lay,
                                                                  const double *__restrict__ theta,
                                                                  const double *__restrict__ thetaT,
                                                                  SweepBatch b, double *__restrict__ partial) {
    extern __shared__ double sm[];
    const int tid = threadIdx.x;
    const int64_t p0 = (int64_t)blockIdx.x * SWEEP_TILE;
    const int np = (int)((b.n - p0) < SWEEP_TILE ? (b.n - p0) : SWEEP_TILE);
    if (np <= 0) return;
    const int L = d.L;
    double *zbA = sm + lay.zb_off;
    double *zbxA = zbA + SWEEP_TILE * lay.maxw;
    double *zbB = zbxA + SWEEP_TILE * lay.maxw;
    double *zbxB = zbB + SWEEP_TILE * lay.maxw;

    // ---------------- forward: hidden layers l = 0..L-2 produce T^{l+1}, ZX^{l+1}
    for (int l = 0; l < L - 1; ++l) {
        const int win = d.w[l], wout = d.w[l + 1];
        const double *Wt = thetaT + d.off[l];     // Wt[j][k] = W[k][j], win x wout
        const double *bias = theta + d.off[l] + win * wout;
        double *Tn = sm + lay.act_off[l + 1];
        double *ZXn = Tn + SWEEP_TILE * wout;
        for (int idx = tid; idx < np * wout; idx += SWEEP_THREADS) {
            const int pt = idx / wout, k = idx - pt * wout;
            double z = bias[k], zx = 0.0;
            if (l == 0 && b.phi) {
                // Fourier feature input: z = W phi + b, z_x = W phi_x
                for (int j = 0; j < win; ++j) {
                    const double w = Wt[j * wout + k];
                    z = fma(w, b.phi[j * b.phi_ld + p0 + pt], z);
                    zx = fma(w, b.phi[(win + j) * b.phi_ld + p0 + pt], zx);
                }
            } else if (l == 0) {
                const double x = b.x[p0 + pt];
                z = fma(Wt[k], x, z);
                zx = Wt[k];
            } else {
                const double *Tp = sm + lay.act_off[l] + pt * win;
                const double *ZXp = Tp + SWEEP_TILE * win;
                for (int j = 0; j < win; ++j) {
                    const double tj = Tp[j];
                    const double hxj = (1.0 - tj * tj) * ZXp[j];
                    const double w = Wt[j * wout + k];
                    z = fma(w, tj, z);
                    zx = fma(w, hxj, zx);
                }
            }
            Tn[pt * wout + k] = tanh(z);
            ZXn[pt * wout + k] = zx;
        }
        __syncthreads();
    }

    // ---------------- output layer (width 1): NN, NN_x
    {
        const int l = L - 1;
        const int win = d.w[l];
        const double *W = theta + d.off[l];  // 1 x win
        const double bias = theta[d.off[l] + win];
        // one wave per point: lanes over j, fixed-order butterfly reduction
        const int wave = tid >> 6, lane = tid & 63;
        for (int pt = wave; pt < np; pt += SWEEP_THREADS / 64) {
            double z = 0.0, zx = 0.0;
            if (l == 0 && b.phi) {
                for (int j = lane; j < win; j += 64) {
                    z = fma(W[j], b.phi[j * b.phi_ld + p0 + pt], z);
                    zx = fma(W[j], b.phi[(win + j) * b.phi_ld + p0 + pt], zx);
                }
            } else if (l == 0) {
                if (lane == 0) {
                    z = W[0] * b.x[p0 + pt];
                    zx = W[0];
                }
            } else {
                const double *Tp = sm + lay.act_off[l] + pt * win;
                const double *ZXp = Tp + SWEEP_TILE * win;
                for (int j = lane; j < win; j += 64) {
                    const double tj = Tp[j];
                    z = fma(W[j], tj, z);
                    zx = fma(W[j], (1.0 - tj * tj) * ZXp[j], zx);
                }
            }
            for (int o = 32; o > 0; o >>= 1) {
                z += __shfl_xor(z, o, 64);
                zx += __shfl_xor(zx, o, 64);
            }
            if (lane == 0) {
                if (MODE == SWEEP_FORWARD) {
                    b.nn[p0 + pt] = z + bias;
                    b.nn[b.n + p0 + pt] = zx;
                }
                zbA[pt * lay.maxw] = b.s0 ? b.s0[p0 + pt] : b.s0c;
                zbxA[pt * lay.maxw] = b.s1 ? b.s1[p0 + pt] : b.s1c;
            }
        }
    }
    if (MODE == SWEEP_FORWARD) return;
    __syncthreads();

    // ---------------- adjoint sweep, layer l = L-1 .. 0
    double *zb = zbA, *zbx = zbxA, *zbn = zbB, *zbxn = zbxB;
    const int ldz = lay.maxw;
    for (int l = L - 1; l >= 0; --l) {
        const int win = d.w[l], wout = d.w[l + 1];
        const int nseg = wout * (win + 1);  // W^l then b^l
        const double *Tp = (l > 0) ? sm + lay.act_off[l] : nullptr;
        const double *ZXp = (l > 0) ? Tp + SWEEP_TILE * win : nullptr;
        if (MODE == SWEEP_ROWS) {
            for (int pt = 0; pt < np; ++pt) {
                double *row = b.rows + (p0 + pt) * b.ld + d.off[l];
                const double *zr = zb + pt * ldz;
                const double *zxr = zbx + pt * ldz;
                const double xin = (l == 0 && !b.phi) ? b.x[p0 + pt] : 0.0;
                for (int idx = tid; idx < nseg; idx += SWEEP_THREADS) {
                    double v;
                    if (idx < wout * win) {
                        const int k = idx / win, j = idx - k * win;
                        double h, hx;
                        if (l == 0 && b.phi) {
                            h = b.phi[j * b.phi_ld + p0 + pt];
                            hx = b.phi[(win + j) * b.phi_ld + p0 + pt];
                        } else if (l == 0) {
                            h = xin;
                            hx = 1.0;
                        } else {
                            h = Tp[pt * win + j];
                            hx = (1.0 - h * h) * ZXp[pt * win + j];
                        }
                        v = fma(zr[k], h, zxr[k] * hx);
                    } else {
                        v = zr[idx - wout * win];
                    }
                    row[idx] = v;
                }
            }
        } else {  // SWEEP_VJP: sum over the points of this workgroup
            double *out = partial + (int64_t)blockIdx.x * d.P + d.off[l];
            for (int idx = tid; idx < nseg; idx += SWEEP_THREADS) {
                double acc = 0.0;
                if (idx < wout * win) {
                    const int k = idx / win, j = idx - k * win;
                    for (int pt = 0; pt < np; ++pt) {
                        double h, hx;
                        if (l == 0 && b.phi) {
                            h = b.phi[j * b.phi_ld + p0 + pt];
                            hx = b.phi[(win + j) * b.phi_ld + p0 + pt];
                        } else if (l == 0) {
                            h = b.x[p0 + pt];
                            hx = 1.0;
                        } else {
                            h = Tp[pt * win + j];
                            hx = (1.0 - h * h) * ZXp[pt * win + j];
                        }
                        acc += fma(zb[pt * ldz + k], h, zbx[pt * ldz + k] * hx);
                    }
                } else {
                    const int k = idx - wout * win;
                    for (int pt = 0; pt < np; ++pt) acc += zb[pt * ldz + k];
                }
                out[idx] = acc;
            }
        }
        if (l == 0) break;
        // hbar = W^T zbar, hbar_x = W^T zbar_x; then through h = tanh(z),
        // h_x = (1 - t^2) z_x:
        //   zbar_x' = hbar_x (1 - t^2),  zbar' = hbar (1 - t^2) - 2 t (1 - t^2) z_x hbar_x.
        const double *W = theta + d.off[l];  // wout x win
        for (int idx = tid; idx < np * win; idx += SWEEP_THREADS) {
            const int pt = idx / win, j = idx - pt * win;
            double hb = 0.0, hbx = 0.0;
            for (int k = 0; k < wout; ++k) {
                const double w = W[k * win + j];
                hb = fma(w, zb[pt * ldz + k], hb);
                hbx = fma(w, zbx[pt * ldz + k], hbx);
            }
            const double t = Tp[pt * win + j];
            const double dd = 1.0 - t * t;
            const double zxv = ZXp[pt * win + j];
            zbxn[pt * ldz + j] = hbx * dd;
            zbn[pt * ldz + j] = hb * dd - 2.0 * t * dd * zxv * hbx;
        }
        __syncthreads();
        double *tmp = zb;
        zb = zbn;
        zbn = tmp;
        tmp = zbx;
        zbx = zbxn;
        zbxn = tmp;
    }
}

// ---- Jacobian rows on the matrix cores (scalar input and output, hidden
// widths up to 64, no Fourier features)
// A workgroup takes 16 points at a time.  Forward: per hidden layer, the two
// jet components (value and x-derivative) of the layer's pre-activations,
// Z_c = W H_c (+ bias for c = 0), as 16-unit x 16-point tiles on
// v_mfma_f64_16x16x4f64 (wave w takes unit tile w; A = W from the transposed
// weights through L1/L2, B = H_c from LDS), then th = tanh(z0) and
// h1 = (1 - th^2) z1 in registers, stored in LDS as the next layer's input
// (every hidden layer's jets stay in LDS for the reverse sweep).  The input
// layer (one input, so no product) is formed per lane.  Reverse, from the
// seeds on NN and NN_x: the row entries of (W_l, b_l) are
// ZB_0[k] H_0[j] + ZB_1[k] H_1[j] and ZB_0[k] (lane = j, wave = k mod 4,
// four rows at a time, so each store writes 64 contiguous entries of a row);
// then hb = W_l^T ZB per component on the MFMA tiles and, through the
// reverse tanh rule, zb_1 = (1 - th^2) hb_1 and
// zb_0 = (1 - th^2) hb_0 - 2 th h1 hb_1.
// LDS: planes [c][j][t] with row stride 17 (reads along j spread over the
// banks): one per hidden layer output plus ZB, 2 x wpad x 17 doubles each.
typedef double double4_t __attribute__((ext_vector_type(4)));
static constexpr int RW1_TP = 16, RW1_LD = RW1_TP + 1;

// Pre-activations of layer f for the 16 points of a tile: acc0 (value) and
// acc1 (x-derivative) of units 16 * wave + fk + 4 r at point fr, as
// Z_c = W_f H_c (+ bias for c = 0) on the MFMA tiles (A = W_f from the
// transposed weights, B = H_c from the LDS plane Hf laid out [c][j][t] with
// row stride RW1_LD); the input layer (one input x, Hf null) is formed per
// lane.  Returns false (accumulators zero) for waves past the layer's unit
// tiles (uniform over the wave).
__device__ __forceinline__ bool rows1d_layer_product(const MlpDesc &d, int f, int wpad, const double *__restrict__ theta,
                                                     const double *__restrict__ thetaT, const double *Hf,
                                                     const double *xs, int wave, int fr, int fk, double4_t &acc0,
                                                     double4_t &acc1) {
    const int win = d.w[f], wout = d.w[f + 1];
    const int nut = (wout + 15) / 16;
    acc0 = (double4_t){0.0, 0.0, 0.0, 0.0};
    acc1 = acc0;
    if (wave >= nut) return false;
    const double *bias = theta + d.off[f] + win * wout;
    if (Hf == nullptr) {
        // one input: z0 = W x + b, z1 = W
        const double *W0 = theta + d.off[0];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k = 16 * wave + fk + 4 * r;
            const double wk = k < wout ? W0[k] : 0.0;
            acc0[r] = k < wout ? fma(wk, xs[fr], bias[k]) : 0.0;
            acc1[r] = wk;
        }
        return true;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int k = 16 * wave + fk + 4 * r;
        acc0[r] = k < wout ? bias[k] : 0.0;
    }
    const double *Wt = thetaT + d.off[f];  // Wt[j][k] = W[k][j]
    const int kpad = (win + 3) & ~3;
    const int k = 16 * wave + fr;
    double a[4], an[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int j = 4 * q + fk;
        a[q] = (4 * q < kpad && k < wout && j < win) ? Wt[j * wout + k] : 0.0;
    }
    for (int s0 = 0; s0 < kpad; s0 += 16) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = s0 + 16 + 4 * q + fk;
            an[q] = (s0 + 16 + 4 * q < kpad && k < wout && j < win) ? Wt[j * wout + k] : 0.0;
        }
        double b0[4], b1[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = s0 + 4 * q + fk;
            const bool in = s0 + 4 * q < kpad;
            b0[q] = in ? Hf[j * RW1_LD + fr] : 0.0;
            b1[q] = in ? Hf[(wpad + j) * RW1_LD + fr] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b0[q], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b1[q], acc1, 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = an[q];
    }
    return true;
}

// JOBS: one 16-point tile per workgroup from a work table (job, tile) over
// many sweeps (the instances of a batch), each with its own parameters.
template <bool JOBS>
__global__ __launch_bounds__(256) void mlp_rows_mfma_kernel(MlpDesc d, int wpad, const double *__restrict__ theta0,
                                                            const double *__restrict__ thetaT0, SweepBatch b0,
                                                            const SweepJob *__restrict__ jobs,
                                                            const int2 *__restrict__ work) {
    extern __shared__ double sm[];
    const double *theta = theta0, *thetaT = thetaT0;
    SweepBatch b = b0;
    int64_t tile_first = blockIdx.x, tile_step = gridDim.x;
    if (JOBS) {
        const int2 w = work[blockIdx.x];
        if (w.x < 0) return;
        theta = jobs[w.x].theta;
        thetaT = jobs[w.x].thetaT;
        b = jobs[w.x].b;
        tile_first = w.y;
        tile_step = INT64_MAX / 2;
    }
    __shared__ double xs[RW1_TP];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int fr = lane & 15, fk = lane >> 4;
    const int L = d.L;
    const int plane = 2 * wpad * RW1_LD;
    // H_l (l = 1 .. L-1) at sm + (l - 1) * plane, ZB at sm + (L - 1) * plane
    auto H = [&](int l, int c, int j, int t) -> double & { return sm[(l - 1) * plane + (c * wpad + j) * RW1_LD + t]; };
    double *zs = sm + (L - 1) * plane;
    auto Z = [&](int c, int k, int t) -> double & { return zs[(c * wpad + k) * RW1_LD + t]; };
    const int64_t ntiles = (b.n + RW1_TP - 1) / RW1_TP;
    for (int64_t tile = tile_first; tile < ntiles; tile += tile_step) {
        const int64_t p0 = tile * RW1_TP;
        const int nr = (int)((b.n - p0) < RW1_TP ? (b.n - p0) : RW1_TP);
        __syncthreads();  // the previous tile is done with LDS
        if (tid < RW1_TP) xs[tid] = tid < nr ? b.x[p0 + tid] : 0.0;
        // seeds on NN (c = 0) and NN_x (c = 1); zero past the output and the last point
        for (int idx = tid; idx < 2 * 16 * RW1_TP; idx += 256) {
            const int c = idx / (16 * RW1_TP), o = (idx / RW1_TP) & 15, t = idx % RW1_TP;
            double v = 0.0;
            if (o == 0 && t < nr) v = c == 0 ? (b.s0 ? b.s0[p0 + t] : b.s0c) : (b.s1 ? b.s1[p0 + t] : b.s1c);
            Z(c, o, t) = v;
        }
        __syncthreads();
        // forward through the hidden layers
        for (int f = 0; f + 1 < L; ++f) {
            double4_t acc0, acc1;
            if (rows1d_layer_product(d, f, wpad, theta, thetaT, f > 0 ? &H(f, 0, 0, 0) : nullptr, xs, wave, fr, fk,
                                     acc0, acc1)) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int k = 16 * wave + fk + 4 * r;
                    const double th = tanh(acc0[r]);
                    H(f + 1, 0, k, fr) = th;
                    H(f + 1, 1, k, fr) = (1.0 - th * th) * acc1[r];
                }
            }
            __syncthreads();
        }
        // reverse over the layers
        for (int l = L - 1; l >= 0; --l) {
            const int win = d.w[l], wout = d.w[l + 1];
            double *Jl = b.rows + p0 * b.ld + d.off[l];
            if (l == 0) {
                // one input: entries Z_0[k] x + Z_1[k] of W_0, then b_0
                for (int idx = tid; idx < 2 * wout * nr; idx += 256) {
                    const int t = idx / (2 * wout), e = idx - t * 2 * wout;
                    const int k = e < wout ? e : e - wout;
                    Jl[t * b.ld + e] = e < wout ? fma(Z(0, k, t), xs[t], Z(1, k, t)) : Z(0, k, t);
                }
                break;
            }
            if (wout < 4 || win < 32) {
                for (int idx = tid; idx < wout * win * nr; idx += 256) {
                    const int t = idx / (wout * win), e = idx - t * wout * win, k = e / win, j = e - k * win;
                    Jl[t * b.ld + e] = fma(Z(0, k, t), H(l, 0, j, t), Z(1, k, t) * H(l, 1, j, t));
                }
            } else if (lane < win) {
                for (int t0 = 0; t0 < nr; t0 += 4) {
                    double h0[4], h1[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        h0[q] = H(l, 0, lane, t0 + q);
                        h1[q] = H(l, 1, lane, t0 + q);
                    }
                    for (int k = wave; k < wout; k += 4) {
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if (t0 + q < nr)
                                Jl[(t0 + q) * b.ld + k * win + lane] = fma(Z(0, k, t0 + q), h0[q], Z(1, k, t0 + q) * h1[q]);
                    }
                }
            }
            for (int idx = tid; idx < wout * nr; idx += 256) {
                const int t = idx / wout, k = idx - t * wout;
                Jl[t * b.ld + wout * win + k] = Z(0, k, t);
            }
            // hb = W_l^T ZB per component (j-tile = wave), then back through tanh
            const double *W = theta + d.off[l];  // W[k][j], wout x win
            const int kpad = (wout + 3) & ~3, nut = (win + 15) / 16;
            const bool mine = wave < nut;
            double4_t acc0 = (double4_t){0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
            if (mine) {
                const int j = 16 * wave + fr;
                double a[4], an[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int k = 4 * q + fk;
                    a[q] = (4 * q < kpad && k < wout && j < win) ? W[k * win + j] : 0.0;
                }
                for (int s0 = 0; s0 < kpad; s0 += 16) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int k = s0 + 16 + 4 * q + fk;
                        an[q] = (s0 + 16 + 4 * q < kpad && k < wout && j < win) ? W[k * win + j] : 0.0;
                    }
                    double b0[4], b1[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int k = s0 + 4 * q + fk;
                        const bool in = s0 + 4 * q < kpad;
                        b0[q] = in ? Z(0, k, fr) : 0.0;
                        b1[q] = in ? Z(1, k, fr) : 0.0;
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b0[q], acc0, 0, 0, 0);
                        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b1[q], acc1, 0, 0, 0);
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) a[q] = an[q];
                }
            }
            __syncthreads();  // every read of ZB (this layer's rows and products) is done
            if (mine) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int j = 16 * wave + fk + 4 * r;
                    const double th = H(l, 0, j, fr), h1 = H(l, 1, j, fr);
                    const double sd = 1.0 - th * th;
                    Z(1, j, fr) = sd * acc1[r];
                    Z(0, j, fr) = sd * acc0[r] - 2.0 * th * h1 * acc1[r];
                }
            }
            __syncthreads();
        }
    }
}

// Forward jets on the matrix cores (the same networks as the rows kernel):
// the hidden layers as there, then the output layer's value and
// x-derivative, NN and NN_x, from the same product (one unit: wave 0, lanes
// of the first unit row).
template <bool JOBS>
__global__ __launch_bounds__(256) void mlp_forward_mfma_kernel(MlpDesc d, int wpad, const double *__restrict__ theta0,
                                                               const double *__restrict__ thetaT0, SweepBatch b0,
                                                               const SweepJob *__restrict__ jobs,
                                                               const int2 *__restrict__ work) {
    extern __shared__ double sm[];
    const double *theta = theta0, *thetaT = thetaT0;
    SweepBatch b = b0;
    int64_t tile_first = blockIdx.x, tile_step = gridDim.x;
    if (JOBS) {
        const int2 w = work[blockIdx.x];
        if (w.x < 0) return;
        theta = jobs[w.x].theta;
        thetaT = jobs[w.x].thetaT;
        b = jobs[w.x].b;
        tile_first = w.y;
        tile_step = INT64_MAX / 2;
    }
    __shared__ double xs[RW1_TP];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int fr = lane & 15, fk = lane >> 4;
    const int L = d.L;
    const int plane = 2 * wpad * RW1_LD;
    auto H = [&](int l, int c, int j, int t) -> double & { return sm[(l - 1) * plane + (c * wpad + j) * RW1_LD + t]; };
    const int64_t ntiles = (b.n + RW1_TP - 1) / RW1_TP;
    for (int64_t tile = tile_first; tile < ntiles; tile += tile_step) {
        const int64_t p0 = tile * RW1_TP;
        const int nr = (int)((b.n - p0) < RW1_TP ? (b.n - p0) : RW1_TP);
        __syncthreads();  // the previous tile is done with LDS
        if (tid < RW1_TP) xs[tid] = tid < nr ? b.x[p0 + tid] : 0.0;
        __syncthreads();
        for (int f = 0; f + 1 < L; ++f) {
            double4_t acc0, acc1;
            if (rows1d_layer_product(d, f, wpad, theta, thetaT, f > 0 ? &H(f, 0, 0, 0) : nullptr, xs, wave, fr, fk,
                                     acc0, acc1)) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int k = 16 * wave + fk + 4 * r;
                    const double th = tanh(acc0[r]);
                    H(f + 1, 0, k, fr) = th;
                    H(f + 1, 1, k, fr) = (1.0 - th * th) * acc1[r];
                }
            }
            __syncthreads();
        }
        double4_t acc0, acc1;
        if (rows1d_layer_product(d, L - 1, wpad, theta, thetaT, &H(L - 1, 0, 0, 0), xs, wave, fr, fk, acc0, acc1) &&
            fk == 0 && fr < nr) {
            b.nn[p0 + fr] = acc0[0];
            b.nn[b.n + p0 + fr] = acc1[0];
        }
    }
}

// wpad of the matrix-core rows sweep, or 0 if the network does not fit it
static int rows1d_mfma_wpad(const MlpDesc &d) {
    if (d.L < 2 || d.w[0] != 1 || d.w[d.L] != 1) return 0;
    int m = 16;
    for (int l = 1; l < d.L; ++l) m = d.w[l] > m ? d.w[l] : m;
    const int wpad = (m + 15) / 16 * 16;
    if (wpad > 64) return 0;
    const size_t bytes = sizeof(double) * (size_t)d.L * 2 * wpad * RW1_LD;
    return bytes <= 150 * 1024 ? wpad : 0;
}

// W^T per layer (same offsets as theta; biases copied).
__global__ void transpose_weights_kernel(MlpDesc d, const double *__restrict__ theta, double *__restrict__ out) {
    for (int l = 0; l < d.L; ++l) {
        const int win = d.w[l], wout = d.w[l + 1];
        const int nseg = wout * (win + 1);
        for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < nseg; idx += gridDim.x * blockDim.x) {
            if (idx < wout * win) {
                const int j = idx / wout, k = idx - j * wout;  // out[j][k] = W[k][j]
                out[d.off[l] + idx] = theta[d.off[l] + k * win + j];
            } else {
                out[d.off[l] + idx] = theta[d.off[l] + idx];
            }
        }
    }
}

template <int MODE>
static hipError_t launch_sweep_mode(hipStream_t st, const MlpDesc &d, const double *theta, const double *thetaT,
                                    SweepBatch b, double *partial) {
    SweepLds lay = sweep_lds_layout(d);
    const size_t shm = sizeof(double) * (size_t)lay.total;
    static bool attr_set = false;
    if (!attr_set) {
        // allow up to the full 160 KB of LDS of a gfx950 workgroup
        (void)hipFuncSetAttribute((const void *)mlp_sweep_kernel<MODE>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
        attr_set = true;
    }
    const int64_t blocks = (b.n + SWEEP_TILE - 1) / SWEEP_TILE;
    hipLaunchKernelGGL(mlp_sweep_kernel<MODE>, dim3((unsigned)blocks), dim3(SWEEP_THREADS), shm, st, d, lay, theta,
                       thetaT, b, partial);
    return hipGetLastError();
}

size_t mlp_sweep_lds_bytes(const MlpDesc &d) { return sizeof(double) * (size_t)sweep_lds_layout(d).total; }

hipError_t launch_transpose_weights(hipStream_t st, const MlpDesc &d, const double *theta, double *thetaT) {
    hipLaunchKernelGGL(transpose_weights_kernel, dim3(8), dim3(256), 0, st, d, theta, thetaT);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(hipStream_t st, const MlpDesc &d, const double *theta, const double *thetaT,
                              SweepBatch b) {
    if (b.n <= 0) return hipSuccess;
    const int wpad = b.phi ? 0 : rows1d_mfma_wpad(d);
    if (wpad == 0) return launch_sweep_mode<SWEEP_FORWARD>(st, d, theta, thetaT, b, nullptr);
    const size_t shm = sizeof(double) * (size_t)(d.L - 1) * 2 * wpad * RW1_LD;
    if (shm > 64 * 1024) {
        static bool attr = false;
        if (!attr) {
            (void)hipFuncSetAttribute((const void *)mlp_forward_mfma_kernel<false>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, 152 * 1024);
            attr = true;
        }
    }
    const int64_t ntiles = (b.n + RW1_TP - 1) / RW1_TP;
    const unsigned grid = (unsigned)(ntiles < 16384 ? ntiles : 16384);
    hipLaunchKernelGGL(mlp_forward_mfma_kernel<false>, dim3(grid), dim3(256), shm, st, d, wpad, theta, thetaT, b,
                       nullptr, nullptr);
    return hipGetLastError();
}
hipError_t launch_mlp_rows(hipStream_t st, const MlpDesc &d, const double *theta, const double *thetaT,
                           SweepBatch b) {
    if (b.n <= 0) return hipSuccess;
    const int wpad = b.phi ? 0 : rows1d_mfma_wpad(d);
    if (wpad == 0) return launch_sweep_mode<SWEEP_ROWS>(st, d, theta, thetaT, b, nullptr);
    static bool attr = false;
    if (!attr) {
        // the kernel's static LDS (the tile's inputs) comes on top
        (void)hipFuncSetAttribute((const void *)mlp_rows_mfma_kernel<false>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 152 * 1024);
        attr = true;
    }
    const size_t shm = sizeof(double) * (size_t)d.L * 2 * wpad * RW1_LD;
    const int64_t ntiles = (b.n + RW1_TP - 1) / RW1_TP;
    const unsigned grid = (unsigned)(ntiles < 16384 ? ntiles : 16384);
    hipLaunchKernelGGL(mlp_rows_mfma_kernel<false>, dim3(grid), dim3(256), shm, st, d, wpad, theta, thetaT, b, nullptr,
                       nullptr);
    return hipGetLastError();
}

bool mlp_jobs_supported(const MlpDesc &d) { return rows1d_mfma_wpad(d) != 0; }

void mlp_jobs_work(const std::vector<SweepJob> &jobs, std::vector<int2> &work) {
    work.clear();
    for (size_t j = 0; j < jobs.size(); ++j)
        for (int64_t t = 0; t * RW1_TP < jobs[j].b.n; ++t) work.push_back(make_int2((int)j, (int)t));
}

hipError_t launch_mlp_forward_jobs(hipStream_t st, const MlpDesc &d, const SweepJob *d_jobs, const int2 *d_work,
                                   int64_t nwork) {
    const int wpad = rows1d_mfma_wpad(d);
    if (wpad == 0) return hipErrorInvalidValue;
    if (nwork <= 0) return hipSuccess;
    const size_t shm = sizeof(double) * (size_t)(d.L - 1) * 2 * wpad * RW1_LD;
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)mlp_forward_mfma_kernel<true>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 152 * 1024);
        attr = true;
    }
    hipLaunchKernelGGL(mlp_forward_mfma_kernel<true>, dim3((unsigned)nwork), dim3(256), shm, st, d, wpad, nullptr,
                       nullptr, SweepBatch{}, d_jobs, d_work);
    return hipGetLastError();
}

hipError_t launch_mlp_rows_jobs(hipStream_t st, const MlpDesc &d, const SweepJob *d_jobs, const int2 *d_work,
                                int64_t nwork) {
    const int wpad = rows1d_mfma_wpad(d);
    if (wpad == 0) return hipErrorInvalidValue;
    if (nwork <= 0) return hipSuccess;
    const size_t shm = sizeof(double) * (size_t)d.L * 2 * wpad * RW1_LD;
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)mlp_rows_mfma_kernel<true>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 152 * 1024);
        attr = true;
    }
    hipLaunchKernelGGL(mlp_rows_mfma_kernel<true>, dim3((unsigned)nwork), dim3(256), shm, st, d, wpad, nullptr,
                       nullptr, SweepBatch{}, d_jobs, d_work);
    return hipGetLastError();
}
int64_t mlp_vjp_partials(const MlpDesc &, int64_t n) { return (n + SWEEP_TILE - 1) / SWEEP_TILE; }
hipError_t launch_mlp_vjp(hipStream_t st, const MlpDesc &d, const double *theta, const double *thetaT,
                          SweepBatch b, double *partial, int64_t *n_partials) {
    *n_partials = mlp_vjp_partials(d, b.n);
    if (b.n <= 0) return hipSuccess;
    return launch_sweep_mode<SWEEP_VJP>(st, d, theta, thetaT, b, partial);
}

// Fourier features of the network input q: rows k < F cos(b_k q), F <= k < 2F
// sin(b_k q), then their q-derivatives in rows 2F .. 4F-1 (out[k * ld + i]).
__global__ void fourier_features_kernel(int64_t n, const double *__restrict__ q, int F, const double *__restrict__ b,
                                        double *__restrict__ out, int64_t ld) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = q[i];
    for (int k = 0; k < F; ++k) {
        double sn, cs;
        sincos(b[k] * x, &sn, &cs);
        out[k * ld + i] = cs;
        out[(F + k) * ld + i] = sn;
        out[(2 * F + k) * ld + i] = -b[k] * sn;
        out[(3 * F + k) * ld + i] = b[k] * cs;
    }
}

hipError_t launch_fourier_features(hipStream_t st, int64_t n, const double *q, int F, const double *b, double *out,
                                   int64_t ld) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fourier_features_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, q, F, b, out, ld);
    return hipGetLastError();
}

// ------------------------------------------------------------------ residual
__device__ __forceinline__ void atomic_max_nonneg(unsigned long long *p, double v) {
    if (p == nullptr) return;
    if (!(v == v)) v = __builtin_inf();  // NaN counts as +inf so it is visible
    atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

// 64 points per workgroup of four waves.  The nodes are staged through LDS
// in chunks of RES_PTS (t_j, w_j, Theta_j); each wave sums its points' Hilbert
// terms over its quarter of every chunk in node order, and the four partial
// sums are added in wave order (deterministic).  The node values are LDS
// broadcasts and consecutive terms are independent, so the divisions
// pipeline; four waves per point give the small point sets (8192 collocation
// points, or one instance of a batch) four times as many waves as one thread
// per point would.
static constexpr int RES_PTS = 256;                 // nodes staged per chunk
static constexpr int RES_WG_PTS = 64, RES_SPLIT = 4;  // points per workgroup, waves per point
// JOBS: one 64-point block per workgroup from a work table (job, block) over
// the residuals of many point sets (the instances of a batch).
template <bool JOBS>
__global__ __launch_bounds__(RES_PTS) void ccf_residual_kernel(ResidualArgs a0, const ResidualArgs *__restrict__ jobs,
                                                               const int2 *__restrict__ work) {
    __shared__ double tn[RES_PTS], wn[RES_PTS], thn[RES_PTS];
    __shared__ double Us[RES_SPLIT][RES_WG_PTS], cs[RES_SPLIT][RES_WG_PTS];
    int64_t blk = blockIdx.x;
    if (JOBS) {
        const int2 wk = work[blockIdx.x];
        if (wk.x < 0) return;
        blk = wk.y;
    }
    const ResidualArgs a = JOBS ? jobs[work[blockIdx.x].x] : a0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i = blk * RES_WG_PTS + lane;
    const bool valid = i < a.n;
    const int64_t ii = valid ? i : a.n - 1;
    const double yi = a.pts.y[ii];
    const double Ei = a.pts.E[ii];
    const double NNi = a.nn[ii];
    const double Thi = Ei * NNi;
    const double y2 = 2.0 * yi;
    // the four waves of a workgroup take the same 64 points and a quarter of
    // each staged chunk of nodes each; their partial sums are added in wave
    // order (deterministic)
    double U = 0.0, c = 0.0;
    for (int64_t j0 = 0; j0 < a.m; j0 += RES_PTS) {
        const int64_t j = j0 + threadIdx.x;
        if (j < a.m) {
            tn[threadIdx.x] = a.nodes.y[j];
            wn[threadIdx.x] = a.nodes.wh[j];
            thn[threadIdx.x] = a.nodes.E[j] * a.nn_nodes[j];
        }
        __syncthreads();
        const int cnt = (a.m - j0) < RES_PTS ? (int)(a.m - j0) : RES_PTS;
        const int kb = w * (RES_PTS / RES_SPLIT), ke = kb + RES_PTS / RES_SPLIT < cnt ? kb + RES_PTS / RES_SPLIT : cnt;
#pragma unroll 4
        for (int k = kb; k < ke; ++k) {
            const double tj = tn[k];
            const double qij = wn[k] * y2 / ((yi - tj) * (yi + tj));
            U = fma(qij, thn[k] - Thi, U);
            c += qij;
        }
        __syncthreads();
    }
    Us[w][lane] = U;
    cs[w][lane] = c;
    __syncthreads();
    if (w != 0) return;
    U = ((Us[0][lane] + Us[1][lane]) + Us[2][lane]) + Us[3][lane];
    c = ((cs[0][lane] + cs[1][lane]) + cs[2][lane]) + cs[3][lane];
    const double lam = a.lam;
    const double NNq = a.nn[a.n + ii];
    const double Eyi = a.pts.Ey[ii], qyi = a.pts.qy[ii];
    const double Thy = Eyi * NNi + Ei * qyi * NNq;
    // second stage: R_1 + eps D[Theta_1] Theta, D Phi = -lam Phi + V_1 Phi' + U[Phi] Theta_1'
    const bool lin = a.R1 != nullptr;
    const double V = lin ? a.V1[ii] : (1.0 + lam) * yi + U;
    const double Ty = lin ? a.T1y[ii] : Thy;     // coefficient of U (and its seed)
    const double g = lin ? a.eps : 1.0;
    const double R = lin ? a.R1[ii] + a.eps * (-lam * Thi + V * Thy + U * Ty) : -lam * Thi + V * Thy;
    // max |R| over the wave on the bit patterns (a NaN stays largest), one atomic per wave
    unsigned long long mb = valid ? (unsigned long long)__double_as_longlong(fabs(R)) : 0ull;
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long other = __shfl_xor(mb, o, 64);
        mb = other > mb ? other : mb;
    }
    if ((threadIdx.x & 63) == 0 && mb != 0ull) atomic_max_nonneg(a.max_out, __longlong_as_double((long long)mb));
    if (!valid) return;
    if (a.R) a.R[i] = R;
    if (a.V_out) a.V_out[i] = V;
    if (a.Ty_out) a.Ty_out[i] = Thy;
    if (a.r) {
        const double sc = sqrt((a.rho ? a.rho[i] : 1.0) * a.inv_n);
        a.r[i * a.r_stride] = sc * (R - (a.f ? a.f[i] : 0.0));
        if (a.seed0) {
            // dR/dNN_i (including U's dependence on Theta_i via -c_i E_i) and dR/dNN_q,i
            a.seed0[i] = sc * g * (-lam * Ei + V * Eyi - Ty * c * Ei);
            a.seed1[i] = sc * g * (V * Ei * qyi);
        }
        if (a.cscale) a.cscale[i] = sc * g * Ty;
    }
}

// Local variant: R = -lam U + ((1+lam) y + U) U_y with U = Theta.
__global__ void burgers_residual_kernel(ResidualArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const double lam = a.lam;
    const double yi = a.pts.y[i], Ei = a.pts.E[i], Eyi = a.pts.Ey[i], qyi = a.pts.qy[i];
    const double NNi = a.nn[i], NNq = a.nn[a.n + i];
    const double Th = Ei * NNi;
    const double Thy = Eyi * NNi + Ei * qyi * NNq;
    // second stage (U[Phi] = Phi): R_1 + eps (-lam Phi + V_1 Phi' + Phi Theta_1')
    const bool lin = a.R1 != nullptr;
    const double V = lin ? a.V1[i] : (1.0 + lam) * yi + Th;
    const double Ty = lin ? a.T1y[i] : Thy;
    const double g = lin ? a.eps : 1.0;
    const double R = lin ? a.R1[i] + a.eps * (-lam * Th + V * Thy + Th * Ty) : -lam * Th + V * Thy;
    if (a.R) a.R[i] = R;
    if (a.V_out) a.V_out[i] = V;
    if (a.Ty_out) a.Ty_out[i] = Thy;
    atomic_max_nonneg(a.max_out, fabs(R));
    if (a.r) {
        const double sc = sqrt((a.rho ? a.rho[i] : 1.0) * a.inv_n);
        a.r[i * a.r_stride] = sc * (R - (a.f ? a.f[i] : 0.0));
        if (a.seed0) {
            a.seed0[i] = sc * g * ((Ty - lam) * Ei + V * Eyi);
            a.seed1[i] = sc * g * (V * Ei * qyi);
        }
        if (a.cscale) a.cscale[i] = 0.0;
    }
}

hipError_t launch_residual(hipStream_t st, const ResidualArgs &a) {
    if (a.n <= 0) return hipSuccess;
    if (a.equation == GN_EQ_CCF1D) {
        hipLaunchKernelGGL(ccf_residual_kernel<false>, dim3((unsigned)((a.n + RES_WG_PTS - 1) / RES_WG_PTS)),
                           dim3(RES_PTS), 0, st, a, nullptr, nullptr);
    } else {
        hipLaunchKernelGGL(burgers_residual_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

void residual_jobs_work(const ResidualArgs *jobs, int n, std::vector<int2> &work) {
    work.clear();
    for (int j = 0; j < n; ++j)
        for (int64_t k = 0; k * RES_WG_PTS < jobs[j].n; ++k) work.push_back(make_int2(j, (int)k));
}

hipError_t launch_residual_jobs(hipStream_t st, const ResidualArgs *d_jobs, const int2 *d_work, int64_t nwork) {
    if (nwork <= 0) return hipSuccess;
    hipLaunchKernelGGL(ccf_residual_kernel<true>, dim3((unsigned)nwork), dim3(RES_PTS), 0, st, ResidualArgs{}, d_jobs,
                       d_work);
    return hipGetLastError();
}

__global__ void norm_row_kernel(const double *nn1, double sqrt_c, double target, double *r_out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) r_out[0] = sqrt_c * (nn1[0] - target);
}

hipError_t launch_norm_row(hipStream_t st, const double *nn1, double sqrt_c, double target, double *r_out) {
    hipLaunchKernelGGL(norm_row_kernel, dim3(1), dim3(64), 0, st, nn1, sqrt_c, target, r_out);
    return hipGetLastError();
}

// out_j = E_j sum_i Q_ij v_i cscale_i: one wave per node j, lanes stride over
// the points of row j of Q^T in order, then a fixed butterfly (deterministic).
__global__ __launch_bounds__(256) void hilbert_adjoint_kernel(int64_t n, int64_t m, const double *__restrict__ QT,
                                                              int64_t ld, const double *__restrict__ v,
                                                              const double *__restrict__ cs,
                                                              const double *__restrict__ E, double *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= m) return;
    const double *row = QT + j * ld;
    double acc = 0.0;
    for (int64_t i = lane; i < n; i += 64) acc = fma(row[i], v[i] * cs[i], acc);
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) out[j] = E[j] * acc;
}

int64_t hilbert_adjoint_work_size(int64_t) { return 0; }

hipError_t launch_hilbert_adjoint(hipStream_t st, int64_t n, int64_t m, const double *QT, int64_t ld,
                                  const double *v, const double *cscale, const double *E_nodes, double *out,
                                  double *) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(hilbert_adjoint_kernel, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st, n, m, QT, ld, v,
                       cscale, E_nodes, out);
    return hipGetLastError();
}

}  // namespace gn
