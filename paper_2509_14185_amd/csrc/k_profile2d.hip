// 2D self-similar profile stand-ins on gfx950 (paper, Methods, "Solution
// Modeling and Equation Factorisation"): compactified network inputs
// q = (1+|y|^2)^{-1/(2(1+lam))}, beta = y2 / sqrt(1+|y|^2); tanh MLP; each
// field is a symmetry prefactor times a network output times a decay factor.
//
// Everything is carried as second-order jets in y: 6 components
// (f, f_1, f_2, f_11, f_12, f_22), composed by the product and chain rules.
//   - geometry2d: y from the s-coordinates and the input jets of (q, beta);
//   - jet sweeps: forward jets of the network outputs at points, and per row
//     a reverse sweep of the row's seeds (dR/d(output jets)) through the jets,
//     which is that row of the parameter Jacobian;
//   - residual2d: residual rows and their seeds (IPM-style: equation, d1 and
//     symmetry rows; Boussinesq-type: three equations per point and y2 = 0
//     boundary rows), the normalisation row, max |R|.
#include "gn_internal.h"
#include "tile_loader.h"

namespace gn {

struct J6 {
    double c[6];
};

__device__ __forceinline__ J6 j6_zero() { return J6{{0.0, 0.0, 0.0, 0.0, 0.0, 0.0}}; }

__device__ __forceinline__ J6 j6_var(double y, int a) {
    J6 r = j6_zero();
    r.c[0] = y;
    r.c[a] = 1.0;
    return r;
}

__device__ __forceinline__ J6 j6_add(const J6 &f, const J6 &g) {
    J6 r;
#pragma unroll
    for (int i = 0; i < 6; ++i) r.c[i] = f.c[i] + g.c[i];
    return r;
}

__device__ __forceinline__ J6 j6_mul(const J6 &f, const J6 &g) {
    J6 r;
    r.c[0] = f.c[0] * g.c[0];
    r.c[1] = f.c[1] * g.c[0] + f.c[0] * g.c[1];
    r.c[2] = f.c[2] * g.c[0] + f.c[0] * g.c[2];
    r.c[3] = f.c[3] * g.c[0] + 2.0 * f.c[1] * g.c[1] + f.c[0] * g.c[3];
    r.c[4] = f.c[4] * g.c[0] + f.c[1] * g.c[2] + f.c[2] * g.c[1] + f.c[0] * g.c[4];
    r.c[5] = f.c[5] * g.c[0] + 2.0 * f.c[2] * g.c[2] + f.c[0] * g.c[5];
    return r;
}

// phi(f) from phi(f0) = v, phi'(f0) = d1, phi''(f0) = d2
__device__ __forceinline__ J6 j6_chain(const J6 &f, double v, double d1, double d2) {
    J6 r;
    r.c[0] = v;
    r.c[1] = d1 * f.c[1];
    r.c[2] = d1 * f.c[2];
    r.c[3] = d2 * f.c[1] * f.c[1] + d1 * f.c[3];
    r.c[4] = d2 * f.c[1] * f.c[2] + d1 * f.c[4];
    r.c[5] = d2 * f.c[2] * f.c[2] + d1 * f.c[5];
    return r;
}

__device__ __forceinline__ J6 j6_pow(const J6 &f, double m) {
    const double x = f.c[0], v = pow(x, m);
    return j6_chain(f, v, m * v / x, m * (m - 1.0) * v / (x * x));
}

// y1, y2, u = 1 + |y|^2
__device__ __forceinline__ void base_jets(double y1, double y2, J6 &Y1, J6 &Y2, J6 &U) {
    Y1 = j6_var(y1, 1);
    Y2 = j6_var(y2, 2);
    U = j6_add(j6_mul(Y1, Y1), j6_mul(Y2, Y2));
    U.c[0] += 1.0;
}

// Envelope jets of the fields (same readings as the oracle):
//   IPM-style: (y1/rho) q;  Boussinesq-type: (y1/rho) q, q, (y1/rho) q u.
__device__ __forceinline__ int envelopes2d(int equation, double y1, double y2, double lam, J6 *E) {
    J6 Y1, Y2, U;
    base_jets(y1, y2, Y1, Y2, U);
    const J6 q = j6_pow(U, -1.0 / (2.0 * (1.0 + lam)));
    const J6 odd = j6_mul(Y1, j6_pow(U, -0.5));
    E[0] = j6_mul(odd, q);
    if (equation == GN_EQ_IPM2D) return 1;
    E[1] = q;
    E[2] = j6_mul(E[0], U);
    return 3;
}

// ------------------------------------------------------------ geometry
__global__ void geometry2d_kernel(int64_t n, const double *__restrict__ s, int edge, double lam, Pts2D p,
                                  int64_t off) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double s1 = edge ? s[i] : s[2 * i], s2 = edge ? 0.0 : s[2 * i + 1];
    const double y1 = s1 / (1.0 - s1), y2 = s2 / (1.0 - s2);
    J6 Y1, Y2, U;
    base_jets(y1, y2, Y1, Y2, U);
    const J6 q = j6_pow(U, -1.0 / (2.0 * (1.0 + lam)));
    const J6 beta = j6_mul(Y2, j6_pow(U, -0.5));
    const int64_t k = off + i;
    p.y1[k] = y1;
    p.y2[k] = y2;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        p.xin[c * p.ld + k] = q.c[c];
        p.xin[(6 + c) * p.ld + k] = beta.c[c];
    }
}

hipError_t launch_geometry2d(hipStream_t st, int64_t n, const double *s, int edge, double lam, Pts2D p,
                             int64_t off) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(geometry2d_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, s, edge, lam, p,
                       off);
    return hipGetLastError();
}

// ------------------------------------------------------------ residual rows and seeds
// Seeds on the network-output jets from seeds on the field jets
// (Phi = E N by the product rule, transposed).
__device__ __forceinline__ void field_to_output_seeds(const J6 &E, const double *sp, double *sn) {
    sn[0] = E.c[0] * sp[0] + E.c[1] * sp[1] + E.c[2] * sp[2] + E.c[3] * sp[3] + E.c[4] * sp[4] + E.c[5] * sp[5];
    sn[1] = E.c[0] * sp[1] + 2.0 * E.c[1] * sp[3] + E.c[2] * sp[4];
    sn[2] = E.c[0] * sp[2] + E.c[1] * sp[4] + 2.0 * E.c[2] * sp[5];
    sn[3] = E.c[0] * sp[3];
    sn[4] = E.c[0] * sp[4];
    sn[5] = E.c[0] * sp[5];
}

// One thread per row.  Rows (RowMap2D): n points x n_eq equation rows
// (fields interleaved per point), 2 n1 d1 rows, ne y2 = 0 rows, the
// normalisation row.  In validation mode (a.validation) the rows are the
// n x n_eq equation rows at the validation points and only max |R| is kept.
__global__ void residual2d_kernel(Res2DArgs a) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nrow = a.validation ? a.map.n * a.map.n_eq : a.map.rows();
    if (row >= nrow) return;
    int kind, comp;
    const int64_t pt = a.map.point_of(row, kind, comp);
    const double lam = a.lam;
    const int nout = a.nout;
    double nn[3][6];
    for (int f = 0; f < nout; ++f)
#pragma unroll
        for (int c = 0; c < 6; ++c) nn[f][c] = a.nn[(f * 6 + c) * a.ldn + pt];
    double sn[3][6];
    for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int c = 0; c < 6; ++c) sn[f][c] = 0.0;
    double value = 0.0, scale = 1.0;
    if (kind == 3) {  // normalisation row: sqrt(c) (NN_0(origin) - target)
        scale = sqrt(a.c_norm);
        value = nn[0][0] - a.c_target;
        sn[0][0] = 1.0;
    } else {
        const double y1 = a.pts.y1[pt], y2 = a.pts.y2[pt];
        J6 E[3];
        envelopes2d(a.equation, y1, y2, lam, E);
        double F[3][6];  // field jets
        for (int f = 0; f < nout; ++f) {
            J6 N;
#pragma unroll
            for (int c = 0; c < 6; ++c) N.c[c] = nn[f][c];
            const J6 Ph = j6_mul(E[f], N);
#pragma unroll
            for (int c = 0; c < 6; ++c) F[f][c] = Ph.c[c];
        }
        double sp[3][6];  // seeds on the field jets
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int c = 0; c < 6; ++c) sp[f][c] = 0.0;
        if (a.equation == GN_EQ_IPM2D) {
            const double *P = F[0];
            const double V1 = (1.0 + lam) * y1 + P[0], V2 = (1.0 + lam) * y2;
            if (kind == 0) {  // R = Phi + V1 Phi_1 + V2 Phi_2
                value = P[0] + V1 * P[1] + V2 * P[2];
                sp[0][0] = 1.0 + P[1];
                sp[0][1] = V1;
                sp[0][2] = V2;
                scale = a.scale_eq;
            } else if (kind == 1 && comp == 0) {  // dR/dy1
                value = P[1] + (1.0 + lam + P[1]) * P[1] + V1 * P[3] + V2 * P[4];
                sp[0][0] = P[3];
                sp[0][1] = 2.0 + lam + 2.0 * P[1];
                sp[0][3] = V1;
                sp[0][4] = V2;
                scale = a.scale_d1;
            } else if (kind == 1) {  // dR/dy2
                value = P[2] + P[2] * P[1] + V1 * P[4] + (1.0 + lam) * P[2] + V2 * P[5];
                sp[0][0] = P[4];
                sp[0][1] = P[2];
                sp[0][2] = 2.0 + lam + P[1];
                sp[0][4] = V1;
                sp[0][5] = V2;
                scale = a.scale_d1;
            } else {  // dPhi/dy2 on y2 = 0
                value = P[2];
                sp[0][2] = 1.0;
                scale = a.scale_edge;
            }
        } else {
            const double *Om = F[0], *Th = F[1], *Ps = F[2];
            const double V1 = (1.0 + lam) * y1 - Ps[2], V2 = (1.0 + lam) * y2 + Ps[1];
            if (kind == 0 && comp == 0) {  // R_Omega = Omega + V.grad Omega - Theta_1
                value = Om[0] + V1 * Om[1] + V2 * Om[2] - Th[1];
                sp[0][0] = 1.0;
                sp[0][1] = V1;
                sp[0][2] = V2;
                sp[1][1] = -1.0;
                sp[2][2] = -Om[1];
                sp[2][1] = Om[2];
            } else if (kind == 0 && comp == 1) {  // R_Theta = (1-lam) Theta + V.grad Theta
                value = (1.0 - lam) * Th[0] + V1 * Th[1] + V2 * Th[2];
                sp[1][0] = 1.0 - lam;
                sp[1][1] = V1;
                sp[1][2] = V2;
                sp[2][2] = -Th[1];
                sp[2][1] = Th[2];
            } else if (kind == 0) {  // R_Psi = Psi_11 + Psi_22 - Omega
                value = Ps[3] + Ps[5] - Om[0];
                sp[2][3] = 1.0;
                sp[2][5] = 1.0;
                sp[0][0] = -1.0;
            } else {  // Psi(y1, 0)
                value = Ps[0];
                sp[2][0] = 1.0;
            }
            scale = (kind == 0) ? a.scale_eq : a.scale_edge;
        }
        for (int f = 0; f < nout; ++f) {
            J6 Ef = E[f];
            field_to_output_seeds(Ef, sp[f], sn[f]);
        }
        if (kind == 0 && a.max_out) atomic_max_abs(a.max_out, value);
    }
    if (a.validation) return;
    if (a.r) a.r[row * a.r_stride] = scale * value;
    if (a.seeds) {
        for (int f = 0; f < nout; ++f)
#pragma unroll
            for (int c = 0; c < 6; ++c) a.seeds[(f * 6 + c) * a.lds + row] = scale * sn[f][c];
    }
}

hipError_t launch_residual2d(hipStream_t st, const Res2DArgs &a) {
    const int64_t nrow = a.validation ? a.map.n * a.map.n_eq : a.map.rows();
    if (nrow <= 0) return hipSuccess;
    hipLaunchKernelGGL(residual2d_kernel, dim3((unsigned)((nrow + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

// ------------------------------------------------------------ jet sweeps
// A workgroup handles T rows (or points).  LDS per row: the input jets
// (6 x 2), the hidden activations as h-jets (6 x w per hidden layer), and
// two adjoint buffers (6 x maxw).  The reverse rule of h = tanh(z) in jet
// form needs only the h-jets (s = 1 - t^2, t = h):
//   zb_ab = s hb_ab,
//   zb_1 = s hb_1 - 2t (2 h_1 hb_11 + h_2 hb_12),
//   zb_2 = s hb_2 - 2t (h_1 hb_12 + 2 h_2 hb_22),
//   zb_0 = s hb_0 - 2t (h_1 hb_1 + h_2 hb_2) - sum_ab hb_ab (2t h_ab + 2 h_a h_b).
enum Sweep2DMode { SW2_FORWARD = 0, SW2_ROWS = 1, SW2_VJP = 2 };
static constexpr int64_t VJP2D_MAX_BLOCKS = 1024;  // partial P-vectors of a VJP

struct Sweep2DLds {
    int in_off;
    int act_off[GN_MAX_LAYERS + 1];
    int zb_off;
    int maxw;
    int tile;
    int total;
};

static Sweep2DLds sweep2d_layout(const MlpDesc &d) {
    Sweep2DLds s{};
    int per = 12, maxw = 1;
    for (int l = 1; l < d.L; ++l) {
        per += 6 * d.w[l];
        if (d.w[l] > maxw) maxw = d.w[l];
    }
    if (d.w[d.L] > maxw) maxw = d.w[d.L];
    per += 12 * maxw;
    int tile = (int)((160 * 1024 / 8 - 64) / per);
    if (tile > 8) tile = 8;
    s.tile = tile;
    s.maxw = maxw;
    int o = 0;
    s.in_off = o;
    o += 12 * tile;
    for (int l = 1; l < d.L; ++l) {
        s.act_off[l] = o;
        o += 6 * tile * d.w[l];
    }
    s.zb_off = o;
    o += 12 * tile * maxw;
    s.total = o;
    return s;
}

template <int MODE>
__global__ __launch_bounds__(256) void jet_sweep2d_kernel(MlpDesc d, Sweep2DLds lay, const double *__restrict__ theta,
                                                          const double *__restrict__ thetaT, Sweep2DArgs b) {
    extern __shared__ double sm[];
    const int tid = threadIdx.x;
    const int T = lay.tile;
    const int L = d.L;
    // Tiles of T rows; a workgroup takes tiles blockIdx.x, + gridDim.x, ...
    // (VJP grids are capped; the workgroup's partial sums its tiles in order).
    const int64_t ntiles = (b.nrows + T - 1) / T;
    for (int64_t tile = blockIdx.x, it = 0; tile < ntiles; tile += gridDim.x, ++it) {
    if (it > 0) __syncthreads();  // LDS of the previous tile is no longer read
    const int64_t r0 = tile * T;
    const int nr = (int)((b.nrows - r0) < T ? (b.nrows - r0) : T);
    // rows -> points, input jets
    for (int idx = tid; idx < nr * 12; idx += 256) {
        const int t = idx / 12, c = idx - t * 12;
        const int64_t row = b.row0 + r0 + t;
        int64_t pt = row;
        if (MODE != SW2_FORWARD) {
            int kind, comp;
            pt = b.map.point_of(row, kind, comp);
        }
        sm[lay.in_off + t * 12 + c] = b.pts.xin[c * b.pts.ld + pt];
    }
    __syncthreads();
    // input jet c of unit j of the layer-l input, row t
    auto hin = [&](int l, int t, int c, int j) -> double {
        return (l == 0) ? sm[lay.in_off + t * 12 + j * 6 + c] : sm[lay.act_off[l] + (t * 6 + c) * d.w[l] + j];
    };

    // ---------------- forward through the hidden layers
    for (int l = 0; l < L - 1; ++l) {
        const int win = d.w[l], wout = d.w[l + 1];
        const double *Wt = thetaT + d.off[l];  // Wt[j][k] = W[k][j]
        const double *bias = theta + d.off[l] + win * wout;
        for (int idx = tid; idx < nr * wout; idx += 256) {
            const int t = idx / wout, k = idx - t * wout;
            double z[6] = {bias[k], 0.0, 0.0, 0.0, 0.0, 0.0};
            for (int j = 0; j < win; ++j) {
                const double w = Wt[j * wout + k];
#pragma unroll
                for (int c = 0; c < 6; ++c) z[c] = fma(w, hin(l, t, c, j), z[c]);
            }
            const double th = tanh(z[0]), s = 1.0 - th * th;
            const double h1 = s * z[1], h2 = s * z[2];
            double *o = sm + lay.act_off[l + 1] + t * 6 * wout + k;
            o[0] = th;
            o[wout] = h1;
            o[2 * wout] = h2;
            o[3 * wout] = s * z[3] - 2.0 * th * h1 * z[1];
            o[4 * wout] = s * z[4] - 2.0 * th * h1 * z[2];
            o[5 * wout] = s * z[5] - 2.0 * th * h2 * z[2];
        }
        __syncthreads();
    }
    // ---------------- output layer (linear)
    const int lo = L - 1, win_o = d.w[lo], nout = d.w[L];
    double *zb = sm + lay.zb_off, *zbn = zb + 6 * T * lay.maxw;
    const int ldz = lay.maxw;  // zb[(t*6 + c)*ldz + k]
    if (MODE == SW2_FORWARD) {
        const double *W = theta + d.off[lo];
        const double *bias = W + win_o * nout;
        for (int idx = tid; idx < nr * nout * 6; idx += 256) {
            const int t = idx / (nout * 6), rem = idx - t * nout * 6, o = rem / 6, c = rem - o * 6;
            double z = (c == 0) ? bias[o] : 0.0;
            for (int j = 0; j < win_o; ++j) z = fma(W[o * win_o + j], hin(lo, t, c, j), z);
            b.nn[(o * 6 + c) * b.ldn + r0 + t] = z;
        }
        continue;
    }
    for (int idx = tid; idx < nr * nout * 6; idx += 256) {
        const int t = idx / (nout * 6), rem = idx - t * nout * 6, o = rem / 6, c = rem - o * 6;
        const int64_t row = b.row0 + r0 + t;
        double sd = b.seeds[(o * 6 + c) * b.lds + row];
        if (MODE == SW2_VJP) sd *= b.v[row];
        zb[(t * 6 + c) * ldz + o] = sd;
    }
    __syncthreads();

    // ---------------- reverse sweep, layer l = L-1 .. 0
    for (int l = L - 1; l >= 0; --l) {
        const int win = d.w[l], wout = d.w[l + 1];
        const int nseg = wout * (win + 1);  // W^l then b^l
        if (MODE == SW2_ROWS) {
            for (int t = 0; t < nr; ++t) {
                double *row = b.J + (r0 + t) * b.ldJ + d.off[l];
                for (int idx = tid; idx < nseg; idx += 256) {
                    double v;
                    if (idx < wout * win) {
                        const int k = idx / win, j = idx - k * win;
                        v = 0.0;
#pragma unroll
                        for (int c = 0; c < 6; ++c) v = fma(zb[(t * 6 + c) * ldz + k], hin(l, t, c, j), v);
                    } else {
                        v = zb[(t * 6) * ldz + (idx - wout * win)];
                    }
                    row[idx] = v;
                }
            }
        } else {  // SW2_VJP: sum over the rows of this workgroup, fixed order
            double *out = b.partial + (int64_t)blockIdx.x * d.P + d.off[l];
            for (int idx = tid; idx < nseg; idx += 256) {
                double acc = 0.0;
                if (idx < wout * win) {
                    const int k = idx / win, j = idx - k * win;
                    for (int t = 0; t < nr; ++t) {
                        double v = 0.0;
#pragma unroll
                        for (int c = 0; c < 6; ++c) v = fma(zb[(t * 6 + c) * ldz + k], hin(l, t, c, j), v);
                        acc += v;
                    }
                } else {
                    const int k = idx - wout * win;
                    for (int t = 0; t < nr; ++t) acc += zb[(t * 6) * ldz + k];
                }
                out[idx] = (it == 0) ? acc : out[idx] + acc;
            }
        }
        if (l == 0) break;
        // hbar = W^T zbar per jet component, then back through tanh
        const double *W = theta + d.off[l];  // wout x win
        for (int idx = tid; idx < nr * win; idx += 256) {
            const int t = idx / win, j = idx - t * win;
            double hb[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            for (int k = 0; k < wout; ++k) {
                const double w = W[k * win + j];
#pragma unroll
                for (int c = 0; c < 6; ++c) hb[c] = fma(w, zb[(t * 6 + c) * ldz + k], hb[c]);
            }
            const double *h = sm + lay.act_off[l] + t * 6 * win + j;
            const double th = h[0], h1 = h[win], h2 = h[2 * win], h11 = h[3 * win], h12 = h[4 * win],
                         h22 = h[5 * win];
            const double s = 1.0 - th * th, t2 = 2.0 * th;
            double *o = zbn + (t * 6) * ldz + j;
            o[3 * ldz] = s * hb[3];
            o[4 * ldz] = s * hb[4];
            o[5 * ldz] = s * hb[5];
            o[ldz] = s * hb[1] - t2 * (2.0 * h1 * hb[3] + h2 * hb[4]);
            o[2 * ldz] = s * hb[2] - t2 * (h1 * hb[4] + 2.0 * h2 * hb[5]);
            o[0] = s * hb[0] - t2 * (h1 * hb[1] + h2 * hb[2]) - hb[3] * (t2 * h11 + 2.0 * h1 * h1) -
                   hb[4] * (t2 * h12 + 2.0 * h1 * h2) - hb[5] * (t2 * h22 + 2.0 * h2 * h2);
        }
        __syncthreads();
        double *tmp = zb;
        zb = zbn;
        zbn = tmp;
    }
    }
}

// ---- forward jets on the matrix cores
// Each layer of the forward sweep is a product: for the six jet components
// c of 16 points, Z_c = W H_c (+ bias for c = 0), W wout x win, H_c win x 16.
// A workgroup (four waves) takes 16 points at a time; wave w forms the
// 16-unit tiles w, w + 4 of Z for all six components with
// v_mfma_f64_16x16x4f64 (A = W from the transposed weights through L1/L2,
// B = H_c from LDS), so every lane ends with all six components of its
// (unit, point) entries and applies the tanh jet rules in registers; the
// result overwrites H in LDS (after a barrier) as the next layer's input.
// LDS: H[c][j][t], 6 x wpad x 16 doubles (wpad = the widest layer input
// rounded up to 16, at most 128).  Units beyond a layer's width come out as
// tanh(0) = 0 with zero derivatives, which is the zero padding of the next
// layer's K; the input layer's K is padded from 2 to 4.
static constexpr int FW2_TP = 16;

template <int UT>
__global__ __launch_bounds__(256) void jet_forward2d_mfma_kernel(MlpDesc d, int wpad, const double *__restrict__ theta,
                                                                 const double *__restrict__ thetaT, Sweep2DArgs b) {
    extern __shared__ double hs[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int fr = lane & 15, fk = lane >> 4;
    const int L = d.L;
    auto H = [&](int c, int j, int t) -> double & { return hs[(c * wpad + j) * FW2_TP + t]; };
    const int64_t ntiles = (b.nrows + FW2_TP - 1) / FW2_TP;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t p0 = tile * FW2_TP;
        const int nr = (int)((b.nrows - p0) < FW2_TP ? (b.nrows - p0) : FW2_TP);
        __syncthreads();  // the previous tile's reads of H are done
        for (int idx = tid; idx < 6 * 4 * FW2_TP; idx += 256) {
            const int c = idx / (4 * FW2_TP), j = (idx / FW2_TP) & 3, t = idx % FW2_TP;
            H(c, j, t) = (j < 2 && t < nr) ? b.pts.xin[(j * 6 + c) * b.pts.ld + b.row0 + p0 + t] : 0.0;
        }
        __syncthreads();
        for (int l = 0; l < L; ++l) {
            const int win = d.w[l], wout = d.w[l + 1];
            const int kpad = (win + 3) & ~3, nut = (wout + 15) / 16;
            const double *Wt = thetaT + d.off[l];  // Wt[j][k] = W[k][j]
            const double *bias = theta + d.off[l] + win * wout;
            double4_t acc[UT][6];
#pragma unroll
            for (int u = 0; u < UT; ++u) {
#pragma unroll
                for (int c = 0; c < 6; ++c) acc[u][c] = (double4_t){0.0, 0.0, 0.0, 0.0};
                const int ui = wave + 4 * u;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int k = 16 * ui + fk + 4 * r;
                    acc[u][0][r] = (ui < nut && k < wout) ? bias[k] : 0.0;
                }
            }
            // K in chunks of four k-steps: the chunk's weight and H fragments are
            // all loaded before its MFMAs (steps past kpad contribute zeros)
            for (int s0 = 0; s0 < kpad; s0 += 16) {
                double bf[4][6], a[UT][4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int j = s0 + 4 * q + fk;
                    const bool in = s0 + 4 * q < kpad;
#pragma unroll
                    for (int c = 0; c < 6; ++c) bf[q][c] = in ? H(c, j, fr) : 0.0;
#pragma unroll
                    for (int u = 0; u < UT; ++u) {
                        const int k = 16 * (wave + 4 * u) + fr;
                        a[u][q] = (in && k < wout && j < win) ? Wt[j * wout + k] : 0.0;
                    }
                }
#pragma unroll
                for (int u = 0; u < UT; ++u) {
                    if (wave + 4 * u >= nut) continue;  // uniform over the wave
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int c = 0; c < 6; ++c)
                            acc[u][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][q], bf[q][c], acc[u][c], 0, 0, 0);
                }
            }
            __syncthreads();  // every read of this layer's input is done
            if (l < L - 1) {
#pragma unroll
                for (int u = 0; u < UT; ++u) {
                    const int ui = wave + 4 * u;
                    if (ui >= nut) continue;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int k = 16 * ui + fk + 4 * r;
                        const double z1 = acc[u][1][r], z2 = acc[u][2][r];
                        const double th = tanh(acc[u][0][r]), sd = 1.0 - th * th;
                        const double h1 = sd * z1, h2 = sd * z2;
                        H(0, k, fr) = th;
                        H(1, k, fr) = h1;
                        H(2, k, fr) = h2;
                        H(3, k, fr) = sd * acc[u][3][r] - 2.0 * th * h1 * z1;
                        H(4, k, fr) = sd * acc[u][4][r] - 2.0 * th * h1 * z2;
                        H(5, k, fr) = sd * acc[u][5][r] - 2.0 * th * h2 * z2;
                    }
                }
                __syncthreads();
            } else {
#pragma unroll
                for (int u = 0; u < UT; ++u) {
                    const int ui = wave + 4 * u;
                    if (ui >= nut) continue;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int k = 16 * ui + fk + 4 * r;
                        if (k < wout && fr < nr)
#pragma unroll
                            for (int c = 0; c < 6; ++c) b.nn[(k * 6 + c) * b.ldn + p0 + fr] = acc[u][c][r];
                    }
                }
            }
        }
    }
}

// ---- rows of J on the matrix cores (hidden widths up to 64)
// A workgroup takes 16 rows at a time, with two LDS planes laid out like H
// above (row stride 17 so that reads along j spread over the banks): H_l,
// the activations entering layer l, and ZB, the adjoint of layer l's output
// jets.  Reverse over the layers: H_l is recomputed by the forward products
// from the input (the l layers below it, (L-1)L/2 layer products in all, so
// no activations are kept across layers), the row entries of (W_l, b_l) are
// sum_c ZB_c[k][t] H_c[j][t] and ZB_0[k][t], and then hb = W_l^T ZB per jet
// component on the MFMA tiles, through the reverse tanh jet rule with H_l
// into the next ZB.
static constexpr int RW2_LD = FW2_TP + 1;

__global__ __launch_bounds__(256) void jet_rows2d_mfma_kernel(MlpDesc d, int wpad, const double *__restrict__ theta,
                                                              const double *__restrict__ thetaT, Sweep2DArgs b) {
    extern __shared__ double sm[];
    __shared__ int64_t pt_sh[FW2_TP];
    double *hs = sm, *zs = sm + 6 * wpad * RW2_LD;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int fr = lane & 15, fk = lane >> 4;
    const int L = d.L, nout = d.w[L];
    auto H = [&](int c, int j, int t) -> double & { return hs[(c * wpad + j) * RW2_LD + t]; };
    auto Z = [&](int c, int k, int t) -> double & { return zs[(c * wpad + k) * RW2_LD + t]; };
    const int64_t ntiles = (b.nrows + FW2_TP - 1) / FW2_TP;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t p0 = tile * FW2_TP;
        const int nr = (int)((b.nrows - p0) < FW2_TP ? (b.nrows - p0) : FW2_TP);
        __syncthreads();  // the previous tile is done with the LDS planes
        if (tid < FW2_TP) {
            int kind, comp;
            pt_sh[tid] = tid < nr ? b.map.point_of(b.row0 + p0 + tid, kind, comp) : -1;
        }
        // the output adjoint: the rows' seeds (zero past nout and past the last row)
        for (int idx = tid; idx < 6 * 16 * FW2_TP; idx += 256) {
            const int c = idx / (16 * FW2_TP), o = (idx / FW2_TP) & 15, t = idx % FW2_TP;
            Z(c, o, t) = (o < nout && t < nr) ? b.seeds[(o * 6 + c) * b.lds + b.row0 + p0 + t] : 0.0;
        }
        for (int l = L - 1; l >= 0; --l) {
            // H_l: the input jets, then the forward products of layers 0 .. l-1
            __syncthreads();
            for (int idx = tid; idx < 6 * 4 * FW2_TP; idx += 256) {
                const int c = idx / (4 * FW2_TP), j = (idx / FW2_TP) & 3, t = idx % FW2_TP;
                const int64_t pt = pt_sh[t];
                H(c, j, t) = (j < 2 && pt >= 0) ? b.pts.xin[(j * 6 + c) * b.pts.ld + pt] : 0.0;
            }
            __syncthreads();
            for (int f = 0; f < l; ++f) {
                const int win = d.w[f], wout = d.w[f + 1];
                const int kpad = (win + 3) & ~3, nut = (wout + 15) / 16;
                const double *Wt = thetaT + d.off[f];
                const double *bias = theta + d.off[f] + win * wout;
                const bool mine = wave < nut;  // uniform: one 16-unit tile per wave
                double4_t acc[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) acc[c] = (double4_t){0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int k = 16 * wave + fk + 4 * r;
                    acc[0][r] = (mine && k < wout) ? bias[k] : 0.0;
                }
                if (mine) {
                    // the weight fragments of the next chunk are loaded (from L2)
                    // before the current chunk's MFMAs
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
                        double bf[4][6];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int j = s0 + 4 * q + fk;
                            const bool in = s0 + 4 * q < kpad;
#pragma unroll
                            for (int c = 0; c < 6; ++c) bf[q][c] = in ? H(c, j, fr) : 0.0;
                        }
#pragma unroll
                        for (int q = 0; q < 4; ++q)
#pragma unroll
                            for (int c = 0; c < 6; ++c)
                                acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], bf[q][c], acc[c], 0, 0, 0);
#pragma unroll
                        for (int q = 0; q < 4; ++q) a[q] = an[q];
                    }
                }
                __syncthreads();  // every read of the layer's input is done
                if (mine) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int k = 16 * wave + fk + 4 * r;
                        const double z1 = acc[1][r], z2 = acc[2][r];
                        const double th = tanh(acc[0][r]), sd = 1.0 - th * th;
                        const double h1 = sd * z1, h2 = sd * z2;
                        H(0, k, fr) = th;
                        H(1, k, fr) = h1;
                        H(2, k, fr) = h2;
                        H(3, k, fr) = sd * acc[3][r] - 2.0 * th * h1 * z1;
                        H(4, k, fr) = sd * acc[4][r] - 2.0 * th * h1 * z2;
                        H(5, k, fr) = sd * acc[5][r] - 2.0 * th * h2 * z2;
                    }
                }
                __syncthreads();
            }
            // the rows' entries of W_l (lane = j, wave = k mod 4, four rows at a
            // time: each lane keeps its H values of the four rows, and the four
            // rows' sums are independent) and of b_l
            const int win = d.w[l], wout = d.w[l + 1];
            double *Jl = b.J + p0 * b.ldJ + d.off[l];
            if (win < 32) {
                // narrow inputs (the first layer): entries spread flat over the threads
                for (int idx = tid; idx < wout * win * nr; idx += 256) {
                    const int t = idx / (wout * win), e = idx - t * wout * win, k = e / win, j = e - k * win;
                    double v = 0.0;
#pragma unroll
                    for (int c = 0; c < 6; ++c) v = fma(Z(c, k, t), H(c, j, t), v);
                    Jl[t * b.ldJ + e] = v;
                }
            } else if (lane < win) {
                for (int t0 = 0; t0 < nr; t0 += 4) {
                    double hv[6][4];
#pragma unroll
                    for (int c = 0; c < 6; ++c)
#pragma unroll
                        for (int q = 0; q < 4; ++q) hv[c][q] = H(c, lane, t0 + q);
                    for (int k = wave; k < wout; k += 4) {
                        double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                        for (int c = 0; c < 6; ++c)
#pragma unroll
                            for (int q = 0; q < 4; ++q) v[q] = fma(Z(c, k, t0 + q), hv[c][q], v[q]);
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if (t0 + q < nr) Jl[(t0 + q) * b.ldJ + k * win + lane] = v[q];
                    }
                }
            }
            for (int idx = tid; idx < wout * nr; idx += 256) {
                const int t = idx / wout, k = idx - t * wout;
                Jl[t * b.ldJ + wout * win + k] = Z(0, k, t);
            }
            if (l == 0) break;
            // hb = W_l^T ZB per jet component (j-tile = wave), then back through tanh
            {
                const double *W = theta + d.off[l];  // W[k][j], wout x win
                const int kpad = (wout + 3) & ~3, nut = (win + 15) / 16;
                const bool mine = wave < nut;
                double4_t acc[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) acc[c] = (double4_t){0.0, 0.0, 0.0, 0.0};
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
                        double bf[4][6];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int k = s0 + 4 * q + fk;
                            const bool in = s0 + 4 * q < kpad;
#pragma unroll
                            for (int c = 0; c < 6; ++c) bf[q][c] = in ? Z(c, k, fr) : 0.0;
                        }
#pragma unroll
                        for (int q = 0; q < 4; ++q)
#pragma unroll
                            for (int c = 0; c < 6; ++c)
                                acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], bf[q][c], acc[c], 0, 0, 0);
#pragma unroll
                        for (int q = 0; q < 4; ++q) a[q] = an[q];
                    }
                }
                __syncthreads();  // every read of ZB (and of this layer's row entries) is done
                if (mine) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int j = 16 * wave + fk + 4 * r;
                        const double th = H(0, j, fr), h1 = H(1, j, fr), h2 = H(2, j, fr);
                        const double h11 = H(3, j, fr), h12 = H(4, j, fr), h22 = H(5, j, fr);
                        const double hb0 = acc[0][r], hb1 = acc[1][r], hb2 = acc[2][r];
                        const double hb3 = acc[3][r], hb4 = acc[4][r], hb5 = acc[5][r];
                        const double sd = 1.0 - th * th, t2 = 2.0 * th;
                        Z(3, j, fr) = sd * hb3;
                        Z(4, j, fr) = sd * hb4;
                        Z(5, j, fr) = sd * hb5;
                        Z(1, j, fr) = sd * hb1 - t2 * (2.0 * h1 * hb3 + h2 * hb4);
                        Z(2, j, fr) = sd * hb2 - t2 * (h1 * hb4 + 2.0 * h2 * hb5);
                        Z(0, j, fr) = sd * hb0 - t2 * (h1 * hb1 + h2 * hb2) - hb3 * (t2 * h11 + 2.0 * h1 * h1) -
                                      hb4 * (t2 * h12 + 2.0 * h1 * h2) - hb5 * (t2 * h22 + 2.0 * h2 * h2);
                    }
                }
            }
        }
    }
}

// wpad of the matrix-core rows sweep (hidden widths up to 64), or 0
static int rows2d_mfma_wpad(const MlpDesc &d) {
    if (d.w[0] != 2 || d.L < 1 || d.w[d.L] > 16) return 0;
    int m = 16;
    for (int l = 1; l < d.L; ++l) m = d.w[l] > m ? d.w[l] : m;
    const int wpad = (m + 15) / 16 * 16;
    return wpad <= 64 ? wpad : 0;
}

// wpad of the matrix-core forward sweep, or 0 if the network does not fit it
static int forward2d_mfma_wpad(const MlpDesc &d) {
    if (d.w[0] != 2 || d.L < 1) return 0;
    int m = 4;
    for (int l = 1; l < d.L; ++l) m = d.w[l] > m ? d.w[l] : m;
    const int wpad = (m + 15) / 16 * 16;
    return (wpad <= 128 && d.w[d.L] <= 16 * 4 * 2) ? wpad : 0;
}

template <int MODE>
static hipError_t launch_sweep2d(hipStream_t st, const MlpDesc &d, const double *theta, const double *thetaT,
                                 const Sweep2DArgs &b, int64_t *nblocks) {
    const Sweep2DLds lay = sweep2d_layout(d);
    if (lay.tile < 1) return hipErrorInvalidValue;
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)jet_sweep2d_kernel<MODE>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr = true;
    }
    int64_t blocks = (b.nrows + lay.tile - 1) / lay.tile;
    if (MODE == SW2_VJP && blocks > VJP2D_MAX_BLOCKS) blocks = VJP2D_MAX_BLOCKS;
    if (nblocks) *nblocks = blocks;
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(jet_sweep2d_kernel<MODE>, dim3((unsigned)blocks), dim3(256), sizeof(double) * lay.total, st, d,
                       lay, theta, thetaT, b);
    return hipGetLastError();
}

hipError_t launch_jets2d_forward(hipStream_t st, const MlpDesc &d, const double *theta, const double *thetaT,
                                 const Sweep2DArgs &b) {
    const int wpad = forward2d_mfma_wpad(d);
    if (wpad == 0) return launch_sweep2d<SW2_FORWARD>(st, d, theta, thetaT, b, nullptr);
    if (b.nrows <= 0) return hipSuccess;
    const size_t shm = sizeof(double) * 6 * wpad * FW2_TP;
    const int64_t ntiles = (b.nrows + FW2_TP - 1) / FW2_TP;
    const unsigned grid = (unsigned)(ntiles < 16384 ? ntiles : 16384);
    static bool attr1 = false, attr2 = false;
    if (wpad <= 64) {
        if (!attr1) {
            (void)hipFuncSetAttribute((const void *)jet_forward2d_mfma_kernel<1>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            attr1 = true;
        }
        hipLaunchKernelGGL(jet_forward2d_mfma_kernel<1>, dim3(grid), dim3(256), shm, st, d, wpad, theta, thetaT, b);
    } else {
        if (!attr2) {
            (void)hipFuncSetAttribute((const void *)jet_forward2d_mfma_kernel<2>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            attr2 = true;
        }
        hipLaunchKernelGGL(jet_forward2d_mfma_kernel<2>, dim3(grid), dim3(256), shm, st, d, wpad, theta, thetaT, b);
    }
    return hipGetLastError();
}

hipError_t launch_jets2d_rows(hipStream_t st, const MlpDesc &d, const double *theta, const double *thetaT,
                              const Sweep2DArgs &b) {
    const int wpad = rows2d_mfma_wpad(d);
    if (wpad == 0) return launch_sweep2d<SW2_ROWS>(st, d, theta, thetaT, b, nullptr);
    if (b.nrows <= 0) return hipSuccess;
    const size_t shm = sizeof(double) * 2 * 6 * wpad * RW2_LD;
    const int64_t ntiles = (b.nrows + FW2_TP - 1) / FW2_TP;
    const unsigned grid = (unsigned)(ntiles < 16384 ? ntiles : 16384);
    static bool attr = false;
    if (!attr) {
        // the kernel's static LDS (the rows' point indices) comes on top
        (void)hipFuncSetAttribute((const void *)jet_rows2d_mfma_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  159 * 1024);
        attr = true;
    }
    hipLaunchKernelGGL(jet_rows2d_mfma_kernel, dim3(grid), dim3(256), shm, st, d, wpad, theta, thetaT, b);
    return hipGetLastError();
}

hipError_t launch_jets2d_vjp(hipStream_t st, const MlpDesc &d, const double *theta, const double *thetaT,
                             const Sweep2DArgs &b, int64_t *nblocks) {
    return launch_sweep2d<SW2_VJP>(st, d, theta, thetaT, b, nblocks);
}

int64_t jets2d_vjp_partials(const MlpDesc &d, int64_t nrows) {
    const Sweep2DLds lay = sweep2d_layout(d);
    if (lay.tile < 1) return 0;
    const int64_t blocks = (nrows + lay.tile - 1) / lay.tile;
    return blocks < VJP2D_MAX_BLOCKS ? blocks : VJP2D_MAX_BLOCKS;
}

}  // namespace gn
