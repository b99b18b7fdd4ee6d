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
    return launch_sweep2d<SW2_FORWARD>(st, d, theta, thetaT, b, nullptr);
}

hipError_t launch_jets2d_rows(hipStream_t st, const MlpDesc &d, const double *theta, const double *thetaT,
                              const Sweep2DArgs &b) {
    return launch_sweep2d<SW2_ROWS>(st, d, theta, thetaT, b, nullptr);
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
