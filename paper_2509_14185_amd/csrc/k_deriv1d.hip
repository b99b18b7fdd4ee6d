// Derivative (d1, d2) rows of the 1D profile problems (Methods, "Training
// Loss": losses on the first and second y-derivatives of the residual, each
// on its own point batch).  For R = -lam Theta + V Theta', V = (1+lam) y + U:
//   R'  = (1 + U') Theta' + V Theta'',
//   R'' = U'' Theta' + (2 + lam + 2 U') Theta'' + V Theta''',
// U = H Theta (CCF; U' = H[Theta'] by the odd half-line form, U'' = H[Theta''])
// or U = Theta (local variant).  The network is swept with third-order jets
// in its input q; the chain rule to y and the envelope's Leibniz rule are
// applied per point.
#include <hip/hip_runtime.h>

#include "gn_internal.h"

namespace gn {

static constexpr int J3_THREADS = 256;
static constexpr int J3_TILE = 4;  // points per workgroup

// w^p and its first three derivatives in w (p(p-1)... w^(p-k)), given w^p.
__device__ __forceinline__ void pow_derivs(double wp, double w, double p, double *F) {
    F[0] = wp;
    F[1] = p * wp / w;
    F[2] = (p - 1.0) * F[1] / w;
    F[3] = (p - 2.0) * F[2] / w;
}

// f(w(y)) for w = 1 + y^2 (w' = 2y, w'' = 2, w''' = 0), by Faa di Bruno.
__device__ __forceinline__ void compose_w(const double *F, double y, double *f) {
    const double w1 = 2.0 * y, w2 = 2.0;
    f[0] = F[0];
    f[1] = F[1] * w1;
    f[2] = F[2] * w1 * w1 + F[1] * w2;
    f[3] = F[3] * w1 * w1 * w1 + 3.0 * F[2] * w1 * w2;
}

// Geometry of a point set to third order: y, q^(k) and E^(k) (k = 0..3), y-derivatives.
__global__ void geometry3_kernel(int equation, double lam, int64_t n, const double *__restrict__ s, Geo3 g) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double si = s[i];
    const double q = 1.0 - si;
    const double y2 = expm1(-2.0 * (1.0 + lam) * log1p(-si));
    const double y = sqrt(y2);
    const double w = 1.0 + y2;  // = q^{-2(1+lam)}
    double F[4], qd[4], P[4], Pd[4];
    pow_derivs(q, w, -1.0 / (2.0 * (1.0 + lam)), F);  // q = w^a
    compose_w(F, y, qd);
    const double e = lam / (2.0 * (1.0 + lam));
    double m[4];
    if (equation == GN_EQ_CCF1D) {
        pow_derivs(pow(q, 2.0 + lam), w, e - 1.0, P);  // w^(e-1) = q^(2+lam)
        m[0] = y2; m[1] = 2.0 * y; m[2] = 2.0; m[3] = 0.0;
    } else {
        pow_derivs(q, w, e - 0.5, P);                  // w^(e-1/2) = q
        m[0] = y; m[1] = 1.0; m[2] = 0.0; m[3] = 0.0;
    }
    compose_w(P, y, Pd);
    g.y[i] = y;
#pragma unroll
    for (int k = 0; k < 4; ++k) g.q[k * g.ld + i] = qd[k];
    // E = m(y) P(w(y)): Leibniz
    g.E[0 * g.ld + i] = m[0] * Pd[0];
    g.E[1 * g.ld + i] = m[1] * Pd[0] + m[0] * Pd[1];
    g.E[2 * g.ld + i] = m[2] * Pd[0] + 2.0 * m[1] * Pd[1] + m[0] * Pd[2];
    g.E[3 * g.ld + i] = m[3] * Pd[0] + 3.0 * m[2] * Pd[1] + 3.0 * m[1] * Pd[2] + m[0] * Pd[3];
}

hipError_t launch_geometry3(hipStream_t st, int equation, double lam, int64_t n, const double *s, Geo3 g) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(geometry3_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, equation, lam, n, s, g);
    return hipGetLastError();
}

// y-derivatives of NN (k = 0..3) from its q-derivatives N and q^(k) (chain rule).
__device__ __forceinline__ void nn_in_y(const double *N, const double *qd, double *Ny) {
    const double q1 = qd[1], q2 = qd[2], q3 = qd[3];
    Ny[0] = N[0];
    Ny[1] = N[1] * q1;
    Ny[2] = N[2] * q1 * q1 + N[1] * q2;
    Ny[3] = N[3] * q1 * q1 * q1 + 3.0 * N[2] * q1 * q2 + N[1] * q3;
}

// Theta^(k) = sum_j C(k,j) E^(j) NN_y^(k-j).
__device__ __forceinline__ void field_in_y(const double *E, const double *Ny, double *T) {
    T[0] = E[0] * Ny[0];
    T[1] = E[1] * Ny[0] + E[0] * Ny[1];
    T[2] = E[2] * Ny[0] + 2.0 * E[1] * Ny[1] + E[0] * Ny[2];
    T[3] = E[3] * Ny[0] + 3.0 * E[2] * Ny[1] + 3.0 * E[1] * Ny[2] + E[0] * Ny[3];
}

// Seeds on the q-derivatives of NN from seeds g on Theta^(k) (transpose of
// field_in_y then nn_in_y).
__device__ __forceinline__ void seeds_to_q(const double *g, const double *E, const double *qd, double *sN) {
    double gy[4];
    gy[0] = g[0] * E[0] + g[1] * E[1] + g[2] * E[2] + g[3] * E[3];
    gy[1] = g[1] * E[0] + 2.0 * g[2] * E[1] + 3.0 * g[3] * E[2];
    gy[2] = g[2] * E[0] + 3.0 * g[3] * E[1];
    gy[3] = g[3] * E[0];
    const double q1 = qd[1], q2 = qd[2], q3 = qd[3];
    sN[0] = gy[0];
    sN[1] = gy[1] * q1 + gy[2] * q2 + gy[3] * q3;
    sN[2] = gy[2] * q1 * q1 + 3.0 * gy[3] * q1 * q2;
    sN[3] = gy[3] * q1 * q1 * q1;
}

// ------------------------------------------------------------ jet sweep
// LDS per workgroup (T = J3_TILE points): for each hidden layer output
// l = 1..L-1, seven arrays [T][w_l]: h0 = tanh z, h1, h2, h3 (q-derivatives
// of the activation) and z1, z2, z3 (of the pre-activation); then two sets of
// four adjoint buffers [T][maxw].
struct J3Lds {
    int off[GN_MAX_LAYERS + 1];
    int zb_off;
    int maxw;
    int total;
};

static J3Lds j3_layout(const MlpDesc &d) {
    J3Lds s{};
    int o = 0, maxw = 1;
    for (int l = 1; l < d.L; ++l) {
        s.off[l] = o;
        o += 7 * J3_TILE * d.w[l];
        if (d.w[l] > maxw) maxw = d.w[l];
    }
    s.zb_off = o;
    s.maxw = maxw;
    s.total = o + 8 * J3_TILE * maxw;
    return s;
}

enum J3Mode { J3_FORWARD = 0, J3_ROWS = 1, J3_VJP = 2 };

template <int MODE>
__global__ __launch_bounds__(J3_THREADS) void mlp_jet3_kernel(MlpDesc d, J3Lds lay, const double *__restrict__ theta,
                                                              const double *__restrict__ thetaT, Sweep3 b,
                                                              double *__restrict__ partial) {
    extern __shared__ double sm[];
    const int tid = threadIdx.x;
    const int64_t p0 = (int64_t)blockIdx.x * J3_TILE;
    const int np = (int)((b.n - p0) < J3_TILE ? (b.n - p0) : J3_TILE);
    if (np <= 0) return;
    const int L = d.L;
    const int ldz = lay.maxw;
    double *zbuf[2][4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        zbuf[0][c] = sm + lay.zb_off + c * J3_TILE * ldz;
        zbuf[1][c] = sm + lay.zb_off + (4 + c) * J3_TILE * ldz;
    }
    auto arr = [&](int l, int a) { return sm + lay.off[l] + a * J3_TILE * d.w[l]; };  // a: h0 h1 h2 h3 z1 z2 z3

    // ---------------- forward: hidden layers
    for (int l = 0; l < L - 1; ++l) {
        const int win = d.w[l], wout = d.w[l + 1];
        const double *Wt = thetaT + d.off[l];
        const double *bias = theta + d.off[l] + win * wout;
        for (int idx = tid; idx < np * wout; idx += J3_THREADS) {
            const int pt = idx / wout, k = idx - pt * wout;
            double z0 = bias[k], z1 = 0.0, z2 = 0.0, z3 = 0.0;
            if (l == 0) {
                z0 = fma(Wt[k], b.x[p0 + pt], z0);  // input jets (x, 1, 0, 0)
                z1 = Wt[k];
            } else {
                const double *H0 = arr(l, 0) + pt * win, *H1 = arr(l, 1) + pt * win;
                const double *H2 = arr(l, 2) + pt * win, *H3 = arr(l, 3) + pt * win;
                for (int j = 0; j < win; ++j) {
                    const double w = Wt[j * wout + k];
                    z0 = fma(w, H0[j], z0);
                    z1 = fma(w, H1[j], z1);
                    z2 = fma(w, H2[j], z2);
                    z3 = fma(w, H3[j], z3);
                }
            }
            // tanh jets: f' = s, f'' = -2ts, f''' = (6t^2 - 2)s
            const double t = tanh(z0), s = 1.0 - t * t;
            const double f2 = -2.0 * t * s, f3 = (6.0 * t * t - 2.0) * s;
            const int o = pt * wout + k;
            arr(l + 1, 0)[o] = t;
            arr(l + 1, 1)[o] = s * z1;
            arr(l + 1, 2)[o] = fma(s, z2, f2 * z1 * z1);
            arr(l + 1, 3)[o] = s * z3 + 3.0 * f2 * z1 * z2 + f3 * z1 * z1 * z1;
            arr(l + 1, 4)[o] = z1;
            arr(l + 1, 5)[o] = z2;
            arr(l + 1, 6)[o] = z3;
        }
        __syncthreads();
    }

    // ---------------- output layer (width 1)
    {
        const int l = L - 1;
        const int win = d.w[l];
        const double *W = theta + d.off[l];
        const double bias = theta[d.off[l] + win];
        const int wave = tid >> 6, lane = tid & 63;
        for (int pt = wave; pt < np; pt += J3_THREADS / 64) {
            double z[4] = {0.0, 0.0, 0.0, 0.0};
            if (l == 0) {
                if (lane == 0) {
                    z[0] = W[0] * b.x[p0 + pt];
                    z[1] = W[0];
                }
            } else {
                for (int j = lane; j < win; j += 64) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) z[c] = fma(W[j], arr(l, c)[pt * win + j], z[c]);
                }
            }
#pragma unroll
            for (int c = 0; c < 4; ++c)
                for (int o = 32; o > 0; o >>= 1) z[c] += __shfl_xor(z[c], o, 64);
            if (lane == 0) {
                if (MODE == J3_FORWARD) {
                    b.nn[p0 + pt] = z[0] + bias;
#pragma unroll
                    for (int c = 1; c < 4; ++c) b.nn[c * b.n + p0 + pt] = z[c];
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c) zbuf[0][c][pt * ldz] = b.seed[c * b.seed_ld + p0 + pt];
                }
            }
        }
    }
    if (MODE == J3_FORWARD) return;
    __syncthreads();

    // ---------------- adjoint sweep
    int cur = 0;
    for (int l = L - 1; l >= 0; --l) {
        const int win = d.w[l], wout = d.w[l + 1];
        const int nseg = wout * (win + 1);
        double *const *zb = zbuf[cur];
        // input jets of layer l at point pt, unit j
        auto hin = [&](int pt, int j, double *h) {
            if (l == 0) {
                h[0] = b.x[p0 + pt]; h[1] = 1.0; h[2] = 0.0; h[3] = 0.0;
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) h[c] = arr(l, c)[pt * win + j];
            }
        };
        if (MODE == J3_ROWS) {
            for (int pt = 0; pt < np; ++pt) {
                double *row = b.rows + (p0 + pt) * b.ld + d.off[l];
                for (int idx = tid; idx < nseg; idx += J3_THREADS) {
                    double v;
                    if (idx < wout * win) {
                        const int k = idx / win, j = idx - k * win;
                        double h[4];
                        hin(pt, j, h);
                        v = zb[0][pt * ldz + k] * h[0];
#pragma unroll
                        for (int c = 1; c < 4; ++c) v = fma(zb[c][pt * ldz + k], h[c], v);
                    } else {
                        v = zb[0][pt * ldz + idx - wout * win];
                    }
                    row[idx] = v;
                }
            }
        } else {  // J3_VJP
            double *out = partial + (int64_t)blockIdx.x * d.P + d.off[l];
            for (int idx = tid; idx < nseg; idx += J3_THREADS) {
                double acc = 0.0;
                if (idx < wout * win) {
                    const int k = idx / win, j = idx - k * win;
                    for (int pt = 0; pt < np; ++pt) {
                        double h[4];
                        hin(pt, j, h);
                        double v = zb[0][pt * ldz + k] * h[0];
#pragma unroll
                        for (int c = 1; c < 4; ++c) v = fma(zb[c][pt * ldz + k], h[c], v);
                        acc += v;
                    }
                } else {
                    const int k = idx - wout * win;
                    for (int pt = 0; pt < np; ++pt) acc += zb[0][pt * ldz + k];
                }
                out[idx] = acc;
            }
        }
        if (l == 0) break;
        // hbar_c = W^T zbar_c, then through the tanh jets of layer l's input:
        //   zb3 = hb3 f1
        //   zb2 = hb2 f1 + 3 hb3 f2 z1
        //   zb1 = hb1 f1 + 2 hb2 f2 z1 + hb3 (3 f2 z2 + 3 f3 z1^2)
        //   zb0 = hb0 f1 + hb1 f2 z1 + hb2 (f2 z2 + f3 z1^2) + hb3 (f2 z3 + 3 f3 z1 z2 + f4 z1^3)
        // with f1 = s, f2 = -2ts, f3 = (6t^2 - 2)s, f4 = ts(16 - 24t^2).
        const double *W = theta + d.off[l];
        double *const *zn = zbuf[cur ^ 1];
        for (int idx = tid; idx < np * win; idx += J3_THREADS) {
            const int pt = idx / win, j = idx - pt * win;
            double hb[4] = {0.0, 0.0, 0.0, 0.0};
            for (int k = 0; k < wout; ++k) {
                const double w = W[k * win + j];
#pragma unroll
                for (int c = 0; c < 4; ++c) hb[c] = fma(w, zb[c][pt * ldz + k], hb[c]);
            }
            const int o = pt * win + j;
            const double t = arr(l, 0)[o], z1 = arr(l, 4)[o], z2 = arr(l, 5)[o], z3 = arr(l, 6)[o];
            const double s = 1.0 - t * t;
            const double f2 = -2.0 * t * s, f3 = (6.0 * t * t - 2.0) * s, f4 = t * s * (16.0 - 24.0 * t * t);
            zn[3][pt * ldz + j] = hb[3] * s;
            zn[2][pt * ldz + j] = hb[2] * s + 3.0 * hb[3] * f2 * z1;
            zn[1][pt * ldz + j] = hb[1] * s + 2.0 * hb[2] * f2 * z1 + hb[3] * (3.0 * f2 * z2 + 3.0 * f3 * z1 * z1);
            zn[0][pt * ldz + j] = hb[0] * s + hb[1] * f2 * z1 + hb[2] * (f2 * z2 + f3 * z1 * z1) +
                                  hb[3] * (f2 * z3 + 3.0 * f3 * z1 * z2 + f4 * z1 * z1 * z1);
        }
        __syncthreads();
        cur ^= 1;
    }
}

template <int MODE>
static hipError_t launch_jet3_mode(hipStream_t st, const MlpDesc &d, const double *theta, const double *thetaT,
                                   Sweep3 b, double *partial) {
    const J3Lds lay = j3_layout(d);
    const size_t shm = sizeof(double) * (size_t)lay.total;
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)mlp_jet3_kernel<MODE>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024);
        attr_set = true;
    }
    if (shm > 160 * 1024) return hipErrorInvalidValue;
    const int64_t blocks = (b.n + J3_TILE - 1) / J3_TILE;
    hipLaunchKernelGGL(mlp_jet3_kernel<MODE>, dim3((unsigned)blocks), dim3(J3_THREADS), shm, st, d, lay, theta, thetaT,
                       b, partial);
    return hipGetLastError();
}

hipError_t launch_jet3_forward(hipStream_t st, const MlpDesc &d, const double *theta, const double *thetaT,
                               Sweep3 b) {
    if (b.n <= 0) return hipSuccess;
    return launch_jet3_mode<J3_FORWARD>(st, d, theta, thetaT, b, nullptr);
}
hipError_t launch_jet3_rows(hipStream_t st, const MlpDesc &d, const double *theta, const double *thetaT, Sweep3 b) {
    if (b.n <= 0) return hipSuccess;
    return launch_jet3_mode<J3_ROWS>(st, d, theta, thetaT, b, nullptr);
}
int64_t jet3_vjp_partials(int64_t n) { return (n + J3_TILE - 1) / J3_TILE; }
hipError_t launch_jet3_vjp(hipStream_t st, const MlpDesc &d, const double *theta, const double *thetaT, Sweep3 b,
                           double *partial, int64_t *n_partials) {
    *n_partials = jet3_vjp_partials(b.n);
    if (b.n <= 0) return hipSuccess;
    return launch_jet3_mode<J3_VJP>(st, d, theta, thetaT, b, partial);
}

// ------------------------------------------------------------ node fields
// Theta^(k)(t_j), k = 0..2, at the Hilbert nodes; out[k * m + j].
__global__ void node_fields_kernel(int64_t m, const double *__restrict__ nn, Geo3 g, double *__restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    double N[4], qd[4], E[4], Ny[4], T[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        N[c] = nn[c * m + j];
        qd[c] = g.q[c * g.ld + j];
        E[c] = g.E[c * g.ld + j];
    }
    nn_in_y(N, qd, Ny);
    field_in_y(E, Ny, T);
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c * m + j] = T[c];
}

hipError_t launch_node_fields(hipStream_t st, int64_t m, const double *nn, Geo3 g, double *out) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(node_fields_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, m, nn, g, out);
    return hipGetLastError();
}

// Seeds of the node Jacobians B1_j = t_j dTheta'(t_j)/dtheta and
// B2_j = dTheta''(t_j)/dtheta on the q-derivatives of NN: seed[c * ld + j]
// (B1 in columns 0..m-1, B2 in m..2m-1).
__global__ void node_seeds_kernel(int64_t m, Geo3 g, const double *__restrict__ t, double *__restrict__ seed,
                                  int64_t ld) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    double qd[4], E[4], s1[4], s2[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        qd[c] = g.q[c * g.ld + j];
        E[c] = g.E[c * g.ld + j];
    }
    const double g1[4] = {0.0, t[j], 0.0, 0.0}, g2[4] = {0.0, 0.0, 1.0, 0.0};
    seeds_to_q(g1, E, qd, s1);
    seeds_to_q(g2, E, qd, s2);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        seed[c * ld + j] = s1[c];
        seed[c * ld + m + j] = s2[c];
    }
}

hipError_t launch_node_seeds(hipStream_t st, int64_t m, Geo3 g, const double *t, double *seed, int64_t ld) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(node_seeds_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, m, g, t, seed, ld);
    return hipGetLastError();
}

// ------------------------------------------------------------ residual rows
__device__ __forceinline__ double hq(double yi, double tj, double whj) {
    return whj * (2.0 * yi) / ((yi - tj) * (yi + tj));
}
__device__ __forceinline__ double hq1(double yi, double tj, double whj) {
    return whj * 2.0 / ((yi - tj) * (yi + tj));
}

// One wave per derivative point: rows 0..n1-1 are d1 rows, n1..n1+n2-1 d2 rows.
__global__ __launch_bounds__(256) void deriv_residual_kernel(DerivArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t nd = a.n1 + a.n2;
    if (i >= nd) return;
    double N[4], qd[4], E[4], Ny[4], T[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        N[c] = a.nn[c * nd + i];
        qd[c] = a.geo.q[c * a.geo.ld + i];
        E[c] = a.geo.E[c * a.geo.ld + i];
    }
    nn_in_y(N, qd, Ny);
    field_in_y(E, Ny, T);
    const double yi = a.geo.y[i];
    const bool ccf = a.equation == GN_EQ_CCF1D;
    double U = T[0], U1 = T[1], U2 = T[2], c = 0.0, c1 = 0.0;
    if (ccf) {
        double su = 0.0, su1 = 0.0, su2 = 0.0;
        for (int64_t j = lane; j < a.m; j += 64) {
            const double tj = a.nodes_y[j], wj = a.nodes_wh[j];
            const double qij = hq(yi, tj, wj), q1ij = hq1(yi, tj, wj);
            su = fma(qij, a.node_fields[j] - T[0], su);
            su1 = fma(q1ij, tj * a.node_fields[a.m + j] - yi * T[1], su1);
            su2 = fma(qij, a.node_fields[2 * a.m + j] - T[2], su2);
            c += qij;
            c1 += q1ij;
        }
        for (int o = 32; o > 0; o >>= 1) {
            su += __shfl_xor(su, o, 64);
            su1 += __shfl_xor(su1, o, 64);
            su2 += __shfl_xor(su2, o, 64);
            c += __shfl_xor(c, o, 64);
            c1 += __shfl_xor(c1, o, 64);
        }
        U = su;
        U1 = su1;
        U2 = su2;
    }
    if (lane != 0) return;
    const double lam = a.lam;
    const double V = (1.0 + lam) * yi + U;
    const bool second = i >= a.n1;
    const double R = second ? U2 * T[1] + (2.0 + lam + 2.0 * U1) * T[2] + V * T[3] : (1.0 + U1) * T[1] + V * T[2];
    const double sc = second ? a.scale2 : a.scale1;
    if (a.max_out) atomic_max_abs(a.max_out, R);
    if (a.r) a.r[i * a.r_stride] = sc * R;
    if (!a.seed) return;
    // seeds on Theta^(k) at the point and the coupling coefficients of
    // sum_j Q_ij B_j, sum_j Q1_ij t_j B1_j, sum_j Q_ij B2_j
    double g[4], cB, cB1, cB2;
    if (ccf) {
        if (second) {
            g[0] = -c * T[3];
            g[1] = U2 - 2.0 * T[2] * yi * c1;
            g[2] = -c * T[1] + (2.0 + lam + 2.0 * U1);
            g[3] = V;
            cB = T[3]; cB1 = 2.0 * T[2]; cB2 = T[1];
        } else {
            g[0] = -c * T[2];
            g[1] = (1.0 + U1) - T[1] * yi * c1;
            g[2] = V;
            g[3] = 0.0;
            cB = T[2]; cB1 = T[1]; cB2 = 0.0;
        }
    } else {  // U = Theta
        if (second) {
            g[0] = T[3]; g[1] = 3.0 * T[2]; g[2] = 2.0 + lam + 3.0 * T[1]; g[3] = V;
        } else {
            g[0] = T[2]; g[1] = 1.0 + 2.0 * T[1]; g[2] = V; g[3] = 0.0;
        }
        cB = cB1 = cB2 = 0.0;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) g[k] *= sc;
    double sN[4];
    seeds_to_q(g, E, qd, sN);
#pragma unroll
    for (int k = 0; k < 4; ++k) a.seed[k * nd + i] = sN[k];
    if (a.coef) {
        a.coef[i] = sc * cB;
        a.coef[nd + i] = sc * cB1;
        a.coef[2 * nd + i] = sc * cB2;
    }
}

hipError_t launch_deriv_residual(hipStream_t st, const DerivArgs &a) {
    const int64_t nd = a.n1 + a.n2;
    if (nd <= 0) return hipSuccess;
    hipLaunchKernelGGL(deriv_residual_kernel, dim3((unsigned)((nd + 3) / 4)), dim3(256), 0, st, a);
    return hipGetLastError();
}

// Coupling matrix of the derivative rows, stored transposed (node-major):
// AT[j][i] = cB_i Q_ij, AT[m + j][i] = cB1_i Q1_ij, AT[2m + j][i] = cB2_i Q_ij.
__global__ void deriv_coupling_kernel(int64_t nd, int64_t m, const double *__restrict__ y,
                                      const double *__restrict__ t, const double *__restrict__ wh,
                                      const double *__restrict__ coef, double *__restrict__ AT, int64_t ld) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t j = blockIdx.y;
    if (i >= nd || j >= m) return;
    const double yi = y[i], tj = t[j], wj = wh[j];
    const double qij = hq(yi, tj, wj), q1ij = hq1(yi, tj, wj);
    AT[j * ld + i] = coef[i] * qij;
    AT[(m + j) * ld + i] = coef[nd + i] * q1ij;
    AT[(2 * m + j) * ld + i] = coef[2 * nd + i] * qij;
}

hipError_t launch_deriv_coupling(hipStream_t st, int64_t nd, int64_t m, const double *y, const double *t,
                                 const double *wh, const double *coef, double *AT, int64_t ld) {
    if (nd <= 0 || m <= 0) return hipSuccess;
    if (m > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(deriv_coupling_kernel, dim3((unsigned)((nd + 255) / 256), (unsigned)m), dim3(256), 0, st, nd, m,
                       y, t, wh, coef, AT, ld);
    return hipGetLastError();
}

// Adjoint of the coupling for a vector v over the derivative rows: node
// seeds on the q-derivatives of NN,
//   u_j (E_j, 0, 0, 0) + u1_j (seed of B1_j) + u2_j (seed of B2_j),
// u_j = sum_i v_i AT[j][i] etc.  One wave per node, points in fixed order.
__global__ __launch_bounds__(256) void deriv_coupling_adjoint_kernel(int64_t nd, int64_t m, const double *__restrict__ AT,
                                                                     int64_t ld, const double *__restrict__ v,
                                                                     const double *__restrict__ nodeE,
                                                                     const double *__restrict__ bseed, int64_t sld,
                                                                     double *__restrict__ out, int64_t old) {
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= m) return;
    double u[3] = {0.0, 0.0, 0.0};
    for (int64_t i = lane; i < nd; i += 64) {
        const double vi = v[i];
#pragma unroll
        for (int k = 0; k < 3; ++k) u[k] = fma(AT[(k * m + j) * ld + i], vi, u[k]);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
        for (int o = 32; o > 0; o >>= 1) u[k] += __shfl_xor(u[k], o, 64);
    if (lane != 0) return;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double s = u[1] * bseed[c * sld + j] + u[2] * bseed[c * sld + m + j];
        if (c == 0) s = fma(u[0], nodeE[j], s);
        out[c * old + j] = s;
    }
}

hipError_t launch_deriv_coupling_adjoint(hipStream_t st, int64_t nd, int64_t m, const double *AT, int64_t ld,
                                         const double *v, const double *nodeE, const double *bseed, int64_t sld,
                                         double *out, int64_t old) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(deriv_coupling_adjoint_kernel, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st, nd, m, AT, ld,
                       v, nodeE, bseed, sld, out, old);
    return hipGetLastError();
}

// out[c * ld + i] = v_i seed[c * ld + i], c = 0..3.
__global__ void scale_seeds_kernel(int64_t n, const double *__restrict__ v, const double *__restrict__ seed,
                                   double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
#pragma unroll
    for (int c = 0; c < 4; ++c) out[c * n + i] = v[i] * seed[c * n + i];
}

hipError_t launch_scale_seeds(hipStream_t st, int64_t n, const double *v, const double *seed, double *out) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(scale_seeds_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, v, seed, out);
    return hipGetLastError();
}

// ------------------------------------------------------------ lambda inference
// U'(0) = H[Theta'](0) by the odd half-line form at y = 0:
// sum_j (-2 w_j / t_j) Theta'(t_j), Theta' = E' NN + E q' NN_q at the nodes;
// one workgroup, fixed per-thread order and tree (deterministic).
__global__ __launch_bounds__(256) void lambda_estimate_kernel(int64_t m, Geo1D nodes, const double *__restrict__ nn,
                                                              double *__restrict__ out) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t j = threadIdx.x; j < m; j += 256) {
        const double thy = nodes.Ey[j] * nn[j] + nodes.E[j] * nodes.qy[j] * nn[m + j];
        acc = fma(-2.0 * nodes.wh[j] / nodes.y[j], thy, acc);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = -2.0 * (1.0 + red[0]);
        out[1] = red[0];
    }
}

hipError_t launch_lambda_estimate(hipStream_t st, int64_t m, Geo1D nodes, const double *nn, double *out) {
    if (m <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(lambda_estimate_kernel, dim3(1), dim3(256), 0, st, m, nodes, nn, out);
    return hipGetLastError();
}

// ------------------------------------------------------------ funnel inference
// Proxy r_hat(lam): over the points with y_i <= y_max, the R_i of largest
// |R_i| (a NaN counts as largest; the smallest index on ties) and its y_i.
// One workgroup, fixed per-thread order and tree (deterministic).
// out[0] = R_i, out[1] = y_i, out[2] = number of points with y_i <= y_max.
__global__ __launch_bounds__(1024) void funnel_residual_kernel(int64_t n, const double *__restrict__ R,
                                                              const double *__restrict__ y, double y_max,
                                                              double *__restrict__ out) {
    __shared__ double key[1024];
    __shared__ int64_t idx[1024];
    __shared__ int64_t cnt[1024];
    double best = -1.0;  // |R| of the candidate, +inf for NaN; -1: none
    int64_t bi = n, c = 0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) {
        if (!(y[i] <= y_max)) continue;
        ++c;
        const double r = R[i];
        const double a = r != r ? __builtin_huge_val() : fabs(r);
        if (a > best) {  // i increases along the loop: the first of equal values stays
            best = a;
            bi = i;
        }
    }
    key[threadIdx.x] = best;
    idx[threadIdx.x] = bi;
    cnt[threadIdx.x] = c;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const int t = threadIdx.x + o;
            if (key[t] > key[threadIdx.x] || (key[t] == key[threadIdx.x] && idx[t] < idx[threadIdx.x])) {
                key[threadIdx.x] = key[t];
                idx[threadIdx.x] = idx[t];
            }
            cnt[threadIdx.x] += cnt[t];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t i = idx[0];
        out[0] = i < n ? R[i] : 0.0;
        out[1] = i < n ? y[i] : 0.0;
        out[2] = (double)cnt[0];
    }
}

hipError_t launch_funnel_residual(hipStream_t st, int64_t n, const double *R, const double *y, double y_max,
                                  double *out) {
    if (n <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(funnel_residual_kernel, dim3(1), dim3(1024), 0, st, n, R, y, y_max, out);
    return hipGetLastError();
}

}  // namespace gn
