// C ABI of the gfx950 damped Gauss-Newton library (declared in include/gn.h).
// Argument checking, workspace ownership and the order of kernel launches for
// each entry point.  Every arithmetic step runs in the HIP kernels of
// k_profile1d.hip, k_dgemm.hip and k_solve.hip.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <type_traits>
#include <vector>

#include "gn_internal.h"

using namespace gn;


struct gn_context {
    int equation = 0, precision = 0;
    double lam = 0, c_norm = 0, c_target = 0;
    MlpDesc md{};
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;           // look-ahead stream of the Cholesky (default priority)
    hipEvent_t ev_panel = nullptr, ev_trail = nullptr;
    int device = 0;
    std::string err;
    std::vector<void *> allocs;       // problem-lifetime allocations
    std::vector<void *> pt_allocs;    // point-set allocations
    uint64_t points_gen = 0;          // bumped by every gn_set_points
    // P-dependent workspace (gn_create)
    int64_t cap = 0;                  // largest p accepted by gn_gram/gn_solve work buffers (P + 1)
    double *thetaT = nullptr, *linv = nullptr, *ybuf = nullptr, *zbuf = nullptr, *delta = nullptr;
    double *theta_trial = nullptr, *gdiag = nullptr;   // damping retries: trial point, saved diagonal of G
    double *r1_g = nullptr, *r1_u = nullptr, *r1_D = nullptr, *r1_b = nullptr;  // stochastic step vectors (P)
    double *r1_dots = nullptr, *r1_work = nullptr;
    double *r1_w1 = nullptr, *r1_w2 = nullptr;           // J Delta, J d_prev (rows)
    bool r1_factored = false;                           // the Gram workspace holds the factor of G_ema + gamma I
    double *gemv_work = nullptr, *red_work = nullptr, *chol_tmp = nullptr, *one_x = nullptr, *nn_one = nullptr, *seed_one = nullptr;
    DevStatus *status = nullptr;
    unsigned *solve_sync = nullptr;   // epoch and published-block markers of the one-launch back substitution
    // point-set data (gn_set_points)
    int64_t n = 0, m = 0, nv = 0;
    Geo1D pts{}, nodes{}, val{};
    double *rho = nullptr, *f = nullptr;
    double *Q = nullptr;              // Q^T of the Hilbert quadrature (m rows, stride ldQ)
    int64_t ldQ = 0;
    double *nn_pts = nullptr, *nn_nodes = nullptr, *nn_val = nullptr;
    double *R = nullptr, *seed0 = nullptr, *seed1 = nullptr, *cscale = nullptr, *r_tmp = nullptr;
    double *vseed0 = nullptr, *vseed1 = nullptr, *useed = nullptr;
    double *J = nullptr, *Bm = nullptr, *G = nullptr, *partial = nullptr;
    // the stochastic step's Hilbert coupling applied through products (1D CCF):
    // two n-vectors, two m-vectors, and the partial sums of a paired
    // transposed product over n columns
    double *cp_t = nullptr, *cp_z = nullptr, *cp_work = nullptr;
    float *Jhi = nullptr, *Jlo = nullptr;   // split-precision parts of J (GN_SPLIT32)
    ModgramWork mg{};                        // int8 residue workspaces (GN_INT8_CRT)
    TilePlan gplan{};                        // work plan of the FP64 Gram of order P + 1 (set at creation)
    TilePlan cplan{};                        // work plan of the Hilbert coupling, N x P (set with the points)
    TilePlan dplan{};                        // work plan of the derivative rows' coupling, (n1 + n2) x P
    int64_t ldJ = 0, ldG = 0, n_partial_cap = 0;
    // 2D problems (gn_set_points_2d)
    int dim = 1, nout = 1, n_eq = 1;
    int64_t row_chunk = 0;            // rows of J per chunk in gn_step (0: all)
    RowMap2D map2{};
    Pts2D pts2{}, val2{};
    double *origin_s = nullptr;       // (0, 0): the normalisation point
    double *nn2 = nullptr, *nn2v = nullptr, *seeds2 = nullptr, *r2 = nullptr;
    int64_t ldn2 = 0, ldnv2 = 0, rows_ws = 0;
    // 1D derivative rows (gn_set_points_ex): d1 rows then d2 rows after the d0 rows
    int64_t nd1 = 0, nd2 = 0;
    double c_d1 = 1.0, c_d2 = 1.0;
    Geo3 geo3{}, geo3n{};              // derivative points; Hilbert nodes
    double *nn3 = nullptr, *nn3n = nullptr;   // NN^(c) (4 x nd, 4 x m)
    double *nfield = nullptr;          // Theta, Theta', Theta'' at the nodes (3 x m)
    double *dseed = nullptr, *dvseed = nullptr, *dcoef = nullptr;  // 4 x nd, 4 x nd, 3 x nd
    double *bseed = nullptr;           // seeds of the node Jacobians B1, B2 (4 x 2m)
    double *dAT = nullptr;             // coupling matrix of the derivative rows (3m x ldA)
    int64_t ldA = 0;
    double *nvseed = nullptr;          // node seeds of the coupling adjoint (4 x m)
    // Fourier feature input (gn_problem.n_fourier > 0): features of q per point set
    int nf = 0;
    double *fb = nullptr;              // frequencies b_k (nf)
    double *phi_one = nullptr, *phi_pts = nullptr, *phi_nodes = nullptr, *phi_val = nullptr;
    // second stage (gn_set_stage1): first-stage R, V, Theta' at the points and the validation grid
    bool stage2 = false;
    double s1eps = 0.0;
    double *s1R = nullptr, *s1V = nullptr, *s1T = nullptr, *s1Rv = nullptr, *s1Vv = nullptr, *s1Tv = nullptr;
    double *fn_R = nullptr;  // raw residual on the validation grid (funnel proxy), lazily allocated
    Geo3 geo3v{};                      // validation grid (derivative maxima)
    double *nn3v = nullptr;            // NN^(c) on the validation grid (4 x nv)
    // phase timing
    std::vector<hipEvent_t> events;   // max_steps x (GN_PHASE_COUNT + 1)
    int32_t prof_max = 0, prof_count = 0;
};

namespace {

const char *kStatusText[] = {"ok", "invalid argument", "out of device memory", "HIP runtime error",
                             "non-finite value", "call out of order"};

gn_status fail(gn_handle h, gn_status s, const char *fmt, const char *detail = "") {
    if (h) {
        char buf[512];
        snprintf(buf, sizeof buf, fmt, detail);
        h->err = buf;
    }
    return s;
}

#define GN_HIP(h, expr)                                                                 \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) return fail((h), GN_EDEVICE, "HIP: %s", hipGetErrorString(e_)); \
    } while (0)

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

template <class T>
gn_status dev_alloc(gn_handle h, std::vector<void *> &list, T **out, int64_t count) {
    *out = nullptr;
    if (count <= 0) count = 1;
    void *p = nullptr;
    if (hipMalloc(&p, sizeof(T) * (size_t)count) != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, GN_ENOMEM, "hipMalloc of %s failed", std::to_string(sizeof(T) * count).c_str());
    }
    list.push_back(p);
    *out = (T *)p;
    return GN_OK;
}

void free_list(std::vector<void *> &list) {
    for (void *p : list) (void)hipFree(p);
    list.clear();
}

#define GN_TRY(expr)                  \
    do {                              \
        gn_status s_ = (expr);        \
        if (s_ != GN_OK) return s_;   \
    } while (0)

bool points_ready(gn_handle h) { return h->n > 0; }

// 1D rows: d0 rows (n), d1 rows, d2 rows, then the normalisation row.
int64_t norm_row(gn_handle h) { return h->n + h->nd1 + h->nd2; }
int64_t total_rows(gn_handle h) { return h->dim == 2 ? h->map2.rows() : norm_row(h) + 1; }

// Fourier feature input of a 1D sweep over a point set (no-op without features).
void with_phi(gn_handle h, SweepBatch &b, const double *phi, int64_t ld) {
    if (h->nf > 0) {
        b.phi = phi;
        b.phi_ld = ld;
    }
}

// First-stage fields of a second-stage residual (no-op otherwise).
void with_stage1(gn_handle h, ResidualArgs &a, bool validation_grid) {
    if (!h->stage2) return;
    a.R1 = validation_grid ? h->s1Rv : h->s1R;
    a.V1 = validation_grid ? h->s1Vv : h->s1V;
    a.T1y = validation_grid ? h->s1Tv : h->s1T;
    a.eps = h->s1eps;
}

// Forward jets at the nodes (CCF), the collocation points and q = 1.
gn_status forward_all(gn_handle h, const double *theta) {
    hipStream_t st = h->stream;
    GN_HIP(h, launch_transpose_weights(st, h->md, theta, h->thetaT));
    if (h->equation == GN_EQ_CCF1D) {
        SweepBatch b{};
        b.x = h->nodes.q; b.n = h->m; b.nn = h->nn_nodes;
        with_phi(h, b, h->phi_nodes, h->m);
        GN_HIP(h, launch_mlp_forward(st, h->md, theta, h->thetaT, b));
    }
    SweepBatch b{};
    b.x = h->pts.q; b.n = h->n; b.nn = h->nn_pts;
    with_phi(h, b, h->phi_pts, h->n);
    GN_HIP(h, launch_mlp_forward(st, h->md, theta, h->thetaT, b));
    SweepBatch o{};
    o.x = h->one_x; o.n = 1; o.nn = h->nn_one;
    with_phi(h, o, h->phi_one, 1);
    GN_HIP(h, launch_mlp_forward(st, h->md, theta, h->thetaT, o));
    if (h->nd1 + h->nd2 > 0) {
        // third-order jets at the derivative points (and Theta, Theta', Theta'' at the nodes)
        Sweep3 d{};
        d.x = h->geo3.q; d.n = h->nd1 + h->nd2; d.nn = h->nn3;
        GN_HIP(h, launch_jet3_forward(st, h->md, theta, h->thetaT, d));
        if (h->equation == GN_EQ_CCF1D) {
            Sweep3 nb{};
            nb.x = h->geo3n.q; nb.n = h->m; nb.nn = h->nn3n;
            GN_HIP(h, launch_jet3_forward(st, h->md, theta, h->thetaT, nb));
            GN_HIP(h, launch_node_fields(st, h->m, h->nn3n, h->geo3n, h->nfield));
        }
    }
    return GN_OK;
}

DerivArgs deriv_args(gn_handle h) {
    DerivArgs a{};
    a.equation = h->equation; a.lam = h->lam;
    a.n1 = h->nd1; a.n2 = h->nd2; a.m = h->m;
    a.geo = h->geo3; a.nn = h->nn3;
    a.nodes_y = h->nodes.y; a.nodes_wh = h->nodes.wh; a.node_fields = h->nfield;
    a.scale1 = h->nd1 > 0 ? sqrt(h->c_d1 / (double)h->nd1) : 0.0;
    a.scale2 = h->nd2 > 0 ? sqrt(h->c_d2 / (double)h->nd2) : 0.0;
    return a;
}

// Residual rows into r (stride r_stride); seeds/cscale when `seeds`.
ResidualArgs residual_args_pts(gn_handle h, double *r, int64_t r_stride, bool seeds) {
    ResidualArgs a{};
    a.equation = h->equation; a.lam = h->lam; a.n = h->n; a.m = h->m;
    a.pts = h->pts; a.nodes = h->nodes;
    a.nn = h->nn_pts; a.nn_nodes = h->nn_nodes;
    a.rho = h->rho; a.f = h->f; a.inv_n = 1.0 / (double)h->n;
    a.R = h->R; a.r = r; a.r_stride = r_stride;
    a.seed0 = seeds ? h->seed0 : nullptr; a.seed1 = seeds ? h->seed1 : nullptr;
    a.cscale = seeds ? h->cscale : nullptr;
    a.max_out = &h->status->max_R;
    with_stage1(h, a, false);
    return a;
}

ResidualArgs residual_args_val(gn_handle h) {
    ResidualArgs a{};
    a.equation = h->equation; a.lam = h->lam; a.n = h->nv; a.m = h->m;
    a.pts = h->val; a.nodes = h->nodes;
    a.nn = h->nn_val; a.nn_nodes = h->nn_nodes;
    a.inv_n = 1.0;
    a.max_out = &h->status->max_R_val;
    with_stage1(h, a, true);
    return a;
}

gn_status residual_rows(gn_handle h, double *r, int64_t r_stride, bool seeds) {
    GN_HIP(h, launch_residual(h->stream, residual_args_pts(h, r, r_stride, seeds)));
    if (h->nd1 + h->nd2 > 0) {
        DerivArgs d = deriv_args(h);
        d.r = r + h->n * r_stride; d.r_stride = r_stride;
        d.seed = seeds ? h->dseed : nullptr;
        d.coef = seeds ? h->dcoef : nullptr;
        GN_HIP(h, launch_deriv_residual(h->stream, d));
    }
    GN_HIP(h, launch_norm_row(h->stream, h->nn_one, sqrt(h->c_norm), h->c_target, r + norm_row(h) * r_stride));
    return GN_OK;
}

// Jacobian rows of the derivative rows (after residual_rows with seeds and,
// for CCF, the node Jacobian B in rows 0..m-1 of Bm): local rows by the jet
// sweep, then the coupling with B, B1 = t dTheta'/dtheta, B2 = dTheta''/dtheta.
gn_status deriv_jacobian(gn_handle h, const double *theta, double *J, int64_t ldJ) {
    const int64_t nd = h->nd1 + h->nd2;
    if (nd <= 0) return GN_OK;
    hipStream_t st = h->stream;
    Sweep3 d{};
    d.x = h->geo3.q; d.seed = h->dseed; d.seed_ld = nd; d.n = nd; d.rows = J + h->n * ldJ; d.ld = ldJ;
    GN_HIP(h, launch_jet3_rows(st, h->md, theta, h->thetaT, d));
    if (h->equation != GN_EQ_CCF1D) return GN_OK;
    const int64_t m = h->m;
    for (int k = 0; k < 2; ++k) {
        Sweep3 nb{};
        nb.x = h->geo3n.q; nb.seed = h->bseed + k * m; nb.seed_ld = 2 * m; nb.n = m;
        nb.rows = h->Bm + (1 + k) * m * h->ldJ; nb.ld = h->ldJ;
        GN_HIP(h, launch_jet3_rows(st, h->md, theta, h->thetaT, nb));
    }
    GN_HIP(h, launch_deriv_coupling(st, nd, m, h->geo3.y, h->nodes.y, h->nodes.wh, h->dcoef, h->dAT, h->ldA));
    GemmDesc g{};
    g.M = nd; g.N = h->md.P; g.K = 3 * m;
    g.A = h->dAT; g.lda = h->ldA; g.la = 1;
    g.B = h->Bm; g.ldb = h->ldJ; g.lb = 0;
    g.C = J + h->n * ldJ; g.ldc = ldJ;
    g.alpha = 1.0; g.beta = 1.0;
    GN_HIP(h, launch_planned(st, g, h->dplan));
    return GN_OK;
}

gn_status validation_residual(gn_handle h);

// max |R| on the validation grid (theta's weights already transposed).
gn_status validation(gn_handle h, const double *theta) {
    if (h->nv <= 0) return GN_OK;
    SweepBatch b{};
    b.x = h->val.q; b.n = h->nv; b.nn = h->nn_val;
    with_phi(h, b, h->phi_val, h->nv);
    GN_HIP(h, launch_mlp_forward(h->stream, h->md, theta, h->thetaT, b));
    return validation_residual(h);
}

// The validation residual and its max-norm from the forward jets in nn_val.
gn_status validation_residual(gn_handle h) {
    if (h->nv <= 0) return GN_OK;
    GN_HIP(h, launch_residual(h->stream, residual_args_val(h)));
    return GN_OK;
}

// J (and r when r != null, with stride r_stride) for the current theta.
gn_status jacobian_into(gn_handle h, const double *theta, double *J, int64_t ldJ, double *r, int64_t r_stride) {
    GN_TRY(forward_all(h, theta));
    GN_TRY(residual_rows(h, r ? r : h->r_tmp, r ? r_stride : 1, true));
    hipStream_t st = h->stream;
    SweepBatch b{};
    b.x = h->pts.q; b.s0 = h->seed0; b.s1 = h->seed1; b.n = h->n; b.rows = J; b.ld = ldJ;
    with_phi(h, b, h->phi_pts, h->n);
    GN_HIP(h, launch_mlp_rows(st, h->md, theta, h->thetaT, b));
    SweepBatch o{};
    o.x = h->one_x; o.s0c = sqrt(h->c_norm); o.s1c = 0.0; o.n = 1; o.rows = J + norm_row(h) * ldJ; o.ld = ldJ;
    with_phi(h, o, h->phi_one, 1);
    GN_HIP(h, launch_mlp_rows(st, h->md, theta, h->thetaT, o));
    if (h->equation == GN_EQ_CCF1D) {
        // B_j = dTheta(t_j)/dtheta = E_j dNN(t_j)/dtheta, then J[:N] += diag(sc Theta_y) Q B
        SweepBatch nb{};
        nb.x = h->nodes.q; nb.s0 = h->nodes.E; nb.s1c = 0.0; nb.n = h->m; nb.rows = h->Bm; nb.ld = h->ldJ;
        with_phi(h, nb, h->phi_nodes, h->m);
        GN_HIP(h, launch_mlp_rows(st, h->md, theta, h->thetaT, nb));
        GemmDesc g{};
        g.M = h->n; g.N = h->md.P; g.K = h->m;
        g.A = h->Q; g.lda = h->ldQ; g.la = 1;
        g.B = h->Bm; g.ldb = h->ldJ; g.lb = 0;
        g.C = J; g.ldc = ldJ;
        g.alpha = 1.0; g.beta = 1.0; g.rowscale = h->cscale;
        GN_HIP(h, launch_planned(st, g, h->cplan));
    }
    GN_TRY(deriv_jacobian(h, theta, J, ldJ));
    return GN_OK;
}

gn_status read_status(gn_handle h, DevStatus *out) {
    GN_HIP(h, hipMemcpyAsync(out, h->status, sizeof(DevStatus), hipMemcpyDeviceToHost, h->stream));
    GN_HIP(h, hipStreamSynchronize(h->stream));
    if (out->wait_fail) return fail(h, GN_EDEVICE, "a bounded device wait of the back substitution ran out%s");
    return GN_OK;
}

// Records the boundary event `k` of the current profiled step (no-op when
// profiling is off or the step budget is used up).
void mark(gn_handle h, int k) {
    if (h->prof_count >= h->prof_max) return;
    (void)hipEventRecord(h->events[(size_t)h->prof_count * (GN_PHASE_COUNT + 1) + k], h->stream);
}

// Phase 1 of a step: forward jets, residual rows into column P of the
// workspace J (the Gram of [J | r] then carries g and r^T r), validation
// max-norm, Jacobian rows and the Hilbert coupling.  Marks phase boundaries.
GemmDesc coupling_desc(gn_handle h) {
    GemmDesc c{};
    c.M = h->n; c.N = h->md.P; c.K = h->m;
    c.A = h->Q; c.lda = h->ldQ; c.la = 1;
    c.B = h->Bm; c.ldb = h->ldJ; c.lb = 0;
    c.C = h->J; c.ldc = h->ldJ;
    c.alpha = 1.0; c.beta = 1.0; c.rowscale = h->cscale;
    return c;
}

GemmDesc gram_desc(gn_handle h) {
    const int64_t P = h->md.P;
    GemmDesc g{};
    g.M = P + 1; g.N = P + 1; g.K = total_rows(h);
    g.A = h->J; g.lda = h->ldJ; g.la = 1;
    g.B = h->J; g.ldb = h->ldJ; g.lb = 0;
    g.C = h->G; g.ldc = h->ldG;
    g.alpha = 1.0; g.beta = 0.0; g.lower = 1;
    return g;
}

gn_status build_step_jacobian(gn_handle h, const double *d_theta, bool marks, bool coupling = true) {
    hipStream_t st = h->stream;
    const int64_t P = h->md.P;
    double *J = h->J;
    const int64_t ldJ = h->ldJ;
    GN_TRY(forward_all(h, d_theta));
    GN_TRY(residual_rows(h, J + P, ldJ, true));
    GN_TRY(validation(h, d_theta));
    if (marks) mark(h, 1);
    SweepBatch b{};
    b.x = h->pts.q; b.s0 = h->seed0; b.s1 = h->seed1; b.n = h->n; b.rows = J; b.ld = ldJ;
    with_phi(h, b, h->phi_pts, h->n);
    GN_HIP(h, launch_mlp_rows(st, h->md, d_theta, h->thetaT, b));
    SweepBatch o{};
    o.x = h->one_x; o.s0c = sqrt(h->c_norm); o.s1c = 0.0; o.n = 1; o.rows = J + norm_row(h) * ldJ; o.ld = ldJ;
    with_phi(h, o, h->phi_one, 1);
    GN_HIP(h, launch_mlp_rows(st, h->md, d_theta, h->thetaT, o));
    if (h->equation == GN_EQ_CCF1D) {
        SweepBatch nb{};
        nb.x = h->nodes.q; nb.s0 = h->nodes.E; nb.s1c = 0.0; nb.n = h->m; nb.rows = h->Bm; nb.ld = ldJ;
        with_phi(h, nb, h->phi_nodes, h->m);
        GN_HIP(h, launch_mlp_rows(st, h->md, d_theta, h->thetaT, nb));
    }
    if (marks) mark(h, 2);
    if (coupling && h->equation == GN_EQ_CCF1D) GN_HIP(h, launch_planned(st, coupling_desc(h), h->cplan));
    GN_TRY(deriv_jacobian(h, d_theta, J, ldJ));
    return GN_OK;
}


// ---------------------------------------------------------------- 2D helpers
Sweep2DArgs sweep2d_args(gn_handle h) {
    Sweep2DArgs b{};
    b.map = h->map2;
    b.pts = h->pts2;
    b.seeds = h->seeds2;
    b.lds = total_rows(h);
    return b;
}

// network output jets at every point of the table
gn_status forward2d(gn_handle h, const double *theta) {
    hipStream_t st = h->stream;
    GN_HIP(h, launch_transpose_weights(st, h->md, theta, h->thetaT));
    Sweep2DArgs b = sweep2d_args(h);
    b.nrows = h->map2.n + h->map2.n1 + h->map2.ne + 1;
    b.nn = h->nn2;
    b.ldn = h->ldn2;
    GN_HIP(h, launch_jets2d_forward(st, h->md, theta, h->thetaT, b));
    return GN_OK;
}

Res2DArgs res2d_args(gn_handle h) {
    Res2DArgs a{};
    a.equation = h->equation;
    a.lam = h->lam;
    a.map = h->map2;
    a.nout = h->nout;
    a.c_norm = h->c_norm;
    a.c_target = h->c_target;
    a.scale_eq = sqrt(1.0 / (double)(h->map2.n * h->map2.n_eq));
    a.scale_d1 = h->map2.n1 > 0 ? sqrt(1.0 / (2.0 * (double)h->map2.n1)) : 0.0;
    a.scale_edge = h->map2.ne > 0 ? sqrt(1.0 / (double)h->map2.ne) : 0.0;
    return a;
}

// scaled rows into r (stride), seeds into seeds2 when `seeds`; max |R| on the collocation points
gn_status residual2d_rows(gn_handle h, double *r, int64_t r_stride, bool seeds) {
    Res2DArgs a = res2d_args(h);
    a.pts = h->pts2;
    a.nn = h->nn2;
    a.ldn = h->ldn2;
    a.r = r;
    a.r_stride = r_stride;
    a.seeds = seeds ? h->seeds2 : nullptr;
    a.lds = total_rows(h);
    a.max_out = &h->status->max_R;
    GN_HIP(h, launch_residual2d(h->stream, a));
    return GN_OK;
}

// max |R| over the equations at the validation points (weights already transposed)
gn_status validation2d(gn_handle h, const double *theta) {
    if (h->nv <= 0) return GN_OK;
    Sweep2DArgs b{};
    b.pts = h->val2;
    b.nrows = h->nv;
    b.nn = h->nn2v;
    b.ldn = h->ldnv2;
    GN_HIP(h, launch_jets2d_forward(h->stream, h->md, theta, h->thetaT, b));
    Res2DArgs a = res2d_args(h);
    a.map = RowMap2D{h->nv, 0, 0, h->n_eq};
    a.pts = h->val2;
    a.nn = h->nn2v;
    a.ldn = h->ldnv2;
    a.validation = 1;
    a.max_out = &h->status->max_R_val;
    GN_HIP(h, launch_residual2d(h->stream, a));
    return GN_OK;
}

// rows [row0, row0 + nrows) of J (seeds2 current) into J (row row0 at J)
gn_status jac_rows2d(gn_handle h, const double *theta, int64_t row0, int64_t nrows, double *J, int64_t ldJ) {
    Sweep2DArgs b = sweep2d_args(h);
    b.row0 = row0;
    b.nrows = nrows;
    b.J = J;
    b.ldJ = ldJ;
    GN_HIP(h, launch_jets2d_rows(h->stream, h->md, theta, h->thetaT, b));
    return GN_OK;
}

// The device copies of a work plan (table and partial-tile workspace) into
// *out, or *out left empty when the product takes no plan.
gn_status tile_plan_alloc(gn_handle h, std::vector<void *> &A, int64_t M, int64_t N, bool lower, TilePlan *out) {
    *out = TilePlan{};
    int dev = 0, cus = 0;
    GN_HIP(h, hipGetDevice(&dev));
    GN_HIP(h, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    std::vector<int4> t;
    TilePlan p;
    p.M = M;
    p.N = N;
    p.lower = lower;
    const bool ok = lower ? plan_gram(M, cus, t, p.nwork, p.nsplit, p.pieces, p.tile)
                          : plan_rect(M, N, cus, t, p.nwork, p.nsplit, p.pieces, p.tile);
    if (!ok) return GN_OK;
    GN_TRY(dev_alloc(h, A, &p.d_work, (int64_t)t.size()));
    if (p.nsplit > 0) GN_TRY(dev_alloc(h, A, &p.ws, gram_plan_ws_doubles(p.nsplit, p.pieces, p.tile)));
    GN_HIP(h, hipMemcpy(p.d_work, t.data(), sizeof(int4) * t.size(), hipMemcpyHostToDevice));
    *out = p;
    return GN_OK;
}

// Work plan of the FP64 Gram of order P + 1 (tiles balanced over the XCDs,
// the last round's tiles split along K), with its partial-tile workspace.
gn_status gram_plan_alloc(gn_handle h, std::vector<void *> &A) {
    h->gplan = TilePlan{};
    if (h->precision != GN_FP64) return GN_OK;
    return tile_plan_alloc(h, A, h->md.P + 1, h->md.P + 1, true, &h->gplan);
}

GemmDesc gram_desc_rows(gn_handle h, int64_t rows, double beta) {
    const int64_t P = h->md.P;
    GemmDesc g{};
    g.M = P + 1; g.N = P + 1; g.K = rows;
    g.A = h->J; g.lda = h->ldJ; g.la = 1;
    g.B = h->J; g.ldb = h->ldJ; g.lb = 0;
    g.C = h->G; g.ldc = h->ldG;
    g.alpha = 1.0; g.beta = beta; g.lower = 1;
    return g;
}

// Bordered Gram of [J | r] over all rows of a 2D problem, row chunk by row
// chunk (J of the chunk formed, then accumulated into G); r^T r from r2.
gn_status gram2d(gn_handle h, const double *theta) {
    hipStream_t st = h->stream;
    const int64_t P = h->md.P, m = total_rows(h);
    double *Grow = h->G + P * h->ldG;
    if (h->precision == GN_INT8_CRT) {
        // Column maxima need every row before the first residue: with more
        // than one chunk, J is formed twice (maxima, then residues).
        // G from int8 modular products over the P parameter columns; the
        // border row g = J^T r (chunk by chunk) and r^T r in FP64
        const int b = modgram_bits(m);
        const bool one = h->rows_ws >= m;
        GN_HIP(h, launch_modgram_begin(st, P, h->mg));
        for (int pass = one ? 1 : 0; pass < 2; ++pass)
            for (int64_t r0 = 0, c = 0; r0 < m; r0 += h->rows_ws, ++c) {
                const int64_t nr = (m - r0) < h->rows_ws ? (m - r0) : h->rows_ws;
                GN_TRY(jac_rows2d(h, theta, r0, nr, h->J, h->ldJ));
                if (pass == 0 || one) GN_HIP(h, launch_modgram_colmax(st, h->J, nr, P, h->ldJ, h->mg));
                if (pass == 1) {
                    GN_HIP(h, launch_modgram_chunk(st, h->J, nr, P, h->ldJ, b, h->mg, c > 0));
                    GN_HIP(h, launch_gemv_t(st, h->J, nr, P, h->ldJ, h->r2 + r0, Grow, h->gemv_work, c > 0));
                }
            }
        GN_HIP(h, launch_modgram_finish(st, P, b, h->G, h->ldG, h->mg));
        GN_HIP(h, launch_sumsq(st, h->r2, m, 1, Grow + P, h->red_work));
        return GN_OK;
    }
    for (int64_t r0 = 0, c = 0; r0 < m; r0 += h->rows_ws, ++c) {
        const int64_t nr = (m - r0) < h->rows_ws ? (m - r0) : h->rows_ws;
        GN_TRY(jac_rows2d(h, theta, r0, nr, h->J, h->ldJ));
        if (h->precision == GN_SPLIT32) {
            GN_HIP(h, launch_split(st, h->J, nr, P, h->ldJ, h->Jhi, h->Jlo));
            GN_HIP(h, launch_split_gram(st, h->Jhi, h->Jlo, nr, P, h->ldJ, h->G, h->ldG, c > 0));
            GN_HIP(h, launch_gemv_t(st, h->J, nr, P, h->ldJ, h->r2 + r0, Grow, h->gemv_work, c > 0));
        } else {
            GN_HIP(h, launch_copy_strided(st, h->r2 + r0, nr, 1, h->J + P, h->ldJ, 1.0));
            GN_HIP(h, launch_planned(st, gram_desc_rows(h, nr, c > 0 ? 1.0 : 0.0), h->gplan));
        }
    }
    if (h->precision == GN_SPLIT32) GN_HIP(h, launch_sumsq(st, h->r2, m, 1, Grow + P, h->red_work));
    return GN_OK;
}

double bits_to_double(unsigned long long b) {
    double d;
    memcpy(&d, &b, sizeof d);
    return d;
}

void fill_stats(const DevStatus &ds, gn_stats *o) {
    memset(o, 0, sizeof *o);
    o->half_sq_norm = 0.5 * ds.half_sq_norm;
    o->max_abs_R = bits_to_double(ds.max_R);
    o->max_abs_R_val = bits_to_double(ds.max_R_val);
    o->grad_dot_delta = -ds.grad_dot_delta;
    o->model_sq_norm = ds.model_sq_norm;
    o->chol_info = ds.chol_info;
    o->updated = ds.updated;
    const bool r_finite = (ds.half_sq_norm - ds.half_sq_norm == 0.0);
    o->status = !r_finite ? GN_ENONFINITE : (ds.flag ? GN_ENOTPD : (ds.nonfinite ? GN_ENONFINITE : GN_OK));
}

}  // namespace

struct gn_batch_context {
    std::vector<gn_handle> hs;
    hipStream_t stream = nullptr;
    int64_t P = 0;
    std::vector<BatchChol> h_bc;
    BatchChol *d_bc = nullptr;
    BatchedGemmPlan coupling, gram;          // Hilbert coupling of the CCF instances, bordered Gram
    BatchedGemmPlan gram_tail;               // the bordered Gram's last rows when they are few (thin tiles)
    BatchedGemmPlan coupling_tail;           // the coupling's last columns when they are few (128 x 64 tiles)
    std::vector<BatchedGemmPlan> chol;       // per Cholesky panel: panel solve, trailing update
    std::vector<double *> uploaded_thetas;
    std::vector<DevStatus> ds;
    std::vector<uint64_t> gen;  // point-set generation of every handle when the batch was made
    // the per-instance stage (small, launch-bound kernels) spread over the
    // batch stream and BATCH_LANES more streams of default priority,
    // forked from and joined back into the batch stream by events
    std::vector<hipStream_t> lanes;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    // when the network fits the matrix-core sweeps: the forward jets of every
    // point set of every instance in one launch, and the Jacobian rows in one
    // (work tables of 16-point tiles); job k belongs to instance *_inst[k]
    bool jobs = false;
    std::vector<SweepJob> h_fjobs, h_rjobs;
    std::vector<int> fjob_inst, rjob_inst;
    SweepJob *d_fjobs = nullptr, *d_rjobs = nullptr;
    int2 *d_fwork = nullptr, *d_rwork = nullptr;
    int64_t nfwork = 0, nrwork = 0;
    // CCF batches: the residuals of every instance (collocation points with
    // their seeds, validation grid) in one launch
    bool res_jobs = false;
    ResidualArgs *d_resjobs = nullptr;
    int2 *d_reswork = nullptr;
    int64_t nreswork = 0;
};
static constexpr int BATCH_LANES = 3;

extern "C" {

const char *gn_status_string(int32_t s) {
    if (s == GN_ENOTPD) return "matrix not positive definite";
    if (s == GN_EREJECTED) return "no trial step decreased the objective";
    if (s <= 0 && s >= -5) return kStatusText[-s];
    return "unknown status";
}

const char *gn_last_error(gn_handle h) { return h ? h->err.c_str() : noalloc_last_error(); }

gn_status gn_int8_crt_params(int64_t m, int32_t *bits, int32_t *n_moduli, int32_t *moduli) {
    if (m < 1 || m > GN_INT8_CRT_MAX_TOTAL_ROWS || !bits || !n_moduli || !moduli) return GN_EINVAL;
    *bits = modgram_bits(m);
    *n_moduli = modgram_moduli();
    modgram_list(moduli);
    return GN_OK;
}

gn_status gn_create(const gn_problem *prob, gn_handle *out) {
    if (!prob || !out || !prob->widths) return GN_EINVAL;
    *out = nullptr;
    const int L = prob->n_layers;
    if (L < 1 || L > GN_MAX_LAYERS) return GN_EINVAL;
    const bool two_d = prob->equation == GN_EQ_IPM2D || prob->equation == GN_EQ_BOUSS2D;
    if (!two_d && prob->equation != GN_EQ_CCF1D && prob->equation != GN_EQ_BURGERS1D) return GN_EINVAL;
    if (prob->precision != GN_FP64 && prob->precision != GN_SPLIT32 && prob->precision != GN_INT8_CRT)
        return GN_EINVAL;
    if (!(prob->lam > 0.0) || !(prob->c_norm >= 0.0) || prob->row_chunk < 0) return GN_EINVAL;
    if (two_d) {
        const int nout = prob->equation == GN_EQ_IPM2D ? 1 : 3;
        if (prob->widths[0] != 2 || prob->widths[L] != nout) return GN_EINVAL;
        for (int l = 1; l < L; ++l)
            if (prob->widths[l] < 1 || prob->widths[l] > GN_MAX_WIDTH_2D) return GN_EINVAL;
    } else {
        const int nf = prob->n_fourier;
        if (nf < 0 || (nf > 0 && (!prob->fourier_b || 2 * nf > GN_MAX_WIDTH))) return GN_EINVAL;
        if (prob->widths[0] != (nf > 0 ? 2 * nf : 1) || prob->widths[L] != 1) return GN_EINVAL;
        for (int l = 1; l < L; ++l)
            if (prob->widths[l] < 1 || prob->widths[l] > GN_MAX_WIDTH) return GN_EINVAL;
    }
    if (two_d && prob->n_fourier != 0) return GN_EINVAL;
    gn_handle h = new (std::nothrow) gn_context();
    if (!h) return GN_ENOMEM;
    h->equation = prob->equation;
    h->precision = prob->precision;
    h->lam = prob->lam;
    h->c_norm = prob->c_norm;
    h->c_target = prob->c_target;
    h->dim = two_d ? 2 : 1;
    h->nout = prob->widths[L];
    h->n_eq = prob->equation == GN_EQ_BOUSS2D ? 3 : 1;
    h->row_chunk = prob->row_chunk;
    MlpDesc &d = h->md;
    d.L = L;
    int o = 0;
    for (int l = 0; l <= L; ++l) d.w[l] = prob->widths[l];
    for (int l = 0; l < L; ++l) {
        d.off[l] = o;
        o += d.w[l + 1] * (d.w[l] + 1);
    }
    d.P = o;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return GN_EDEVICE;
    }
    const int64_t P = d.P;
    h->cap = P + 1;
    gn_status s = GN_OK;
    if (s == GN_OK) s = dev_alloc(h, h->allocs, &h->thetaT, P);
    if (s == GN_OK) s = dev_alloc(h, h->allocs, &h->linv, chol_linv_size(h->cap));
    if (s == GN_OK) s = dev_alloc(h, h->allocs, &h->ybuf, h->cap);
    if (s == GN_OK) s = dev_alloc(h, h->allocs, &h->zbuf, h->cap);
    if (s == GN_OK) s = dev_alloc(h, h->allocs, &h->delta, h->cap);
    if (s == GN_OK) s = dev_alloc(h, h->allocs, &h->theta_trial, P);
    if (s == GN_OK) s = dev_alloc(h, h->allocs, &h->r1_g, P);
    if (s == GN_OK) s = dev_alloc(h, h->allocs, &h->r1_u, P);
    if (s == GN_OK) s = dev_alloc(h, h->allocs, &h->r1_D, P);
    if (s == GN_OK) s = dev_alloc(h, h->allocs, &h->r1_b, P);
    if (s == GN_OK) s = dev_alloc(h, h->allocs, &h->r1_dots, DOT_MAX);
    if (s == GN_OK) s = dev_alloc(h, h->allocs, &h->r1_work, dots_work_size());
    if (s == GN_OK) s = dev_alloc(h, h->allocs, &h->gdiag, h->cap);
    if (s == GN_OK)
        s = dev_alloc(h, h->allocs, &h->gemv_work, std::max(gemv_t_work_size(0, h->cap), gemv_t2_work_size(h->cap)));
    if (s == GN_OK) s = dev_alloc(h, h->allocs, &h->red_work, 1024);
    if (s == GN_OK) s = dev_alloc(h, h->allocs, &h->chol_tmp, chol_tmp_size());
    if (s == GN_OK) s = dev_alloc(h, h->allocs, &h->one_x, 1);
    if (s == GN_OK) s = dev_alloc(h, h->allocs, &h->nn_one, 2);
    if (s == GN_OK) s = dev_alloc(h, h->allocs, &h->seed_one, 1);
    if (s == GN_OK) s = dev_alloc(h, h->allocs, &h->status, 1);
    if (s == GN_OK) s = dev_alloc(h, h->allocs, &h->solve_sync, solve_sync_size(h->cap));
    if (s == GN_OK && hipMemset(h->solve_sync, 0, sizeof(unsigned) * (size_t)solve_sync_size(h->cap)) != hipSuccess) {
        (void)hipGetLastError();
        s = GN_EDEVICE;
    }
    if (!two_d && prob->n_fourier > 0) {
        h->nf = prob->n_fourier;
        if (s == GN_OK) s = dev_alloc(h, h->allocs, &h->fb, h->nf);
        if (s == GN_OK) s = dev_alloc(h, h->allocs, &h->phi_one, 4 * h->nf);
    }
    if (s == GN_OK) s = gram_plan_alloc(h, h->allocs);
    if (s != GN_OK) {
        free_list(h->allocs);
        delete h;
        return s;
    }
    const double one = 1.0;
    bool ok = hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&h->ev_panel, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&h->ev_trail, hipEventDisableTiming) == hipSuccess &&
              hipMemcpy(h->one_x, &one, sizeof one, hipMemcpyHostToDevice) == hipSuccess;
    if (ok && h->nf > 0) {
        ok = hipMemcpy(h->fb, prob->fourier_b, sizeof(double) * h->nf, hipMemcpyHostToDevice) == hipSuccess &&
             launch_fourier_features(nullptr, 1, h->one_x, h->nf, h->fb, h->phi_one, 1) == hipSuccess &&
             hipStreamSynchronize(nullptr) == hipSuccess;
    }
    if (!ok) {
        if (h->side) (void)hipStreamDestroy(h->side);
        if (h->ev_panel) (void)hipEventDestroy(h->ev_panel);
        if (h->ev_trail) (void)hipEventDestroy(h->ev_trail);
        free_list(h->allocs);
        delete h;
        return GN_EDEVICE;
    }
    *out = h;
    return GN_OK;
}

gn_status gn_destroy(gn_handle h) {
    if (!h) return GN_EINVAL;
    (void)hipStreamSynchronize(h->stream);
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    if (h->side) {
        (void)hipStreamSynchronize(h->side);
        (void)hipStreamDestroy(h->side);
    }
    if (h->ev_panel) (void)hipEventDestroy(h->ev_panel);
    if (h->ev_trail) (void)hipEventDestroy(h->ev_trail);
    free_list(h->pt_allocs);
    free_list(h->allocs);
    delete h;
    return GN_OK;
}

gn_status gn_set_stream(gn_handle h, void *stream) {
    if (!h) return GN_EINVAL;
    h->stream = (hipStream_t)stream;
    return GN_OK;
}

int64_t gn_num_params(gn_handle h) { return h ? h->md.P : -1; }
int64_t gn_num_rows(gn_handle h) { return (h && h->n > 0) ? total_rows(h) : -1; }

gn_status gn_set_points(gn_handle h, int64_t n, const double *d_s, const double *d_rho, const double *d_f,
                        int64_t m_quad, const double *d_sq, const double *d_wq, int64_t n_val,
                        const double *d_sval) {
    return gn_set_points_ex(h, n, d_s, d_rho, d_f, m_quad, d_sq, d_wq, n_val, d_sval, 0, nullptr, 0, nullptr, 1.0,
                            1.0);
}

gn_status gn_set_points_ex(gn_handle h, int64_t n, const double *d_s, const double *d_rho, const double *d_f,
                           int64_t m_quad, const double *d_sq, const double *d_wq, int64_t n_val,
                           const double *d_sval, int64_t n1, const double *d_s1, int64_t n2, const double *d_s2,
                           double c_d1, double c_d2) {
    if (!h) return GN_EINVAL;
    if (h->dim != 1) return fail(h, GN_EINVAL, "2D problems take gn_set_points_2d%s");
    if (n < 1 || !d_s) return fail(h, GN_EINVAL, "need n >= 1 collocation points%s");
    if (h->equation == GN_EQ_CCF1D && (m_quad < 1 || !d_sq || !d_wq))
        return fail(h, GN_EINVAL, "the CCF Hilbert term needs m_quad >= 1 nodes and weights%s");
    if (n_val < 0 || (n_val > 0 && !d_sval)) return fail(h, GN_EINVAL, "bad validation grid%s");
    if (n1 < 0 || n2 < 0 || (n1 > 0 && !d_s1) || (n2 > 0 && !d_s2))
        return fail(h, GN_EINVAL, "bad derivative point sets%s");
    if (!(c_d1 >= 0.0) || !(c_d2 >= 0.0)) return fail(h, GN_EINVAL, "derivative loss weights must be >= 0%s");
    if (h->equation != GN_EQ_CCF1D) m_quad = 0;
    if (m_quad > 65535 && n1 + n2 > 0) return fail(h, GN_EINVAL, "at most 65535 nodes with derivative rows%s");
    if (h->nf > 0 && n1 + n2 > 0) return fail(h, GN_EINVAL, "derivative rows take the plain network input%s");
    if (h->precision == GN_INT8_CRT && n + n1 + n2 + 1 > GN_INT8_CRT_MAX_ROWS)
        return fail(h, GN_EINVAL, "the int8 Gram takes at most %s rows", std::to_string(GN_INT8_CRT_MAX_ROWS).c_str());
    GN_HIP(h, hipStreamSynchronize(h->stream));
    free_list(h->pt_allocs);
    ++h->points_gen;
    h->r1_factored = false;
    h->n = h->m = h->nv = 0;
    h->nd1 = h->nd2 = 0;
    h->stage2 = false;
    h->s1R = h->s1V = h->s1T = h->s1Rv = h->s1Vv = h->s1Tv = nullptr;
    h->fn_R = nullptr;
    h->cp_t = h->cp_z = h->cp_work = nullptr;
    h->cplan = TilePlan{};
    h->dplan = TilePlan{};
    auto &A = h->pt_allocs;
    const int64_t P = h->md.P;
    const int64_t nd = n1 + n2;
    const int64_t m_rows = n + nd + 1;
    h->ldJ = round_up(P + 1, 32);
    h->ldG = round_up(P + 1, 32);
    h->ldQ = round_up(n, 2);  // Q^T: m_quad rows of n points (even stride: 16-byte aligned rows)
    h->ldA = round_up(nd, 2);
    const int64_t nparts = mlp_vjp_partials(h->md, n) + mlp_vjp_partials(h->md, 1) + mlp_vjp_partials(h->md, m_quad) +
                           (nd > 0 ? jet3_vjp_partials(nd) + jet3_vjp_partials(m_quad) : 0);
    auto geo = [&](Geo1D &g, int64_t cnt, bool with_w) -> gn_status {
        GN_TRY(dev_alloc(h, A, &g.y, cnt));
        GN_TRY(dev_alloc(h, A, &g.q, cnt));
        GN_TRY(dev_alloc(h, A, &g.E, cnt));
        GN_TRY(dev_alloc(h, A, &g.Ey, cnt));
        GN_TRY(dev_alloc(h, A, &g.qy, cnt));
        g.wh = nullptr;
        if (with_w) GN_TRY(dev_alloc(h, A, &g.wh, cnt));
        return GN_OK;
    };
    gn_status s = GN_OK;
    s = geo(h->pts, n, false);
    if (s == GN_OK) s = geo(h->nodes, m_quad, true);
    if (s == GN_OK) s = geo(h->val, n_val, false);
    if (s == GN_OK && d_rho) s = dev_alloc(h, A, &h->rho, n);
    if (s == GN_OK && !d_rho) h->rho = nullptr;
    if (s == GN_OK && d_f) s = dev_alloc(h, A, &h->f, n);
    if (s == GN_OK && !d_f) h->f = nullptr;
    if (s == GN_OK && m_quad > 0) s = dev_alloc(h, A, &h->Q, m_quad * h->ldQ);
    if (s == GN_OK && m_quad > 0) s = dev_alloc(h, A, &h->cp_t, 2 * n);
    if (s == GN_OK && m_quad > 0) s = dev_alloc(h, A, &h->cp_z, 2 * m_quad);
    if (s == GN_OK && m_quad > 0) s = dev_alloc(h, A, &h->cp_work, gemv_t2_work_size(n));
    if (s == GN_OK && m_quad > 0 && h->equation == GN_EQ_CCF1D) s = tile_plan_alloc(h, A, n, P, false, &h->cplan);
    if (s == GN_OK) s = dev_alloc(h, A, &h->nn_pts, 2 * n);
    if (s == GN_OK) s = dev_alloc(h, A, &h->nn_nodes, 2 * m_quad);
    if (s == GN_OK) s = dev_alloc(h, A, &h->nn_val, 2 * n_val);
    if (s == GN_OK) s = dev_alloc(h, A, &h->R, n);
    if (s == GN_OK) s = dev_alloc(h, A, &h->seed0, n);
    if (s == GN_OK) s = dev_alloc(h, A, &h->seed1, n);
    if (s == GN_OK) s = dev_alloc(h, A, &h->cscale, n);
    if (s == GN_OK) s = dev_alloc(h, A, &h->r_tmp, m_rows);
    if (s == GN_OK) s = dev_alloc(h, A, &h->r1_w1, m_rows);
    if (s == GN_OK) s = dev_alloc(h, A, &h->r1_w2, m_rows);
    if (s == GN_OK) s = dev_alloc(h, A, &h->vseed0, n);
    if (s == GN_OK) s = dev_alloc(h, A, &h->vseed1, n);
    if (s == GN_OK) s = dev_alloc(h, A, &h->useed, m_quad);
    if (s == GN_OK) s = dev_alloc(h, A, &h->J, m_rows * h->ldJ);
    // node Jacobians B (and B1, B2 for the derivative rows), stacked
    if (s == GN_OK && m_quad > 0) s = dev_alloc(h, A, &h->Bm, (nd > 0 ? 3 : 1) * m_quad * h->ldJ);
    auto geo3 = [&](Geo3 &g, int64_t cnt) -> gn_status {
        g.ld = cnt;
        GN_TRY(dev_alloc(h, A, &g.y, cnt));
        GN_TRY(dev_alloc(h, A, &g.q, 4 * cnt));
        GN_TRY(dev_alloc(h, A, &g.E, 4 * cnt));
        return GN_OK;
    };
    if (h->nf > 0) {
        if (s == GN_OK) s = dev_alloc(h, A, &h->phi_pts, 4 * h->nf * n);
        if (s == GN_OK && m_quad > 0) s = dev_alloc(h, A, &h->phi_nodes, 4 * h->nf * m_quad);
        if (s == GN_OK && n_val > 0) s = dev_alloc(h, A, &h->phi_val, 4 * h->nf * n_val);
    }
    // third-order data of the nodes and the validation grid (derivative rows and maxima)
    if (m_quad > 0) {
        if (s == GN_OK) s = geo3(h->geo3n, m_quad);
        if (s == GN_OK) s = dev_alloc(h, A, &h->nn3n, 4 * m_quad);
        if (s == GN_OK) s = dev_alloc(h, A, &h->nfield, 3 * m_quad);
    }
    if (n_val > 0) {
        if (s == GN_OK) s = geo3(h->geo3v, n_val);
        if (s == GN_OK) s = dev_alloc(h, A, &h->nn3v, 4 * n_val);
    }
    if (nd > 0) {
        if (s == GN_OK) s = geo3(h->geo3, nd);
        if (s == GN_OK) s = dev_alloc(h, A, &h->nn3, 4 * nd);
        if (s == GN_OK) s = dev_alloc(h, A, &h->dseed, 4 * nd);
        if (s == GN_OK) s = dev_alloc(h, A, &h->dvseed, 4 * nd);
        if (s == GN_OK) s = dev_alloc(h, A, &h->dcoef, 3 * nd);
        if (m_quad > 0) {
            if (s == GN_OK) s = dev_alloc(h, A, &h->bseed, 8 * m_quad);
            if (s == GN_OK) s = dev_alloc(h, A, &h->dAT, 3 * m_quad * h->ldA);
            if (s == GN_OK && h->equation == GN_EQ_CCF1D) s = tile_plan_alloc(h, A, nd, P, false, &h->dplan);
            if (s == GN_OK) s = dev_alloc(h, A, &h->nvseed, 4 * m_quad);
        }
    }
    if (s == GN_OK) s = dev_alloc(h, A, &h->G, (P + 1) * h->ldG);
    if (s == GN_OK && h->precision == GN_SPLIT32) s = dev_alloc(h, A, &h->Jhi, m_rows * h->ldJ);
    if (s == GN_OK && h->precision == GN_SPLIT32) s = dev_alloc(h, A, &h->Jlo, m_rows * h->ldJ);
    h->mg = ModgramWork{};
    if (h->precision == GN_INT8_CRT) {
        h->mg.r_bytes = modgram_r_bytes(m_rows, P + 1);
        h->mg.y_bytes = modgram_y_bytes(P + 1);
        h->mg.cmax_len = modgram_ppad(P + 1);
        h->mg.rows = m_rows;
        if (s == GN_OK) s = dev_alloc(h, A, &h->mg.R, h->mg.r_bytes);
        if (s == GN_OK) s = dev_alloc(h, A, &h->mg.Y, h->mg.y_bytes);
        if (s == GN_OK) s = dev_alloc(h, A, &h->mg.cmax, h->mg.cmax_len);
    }
    if (s == GN_OK) s = dev_alloc(h, A, &h->partial, nparts * P);
    if (s != GN_OK) {
        free_list(A);
        return s;
    }
    h->n_partial_cap = nparts;
    hipStream_t st = h->stream;
    if (d_rho) GN_HIP(h, hipMemcpyAsync(h->rho, d_rho, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    if (d_f) GN_HIP(h, hipMemcpyAsync(h->f, d_f, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    GN_HIP(h, launch_geometry(st, h->equation, h->lam, n, d_s, nullptr, h->pts));
    if (m_quad > 0) {
        GN_HIP(h, launch_geometry(st, h->equation, h->lam, m_quad, d_sq, d_wq, h->nodes));
        GN_HIP(h, launch_hilbert_matrix(st, n, m_quad, h->pts.y, h->nodes.y, h->nodes.wh, h->Q, h->ldQ));
    }
    if (n_val > 0) GN_HIP(h, launch_geometry(st, h->equation, h->lam, n_val, d_sval, nullptr, h->val));
    if (h->nf > 0) {
        GN_HIP(h, launch_fourier_features(st, n, h->pts.q, h->nf, h->fb, h->phi_pts, n));
        if (m_quad > 0) GN_HIP(h, launch_fourier_features(st, m_quad, h->nodes.q, h->nf, h->fb, h->phi_nodes, m_quad));
        if (n_val > 0) GN_HIP(h, launch_fourier_features(st, n_val, h->val.q, h->nf, h->fb, h->phi_val, n_val));
    }
    if (m_quad > 0) GN_HIP(h, launch_geometry3(st, h->equation, h->lam, m_quad, d_sq, h->geo3n));
    if (n_val > 0) GN_HIP(h, launch_geometry3(st, h->equation, h->lam, n_val, d_sval, h->geo3v));
    if (nd > 0) {
        Geo3 g2 = h->geo3;  // the d2 points follow the d1 points
        g2.y += n1; g2.q += n1; g2.E += n1;
        GN_HIP(h, launch_geometry3(st, h->equation, h->lam, n1, d_s1, h->geo3));
        GN_HIP(h, launch_geometry3(st, h->equation, h->lam, n2, d_s2, g2));
        if (m_quad > 0) GN_HIP(h, launch_node_seeds(st, m_quad, h->geo3n, h->nodes.y, h->bseed, 2 * m_quad));
    }
    GN_HIP(h, hipStreamSynchronize(st));
    h->n = n;
    h->m = m_quad;
    h->nv = n_val;
    h->nd1 = n1;
    h->nd2 = n2;
    h->c_d1 = c_d1;
    h->c_d2 = c_d2;
    return GN_OK;
}

gn_status gn_set_points_2d(gn_handle h, int64_t n, const double *d_s, int64_t n1, const double *d_s1, int64_t ne,
                           const double *d_se, int64_t n_val, const double *d_sval) {
    if (!h) return GN_EINVAL;
    if (h->dim != 2) return fail(h, GN_EINVAL, "1D problems take gn_set_points%s");
    if (n < 1 || !d_s) return fail(h, GN_EINVAL, "need n >= 1 collocation points%s");
    if (n1 < 0 || (n1 > 0 && !d_s1)) return fail(h, GN_EINVAL, "bad d1 point set%s");
    if (n1 > 0 && h->equation != GN_EQ_IPM2D) return fail(h, GN_EINVAL, "d1 rows are defined for GN_EQ_IPM2D%s");
    if (ne < 0 || (ne > 0 && !d_se)) return fail(h, GN_EINVAL, "bad boundary point set%s");
    if (n_val < 0 || (n_val > 0 && !d_sval)) return fail(h, GN_EINVAL, "bad validation grid%s");
    if (h->precision == GN_INT8_CRT) {
        const int64_t rows = RowMap2D{n, n1, ne, h->n_eq}.rows();
        const int64_t chunk = (h->row_chunk > 0 && h->row_chunk < rows) ? h->row_chunk : rows;
        if (chunk > GN_INT8_CRT_MAX_ROWS)
            return fail(h, GN_EINVAL, "the int8 Gram takes row chunks of at most %s rows",
                        std::to_string(GN_INT8_CRT_MAX_ROWS).c_str());
    }
    GN_HIP(h, hipStreamSynchronize(h->stream));
    free_list(h->pt_allocs);
    ++h->points_gen;
    h->r1_factored = false;
    h->n = h->m = h->nv = 0;
    auto &A = h->pt_allocs;
    const int64_t P = h->md.P;
    h->map2 = RowMap2D{n, n1, ne, h->n_eq};
    const int64_t m = h->map2.rows(), npt = n + n1 + ne + 1;
    h->rows_ws = (h->row_chunk > 0 && h->row_chunk < m) ? h->row_chunk : m;
    h->ldJ = round_up(P + 1, 32);
    h->ldG = round_up(P + 1, 32);
    const int64_t nparts = jets2d_vjp_partials(h->md, m);
    const int nc = 6 * h->nout;
    gn_status s = GN_OK;
    auto table = [&](Pts2D &p, int64_t cnt) -> gn_status {
        GN_TRY(dev_alloc(h, A, &p.y1, cnt));
        GN_TRY(dev_alloc(h, A, &p.y2, cnt));
        GN_TRY(dev_alloc(h, A, &p.xin, 12 * cnt));
        p.ld = cnt;
        return GN_OK;
    };
    s = table(h->pts2, npt);
    if (s == GN_OK) s = table(h->val2, n_val);
    if (s == GN_OK) s = dev_alloc(h, A, &h->origin_s, 2);
    if (s == GN_OK) s = dev_alloc(h, A, &h->nn2, nc * npt);
    if (s == GN_OK) s = dev_alloc(h, A, &h->nn2v, nc * n_val);
    if (s == GN_OK) s = dev_alloc(h, A, &h->seeds2, nc * m);
    if (s == GN_OK) s = dev_alloc(h, A, &h->r2, m);
    if (s == GN_OK) s = dev_alloc(h, A, &h->J, h->rows_ws * h->ldJ);
    if (s == GN_OK) s = dev_alloc(h, A, &h->G, (P + 1) * h->ldG);
    if (s == GN_OK && h->precision == GN_SPLIT32) s = dev_alloc(h, A, &h->Jhi, h->rows_ws * h->ldJ);
    if (s == GN_OK && h->precision == GN_SPLIT32) s = dev_alloc(h, A, &h->Jlo, h->rows_ws * h->ldJ);
    h->mg = ModgramWork{};
    if (h->precision == GN_INT8_CRT) {
        h->mg.r_bytes = modgram_r_bytes(h->rows_ws, P + 1);
        h->mg.y_bytes = modgram_y_bytes(P + 1);
        h->mg.cmax_len = modgram_ppad(P + 1);
        h->mg.rows = h->rows_ws;
        if (s == GN_OK) s = dev_alloc(h, A, &h->mg.R, h->mg.r_bytes);
        if (s == GN_OK) s = dev_alloc(h, A, &h->mg.Y, h->mg.y_bytes);
        if (s == GN_OK) s = dev_alloc(h, A, &h->mg.cmax, h->mg.cmax_len);
    }
    if (s == GN_OK) s = dev_alloc(h, A, &h->partial, nparts * P);
    if (s != GN_OK) {
        free_list(A);
        return s;
    }
    h->ldn2 = npt;
    h->ldnv2 = n_val;
    h->r_tmp = h->r2;
    h->n_partial_cap = nparts;
    hipStream_t st = h->stream;
    const double zero2[2] = {0.0, 0.0};
    GN_HIP(h, hipMemcpy(h->origin_s, zero2, sizeof zero2, hipMemcpyHostToDevice));
    GN_HIP(h, launch_geometry2d(st, n, d_s, 0, h->lam, h->pts2, 0));
    GN_HIP(h, launch_geometry2d(st, n1, d_s1, 0, h->lam, h->pts2, n));
    GN_HIP(h, launch_geometry2d(st, ne, d_se, 1, h->lam, h->pts2, n + n1));
    GN_HIP(h, launch_geometry2d(st, 1, h->origin_s, 0, h->lam, h->pts2, n + n1 + ne));
    GN_HIP(h, launch_geometry2d(st, n_val, d_sval, 0, h->lam, h->val2, 0));
    GN_HIP(h, hipStreamSynchronize(st));
    h->n = n;
    h->nv = n_val;
    return GN_OK;
}

gn_status gn_residual(gn_handle h, const double *d_theta, double *d_r) {
    if (!h || !d_theta || !d_r) return GN_EINVAL;
    if (!points_ready(h)) return fail(h, GN_ESTATE, "gn_set_points must be called first%s");
    GN_HIP(h, launch_reset_status(h->stream, h->status));
    if (h->dim == 2) {
        GN_TRY(forward2d(h, d_theta));
        return residual2d_rows(h, d_r, 1, false);
    }
    GN_TRY(forward_all(h, d_theta));
    return residual_rows(h, d_r, 1, false);
}

gn_status gn_jacobian(gn_handle h, const double *d_theta, double *d_J, int64_t ldJ, double *d_r) {
    if (!h || !d_theta || !d_J) return GN_EINVAL;
    if (!points_ready(h)) return fail(h, GN_ESTATE, "gn_set_points must be called first%s");
    if (ldJ < h->md.P) return fail(h, GN_EINVAL, "ldJ < P%s");
    GN_HIP(h, launch_reset_status(h->stream, h->status));
    if (h->dim == 2) {
        GN_TRY(forward2d(h, d_theta));
        GN_TRY(residual2d_rows(h, d_r ? d_r : h->r2, 1, true));
        return jac_rows2d(h, d_theta, 0, total_rows(h), d_J, ldJ);
    }
    return jacobian_into(h, d_theta, d_J, ldJ, d_r, 1);
}

gn_status gn_gram(gn_handle h, const double *d_J, int64_t m, int64_t p, int64_t ldJ, const double *d_r,
                  double *d_G, int64_t ldG, double *d_g) {
    if (!h || !d_J || !d_G || m < 0 || p < 1) return GN_EINVAL;
    if (ldJ < p || ldG < p) return fail(h, GN_EINVAL, "leading dimension smaller than p%s");
    if (d_r && !d_g) return fail(h, GN_EINVAL, "d_g is required when d_r is given%s");
    if (d_r && p > h->cap) return fail(h, GN_EINVAL, "p exceeds the gradient workspace (P + 1)%s");
    if (h->precision == GN_SPLIT32) {
        if (!h->Jhi || m > (h->dim == 2 ? h->rows_ws : total_rows(h)) || ldJ > h->ldJ)
            return fail(h, GN_EINVAL, "split-precision gram needs m <= N + 1 and ldJ <= the workspace ld%s");
        GN_HIP(h, launch_split(h->stream, d_J, m, p, ldJ, h->Jhi, h->Jlo));
        GN_HIP(h, launch_split_gram(h->stream, h->Jhi, h->Jlo, m, p, ldJ, d_G, ldG));
    } else if (h->precision == GN_INT8_CRT) {
        if (!h->mg.R || m > h->mg.rows) return fail(h, GN_EINVAL, "int8 gram needs m <= the workspace rows%s");
        GN_HIP(h, launch_modgram(h->stream, d_J, m, p, ldJ, d_G, ldG, h->mg));
    } else {
        GemmDesc g{};
        g.M = p; g.N = p; g.K = m;
        g.A = d_J; g.lda = ldJ; g.la = 1;
        g.B = d_J; g.ldb = ldJ; g.lb = 0;
        g.C = d_G; g.ldc = ldG;
        g.alpha = 1.0; g.beta = 0.0; g.lower = 1;
        GN_HIP(h, launch_planned(h->stream, g, h->gplan));
    }
    if (d_r) GN_HIP(h, launch_gemv_t(h->stream, d_J, m, p, ldJ, d_r, d_g, h->gemv_work));
    return GN_OK;
}

namespace {

// Blocked Cholesky of A + mu I (order n) on the handle's stream, with the
// look-ahead trailing updates on the side stream.
hipError_t factor(gn_handle h, double *A, int64_t n, int64_t lda, double mu, int border) {
    return launch_cholesky(h->stream, h->side, h->ev_panel, h->ev_trail, A, n, lda, mu, border, h->linv, h->chol_tmp,
                           h->status);
}

}  // namespace

gn_status gn_solve(gn_handle h, double *d_G, int64_t p, int64_t ldG, double mu, const double *d_g,
                   double *d_delta, int64_t *h_info) {
    if (!h || !d_G || !d_g || !d_delta || p < 1) return GN_EINVAL;
    if (ldG < p) return fail(h, GN_EINVAL, "ldG < p%s");
    if (p > h->cap) return fail(h, GN_EINVAL, "p exceeds the solver workspace (P + 1)%s");
    if (!(mu >= 0.0)) return fail(h, GN_EINVAL, "mu must be >= 0%s");
    hipStream_t st = h->stream;
    h->r1_factored = false;  // linv is shared with the stochastic step's factor
    GN_HIP(h, launch_reset_status(st, h->status));
    GN_HIP(h, factor(h, d_G, p, ldG, mu, 0));
    GN_HIP(h, launch_copy_strided(st, d_g, p, 1, h->ybuf, 1, -1.0));
    GN_HIP(h, launch_solve_lower_sync(st, d_G, p, ldG, h->linv, h->ybuf, h->zbuf, h->status, h->solve_sync));
    GN_HIP(h, launch_solve_upper_sync(st, d_G, p, ldG, h->linv, h->zbuf, d_delta, h->status, h->solve_sync));
    GN_HIP(h, launch_check_finite(st, d_delta, p, h->status));
    DevStatus ds;
    GN_TRY(read_status(h, &ds));
    if (h_info) *h_info = ds.chol_info;
    if (ds.flag) return fail(h, GN_ENOTPD, "Cholesky pivot %s is not positive", std::to_string(ds.chol_info).c_str());
    if (ds.nonfinite) return fail(h, GN_ENONFINITE, "non-finite update%s");
    return GN_OK;
}

namespace {

// r, J (or its chunks) and the bordered Gram [[G, g], [g^T, r^T r]] at theta,
// with the residual statistics; phase marks 0-4.
gn_status form_system(gn_handle h, const double *d_theta) {
    hipStream_t st = h->stream;
    h->r1_factored = false;  // the Gram overwrites the stochastic step's factor
    const int64_t P = h->md.P, m_rows = total_rows(h);
    double *J = h->J;
    const int64_t ldJ = h->ldJ;
    mark(h, 0);
    GN_HIP(h, launch_reset_status(st, h->status));
    if (h->dim == 2) {
        GN_TRY(forward2d(h, d_theta));
        GN_TRY(residual2d_rows(h, h->r2, 1, true));
        GN_TRY(validation2d(h, d_theta));
        GN_HIP(h, launch_sumsq(st, h->r2, total_rows(h), 1, &h->status->half_sq_norm, h->red_work));
        mark(h, 1);
        mark(h, 2);
        mark(h, 3);
        GN_TRY(gram2d(h, d_theta));  // Jacobian rows and the Gram, chunk by chunk
    } else {
        GN_TRY(build_step_jacobian(h, d_theta, true));
        mark(h, 3);
        if (h->precision == GN_SPLIT32) {
            // G from FP32 hi/lo products; the border row g = J^T r and r^T r stay FP64
            double *Grow = h->G + P * h->ldG;
            GN_HIP(h, launch_split(st, J, m_rows, P, ldJ, h->Jhi, h->Jlo));
            GN_HIP(h, launch_split_gram(st, h->Jhi, h->Jlo, m_rows, P, ldJ, h->G, h->ldG));
            GN_HIP(h, launch_copy_strided(st, J + P, m_rows, ldJ, h->r_tmp, 1, 1.0));
            GN_HIP(h, launch_gemv_t(st, J, m_rows, P, ldJ, h->r_tmp, Grow, h->gemv_work));
            GN_HIP(h, launch_sumsq(st, h->r_tmp, m_rows, 1, Grow + P, h->red_work));
        } else if (h->precision == GN_INT8_CRT) {
            // G from int8 modular products over the P parameter columns; the
            // border row g = J^T r and r^T r in FP64
            double *Grow = h->G + P * h->ldG;
            GN_HIP(h, launch_modgram(st, J, m_rows, P, ldJ, h->G, h->ldG, h->mg));
            GN_HIP(h, launch_copy_strided(st, J + P, m_rows, ldJ, h->r_tmp, 1, 1.0));
            GN_HIP(h, launch_gemv_t(st, J, m_rows, P, ldJ, h->r_tmp, Grow, h->gemv_work));
            GN_HIP(h, launch_sumsq(st, h->r_tmp, m_rows, 1, Grow + P, h->red_work));
        } else {
            GN_HIP(h, launch_planned(st, gram_desc(h), h->gplan));
        }
        GN_HIP(h, launch_sumsq(st, J + P, m_rows, ldJ, &h->status->half_sq_norm, h->red_work));
    }
    mark(h, 4);
    return GN_OK;
}

// r (column P of the workspace J), J and the residual statistics at theta
// (1D problems; no Gram).
// coupling = false: the collocation rows leave out the Hilbert coupling
// diag(cs) Q B (1D CCF), for callers that apply it in their products.
gn_status form_jacobian(gn_handle h, const double *d_theta, bool coupling = true) {
    hipStream_t st = h->stream;
    GN_HIP(h, launch_reset_status(st, h->status));
    GN_TRY(build_step_jacobian(h, d_theta, false, coupling));
    GN_HIP(h, launch_sumsq(st, h->J + h->md.P, total_rows(h), h->ldJ, &h->status->half_sq_norm, h->red_work));
    return GN_OK;
}

// Cholesky of [[G + mu I, g], [g^T, r^T r]]: its last row is (L^{-1} g)^T and
// its corner the Schur complement r^T r - |L^{-1} g|^2; then delta =
// -L^{-T} L^{-1} g into h->delta.  Phase mark 5.
gn_status solve_system(gn_handle h, double mu) {
    hipStream_t st = h->stream;
    const int64_t P = h->md.P;
    GN_HIP(h, factor(h, h->G, P + 1, h->ldG, mu, 1));
    mark(h, 5);
    double *w = h->G + P * h->ldG;
    GN_HIP(h, launch_sumsq(st, w, P, 1, &h->status->grad_dot_delta, h->red_work));
    GN_HIP(h, launch_copy_strided(st, w + P, 1, 1, &h->status->model_sq_norm, 1, 1.0));
    GN_HIP(h, launch_copy_strided(st, w, P, 1, h->ybuf, 1, -1.0));
    GN_HIP(h, launch_solve_upper_sync(st, h->G, P, h->ldG, h->linv, h->ybuf, h->delta, h->status, h->solve_sync));
    return GN_OK;
}

// |r|^2 at theta into status->half_sq_trial (no Jacobian, no seeds).
gn_status trial_objective(gn_handle h, const double *theta) {
    hipStream_t st = h->stream;
    if (h->dim == 2) {
        GN_TRY(forward2d(h, theta));
        GN_TRY(residual2d_rows(h, h->r2, 1, false));
        GN_HIP(h, launch_sumsq(st, h->r2, total_rows(h), 1, &h->status->half_sq_trial, h->red_work));
    } else {
        GN_TRY(forward_all(h, theta));
        GN_TRY(residual_rows(h, h->r_tmp, 1, false));
        GN_HIP(h, launch_sumsq(st, h->r_tmp, total_rows(h), 1, &h->status->half_sq_trial, h->red_work));
    }
    return GN_OK;
}

}  // namespace

gn_status gn_step(gn_handle h, double *d_theta, double mu, gn_stats *h_stats) {
    if (!h || !d_theta) return GN_EINVAL;
    if (!points_ready(h)) return fail(h, GN_ESTATE, "gn_set_points must be called first%s");
    if (!(mu >= 0.0)) return fail(h, GN_EINVAL, "mu must be >= 0%s");
    hipStream_t st = h->stream;
    const int64_t P = h->md.P;
    GN_TRY(form_system(h, d_theta));
    GN_TRY(solve_system(h, mu));
    GN_HIP(h, launch_finalize_step(st, d_theta, h->delta, nullptr, P, 1, h->status));
    mark(h, 6);
    if (h->prof_count < h->prof_max) ++h->prof_count;
    if (!h_stats) return GN_OK;
    DevStatus ds;
    GN_TRY(read_status(h, &ds));
    fill_stats(ds, h_stats);
    const gn_status s = (gn_status)h_stats->status;
    if (s == GN_ENOTPD) return fail(h, s, "Cholesky pivot %s is not positive", std::to_string(ds.chol_info).c_str());
    if (s == GN_ENONFINITE) return fail(h, s, "non-finite residual or update%s");
    return GN_OK;
}

gn_status gn_step_lm(gn_handle h, double *d_theta, gn_lm *lm, gn_stats *h_stats) {
    if (!h || !d_theta || !lm) return GN_EINVAL;
    if (!points_ready(h)) return fail(h, GN_ESTATE, "gn_set_points must be called first%s");
    const bool ok = lm->mu_min > 0.0 && lm->mu_max >= lm->mu_min && lm->mu >= 0.0 && lm->mu <= lm->mu_max &&
                    lm->up > 1.0 && lm->down >= 1.0 && lm->rho_lo >= 0.0 && lm->rho_hi >= lm->rho_lo &&
                    lm->max_tries >= 1 && std::isfinite(lm->mu_max) && std::isfinite(lm->up) &&
                    std::isfinite(lm->down) && std::isfinite(lm->rho_hi);
    if (!ok) return fail(h, GN_EINVAL, "Levenberg-Marquardt constants out of range%s");
    hipStream_t st = h->stream;
    const int64_t P = h->md.P;
    lm->tries = 0;
    lm->rho = std::nan("");
    GN_TRY(form_system(h, d_theta));
    DevStatus ds0, ds;
    GN_TRY(read_status(h, &ds0));
    const double h0 = 0.5 * ds0.half_sq_norm;
    lm->half_sq_norm_new = h0;
    ds = ds0;
    bool accepted = false;
    double mu = lm->mu, h1 = h0;
    if (std::isfinite(h0)) {
        GN_HIP(h, launch_tri_save(st, h->G, P + 1, h->ldG, h->gdiag));
        while (lm->tries < lm->max_tries) {
            if (lm->tries++ > 0) GN_HIP(h, launch_tri_restore(st, h->G, P + 1, h->ldG, h->gdiag));
            GN_HIP(h, launch_reset_solve_status(st, h->status));
            GN_TRY(solve_system(h, mu));
            // trial point theta + delta (left equal to theta when the solve failed)
            GN_HIP(h, hipMemcpyAsync(h->theta_trial, d_theta, sizeof(double) * P, hipMemcpyDeviceToDevice, st));
            GN_HIP(h, launch_finalize_step(st, h->theta_trial, h->delta, nullptr, P, 1, h->status));
            GN_HIP(h, launch_sumsq(st, h->delta, P, 1, &h->status->delta_sq_norm, h->red_work));
            GN_TRY(trial_objective(h, h->theta_trial));
            GN_TRY(read_status(h, &ds));
            double rho = -INFINITY;
            h1 = 0.5 * ds.half_sq_trial;
            if (!ds.flag && !ds.nonfinite && ds.updated) {
                // h(theta) - |r + J delta|^2 / 2 = (|L^{-1} g|^2 + mu |delta|^2) / 2
                const double pred = 0.5 * (ds.grad_dot_delta + mu * ds.delta_sq_norm);
                if (pred > 0.0) rho = (h0 - h1) / pred;
            }
            lm->rho = rho;
            if (std::isfinite(h1) && rho > 0.0) {
                GN_HIP(h, hipMemcpyAsync(d_theta, h->theta_trial, sizeof(double) * P, hipMemcpyDeviceToDevice, st));
                if (rho > lm->rho_hi) mu = std::max(mu / lm->down, lm->mu_min);
                else if (rho < lm->rho_lo) mu = std::min(mu * lm->up, lm->mu_max);
                accepted = true;
                break;
            }
            if (mu >= lm->mu_max) break;
            mu = std::min(std::max(mu * lm->up, lm->mu_min), lm->mu_max);
        }
    }
    mark(h, 5);
    mark(h, 6);
    if (h->prof_count < h->prof_max) ++h->prof_count;
    lm->mu = mu;
    if (accepted) lm->half_sq_norm_new = h1;
    GN_HIP(h, hipStreamSynchronize(st));
    if (h_stats) {
        fill_stats(ds0, h_stats);
        h_stats->grad_dot_delta = -ds.grad_dot_delta;
        h_stats->model_sq_norm = ds.model_sq_norm;
        h_stats->chol_info = ds.chol_info;
        h_stats->updated = accepted ? 1 : 0;
        h_stats->status = accepted ? GN_OK : (std::isfinite(h0) ? GN_EREJECTED : GN_ENONFINITE);
    }
    if (!std::isfinite(h0)) return fail(h, GN_ENONFINITE, "non-finite residual%s");
    if (!accepted) return fail(h, GN_EREJECTED, "no trial decreased the objective (last mu %s)",
                               std::to_string(mu).c_str());
    return GN_OK;
}

gn_status gn_step_rank1(gn_handle h, double *d_theta, double *d_G_ema, int64_t ldG, double *d_prev,
                        const double *d_v, const gn_rank1_args *a, gn_rank1_stats *h_stats) {
    if (!h || !d_theta || !d_G_ema || !d_prev || !d_v || !a) return GN_EINVAL;
    if (!points_ready(h)) return fail(h, GN_ESTATE, "gn_set_points must be called first%s");
    const int64_t P = h->md.P, m_rows = total_rows(h);
    if (h->dim != 1) return fail(h, GN_EINVAL, "the stochastic step takes 1D problems%s");
    if (ldG < P) return fail(h, GN_EINVAL, "ldG < P%s");
    if (P > 65535) return fail(h, GN_EINVAL, "P above 65535%s");
    if (!(a->beta >= 0.0 && a->beta <= 1.0) || !(a->gamma > 0.0) || !std::isfinite(a->gamma))
        return fail(h, GN_EINVAL, "need 0 <= beta <= 1 and a finite gamma > 0%s");
    if (!a->refactor && !h->r1_factored)
        return fail(h, GN_ESTATE, "no factor of G_ema + gamma I is kept: refactor first%s");
    hipStream_t st = h->stream;
    double *J = h->J;
    const int64_t ldJ = h->ldJ;
    // The step uses J only in products, so for the 1D CCF equation the
    // Hilbert coupling of the collocation rows, diag(cs) Q B (the N x M x P
    // product that dominates forming J), is applied inside them instead:
    // J x = J_loc x + cs o Q (B x) and J^T y = J_loc^T y + B^T Q^T (cs o y)
    // (Q^T is kept as M rows of N, B as M rows of P).
    const bool implicit = h->equation == GN_EQ_CCF1D && h->m > 0 && h->cp_t != nullptr;
    const int64_t nc = h->n, mq = h->m;
    GN_TRY(form_jacobian(h, d_theta, !implicit));
    // g = J^T r, u = J^T v
    GN_HIP(h, launch_copy_strided(st, J + P, m_rows, ldJ, h->r_tmp, 1, 1.0));
    GN_HIP(h, launch_gemv_t2(st, J, m_rows, P, ldJ, h->r_tmp, d_v, h->r1_g, h->r1_u, h->gemv_work, 0));
    if (implicit) {
        double *t1 = h->cp_t, *t2 = h->cp_t + nc, *z1 = h->cp_z, *z2 = h->cp_z + mq;
        GN_HIP(h, launch_diag_scale2(st, nc, h->cscale, h->r_tmp, d_v, t1, t2, 0));
        GN_HIP(h, launch_gemv_n2(st, h->Q, mq, nc, h->ldQ, t1, t2, z1, z2));
        GN_HIP(h, launch_gemv_t2(st, h->Bm, mq, P, ldJ, z1, z2, h->r1_g, h->r1_u, h->gemv_work, 1));
    }
    GN_HIP(h, launch_ema_rank1(st, d_G_ema, P, ldG, a->beta, h->r1_u));
    if (a->refactor) {
        GN_HIP(h, launch_copy_lower(st, d_G_ema, ldG, h->G, h->ldG, P));
        GN_HIP(h, factor(h, h->G, P, h->ldG, a->gamma, 0));
    }
    // Delta = -(G_ema + gamma I)^{-1} g
    GN_HIP(h, launch_copy_strided(st, h->r1_g, P, 1, h->r1_b, 1, -1.0));
    GN_HIP(h, launch_solve_lower_sync(st, h->G, P, h->ldG, h->linv, h->r1_b, h->zbuf, h->status, h->solve_sync));
    GN_HIP(h, launch_solve_upper_sync(st, h->G, P, h->ldG, h->linv, h->zbuf, h->r1_D, h->status, h->solve_sync));
    // exact curvature along Delta and d_prev
    GN_HIP(h, launch_gemv_n2(st, J, m_rows, P, ldJ, h->r1_D, d_prev, h->r1_w1, h->r1_w2));
    if (implicit) {
        double *y1 = h->cp_z, *y2 = h->cp_z + mq, *s1 = h->cp_t, *s2 = h->cp_t + nc;
        GN_HIP(h, launch_gemv_n2(st, h->Bm, mq, P, ldJ, h->r1_D, d_prev, y1, y2));
        GN_HIP(h, launch_gemv_t2(st, h->Q, mq, nc, h->ldQ, y1, y2, s1, s2, h->cp_work, 0));
        GN_HIP(h, launch_diag_scale2(st, nc, h->cscale, s1, s2, h->r1_w1, h->r1_w2, 1));
    }
    DotPairs dp{};
    const double *xs[8] = {h->r1_w1, h->r1_w1, h->r1_w2, h->r1_D, h->r1_D, d_prev, h->r1_g, h->r1_g};
    const double *ys[8] = {h->r1_w1, h->r1_w2, h->r1_w2, h->r1_D, d_prev, d_prev, h->r1_D, d_prev};
    dp.count = 3;
    for (int k = 0; k < 3; ++k) { dp.x[k] = xs[k]; dp.y[k] = ys[k]; }
    GN_HIP(h, launch_dots(st, dp, m_rows, h->r1_dots, h->r1_work));
    dp.count = 5;
    for (int k = 0; k < 5; ++k) { dp.x[k] = xs[3 + k]; dp.y[k] = ys[3 + k]; }
    GN_HIP(h, launch_dots(st, dp, P, h->r1_dots + 3, h->r1_work));
    DevStatus ds;
    double dots[8];
    GN_HIP(h, hipMemcpyAsync(dots, h->r1_dots, sizeof dots, hipMemcpyDeviceToHost, st));
    GN_TRY(read_status(h, &ds));
    gn_rank1_stats o{};
    o.half_sq_norm = 0.5 * ds.half_sq_norm;
    o.max_abs_R = bits_to_double(ds.max_R);
    o.max_abs_R_val = bits_to_double(ds.max_R_val);
    o.chol_info = ds.chol_info;
    gn_status rc = GN_OK;
    if (a->refactor) h->r1_factored = !ds.flag;
    if (ds.flag) {
        rc = GN_ENOTPD;
    } else {
        // the 2 x 2 model in (alpha, mu): C = J^T J + gamma I
        const double g = a->gamma;
        const double a11 = dots[0] + g * dots[3], b1 = dots[6];
        const double a12 = dots[1] + g * dots[4], a22 = dots[2] + g * dots[5], b2 = dots[7];
        double alpha = -b1 / a11, mu = 0.0, model = 0.5 * alpha * alpha * a11 + alpha * b1;
        const double det = a11 * a22 - a12 * a12;
        if (a->momentum && dots[5] > 0.0 && det > 1e-12 * a11 * a22) {
            alpha = (-b1 * a22 + b2 * a12) / det;
            mu = (-b2 * a11 + b1 * a12) / det;
            model = 0.5 * (alpha * alpha * a11 + 2 * alpha * mu * a12 + mu * mu * a22) + alpha * b1 + mu * b2;
            o.used_momentum = 1;
        }
        o.alpha = alpha;
        o.mu = mu;
        o.model = model;
        if (!std::isfinite(alpha) || !std::isfinite(mu) || !std::isfinite(o.half_sq_norm)) {
            rc = GN_ENONFINITE;
        } else {
            GN_HIP(h, launch_rank1_update(st, d_theta, d_prev, h->r1_D, alpha, mu, P));
        }
    }
    o.status = rc;
    if (h_stats) *h_stats = o;
    if (rc == GN_ENOTPD)
        return fail(h, rc, "G_ema + gamma I: pivot %s is not positive", std::to_string(ds.chol_info).c_str());
    if (rc == GN_ENONFINITE) return fail(h, rc, "non-finite residual or coefficients%s");
    return GN_OK;
}

gn_status gn_fields(gn_handle h, const double *d_theta, int32_t which, double *d_R, double *d_V, double *d_Ty) {
    if (!h || !d_theta || !d_R || !d_V || !d_Ty || (which != 0 && which != 1)) return GN_EINVAL;
    if (!points_ready(h)) return fail(h, GN_ESTATE, "gn_set_points must be called first%s");
    if (h->dim != 1 || h->stage2) return fail(h, GN_EINVAL, "fields are exported by 1D first-stage handles%s");
    if (which == 1 && h->nv <= 0) return fail(h, GN_ESTATE, "no validation grid%s");
    hipStream_t st = h->stream;
    GN_HIP(h, launch_reset_status(st, h->status));
    GN_TRY(forward_all(h, d_theta));
    if (which == 1) {
        SweepBatch b{};
        b.x = h->val.q; b.n = h->nv; b.nn = h->nn_val;
        with_phi(h, b, h->phi_val, h->nv);
        GN_HIP(h, launch_mlp_forward(st, h->md, d_theta, h->thetaT, b));
    }
    ResidualArgs a{};
    a.equation = h->equation; a.lam = h->lam; a.m = h->m;
    a.nodes = h->nodes; a.nn_nodes = h->nn_nodes;
    a.n = which ? h->nv : h->n;
    a.pts = which ? h->val : h->pts;
    a.nn = which ? h->nn_val : h->nn_pts;
    a.inv_n = 1.0;
    a.R = d_R; a.V_out = d_V; a.Ty_out = d_Ty;
    a.max_out = &h->status->max_R;
    GN_HIP(h, launch_residual(st, a));
    GN_HIP(h, hipStreamSynchronize(st));
    return GN_OK;
}

gn_status gn_set_stage1(gn_handle h, double eps, const double *d_R1, const double *d_V1, const double *d_T1y,
                        const double *d_R1v, const double *d_V1v, const double *d_T1yv) {
    if (!h || !d_R1 || !d_V1 || !d_T1y) return GN_EINVAL;
    if (!points_ready(h)) return fail(h, GN_ESTATE, "gn_set_points must be called first%s");
    if (h->dim != 1 || h->nd1 + h->nd2 > 0) return fail(h, GN_EINVAL, "second stages take 1D d0 problems%s");
    if (!std::isfinite(eps)) return fail(h, GN_EINVAL, "eps must be finite%s");
    if (h->nv > 0 && (!d_R1v || !d_V1v || !d_T1yv)) return fail(h, GN_EINVAL, "validation-grid fields needed%s");
    auto &A = h->pt_allocs;
    const int64_t n = h->n, nv = h->nv;
    if (!h->s1R) {
        gn_status s = GN_OK;
        if (s == GN_OK) s = dev_alloc(h, A, &h->s1R, n);
        if (s == GN_OK) s = dev_alloc(h, A, &h->s1V, n);
        if (s == GN_OK) s = dev_alloc(h, A, &h->s1T, n);
        if (s == GN_OK && nv > 0) s = dev_alloc(h, A, &h->s1Rv, nv);
        if (s == GN_OK && nv > 0) s = dev_alloc(h, A, &h->s1Vv, nv);
        if (s == GN_OK && nv > 0) s = dev_alloc(h, A, &h->s1Tv, nv);
        if (s != GN_OK) {
            h->s1R = nullptr;
            return s;
        }
    }
    hipStream_t st = h->stream;
    const size_t bn = sizeof(double) * n, bv = sizeof(double) * nv;
    GN_HIP(h, hipMemcpyAsync(h->s1R, d_R1, bn, hipMemcpyDeviceToDevice, st));
    GN_HIP(h, hipMemcpyAsync(h->s1V, d_V1, bn, hipMemcpyDeviceToDevice, st));
    GN_HIP(h, hipMemcpyAsync(h->s1T, d_T1y, bn, hipMemcpyDeviceToDevice, st));
    if (nv > 0) {
        GN_HIP(h, hipMemcpyAsync(h->s1Rv, d_R1v, bv, hipMemcpyDeviceToDevice, st));
        GN_HIP(h, hipMemcpyAsync(h->s1Vv, d_V1v, bv, hipMemcpyDeviceToDevice, st));
        GN_HIP(h, hipMemcpyAsync(h->s1Tv, d_T1yv, bv, hipMemcpyDeviceToDevice, st));
    }
    GN_HIP(h, hipStreamSynchronize(st));
    h->s1eps = eps;
    h->stage2 = true;
    return GN_OK;
}

gn_status gn_eval_derivs(gn_handle h, const double *d_theta, double *h_max_d1, double *h_max_d2) {
    if (!h || !d_theta || !h_max_d1 || !h_max_d2) return GN_EINVAL;
    if (!points_ready(h)) return fail(h, GN_ESTATE, "gn_set_points must be called first%s");
    if (h->dim != 1 || h->nf > 0 || h->stage2)
        return fail(h, GN_EINVAL, "derivative maxima are defined for 1D first-stage problems%s");
    if (h->nv <= 0) return fail(h, GN_ESTATE, "no validation grid%s");
    hipStream_t st = h->stream;
    GN_HIP(h, launch_reset_status(st, h->status));
    GN_HIP(h, launch_transpose_weights(st, h->md, d_theta, h->thetaT));
    if (h->equation == GN_EQ_CCF1D) {
        Sweep3 nb{};
        nb.x = h->geo3n.q; nb.n = h->m; nb.nn = h->nn3n;
        GN_HIP(h, launch_jet3_forward(st, h->md, d_theta, h->thetaT, nb));
        GN_HIP(h, launch_node_fields(st, h->m, h->nn3n, h->geo3n, h->nfield));
    }
    Sweep3 v{};
    v.x = h->geo3v.q; v.n = h->nv; v.nn = h->nn3v;
    GN_HIP(h, launch_jet3_forward(st, h->md, d_theta, h->thetaT, v));
    DerivArgs a = deriv_args(h);
    a.geo = h->geo3v; a.nn = h->nn3v;
    a.scale1 = a.scale2 = 1.0;
    a.n1 = h->nv; a.n2 = 0; a.max_out = &h->status->max_d1_val;
    GN_HIP(h, launch_deriv_residual(st, a));
    a.n1 = 0; a.n2 = h->nv; a.max_out = &h->status->max_d2_val;
    GN_HIP(h, launch_deriv_residual(st, a));
    DevStatus ds;
    GN_TRY(read_status(h, &ds));
    *h_max_d1 = bits_to_double(ds.max_d1_val);
    *h_max_d2 = bits_to_double(ds.max_d2_val);
    return GN_OK;
}

gn_status gn_lambda_estimate(gn_handle h, const double *d_theta, double *h_lam, double *h_dU0) {
    if (!h || !d_theta || !h_lam) return GN_EINVAL;
    if (!points_ready(h)) return fail(h, GN_ESTATE, "gn_set_points must be called first%s");
    if (h->dim != 1 || h->equation != GN_EQ_CCF1D || h->stage2)
        return fail(h, GN_EINVAL, "lambda inference is defined for the 1D CCF problem%s");
    hipStream_t st = h->stream;
    GN_HIP(h, launch_transpose_weights(st, h->md, d_theta, h->thetaT));
    SweepBatch b{};
    b.x = h->nodes.q; b.n = h->m; b.nn = h->nn_nodes;
    with_phi(h, b, h->phi_nodes, h->m);
    GN_HIP(h, launch_mlp_forward(st, h->md, d_theta, h->thetaT, b));
    GN_HIP(h, launch_lambda_estimate(st, h->m, h->nodes, h->nn_nodes, h->r1_dots));
    double out[2];
    GN_HIP(h, hipMemcpyAsync(out, h->r1_dots, sizeof out, hipMemcpyDeviceToHost, st));
    GN_HIP(h, hipStreamSynchronize(st));
    *h_lam = out[0];
    if (h_dU0) *h_dU0 = out[1];
    return GN_OK;
}

gn_status gn_funnel_residual(gn_handle h, const double *d_theta, double y_max, double *h_r_hat, double *h_y_at) {
    if (!h || !d_theta || !h_r_hat || !std::isfinite(y_max)) return GN_EINVAL;
    if (!points_ready(h)) return fail(h, GN_ESTATE, "gn_set_points must be called first%s");
    if (h->dim != 1 || h->stage2) return fail(h, GN_EINVAL, "the funnel proxy is defined for 1D first stages%s");
    if (h->nv <= 0) return fail(h, GN_ESTATE, "no validation grid%s");
    if (!h->fn_R) {
        double *p = nullptr;
        GN_TRY(dev_alloc(h, h->pt_allocs, &p, h->nv));
        h->fn_R = p;
    }
    hipStream_t st = h->stream;
    GN_HIP(h, launch_reset_status(st, h->status));
    GN_TRY(forward_all(h, d_theta));
    SweepBatch b{};
    b.x = h->val.q; b.n = h->nv; b.nn = h->nn_val;
    with_phi(h, b, h->phi_val, h->nv);
    GN_HIP(h, launch_mlp_forward(st, h->md, d_theta, h->thetaT, b));
    ResidualArgs a{};
    a.equation = h->equation; a.lam = h->lam; a.m = h->m;
    a.nodes = h->nodes; a.nn_nodes = h->nn_nodes;
    a.n = h->nv; a.pts = h->val; a.nn = h->nn_val;
    a.inv_n = 1.0;
    a.R = h->fn_R;
    a.max_out = &h->status->max_R;
    GN_HIP(h, launch_residual(st, a));
    GN_HIP(h, launch_funnel_residual(st, h->nv, h->fn_R, h->val.y, y_max, h->r1_dots));
    double out[3];
    GN_HIP(h, hipMemcpyAsync(out, h->r1_dots, sizeof out, hipMemcpyDeviceToHost, st));
    GN_HIP(h, hipStreamSynchronize(st));
    if (out[2] < 1.0) return fail(h, GN_ESTATE, "no validation point with y <= y_max%s");
    *h_r_hat = out[0];
    if (h_y_at) *h_y_at = out[1];
    return GN_OK;
}

gn_status gn_eval(gn_handle h, const double *d_theta, gn_stats *h_stats) {
    if (!h || !d_theta || !h_stats) return GN_EINVAL;
    if (!points_ready(h)) return fail(h, GN_ESTATE, "gn_set_points must be called first%s");
    hipStream_t st = h->stream;
    GN_HIP(h, launch_reset_status(st, h->status));
    if (h->dim == 2) {
        GN_TRY(forward2d(h, d_theta));
        GN_TRY(residual2d_rows(h, h->r2, 1, false));
        GN_HIP(h, launch_sumsq(st, h->r2, total_rows(h), 1, &h->status->half_sq_norm, h->red_work));
        GN_TRY(validation2d(h, d_theta));
    } else {
        GN_TRY(forward_all(h, d_theta));
        GN_TRY(residual_rows(h, h->r_tmp, 1, false));
        GN_HIP(h, launch_sumsq(st, h->r_tmp, total_rows(h), 1, &h->status->half_sq_norm, h->red_work));
        GN_TRY(validation(h, d_theta));
    }
    DevStatus ds;
    GN_TRY(read_status(h, &ds));
    memset(h_stats, 0, sizeof *h_stats);
    h_stats->half_sq_norm = 0.5 * ds.half_sq_norm;
    h_stats->max_abs_R = bits_to_double(ds.max_R);
    h_stats->max_abs_R_val = bits_to_double(ds.max_R_val);
    return GN_OK;
}

gn_status gn_vjp(gn_handle h, const double *d_theta, const double *d_v, double *d_out) {
    if (!h || !d_theta || !d_v || !d_out) return GN_EINVAL;
    if (!points_ready(h)) return fail(h, GN_ESTATE, "gn_set_points must be called first%s");
    hipStream_t st = h->stream;
    const int64_t P = h->md.P;
    GN_HIP(h, launch_reset_status(st, h->status));
    if (h->dim == 2) {
        GN_TRY(forward2d(h, d_theta));
        GN_TRY(residual2d_rows(h, h->r2, 1, true));
        Sweep2DArgs b = sweep2d_args(h);
        b.nrows = total_rows(h);
        b.v = d_v;
        b.partial = h->partial;
        int64_t nb = 0;
        GN_HIP(h, launch_jets2d_vjp(st, h->md, d_theta, h->thetaT, b, &nb));
        GN_HIP(h, launch_reduce_partials(st, h->partial, nb, P, d_out, 0));
        return GN_OK;
    }
    GN_TRY(forward_all(h, d_theta));
    GN_TRY(residual_rows(h, h->r_tmp, 1, true));
    // collocation rows: seeds scaled by v_i
    GN_HIP(h, launch_mul(st, d_v, h->seed0, h->vseed0, h->n, 1.0));
    GN_HIP(h, launch_mul(st, d_v, h->seed1, h->vseed1, h->n, 1.0));
    int64_t c0 = 0, c1 = 0, c2 = 0;
    SweepBatch b{};
    b.x = h->pts.q; b.s0 = h->vseed0; b.s1 = h->vseed1; b.n = h->n;
    with_phi(h, b, h->phi_pts, h->n);
    GN_HIP(h, launch_mlp_vjp(st, h->md, d_theta, h->thetaT, b, h->partial, &c0));
    // normalisation row: seed v_last sqrt(c_norm)
    GN_HIP(h, launch_copy_strided(st, d_v + norm_row(h), 1, 1, h->seed_one, 1, sqrt(h->c_norm)));
    SweepBatch o{};
    o.x = h->one_x; o.s0 = h->seed_one; o.s1c = 0.0; o.n = 1;
    with_phi(h, o, h->phi_one, 1);
    GN_HIP(h, launch_mlp_vjp(st, h->md, d_theta, h->thetaT, o, h->partial + c0 * P, &c1));
    if (h->equation == GN_EQ_CCF1D) {
        // Hilbert coupling adjoint: node seeds E_j sum_i Q_ij v_i sc_i Theta_y,i
        GN_HIP(h, launch_hilbert_adjoint(st, h->n, h->m, h->Q, h->ldQ, d_v, h->cscale, h->nodes.E, h->useed,
                                         nullptr));
        SweepBatch nb{};
        nb.x = h->nodes.q; nb.s0 = h->useed; nb.s1c = 0.0; nb.n = h->m;
        with_phi(h, nb, h->phi_nodes, h->m);
        GN_HIP(h, launch_mlp_vjp(st, h->md, d_theta, h->thetaT, nb, h->partial + (c0 + c1) * P, &c2));
    }
    int64_t c3 = 0, c4 = 0;
    const int64_t nd = h->nd1 + h->nd2;
    if (nd > 0) {
        // derivative rows: seeds scaled by v, then the adjoint of their coupling
        const double *vd = d_v + h->n;
        GN_HIP(h, launch_scale_seeds(st, nd, vd, h->dseed, h->dvseed));
        Sweep3 d{};
        d.x = h->geo3.q; d.seed = h->dvseed; d.seed_ld = nd; d.n = nd;
        GN_HIP(h, launch_jet3_vjp(st, h->md, d_theta, h->thetaT, d, h->partial + (c0 + c1 + c2) * P, &c3));
        if (h->equation == GN_EQ_CCF1D) {
            const int64_t m = h->m;
            GN_HIP(h, launch_deriv_coupling(st, nd, m, h->geo3.y, h->nodes.y, h->nodes.wh, h->dcoef, h->dAT, h->ldA));
            GN_HIP(h, launch_deriv_coupling_adjoint(st, nd, m, h->dAT, h->ldA, vd, h->nodes.E, h->bseed, 2 * m,
                                                    h->nvseed, m));
            Sweep3 nb{};
            nb.x = h->geo3n.q; nb.seed = h->nvseed; nb.seed_ld = m; nb.n = m;
            GN_HIP(h, launch_jet3_vjp(st, h->md, d_theta, h->thetaT, nb, h->partial + (c0 + c1 + c2 + c3) * P, &c4));
        }
    }
    GN_HIP(h, launch_reduce_partials(st, h->partial, c0 + c1 + c2 + c3 + c4, P, d_out, 0));
    return GN_OK;
}

static void batch_free(gn_batch b) {
    for (void *q : {(void *)b->d_fjobs, (void *)b->d_rjobs, (void *)b->d_fwork, (void *)b->d_rwork,
                    (void *)b->d_resjobs, (void *)b->d_reswork})
        if (q) (void)hipFree(q);
    for (hipStream_t l : b->lanes) (void)hipStreamDestroy(l);
    for (hipEvent_t e : b->join) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->d_bc) (void)hipFree(b->d_bc);
    batched_plan_free(b->coupling);
    batched_plan_free(b->gram);
    batched_plan_free(b->gram_tail);
    batched_plan_free(b->coupling_tail);
    for (auto &p : b->chol) batched_plan_free(p);
    delete b;
}

gn_status gn_batch_create(gn_handle *hs, int32_t n, void *stream, gn_batch *out) {
    if (!hs || n < 1 || !out) return GN_EINVAL;
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        if (!hs[i] || hs[i]->dim != 1) return GN_EINVAL;
        if (hs[i]->n <= 0) return GN_ESTATE;
        // derivative rows, Fourier inputs and second stages are not batched
        if (hs[i]->nd1 + hs[i]->nd2 > 0 || hs[i]->nf > 0 || hs[i]->stage2) return GN_EINVAL;
        if (hs[i]->md.P != hs[0]->md.P || hs[i]->precision != GN_FP64) return GN_EINVAL;
    }
    gn_batch b = new (std::nothrow) gn_batch_context();
    if (!b) return GN_ENOMEM;
    b->hs.assign(hs, hs + n);
    b->stream = (hipStream_t)stream;
    b->P = hs[0]->md.P;
    const int64_t P = b->P;
    // A bordered order just above a multiple of 128 (1154 = 9 x 128 + 2 for the
    // small CCF network) would give the Gram a last row of 128-row tiles with
    // a few valid rows: those rows go to a second product of 32-row tiles,
    // masked to the lower triangle (C starts `head` rows below the diagonal).
    const int64_t order = P + 1, head = order / 128 * 128, tail = order - head;
    const bool split_tail = head >= 128 && tail >= 1 && tail <= 32;
    // likewise the coupling's last columns (P = 1153 = 9 x 128 + 1): 128 x 64 tiles
    const int64_t chead = P / 128 * 128, ctail = P - chead;
    const bool split_ctail = chead >= 128 && ctail >= 1 && ctail <= 32;
    for (int i = 0; i < n; ++i) {
        gn_handle h = hs[i];
        if (h->equation == GN_EQ_CCF1D) {
            GemmDesc c = coupling_desc(h);
            if (split_ctail) {
                GemmDesc t = c;
                t.N = ctail;
                t.B = h->Bm + chead;
                t.C = h->J + chead;
                b->coupling_tail.h_descs.push_back(t);
                c.N = chead;
            }
            b->coupling.h_descs.push_back(c);
        }
        GemmDesc g = gram_desc(h);
        if (split_tail) {
            GemmDesc t = g;
            t.M = tail;
            t.A = h->J + head;
            t.C = h->G + head * h->ldG;
            t.lower = 0;
            t.mask_lower = 1;
            t.mask_shift = head;
            b->gram_tail.h_descs.push_back(t);
            g.M = g.N = head;
        }
        b->gram.h_descs.push_back(g);
        BatchChol c{};
        c.A = h->G; c.lda = h->ldG; c.linv = h->linv; c.y = h->ybuf; c.x = h->delta; c.theta = nullptr;
        c.status = h->status;
        b->h_bc.push_back(c);
    }
    cholesky_batched_plans(b->h_bc.data(), n, P + 1, b->chol);
    hipError_t e = hipMalloc((void **)&b->d_bc, sizeof(BatchChol) * n);
    if (e == hipSuccess) e = hipMemcpy(b->d_bc, b->h_bc.data(), sizeof(BatchChol) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = batched_plan_upload(b->coupling);
    if (e == hipSuccess) e = batched_plan_upload(b->gram);
    if (e == hipSuccess) e = batched_plan_upload(b->gram_tail);
    if (e == hipSuccess) e = batched_plan_upload(b->coupling_tail);
    for (auto &p : b->chol)
        if (e == hipSuccess) e = batched_plan_upload(p);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    for (int l = 0; l < BATCH_LANES && e == hipSuccess; ++l) {
        hipStream_t s_ = nullptr;
        hipEvent_t j_ = nullptr;
        e = hipStreamCreateWithFlags(&s_, hipStreamNonBlocking);
        if (e == hipSuccess) b->lanes.push_back(s_);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&j_, hipEventDisableTiming);
        if (e == hipSuccess) b->join.push_back(j_);
    }
    b->jobs = mlp_jobs_supported(hs[0]->md);
    if (b->jobs) {
        for (int i = 0; i < n; ++i) {
            gn_handle h = hs[i];
            auto fjob = [&](const double *x, int64_t np, double *nn) {
                SweepJob j{};
                j.thetaT = h->thetaT;
                j.b.x = x; j.b.n = np; j.b.nn = nn;
                b->h_fjobs.push_back(j);
                b->fjob_inst.push_back(i);
            };
            if (h->equation == GN_EQ_CCF1D) fjob(h->nodes.q, h->m, h->nn_nodes);
            fjob(h->pts.q, h->n, h->nn_pts);
            fjob(h->one_x, 1, h->nn_one);
            if (h->nv > 0) fjob(h->val.q, h->nv, h->nn_val);
            auto rjob = [&](const SweepBatch &sb) {
                SweepJob j{};
                j.thetaT = h->thetaT;
                j.b = sb;
                b->h_rjobs.push_back(j);
                b->rjob_inst.push_back(i);
            };
            SweepBatch pb{};
            pb.x = h->pts.q; pb.s0 = h->seed0; pb.s1 = h->seed1; pb.n = h->n; pb.rows = h->J; pb.ld = h->ldJ;
            rjob(pb);
            SweepBatch ob{};
            ob.x = h->one_x; ob.s0c = sqrt(h->c_norm); ob.s1c = 0.0; ob.n = 1; ob.rows = h->J + norm_row(h) * h->ldJ;
            ob.ld = h->ldJ;
            rjob(ob);
            if (h->equation == GN_EQ_CCF1D) {
                SweepBatch nb{};
                nb.x = h->nodes.q; nb.s0 = h->nodes.E; nb.s1c = 0.0; nb.n = h->m; nb.rows = h->Bm; nb.ld = h->ldJ;
                rjob(nb);
            }
        }
        std::vector<int2> fw, rw;
        mlp_jobs_work(b->h_fjobs, fw);
        mlp_jobs_work(b->h_rjobs, rw);
        b->nfwork = (int64_t)fw.size();
        b->nrwork = (int64_t)rw.size();
        if (e == hipSuccess) e = hipMalloc((void **)&b->d_fjobs, sizeof(SweepJob) * b->h_fjobs.size());
        if (e == hipSuccess) e = hipMalloc((void **)&b->d_rjobs, sizeof(SweepJob) * b->h_rjobs.size());
        if (e == hipSuccess) e = hipMalloc((void **)&b->d_fwork, sizeof(int2) * fw.size());
        if (e == hipSuccess) e = hipMalloc((void **)&b->d_rwork, sizeof(int2) * rw.size());
        if (e == hipSuccess) e = hipMemcpy(b->d_fwork, fw.data(), sizeof(int2) * fw.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(b->d_rwork, rw.data(), sizeof(int2) * rw.size(), hipMemcpyHostToDevice);
        b->res_jobs = true;
        for (int i = 0; i < n; ++i) b->res_jobs = b->res_jobs && hs[i]->equation == GN_EQ_CCF1D;
        if (b->res_jobs) {
            std::vector<ResidualArgs> ra;
            for (int i = 0; i < n; ++i) {
                gn_handle h = hs[i];
                ra.push_back(residual_args_pts(h, h->J + P, h->ldJ, true));
                if (h->nv > 0) ra.push_back(residual_args_val(h));
            }
            std::vector<int2> resw;
            residual_jobs_work(ra.data(), (int)ra.size(), resw);
            b->nreswork = (int64_t)resw.size();
            if (e == hipSuccess) e = hipMalloc((void **)&b->d_resjobs, sizeof(ResidualArgs) * ra.size());
            if (e == hipSuccess) e = hipMalloc((void **)&b->d_reswork, sizeof(int2) * resw.size());
            if (e == hipSuccess)
                e = hipMemcpy(b->d_resjobs, ra.data(), sizeof(ResidualArgs) * ra.size(), hipMemcpyHostToDevice);
            if (e == hipSuccess)
                e = hipMemcpy(b->d_reswork, resw.data(), sizeof(int2) * resw.size(), hipMemcpyHostToDevice);
        }
    }
    if (e != hipSuccess) {
        batch_free(b);
        return e == hipErrorOutOfMemory ? GN_ENOMEM : GN_EDEVICE;
    }
    b->uploaded_thetas.assign(n, nullptr);
    b->ds.resize(n);
    for (int i = 0; i < n; ++i) b->gen.push_back(hs[i]->points_gen);
    *out = b;
    return GN_OK;
}

gn_status gn_batch_destroy(gn_batch b) {
    if (!b) return GN_EINVAL;
    (void)hipStreamSynchronize(b->stream);
    batch_free(b);
    return GN_OK;
}

gn_status gn_step_batched(gn_batch b, double *const *d_thetas, double mu, gn_stats *h_stats) {
    if (!b || !d_thetas || !(mu >= 0.0)) return GN_EINVAL;
    const int n = (int)b->hs.size();
    const int64_t P = b->P;
    hipStream_t st = b->stream;
    gn_handle h0 = b->hs[0];
    for (int i = 0; i < n; ++i) {
        if (!d_thetas[i]) return GN_EINVAL;
        if (b->hs[i]->points_gen != b->gen[i]) return GN_ESTATE;
    }
    for (int i = 0; i < n; ++i) b->hs[i]->r1_factored = false;
    // parameter pointers live in the device descriptors; re-upload when they change
    bool changed = false;
    for (int i = 0; i < n; ++i) changed |= (b->uploaded_thetas[i] != d_thetas[i]);
    if (changed) {
        GN_HIP(h0, hipStreamSynchronize(st));
        for (int i = 0; i < n; ++i) b->h_bc[i].theta = d_thetas[i];
        GN_HIP(h0, hipMemcpy(b->d_bc, b->h_bc.data(), sizeof(BatchChol) * n, hipMemcpyHostToDevice));
        if (b->jobs) {
            for (size_t k = 0; k < b->h_fjobs.size(); ++k) b->h_fjobs[k].theta = d_thetas[b->fjob_inst[k]];
            for (size_t k = 0; k < b->h_rjobs.size(); ++k) b->h_rjobs[k].theta = d_thetas[b->rjob_inst[k]];
            GN_HIP(h0, hipMemcpy(b->d_fjobs, b->h_fjobs.data(), sizeof(SweepJob) * b->h_fjobs.size(),
                                 hipMemcpyHostToDevice));
            GN_HIP(h0, hipMemcpy(b->d_rjobs, b->h_rjobs.data(), sizeof(SweepJob) * b->h_rjobs.size(),
                                 hipMemcpyHostToDevice));
        }
        b->uploaded_thetas.assign(d_thetas, d_thetas + n);
    }
    // phase events of the batch step go on the first handle's event list
    auto bmark = [&](int k) {
        if (h0->prof_count < h0->prof_max)
            (void)hipEventRecord(h0->events[(size_t)h0->prof_count * (GN_PHASE_COUNT + 1) + k], st);
    };
    bmark(GN_PHASE_FORWARD);
    // per instance: residual, validation, local Jacobian rows with r in column P;
    // instance i on the batch stream (i % (lanes + 1) == 0) or on lane i % (lanes + 1) - 1
    const int nl = (int)b->lanes.size();
    // runs body(h, i, stream) for every instance, spread over the lanes, and
    // joins every lane back into the batch stream, also after an error
    auto per_instance = [&](auto body) -> gn_status {
        GN_HIP(h0, hipEventRecord(b->fork, st));
        for (int l = 0; l < nl; ++l) GN_HIP(h0, hipStreamWaitEvent(b->lanes[l], b->fork, 0));
        gn_status err = GN_OK;
        for (int i = 0; i < n && err == GN_OK; ++i) {
            gn_handle h = b->hs[i];
            const int q = i % (nl + 1);
            hipStream_t s_ = q == 0 ? st : b->lanes[q - 1];
            hipStream_t own = h->stream;
            h->stream = s_;
            err = body(h, i, s_);
            h->stream = own;
        }
        for (int l = 0; l < nl; ++l) {
            GN_HIP(h0, hipEventRecord(b->join[l], b->lanes[l]));
            GN_HIP(h0, hipStreamWaitEvent(st, b->join[l], 0));
        }
        return err;
    };
    auto sumsq = [&](gn_handle h, int, hipStream_t s_) -> gn_status {
        return launch_sumsq(s_, h->J + P, total_rows(h), h->ldJ, &h->status->half_sq_norm, h->red_work) == hipSuccess
                   ? GN_OK
                   : GN_EDEVICE;
    };
    if (b->jobs) {
        // per instance: status, transposed weights; then every forward sweep in
        // one launch; per instance: residual rows (seeds, r in column P) and the
        // validation residual; then every Jacobian-row sweep in one launch
        GN_TRY(per_instance([&](gn_handle h, int i, hipStream_t s_) -> gn_status {
            if (launch_reset_status(s_, h->status) != hipSuccess) return GN_EDEVICE;
            return launch_transpose_weights(s_, h->md, d_thetas[i], h->thetaT) == hipSuccess ? GN_OK : GN_EDEVICE;
        }));
        GN_HIP(h0, launch_mlp_forward_jobs(st, h0->md, b->d_fjobs, b->d_fwork, b->nfwork));
        if (b->res_jobs) {
            // every residual in one launch; the data rows (one value each) on the batch stream
            GN_HIP(h0, launch_residual_jobs(st, b->d_resjobs, b->d_reswork, b->nreswork));
            for (int i = 0; i < n; ++i) {
                gn_handle h = b->hs[i];
                GN_HIP(h0, launch_norm_row(st, h->nn_one, sqrt(h->c_norm), h->c_target,
                                           h->J + norm_row(h) * h->ldJ + P));
            }
        } else {
            GN_TRY(per_instance([&](gn_handle h, int, hipStream_t) -> gn_status {
                GN_TRY(residual_rows(h, h->J + P, h->ldJ, true));
                return validation_residual(h);
            }));
        }
        GN_HIP(h0, launch_mlp_rows_jobs(st, h0->md, b->d_rjobs, b->d_rwork, b->nrwork));
        GN_TRY(per_instance(sumsq));
    } else {
        // per instance: residual, validation, local Jacobian rows with r in column P
        GN_TRY(per_instance([&](gn_handle h, int i, hipStream_t s_) -> gn_status {
            if (launch_reset_status(s_, h->status) != hipSuccess) return GN_EDEVICE;
            GN_TRY(build_step_jacobian(h, d_thetas[i], false, false));
            return sumsq(h, i, s_);
        }));
    }
    // batched Hilbert coupling, Gram, bordered Cholesky, back substitution and update
    bmark(GN_PHASE_JLOCAL);  // the local rows are timed with the forward phase
    // The tail products (the coupling's last column, the bordered Gram's last
    // rows: memory-bound, on their own tile shapes) run on a lane beside the
    // main products; their outputs are disjoint from the main ones and both
    // read inputs complete before the fork.
    auto beside = [&](const BatchedGemmPlan &main, const BatchedGemmPlan &tail) -> gn_status {
        if (tail.h_work.empty() || nl == 0) {
            GN_HIP(h0, launch_batched_plan(st, main));
            GN_HIP(h0, launch_batched_plan(st, tail));
            return GN_OK;
        }
        GN_HIP(h0, hipEventRecord(b->fork, st));
        GN_HIP(h0, hipStreamWaitEvent(b->lanes[0], b->fork, 0));
        // the join is recorded whatever the launches return, so st never runs ahead of the lane
        hipError_t e = launch_batched_plan(b->lanes[0], tail);
        const hipError_t e2 = launch_batched_plan(st, main);
        if (e == hipSuccess) e = e2;
        GN_HIP(h0, hipEventRecord(b->join[0], b->lanes[0]));
        GN_HIP(h0, hipStreamWaitEvent(st, b->join[0], 0));
        GN_HIP(h0, e);
        return GN_OK;
    };
    bmark(GN_PHASE_COUPLING);
    GN_TRY(beside(b->coupling, b->coupling_tail));
    bmark(GN_PHASE_GRAM);
    GN_TRY(beside(b->gram, b->gram_tail));
    bmark(GN_PHASE_CHOLESKY);
    GN_HIP(h0, launch_cholesky_batched(st, b->h_bc.data(), b->d_bc, b->chol, n, P + 1, mu, 1));
    bmark(GN_PHASE_SOLVE);
    GN_HIP(h0, launch_solve_upper_batched(st, b->d_bc, n, P));
    bmark(GN_PHASE_COUNT);
    if (h0->prof_count < h0->prof_max) ++h0->prof_count;
    if (!h_stats) return GN_OK;
    for (int i = 0; i < n; ++i)
        GN_HIP(h0, hipMemcpyAsync(&b->ds[i], b->hs[i]->status, sizeof(DevStatus), hipMemcpyDeviceToHost, st));
    GN_HIP(h0, hipStreamSynchronize(st));
    for (int i = 0; i < n; ++i) fill_stats(b->ds[i], &h_stats[i]);
    return GN_OK;
}

gn_status gn_probe_fp64_mfma(void *stream, double *h_tflops) {
    if (!h_tflops) return GN_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                  hipSuccess || cus <= 0)
        return GN_EDEVICE;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double flops = 0.0;
    bool ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    ok = ok && launch_mfma_probe(st, cus, 256, nullptr) == hipSuccess;  // warm-up
    ok = ok && hipEventRecord(e0, st) == hipSuccess && launch_mfma_probe(st, cus, 16384, &flops) == hipSuccess &&
         hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    float ms = 0.f;
    ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms > 0.f;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (!ok) return GN_EDEVICE;
    *h_tflops = flops / (ms * 1e-3) / 1e12;
    return GN_OK;
}

gn_status gn_profile_enable(gn_handle h, int32_t enable, int32_t max_steps) {
    if (!h) return GN_EINVAL;
    GN_HIP(h, hipStreamSynchronize(h->stream));
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    h->events.clear();
    h->prof_max = h->prof_count = 0;
    if (!enable) return GN_OK;
    if (max_steps < 1) return fail(h, GN_EINVAL, "max_steps must be >= 1%s");
    h->events.resize((size_t)max_steps * (GN_PHASE_COUNT + 1));
    for (auto &e : h->events) GN_HIP(h, hipEventCreate(&e));
    h->prof_max = max_steps;
    return GN_OK;
}

gn_status gn_profile_read(gn_handle h, double *h_ms, int32_t n_phases, int32_t *n_steps) {
    if (!h || !h_ms || n_phases < 0 || n_phases > GN_PHASE_COUNT) return GN_EINVAL;
    GN_HIP(h, hipStreamSynchronize(h->stream));
    for (int k = 0; k < n_phases; ++k) h_ms[k] = 0.0;
    for (int32_t s = 0; s < h->prof_count; ++s) {
        hipEvent_t *ev = &h->events[(size_t)s * (GN_PHASE_COUNT + 1)];
        for (int k = 0; k < n_phases; ++k) {
            float ms = 0.f;
            GN_HIP(h, hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
            h_ms[k] += ms;
        }
    }
    if (n_steps) *n_steps = h->prof_count;
    return GN_OK;
}

}  // extern "C"
