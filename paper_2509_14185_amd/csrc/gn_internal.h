// Internal declarations shared by the HIP kernels and the C-ABI layer of the
// gfx950 damped Gauss-Newton library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "gn.h"

namespace gn {

// Network shape passed by value to kernels.  theta layout per affine layer
// l: W^l row-major (w[l+1] x w[l]) then b^l; off[l] is the offset of W^l.
struct MlpDesc {
    int L;                       // affine layers
    int w[GN_MAX_LAYERS + 1];    // widths, w[0] = input dim, w[L] = outputs
    int off[GN_MAX_LAYERS];      // offset of W^l in theta
    int P;                       // number of parameters
};

// Geometry of one point set (structure of arrays, length n each).
struct Geo1D {
    double *y;    // self-similar coordinate y >= 0
    double *q;    // network input q = 1 - s
    double *E;    // envelope E(y)
    double *Ey;   // dE/dy
    double *qy;   // dq/dy
    double *wh;   // Hilbert node weight (quadrature nodes only), else null
};

// One batch of points swept through the network.
//   x: network inputs; s0/s1: seeds on NN and NN_x (null -> constants
//   s0c/s1c); rows: output (row i at rows + i*ld) in the row mode;
//   partial: per-workgroup gradient partials (P each) in the VJP mode.
struct SweepBatch {
    const double *x;
    const double *s0;
    const double *s1;
    double s0c, s1c;
    int64_t n;
    double *rows;
    int64_t ld;
    double *nn;    // forward outputs (2n: NN then NN_x), forward mode only
    const double *phi;  // Fourier feature input (rows 0..w0-1 phi, w0..2w0-1 phi_x, stride phi_ld), or null
    int64_t phi_ld;
};

// One sweep of a multi-sweep launch: its parameters, their transpose and the batch.
struct SweepJob {
    const double *theta;
    const double *thetaT;
    SweepBatch b;
};

// max |v| into *p as the bit pattern of a non-negative double (such patterns
// order as integers); NaN counts as +inf so that it is visible.
__device__ __forceinline__ void atomic_max_abs(unsigned long long *p, double v) {
    v = fabs(v);
    if (!(v == v)) v = __builtin_inf();
    atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

// Device-side status shared by the kernels of one step.
struct DevStatus {
    unsigned long long max_R;      // bit pattern of max |R| (collocation); non-negative doubles order as integers
    unsigned long long max_R_val;  // same, validation grid
    int64_t chol_info;             // 0 or 1-based first bad pivot
    int32_t flag;                  // nonzero: stop (factorisation failed)
    int32_t nonfinite;             // nonzero: non-finite update found
    int32_t updated;
    int32_t wait_fail;             // nonzero: a bounded device wait of the solve ran out
    double half_sq_norm;
    double grad_dot_delta;
    double model_sq_norm;
    double delta_sq_norm;          // |delta|^2 (damping retries)
    double half_sq_trial;          // |r|^2 at a trial theta + delta (damping retries)
    unsigned long long max_d1_val; // max |R'| and max |R''| on the validation grid (bit patterns)
    unsigned long long max_d2_val;
};

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `st` and return hipGetLastError().

// Geometry of points s (mapped coordinate); nodes additionally get the
// Hilbert weights from quadrature weights ws.
hipError_t launch_geometry(hipStream_t st, int equation, double lam, int64_t n, const double *s,
                           const double *ws, Geo1D g);
// Q[i][j] (n x m, ld) of the half-line Hilbert quadrature.
// Q^T of the half-line Hilbert quadrature: QT[j*ld + i] = Q_ij (m rows of n).
hipError_t launch_hilbert_matrix(hipStream_t st, int64_t n, int64_t m, const double *y,
                                 const double *t, const double *wh, double *QT, int64_t ld);

// Network sweeps.  thetaT holds the per-layer transposed weights written by
// launch_transpose_weights for the same theta (P doubles).
hipError_t launch_transpose_weights(hipStream_t st, const MlpDesc &d, const double *theta, double *thetaT);
size_t mlp_sweep_lds_bytes(const MlpDesc &d);
hipError_t launch_mlp_forward(hipStream_t st, const MlpDesc &d, const double *theta, const double *thetaT,
                              SweepBatch b);
hipError_t launch_mlp_rows(hipStream_t st, const MlpDesc &d, const double *theta, const double *thetaT,
                           SweepBatch b);
// Forward jets / Jacobian rows of many sweeps in one launch (the matrix-core
// kernels: scalar input and output, hidden widths up to 64, no Fourier
// features), one 16-point tile per workgroup from a work table of (job, tile)
// pairs built by mlp_jobs_work.
bool mlp_jobs_supported(const MlpDesc &d);
void mlp_jobs_work(const std::vector<SweepJob> &jobs, std::vector<int2> &work);
hipError_t launch_mlp_forward_jobs(hipStream_t st, const MlpDesc &d, const SweepJob *d_jobs, const int2 *d_work,
                                   int64_t nwork);
hipError_t launch_mlp_rows_jobs(hipStream_t st, const MlpDesc &d, const SweepJob *d_jobs, const int2 *d_work,
                                int64_t nwork);
// VJP: writes ceil(n / tile) partial gradients (P each) to `partial`;
// returns the number of partials via *n_partials.
hipError_t launch_mlp_vjp(hipStream_t st, const MlpDesc &d, const double *theta, const double *thetaT,
                          SweepBatch b, double *partial, int64_t *n_partials);
int64_t mlp_vjp_partials(const MlpDesc &d, int64_t n);

// Residual of the collocation points (train=1: writes r, seeds, Theta_y
// scale; train=0: R only and the validation max).
struct ResidualArgs {
    int equation;
    double lam;
    int64_t n, m;            // points, Hilbert nodes
    Geo1D pts;
    Geo1D nodes;
    const double *nn;        // NN then NN_x at the points (2n)
    const double *nn_nodes;  // NN at the nodes (first m entries of 2m)
    const double *rho, *f;   // may be null
    double inv_n;            // 1/N (row scale uses rho/N)
    double *R;               // raw residual (n), may be null
    double *r;               // scaled residual rows (n), may be null
    int64_t r_stride;        // stride of r (1, or ldJ when written into a J column)
    double *seed0, *seed1;   // Jacobian seeds on NN, NN_x (scaled), may be null
    double *cscale;          // sc_i * Theta_y,i (row scale of the Hilbert coupling), may be null
    unsigned long long *max_out;  // max |R| (bit pattern)
    // second stage (all null otherwise): R = R1 + eps D[Theta_1] Theta with the
    // first stage's R1, V1 = (1+lam) y + U_1 and Theta_1' at these points
    const double *R1, *V1, *T1y;
    double eps;
    double *V_out, *Ty_out;       // V and Theta' of the field, may be null
};
// Fourier features (rows: cos, sin, d cos/dq, d sin/dq; F each) of q.
hipError_t launch_fourier_features(hipStream_t st, int64_t n, const double *q, int F, const double *b, double *out,
                                   int64_t ld);
hipError_t launch_residual(hipStream_t st, const ResidualArgs &a);
// The CCF residuals of many point sets in one launch (one 64-point block per
// workgroup from a work table of (job, block) pairs built by residual_jobs_work).
void residual_jobs_work(const ResidualArgs *jobs, int n, std::vector<int2> &work);
hipError_t launch_residual_jobs(hipStream_t st, const ResidualArgs *d_jobs, const int2 *d_work, int64_t nwork);
// Normalisation row: r = sqrt(c) (NN(1) - target), written to r_out.
hipError_t launch_norm_row(hipStream_t st, const double *nn1, double sqrt_c, double target,
                           double *r_out);
// Node seeds for the coupling adjoint: out_j = E_j * (Q^T w)_j, w_i = v_i cscale_i
// (QT as from launch_hilbert_matrix; work is unused, kept for the interface).
int64_t hilbert_adjoint_work_size(int64_t m);
hipError_t launch_hilbert_adjoint(hipStream_t st, int64_t n, int64_t m, const double *QT, int64_t ld,
                                  const double *v, const double *cscale, const double *E_nodes,
                                  double *out, double *work);

// Generic FP64 MFMA GEMM: C = beta C + alpha diag(rowscale) op(A) op(B).
// la: 0 = A(m,k) at A[m*lda+k], 1 = A(m,k) at A[k*lda+m].
// lb: 0 = B(k,n) at B[k*ldb+n], 1 = B(k,n) at B[n*ldb+k].
// lower: only C entries with n <= m are written (tiles above skipped).
struct GemmDesc {
    int64_t M, N, K;
    const double *A; int64_t lda; int la;
    const double *B; int64_t ldb; int lb;
    double *C; int64_t ldc;
    double alpha, beta;
    const double *rowscale;
    int lower;                 // square lower-triangular tile set (M == N)
    int mask_lower;            // rectangular tile set, write only n <= m + mask_shift
    int64_t mask_shift;        // with mask_lower: C's first row sits mask_shift rows below the diagonal
    const int32_t *stop_flag;  // if non-null and *stop_flag != 0 the kernel does nothing
    // set by launch_planned: work entries with a piece
    // index write their partial product (one of split_pieces K ranges) to
    // split_ws instead of C
    double *split_ws;
    int split_pieces;
};
hipError_t launch_dgemm(hipStream_t st, const GemmDesc &g);
// Work plan of a product with both operands contiguous along m and n: the
// Gram [J | r]^T [J | r] (lower, plan_gram) and the Hilbert coupling (M x N,
// plan_rect), built once per shape, on the tile shape launch_dgemm would use
// (128 x 128 tiles on four-wave workgroups for large products, 64 x 64 on
// eight-wave ones for small ones; two workgroups per CU either way).  Tiles
// are grouped in 4 x 8 super-tiles as in launch_dgemm, the groups dealt to
// the 8 XCDs so that each gets the same number of tiles (entry b of the table
// runs on XCD b % 8); on each XCD the tiles of its last, partly filled round
// of resident workgroups are split into `pieces` K ranges (the count that
// makes the slowest XCD's last round shortest), their partial products
// summed in a fixed order by a second launch.  Table entries: (unit, tile
// row, tile column, piece), unit -1 for a whole tile, tile row -1 for
// padding; then one entry (first unit, tile row, tile column, 0) per split
// tile for the summing launch.  Returns false (no plan: launch_planned falls
// back to launch_dgemm) when the product does not take the four-wave
// configuration or the device's CUs do not split evenly over XCDs.
struct TilePlan {
    int64_t M = 0, N = 0;    // shape of the product the plan is for (M = 0: none)
    bool lower = false;      // lower-triangular tile set (M == N)
    int tile = 128;          // tile edge: 128 or 64
    int64_t nwork = 0;       // entries of the product launch
    int nsplit = 0;          // split tiles (entries of the summing launch)
    int pieces = 1;          // K ranges per split tile
    int4 *d_work = nullptr;  // nwork + nsplit entries (device)
    double *ws = nullptr;    // nsplit * pieces partial tile x tile tiles (device)
};
int plan_tile_size(int64_t M, int64_t N, bool lower);
bool plan_gram(int64_t M, int cus, std::vector<int4> &table, int64_t &nwork, int &nsplit, int &pieces, int &tile);
bool plan_rect(int64_t M, int64_t N, int cus, std::vector<int4> &table, int64_t &nwork, int &nsplit, int &pieces,
               int &tile);
int64_t gram_plan_ws_doubles(int nsplit, int pieces, int tile);
// The product g on plan p when p was built for g's shape and layout, else
// launch_dgemm(st, g).
hipError_t launch_planned(hipStream_t st, const GemmDesc &g, const TilePlan &p);
// FP64 matrix-instruction throughput probe: cus x 8 workgroups of four waves,
// each wave iters rounds of 8 independent v_mfma_f64_16x16x4f64 chains;
// *flops (if not NULL) receives the flop count.
hipError_t launch_mfma_probe(hipStream_t st, int cus, int iters, double *flops);
// n independent GEMMs in one launch.  plan_dgemm_batched builds, once per
// set of shapes, the work table: one int4 (problem, tile row, tile column, 0)
// per workgroup in dispatch order, entry b running on XCD b % 8, padding
// entries with problem -1.  Tiles are grouped by 4 x 8 super-tiles of one
// problem and the groups are spread over XCDs by longest-processing-time on
// their K extent.  Layouts, the lower flag and the tile configuration must
// agree across the batch (else it returns -1); otherwise the table length.
// h_descs is the host copy, d_descs and d_work the device copies.
int64_t plan_dgemm_batched(const GemmDesc *descs, int n, std::vector<int4> &table);
hipError_t launch_dgemm_batched(hipStream_t st, const GemmDesc *h_descs, const GemmDesc *d_descs, int n,
                                const int4 *d_work, int64_t nwork);

// One batched GEMM launch with its descriptors and work table (host copies
// filled by the caller, device copies by batched_plan_upload).
struct BatchedGemmPlan {
    std::vector<GemmDesc> h_descs;
    std::vector<int4> h_work;
    GemmDesc *d_descs = nullptr;
    int4 *d_work = nullptr;
};
// Plans the work table from h_descs and copies both to the device.
hipError_t batched_plan_upload(BatchedGemmPlan &p);
void batched_plan_free(BatchedGemmPlan &p);
hipError_t launch_batched_plan(hipStream_t st, const BatchedGemmPlan &p);

// g = J^T r (J m x p row-major) via deterministic two-pass reduction
// (accumulate: g += J^T r); work must hold gemv_t_work_size(m, p) doubles.
int64_t gemv_t_work_size(int64_t m, int64_t p);
hipError_t launch_gemv_t(hipStream_t st, const double *J, int64_t m, int64_t p, int64_t ldj,
                         const double *r, double *g, double *work, int accumulate = 0);

// Split precision: hi = fl32(J), lo = fl32(J - hi) for the first p columns
// (same leading dimension), and the lower triangle of
// Jhi^T Jhi + Jhi^T Jlo + Jlo^T Jhi (FP32 MFMA products, FP64 accumulation
// per 32-row chunk); accumulate adds it to C (streamed row chunks).
// Gram from int8 modular products (k_modgram.hip): workspace sizes in bytes
// for m rows and p columns, and the launch (GN_INT8_CRT).
struct ModgramWork {
    int8_t *R = nullptr;                 // residues, MODS x ppad x kpad
    int64_t r_bytes = 0;
    uint8_t *Y = nullptr;                // product residues, MODS x packed lower 256 x 256 tiles
    int64_t y_bytes = 0;
    unsigned long long *cmax = nullptr;  // column maxima (bit patterns), ppad
    int64_t cmax_len = 0;
    int64_t rows = 0;                    // largest m the workspaces hold
};
int64_t modgram_r_bytes(int64_t m, int64_t p);
int64_t modgram_y_bytes(int64_t p);
int64_t modgram_ppad(int64_t p);
int modgram_bits(int64_t m);
int modgram_moduli();
void modgram_list(int32_t *out);
hipError_t launch_modgram(hipStream_t st, const double *J, int64_t m, int64_t p, int64_t ldj, double *G, int64_t ldg,
                          const ModgramWork &w);
hipError_t launch_modgram_begin(hipStream_t st, int64_t p, const ModgramWork &w);
hipError_t launch_modgram_colmax(hipStream_t st, const double *J, int64_t m, int64_t p, int64_t ldj,
                                 const ModgramWork &w);
hipError_t launch_modgram_chunk(hipStream_t st, const double *J, int64_t m, int64_t p, int64_t ldj, int b,
                                const ModgramWork &w, int accumulate);
hipError_t launch_modgram_finish(hipStream_t st, int64_t p, int b, double *G, int64_t ldg, const ModgramWork &w);

hipError_t launch_split(hipStream_t st, const double *J, int64_t m, int64_t p, int64_t ldj, float *hi, float *lo);
hipError_t launch_split_gram(hipStream_t st, const float *hi, const float *lo, int64_t m, int64_t p, int64_t lda,
                             double *C, int64_t ldc, int accumulate = 0);

// Blocked Cholesky of the lower triangle of A (n x n) after adding mu to the
// first n - border diagonal entries.  border = 1: the last row is a border
// row whose final diagonal entry receives the Schur complement (no sqrt).
// linv receives the inverses of the 128x128 diagonal blocks; tmp holds
// chol_tmp_size() doubles of scratch.
int64_t chol_linv_size(int64_t n);
int64_t chol_tmp_size();
// The trailing update of each panel runs on `side` (a second stream of
// default priority) while the next diagonal block is factored on `st`
// (look-ahead); ev_panel / ev_trail order the two streams.  On return all
// work is ordered before later work on `st`.
hipError_t launch_cholesky(hipStream_t st, hipStream_t side, hipEvent_t ev_panel, hipEvent_t ev_trail, double *A,
                           int64_t n, int64_t lda, double mu, int border, double *linv, double *tmp,
                           DevStatus *status);
// Batched bordered Cholesky and back substitution over instances that share
// the order n (one instance = one problem of a batch).
struct BatchChol {
    double *A;          // bordered Gram, (n+1) x lda, factored in place
    int64_t lda;
    double *linv;       // diagonal-block inverses
    double *y, *x;      // right-hand side workspace, solution (delta)
    double *theta;      // parameters updated in place
    DevStatus *status;
};
// plans[2 * panel + pass]: pass 0 the panel solve L21 = A21 X^T, pass 1 the
// trailing update, over all instances (from cholesky_batched_plans, uploaded).
hipError_t launch_cholesky_batched(hipStream_t st, const BatchChol *h_bc, const BatchChol *d_bc,
                                   const std::vector<BatchedGemmPlan> &plans, int nb, int64_t n, double mu,
                                   int border);
// Host descriptors of those GEMMs (work tables and device copies not yet made).
void cholesky_batched_plans(const BatchChol *bc, int nb, int64_t n, std::vector<BatchedGemmPlan> &out);
// y = -(border row), |w|^2 and the Schur complement into status, L^T x = y,
// then theta += x when finite and the factorisation succeeded.
hipError_t launch_solve_upper_batched(hipStream_t st, const BatchChol *d_bc, int nb, int64_t n);

// L z = b (forward), then L^T x = z (back), using the factor and the
// diagonal-block inverses from launch_cholesky.  b is overwritten.
hipError_t launch_solve_lower(hipStream_t st, const double *L, int64_t n, int64_t ldl,
                              const double *linv, double *b, double *z, DevStatus *status);
hipError_t launch_solve_upper(hipStream_t st, const double *L, int64_t n, int64_t ldl,
                              const double *linv, double *y, double *x, DevStatus *status);
// L^T x = y in one launch (one workgroup per column block, each waiting for
// the blocks below it to be published); bitwise the result of
// launch_solve_upper.  sync holds solve_sync_size(n) words, zeroed once when
// allocated; y is not modified.  Calls that share sync must not overlap.
int64_t solve_sync_size(int64_t n);
// L z = b in one launch (one workgroup per row block, each waiting for the
// blocks above it); bitwise the result of launch_solve_lower; b is not
// modified.  Same sync words and rules as launch_solve_upper_sync.
hipError_t launch_solve_lower_sync(hipStream_t st, const double *L, int64_t n, int64_t ldl,
                                   const double *linv, const double *b, double *z, DevStatus *status,
                                   unsigned *sync);
hipError_t launch_solve_upper_sync(hipStream_t st, const double *L, int64_t n, int64_t ldl,
                                   const double *linv, const double *y, double *x, DevStatus *status,
                                   unsigned *sync);

// Small kernels.
hipError_t launch_sumsq(hipStream_t st, const double *x, int64_t n, int64_t stride, double *out,
                        double *work);
hipError_t launch_finalize_step(hipStream_t st, double *theta, const double *delta,
                                const double *grad, int64_t p, int apply, DevStatus *status);
hipError_t launch_check_finite(hipStream_t st, const double *x, int64_t n, DevStatus *status);
hipError_t launch_reduce_partials(hipStream_t st, const double *partial, int64_t count, int64_t p,
                                  double *out, int accumulate);
hipError_t launch_copy_strided(hipStream_t st, const double *src, int64_t n, int64_t src_stride,
                               double *dst, int64_t dst_stride, double scale);

}  // namespace gn

namespace gn {
hipError_t launch_reset_status(hipStream_t st, DevStatus *s);
// Text of the calling thread's last gn_solve_noalloc error (gn_noalloc.hip).
const char *noalloc_last_error();
hipError_t launch_reset_solve_status(hipStream_t st, DevStatus *s);
// Copy of the lower triangle of the n x n matrix A into its strictly upper
// triangle (transposed), the diagonal into diag (n); restore writes it back.
hipError_t launch_tri_save(hipStream_t st, double *A, int64_t n, int64_t lda, double *diag);
hipError_t launch_tri_restore(hipStream_t st, double *A, int64_t n, int64_t lda, const double *diag);
hipError_t launch_mul(hipStream_t st, const double *a, const double *b, double *out, int64_t n, double scale);

// ------------------------------------------------ 1D derivative (d1, d2) rows
// Geometry to third order: y, then q^(k) and E^(k) (k = 0..3, y-derivatives)
// at q[k * ld + i], E[k * ld + i].
struct Geo3 {
    double *y;
    double *q;
    double *E;
    int64_t ld;
};
hipError_t launch_geometry3(hipStream_t st, int equation, double lam, int64_t n, const double *s, Geo3 g);

// Third-order jet sweep of the 1D network in its input q: forward outputs
// nn[c * n + i] (NN^(c), q-derivatives), rows with seeds seed[c * seed_ld + i]
// on them, or per-workgroup gradient partials.
struct Sweep3 {
    const double *x;
    const double *seed;
    int64_t seed_ld;
    int64_t n;
    double *rows;
    int64_t ld;
    double *nn;
};
hipError_t launch_jet3_forward(hipStream_t st, const MlpDesc &d, const double *theta, const double *thetaT, Sweep3 b);
hipError_t launch_jet3_rows(hipStream_t st, const MlpDesc &d, const double *theta, const double *thetaT, Sweep3 b);
int64_t jet3_vjp_partials(int64_t n);
hipError_t launch_jet3_vjp(hipStream_t st, const MlpDesc &d, const double *theta, const double *thetaT, Sweep3 b,
                           double *partial, int64_t *n_partials);
// Theta, Theta', Theta'' at the nodes (out[k * m + j]) from their NN jets.
hipError_t launch_node_fields(hipStream_t st, int64_t m, const double *nn, Geo3 g, double *out);
// Seeds of B1_j = t_j dTheta'(t_j)/dtheta (columns 0..m-1) and B2_j = dTheta''(t_j)/dtheta (m..2m-1).
hipError_t launch_node_seeds(hipStream_t st, int64_t m, Geo3 g, const double *t, double *seed, int64_t ld);

struct DerivArgs {
    int equation;
    double lam;
    int64_t n1, n2, m;             // d1 points, d2 points, Hilbert nodes
    Geo3 geo;                      // geometry of the n1 + n2 points
    const double *nn;              // NN^(c) at the points, [c * (n1 + n2) + i]
    const double *nodes_y, *nodes_wh, *node_fields;
    double scale1, scale2;         // sqrt(c_d1 / n1), sqrt(c_d2 / n2)
    double *r;                     // scaled rows (stride r_stride), may be null
    int64_t r_stride;
    double *seed;                  // seeds on NN^(c) per row [c * nd + i], may be null
    double *coef;                  // coupling coefficients [k * nd + i], k: B, B1, B2, may be null
    unsigned long long *max_out;   // max |raw row| (bit pattern), may be null
};
hipError_t launch_deriv_residual(hipStream_t st, const DerivArgs &a);
// AT (3m x ld, node-major) of the derivative rows' coupling product.
hipError_t launch_deriv_coupling(hipStream_t st, int64_t nd, int64_t m, const double *y, const double *t,
                                 const double *wh, const double *coef, double *AT, int64_t ld);
hipError_t launch_deriv_coupling_adjoint(hipStream_t st, int64_t nd, int64_t m, const double *AT, int64_t ld,
                                         const double *v, const double *nodeE, const double *bseed, int64_t sld,
                                         double *out, int64_t old);
hipError_t launch_scale_seeds(hipStream_t st, int64_t n, const double *v, const double *seed, double *out);
// out[0] = -2 (1 + U'(0)), out[1] = U'(0) from NN, NN_q at the nodes (nn: 2m).
hipError_t launch_lambda_estimate(hipStream_t st, int64_t m, Geo1D nodes, const double *nn, double *out);
// Funnel proxy over the n points with y <= y_max: out[0] = the R of largest
// |R|, out[1] = its y, out[2] = how many points qualify.
hipError_t launch_funnel_residual(hipStream_t st, int64_t n, const double *R, const double *y, double y_max,
                                  double *out);

// ------------------------------------------- stochastic full-matrix GN step
// Lower triangle of G <- beta G + (1 - beta) u u^T (p <= 65535).
hipError_t launch_ema_rank1(hipStream_t st, double *G, int64_t p, int64_t ldg, double beta, const double *u);
// Lower triangle (with the diagonal) of the n x n src into dst (n <= 65535).
hipError_t launch_copy_lower(hipStream_t st, const double *src, int64_t lds, double *dst, int64_t ldd, int64_t n);
// y1 = J x1, y2 = J x2 (J row-major m x p, leading dimension ld).
hipError_t launch_gemv_n2(hipStream_t st, const double *J, int64_t m, int64_t p, int64_t ld, const double *x1,
                          const double *x2, double *y1, double *y2);
// out[k] = x[k] . y[k] (length n) for k < count <= DOT_MAX; work of dots_work_size() doubles.
constexpr int DOT_MAX = 8;
struct DotPairs {
    const double *x[DOT_MAX];
    const double *y[DOT_MAX];
    int count;
};
hipError_t launch_dots(hipStream_t st, const DotPairs &d, int64_t n, double *out, double *work);
int64_t dots_work_size();
// delta = alpha D + mu prev (over prev), theta += delta.
// g1 = J^T r1, g2 = J^T r2 (accumulate: g += ...) in one pass over J, each
// bitwise equal to launch_gemv_t's result; work holds gemv_t2_work_size(p).
int64_t gemv_t2_work_size(int64_t p);
hipError_t launch_gemv_t2(hipStream_t st, const double *J, int64_t m, int64_t p, int64_t ldj, const double *r1,
                          const double *r2, double *g1, double *g2, double *work, int accumulate);
// y_k = cs o x_k (accumulate = 0) or y_k += cs o x_k, k = 1, 2, over n entries.
hipError_t launch_diag_scale2(hipStream_t st, int64_t n, const double *cs, const double *x1, const double *x2,
                              double *y1, double *y2, int accumulate);
hipError_t launch_rank1_update(hipStream_t st, double *theta, double *prev, const double *D, double alpha, double mu,
                               int64_t p);

// ------------------------------------------------------------ 2D problems
// Point table (structure of arrays, stride ld): y1, y2 and the input jets
// of the network inputs q (xin[0..5]) and beta (xin[6..11]), component c of
// input u at xin[(6u + c) * ld + point].
struct Pts2D {
    double *y1, *y2, *xin;
    int64_t ld;
};

// Rows of a 2D problem and the point each one is evaluated at.  Table order:
// n collocation points, n1 d1 points, ne y2 = 0 points, the origin.
// Rows: n x n_eq equation rows (equations interleaved per point), 2 n1 d1
// rows (dR/dy1, dR/dy2 per point), ne boundary rows, the normalisation row.
struct RowMap2D {
    int64_t n, n1, ne;
    int n_eq;
    __host__ __device__ int64_t rows() const { return n * n_eq + 2 * n1 + ne + 1; }
    __host__ __device__ int64_t point_of(int64_t row, int &kind, int &comp) const {
        const int64_t e0 = n * n_eq, d0 = e0 + 2 * n1, b0 = d0 + ne;
        if (row < e0) {
            kind = 0;
            comp = (int)(row % n_eq);
            return row / n_eq;
        }
        if (row < d0) {
            kind = 1;
            comp = (int)((row - e0) & 1);
            return n + (row - e0) / 2;
        }
        if (row < b0) {
            kind = 2;
            comp = 0;
            return n + n1 + (row - d0);
        }
        kind = 3;
        comp = 0;
        return n + n1 + ne;
    }
};

struct Res2DArgs {
    int equation;
    double lam;
    RowMap2D map;
    int nout;
    Pts2D pts;
    const double *nn;        // output jets [(f*6 + c) * ldn + point]
    int64_t ldn;
    double *r;               // scaled rows (may be null)
    int64_t r_stride;
    double *seeds;           // [(f*6 + c) * lds + row], scaled (may be null)
    int64_t lds;
    unsigned long long *max_out;  // max |R| over equation rows (bit pattern)
    double c_norm, c_target;
    double scale_eq, scale_d1, scale_edge;  // row scales sqrt(1/(n n_eq)), sqrt(1/(2 n1)), sqrt(1/ne)
    int validation;          // only the equation rows, only max |R|
};

struct Sweep2DArgs {
    int64_t nrows;           // rows (or points, forward) handled by this launch
    int64_t row0;            // first row (forward: first point, 0)
    RowMap2D map;
    Pts2D pts;
    const double *seeds;     // rows / vjp
    int64_t lds;
    const double *v;         // vjp weights per row
    double *nn;              // forward output jets
    int64_t ldn;
    double *J;               // rows: row (row0 + i) at J + i * ldJ
    int64_t ldJ;
    double *partial;         // vjp: one P-vector per workgroup
};

hipError_t launch_geometry2d(hipStream_t st, int64_t n, const double *s, int edge, double lam, Pts2D p,
                             int64_t off);
hipError_t launch_residual2d(hipStream_t st, const Res2DArgs &a);
hipError_t launch_jets2d_forward(hipStream_t st, const MlpDesc &d, const double *theta, const double *thetaT,
                                 const Sweep2DArgs &b);
hipError_t launch_jets2d_rows(hipStream_t st, const MlpDesc &d, const double *theta, const double *thetaT,
                              const Sweep2DArgs &b);
hipError_t launch_jets2d_vjp(hipStream_t st, const MlpDesc &d, const double *theta, const double *thetaT,
                             const Sweep2DArgs &b, int64_t *nblocks);
int64_t jets2d_vjp_partials(const MlpDesc &d, int64_t nrows);

}  // namespace gn
