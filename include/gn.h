/*
 * gn.h -- C ABI of the MI355X (gfx950) damped Gauss-Newton library for
 * physics-informed networks fitted to self-similar blow-up profiles.
 *
 * Paper: "Discovery of Unstable Singularities" (arXiv 2509.14185), Methods.
 *   - "Self-similar Solutions" and "Solution Modeling and Equation
 *     Factorisation": profile equations in the self-similar variable y, the
 *     compactified coordinate q = (1+|y|^2)^{-1/(2(1+lambda))} fed to a tanh
 *     MLP, envelopes that fix symmetry and far-field behaviour.
 *   - "Training Loss": d0 residual rows weighted by rho/(N N_E) and a
 *     normalisation (data) row.
 *   - "Second-order Optimizer": theta <- theta - (G + gamma I)^{-1} grad h
 *     with the full Gauss-Newton matrix G = J^T J.
 *   - "Validation Metrics for Solutions": max |R| over a validation grid.
 *
 * Conventions
 *   - Pointers named d_* are DEVICE memory owned by the caller; h_* are host
 *     memory.  The library owns only the workspace it allocates in
 *     gn_create/gn_set_points; no other entry point allocates.
 *   - Every call is asynchronous on the handle's stream unless it says it
 *     synchronises.  No C++ exception crosses the ABI; errors are returned
 *     as gn_status and the text of the last error is kept per handle
 *     (gn_last_error).
 *   - theta layout: for each affine layer l = 1..L, W^l row-major
 *     (w_l x w_{l-1}) followed by b^l.  P = sum_l w_l (w_{l-1} + 1).
 *   - Row order of r and J: the N collocation rows in point order, then the
 *     normalisation row (m = N + 1 rows).
 *   - Matrices are row-major: element (i, j) of X with leading dimension ld
 *     is X[i*ld + j].  Only the lower triangle (j <= i) of a Gram matrix or
 *     Cholesky factor is read or written; the strict upper triangle is left
 *     untouched.
 *   - Device pointers must be 8-byte aligned; leading dimensions are in
 *     elements.
 */
#ifndef GN_H
#define GN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gn_context *gn_handle;

typedef enum {
    GN_OK = 0,
    GN_ENOTPD = 1,       /* Cholesky pivot not positive: G + mu I is not numerically PD */
    GN_EREJECTED = 2,    /* gn_step_lm: no trial decreased the objective; theta unchanged */
    GN_EINVAL = -1,      /* bad argument (null pointer, size, leading dimension, widths) */
    GN_ENOMEM = -2,      /* workspace allocation failed */
    GN_EDEVICE = -3,     /* HIP runtime error, or a bounded device wait that ran out */
    GN_ENONFINITE = -4,  /* NaN or Inf in r, g or the update */
    GN_ESTATE = -5       /* call out of order (e.g. no points set) */
} gn_status;

/* Profile equation.  CCF: R = -lam Theta + ((1+lam) y + H Theta) Theta_y with
 * the half-line Hilbert transform of the even field Theta (the Cordoba-
 * Cordoba-Fontelos model under the self-similar ansatz).  BURGERS1D: the
 * local analogue with H Theta replaced by Theta (odd field).
 * 2D stand-ins (paper, Methods, "Solution Modeling and Equation
 * Factorisation": network inputs q = (1+|y|^2)^{-1/(2(1+lam))},
 * beta = y2/sqrt(1+|y|^2), field = symmetry prefactor x NN x decay; the
 * actual IPM and Boussinesq residuals are in unpublished supplementary
 * material).  Points y in the quadrant, y_k = s_k / (1 - s_k):
 *   IPM2D (one output): Phi = (y1/rho) NN q, rho = sqrt(1+|y|^2),
 *     R = Phi + ((1+lam) y + (Phi, 0)) . grad Phi; d1 rows dR/dy1, dR/dy2;
 *     boundary rows dPhi/dy2 = 0 on y2 = 0.
 *   BOUSS2D (three outputs): Omega = (y1/rho) NN_0 q, Theta = NN_1 q,
 *     Psi = (y1/rho) NN_2 q rho^2, U = (-Psi_2, Psi_1),
 *     R_Omega = Omega + ((1+lam) y + U) . grad Omega - Theta_1,
 *     R_Theta = (1-lam) Theta + ((1+lam) y + U) . grad Theta,
 *     R_Psi = Psi_11 + Psi_22 - Omega; boundary rows Psi = 0 on y2 = 0. */
typedef enum { GN_EQ_CCF1D = 0, GN_EQ_BURGERS1D = 1, GN_EQ_IPM2D = 3, GN_EQ_BOUSS2D = 4 } gn_equation;

/* Arithmetic of the Gram bulk.  GN_FP64: FP64 throughout.  GN_SPLIT32: the
 * FP64 Jacobian is split into FP32 parts hi = fl32(J), lo = fl32(J - hi) and
 * G = J^T J is formed as hi^T hi + hi^T lo + lo^T hi with FP32 matrix
 * products, summed in FP64 every 32 rows (about 1e-7 relative error in G);
 * the residual, g = J^T r, the Cholesky and the update stay FP64, so the
 * step is an inexact Newton step with the same fixed point.
 * GN_INT8_CRT (at most 130944 rows per row chunk; a 2D problem streamed in
 * several chunks forms J twice, once for the column maxima): G = J^T J from int8 matrix
 * products by exact modular arithmetic.  Each column of J is scaled by a
 * power of two and rounded to a b-bit integer (b = 54 for 8193 rows), the
 * integer Gram is formed exactly from its residues modulo 16 coprime moduli
 * (int8 products, int32 sums) and rebuilt by the Chinese remainder theorem.
 * Every entry of J keeps the bits above 2^-b times its column's maximum, the
 * integer products and sums are exact, and G is rounded once to FP64 (within
 * 2 ulp of the exact sum of the rounded integers).  A non-finite column gives
 * NaN in its row and column of G.  In gn_step, gn_step_lm and the 2D steps the
 * modular Gram covers the P parameter columns; g = J^T r and r^T r are FP64
 * sums, as for GN_SPLIT32. */
typedef enum { GN_FP64 = 0, GN_SPLIT32 = 1, GN_INT8_CRT = 2 } gn_precision;

#define GN_INT8_CRT_MAX_ROWS 130944  /* rows of J per product of the int8 Gram (one
                                        row chunk): 2^14-bounded products summed in
                                        int32 stay exact; chunks add modulo m_t */
#define GN_INT8_CRT_MAX_TOTAL_ROWS 1099511627776LL  /* 2^40 rows in all (b >= 41) */

/* Host-only parameters of the GN_INT8_CRT Gram for m rows of J in all (the
 * sum over the row chunks of a streamed 2D problem; no GPU call):
 * *bits = b, the bits kept per column (m 2^(2b) < M / 4), *n_moduli = T and
 * moduli[0 .. T-1] (caller-owned, room for 32) the pairwise coprime moduli,
 * M their product.  GN_EINVAL for m < 1, m > GN_INT8_CRT_MAX_TOTAL_ROWS or a
 * NULL pointer. */
gn_status gn_int8_crt_params(int64_t m, int32_t *bits, int32_t *n_moduli, int32_t *moduli);

#define GN_MAX_LAYERS 8   /* affine layers */
#define GN_MAX_WIDTH 64   /* hidden width limit of the 1D kernels */
#define GN_MAX_WIDTH_2D 256  /* hidden width limit of the 2D kernels */

typedef struct {
    int32_t equation;        /* gn_equation */
    int32_t precision;       /* gn_precision */
    int32_t n_layers;        /* L, number of affine layers (1..GN_MAX_LAYERS) */
    const int32_t *widths;   /* host, L+1 entries: [1, w_1, ..., 1] (1D);
                                [2, w_1, ..., n_out] (2D, n_out = 1 IPM2D, 3 BOUSS2D) */
    double lam;              /* self-similar scaling lambda (> 0) */
    double c_norm;           /* weight of the normalisation row (>= 0) */
    double c_target;         /* target value of NN (output 0) at q = 1, beta = 0 (the origin) */
    int64_t row_chunk;       /* 2D: rows of J formed at a time in gn_step (0: all); the
                                Gram is accumulated over the chunks (streamed J) */
    int32_t n_fourier;       /* 1D: F > 0 feeds the network Fourier features [cos(b_k q),
                                sin(b_k q)] of its input q (widths[0] = 2F <= GN_MAX_WIDTH),
                                the second-stage network of the paper (Methods, "Multi-stage
                                Training"); 0: the plain input q */
    const double *fourier_b; /* host, F frequencies b_k (copied at gn_create) */
} gn_problem;

typedef struct {
    double half_sq_norm;     /* |r|^2 / 2 at the input theta */
    double max_abs_R;        /* max |R_i| over collocation points (raw, unscaled) */
    double max_abs_R_val;    /* max |R| over the validation grid (0 if none set) */
    double grad_dot_delta;   /* g^T delta (negative for a descent step) */
    double model_sq_norm;    /* |r + J delta|^2 + mu |delta|^2 (predicted) */
    int64_t chol_info;       /* 0, or 1-based index of the first bad pivot */
    int32_t status;          /* gn_status of the step */
    int32_t updated;         /* 1 if theta was updated */
} gn_stats;

/* Text for a status code (static storage). */
const char *gn_status_string(int32_t status);
/* Text of the last error on this handle (valid until the next call); with
 * h = NULL, of the calling thread's last gn_solve_noalloc call. */
const char *gn_last_error(gn_handle h);

/* Create a handle for one problem on the current HIP device.  Copies *prob
 * (including widths).  With GN_FP64 and a Gram of order P + 1 of at least
 * 64 lower tiles (128 x 128 tiles from 512 of them, P + 1 above about 4000;
 * else 64 x 64), the handle also keeps the Gram's work plan: a tile table
 * and at most one partial tile per resident workgroup (64 MB on 256 CUs).  Errors: GN_EINVAL for bad widths
 * (first/last != 1, hidden width > GN_MAX_WIDTH, L out of range), lam <= 0,
 * c_norm < 0; GN_ENOMEM. */
gn_status gn_create(const gn_problem *prob, gn_handle *out);
gn_status gn_destroy(gn_handle h);

/* Bind a HIP stream (hipStream_t passed as void*; NULL = default stream). */
gn_status gn_set_stream(gn_handle h, void *stream);

/*
 * Set the point sets (paper: collocation batch Y_0 of pairs (y, rho); points
 * are kept fixed for many steps, so geometry is computed once here).
 *   d_s   [n]      collocation points in the mapped coordinate s = 1 - q,
 *                  0 <= s < 1 (y = sqrt(q^{-2(1+lam)} - 1)).
 *   d_rho [n]      loss weights rho_i (NULL: all 1).
 *   d_f   [n]      source term subtracted from R_i (NULL: zero).
 *   d_sq, d_wq [m_quad]  nodes 0 < s_j < 1 and weights of a quadrature for
 *                  integrals over s in (0,1); used by the Hilbert term of
 *                  GN_EQ_CCF1D (ignored, may be NULL with m_quad = 0, for
 *                  GN_EQ_BURGERS1D).
 *   d_sval [n_val] validation grid in s (NULL with n_val = 0: none).
 * The library copies what it needs; caller buffers may be freed afterwards.
 * Allocates the per-step workspace (Jacobian, Gram, factor; for GN_EQ_CCF1D
 * with at least 64 tiles in the n x P Hilbert coupling product (128 x 128
 * tiles from 512 of them, else 64 x 64), also that product's work plan: a
 * tile table and at most 64 MB of partial tiles on 256 CUs).  Synchronises.
 * Errors: GN_EINVAL (n < 1, m_quad < 1 for CCF, null pointers), GN_ENOMEM.
 */
gn_status gn_set_points(gn_handle h, int64_t n, const double *d_s, const double *d_rho,
                        const double *d_f, int64_t m_quad, const double *d_sq,
                        const double *d_wq, int64_t n_val, const double *d_sval);

/* gn_set_points plus derivative (d1, d2) rows for 1D problems.  Paper:
 * Methods, "Training Loss": losses on the first and second y-derivatives of
 * the residual, each on its own point batch, weighted 1/(N_d1 N_E d) and
 * 1/(N_d2 N_E d^2) (here d = N_E = 1) times c_d1, c_d2.  d_s1 (n1) and d_s2
 * (n2): mapped coordinates s in [0, 1) of the d1 and d2 points (device).
 * Rows, in order: the n d0 rows, n1 rows sqrt(c_d1/n1) R'(y), n2 rows
 * sqrt(c_d2/n2) R''(y), the normalisation row; gn_num_rows = n + n1 + n2 + 1.
 * R' = (1 + U') Theta' + V Theta'', R'' = U'' Theta' + (2 + lam + 2 U') Theta''
 * + V Theta''' with V = (1+lam) y + U; for CCF U' = H[Theta'] by the odd
 * half-line form (1/pi) int (t f(t) - y f(y)) 2/(y^2 - t^2) dt and
 * U'' = H[Theta''] by the even form, on the same nodes; U = Theta for the
 * local variant.  The validation max-norm and max_abs_R stay on R.
 * Errors: as gn_set_points, and GN_EINVAL for n1 or n2 < 0, missing point
 * arrays, negative weights, or more than 65535 nodes with derivative rows.
 * With GN_EQ_CCF1D the derivative rows' coupling product ((n1 + n2) x P)
 * takes a work plan of its own, on the same terms as the n x P one.
 * Handles with derivative rows cannot join a batch. */
gn_status gn_set_points_ex(gn_handle h, int64_t n, const double *d_s, const double *d_rho, const double *d_f,
                           int64_t m_quad, const double *d_sq, const double *d_wq, int64_t n_val,
                           const double *d_sval, int64_t n1, const double *d_s1, int64_t n2, const double *d_s2,
                           double c_d1, double c_d2);

/*
 * Point sets of a 2D problem (GN_EQ_IPM2D, GN_EQ_BOUSS2D), s-coordinates in
 * [0,1) mapped per axis to y = s / (1 - s):
 *   d_s    [n x 2]   collocation points (equation rows), n >= 1;
 *   d_s1   [n1 x 2]  points of the d1 rows (IPM2D only; NULL with n1 = 0);
 *   d_se   [ne]      y1-coordinates (as s) of the y2 = 0 boundary rows;
 *   d_sval [n_val x 2] validation grid (NULL with n_val = 0).
 * Row order: n x n_eq equation rows (equations interleaved per point),
 * 2 n1 d1 rows, ne boundary rows, the normalisation row; scales
 * sqrt(1/(n n_eq)), sqrt(1/(2 n1)), sqrt(1/ne), sqrt(c_norm).
 * Allocates the workspace (Jacobian of row_chunk rows, Gram, factor).
 * Synchronises.  Errors: GN_EINVAL (1D handle, n < 1, n1 > 0 for BOUSS2D,
 * null pointers), GN_ENOMEM.
 */
gn_status gn_set_points_2d(gn_handle h, int64_t n, const double *d_s, int64_t n1, const double *d_s1,
                           int64_t ne, const double *d_se, int64_t n_val, const double *d_sval);

int64_t gn_num_params(gn_handle h);  /* P */
int64_t gn_num_rows(gn_handle h);    /* m (1D: N + 1), or -1 before the points are set */

/* Residual rows r (length m): r_i = sqrt(rho_i/N) (R_i - f_i), i < N;
 * r_N = sqrt(c_norm) (NN(q=1) - c_target).  Paper: "Training Loss". */
gn_status gn_residual(gn_handle h, const double *d_theta, double *d_r);

/* Jacobian J = dr/dtheta, m x P, row-major, ldJ >= P.  If d_r is not NULL
 * the residual rows are written too.  Paper: "Second-order Optimizer"
 * (Jacobian of the residual functions). */
gn_status gn_jacobian(gn_handle h, const double *d_theta, double *d_J, int64_t ldJ, double *d_r);

/* Lower triangle of G = J^T J (p x p, ldG >= p) and g = J^T r (p), for any
 * m x p row-major J (ldJ >= p).  d_r may be NULL (then g is not written).
 * With GN_FP64 and p = P + 1 the product runs on the handle's work plan
 * (gn_create); some tiles are then summed from K ranges in a fixed order, so
 * the result is deterministic but may differ in the last bits from another
 * p's tiling of the same entries.
 * With GN_INT8_CRT, m may not exceed the handle's row count (N + 1 + the
 * derivative rows) and p may not exceed P + 1 (GN_EINVAL otherwise). */
gn_status gn_gram(gn_handle h, const double *d_J, int64_t m, int64_t p, int64_t ldJ,
                  const double *d_r, double *d_G, int64_t ldG, double *d_g);

/* Damped solve (G + mu I) delta = -g.  In: lower triangle of G (p x p,
 * ldG >= p); out: its lower Cholesky factor L in place, delta (p).
 * Synchronises to fill *h_info (0, or the 1-based first non-positive pivot).
 * Returns GN_ENOTPD (delta not written) or GN_ENONFINITE; GN_EDEVICE also
 * when a bounded device wait of the substitutions runs out (each triangular
 * solve is one launch whose workgroups wait for the blocks they depend on;
 * this does not happen in normal operation). */
gn_status gn_solve(gn_handle h, double *d_G, int64_t p, int64_t ldG, double mu,
                   const double *d_g, double *d_delta, int64_t *h_info);

/* The damped solve of gn_solve for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): it takes no handle and allocates nothing.  Arguments,
 * results and errors as gn_solve, with the work enqueued on `stream`
 * (hipStream_t as void*, NULL = default stream), for orders
 * 1 <= p <= GN_SOLVE_NOALLOC_MAX_ORDER; a larger p returns GN_EINVAL before
 * any launch.  Its scratch (a status word, the factor's 128 x 128
 * diagonal-block inverses and the two substitution vectors, 17.1 MB) is a
 * static device array that the library holds on every GPU it runs on until
 * the process ends.  All calls on one GPU share that GPU's copy and it keeps
 * the last call's contents (the status word is cleared at the start of each
 * call), so calls that overlap on one GPU, from other threads or streams,
 * race.  The factorisation runs on `stream` alone (no look-ahead stream).
 * Synchronises once to fill *h_info.  gn_last_error(NULL) gives the text of
 * the calling thread's last error from this call. */
#define GN_SOLVE_NOALLOC_MAX_ORDER 16384
gn_status gn_solve_noalloc(void *stream, double *d_G, int64_t p, int64_t ldG, double mu, const double *d_g,
                           double *d_delta, int64_t *h_info);

/* One damped GN step in place: theta <- theta - (J^T J + mu I)^{-1} J^T r.
 * theta is left unchanged when the factorisation fails (GN_ENOTPD) or the
 * update is not finite (GN_ENONFINITE).  Synchronises once to fill *h_stats
 * (may be NULL: then it does not synchronise and returns GN_OK after
 * enqueueing; failures still leave theta unchanged). */
gn_status gn_step(gn_handle h, double *d_theta, double mu, gn_stats *h_stats);

/* Levenberg-Marquardt damping for gn_step_lm.  Paper: Methods, "Second-order
 * Optimizer": the damping sets how far the local quadratic model is trusted
 * and is adapted during training, by the classical Levenberg-Marquardt
 * method for some problems.  The rule, in gain-ratio form: with delta(mu) =
 * -(G + mu I)^{-1} g and h = |r|^2 / 2,
 *   rho = (h(theta) - h(theta + delta)) / (h(theta) - |r + J delta|^2 / 2)
 * (actual over predicted decrease of the Gauss-Newton model).  A trial is
 * accepted iff h(theta + delta) is finite and rho > 0; then mu <- max(mu /
 * down, mu_min) if rho > rho_hi, mu <- min(mu * up, mu_max) if rho < rho_lo.
 * A rejected trial (or a failed factorisation) ends the step if mu == mu_max,
 * else mu <- min(max(mu * up, mu_min), mu_max) and the damped system is
 * solved again with the same G and g.  rho_lo = rho_hi = 0, up = down is
 * Marquardt's rule. */
typedef struct {
    double mu;               /* in: first damping tried (0 <= mu <= mu_max); out: damping for the next step */
    double mu_min;           /* > 0: floor of an increased damping */
    double mu_max;           /* >= mu_min: ceiling; a rejection at mu_max ends the step */
    double up;               /* > 1: factor after a rejection and when rho < rho_lo */
    double down;             /* >= 1: divisor when rho > rho_hi */
    double rho_lo, rho_hi;   /* 0 <= rho_lo <= rho_hi */
    int32_t max_tries;       /* >= 1: factorisations at most */
    int32_t tries;           /* out: factorisations done */
    double rho;              /* out: gain ratio of the last trial (-inf if its solve failed) */
    double half_sq_norm_new; /* out: |r|^2 / 2 at the returned theta */
} gn_lm;

/* One step with Levenberg-Marquardt damping (rule above), theta updated in
 * place on acceptance.  r, J and the bordered Gram are formed once; each
 * trial factors G + mu I again (a copy of G is kept in its own strictly upper
 * triangle, so no extra matrix is allocated) and evaluates the residual at
 * theta + delta.  Synchronises once after forming G and once per trial.
 * *h_stats (may be NULL) describes the input theta and the last trial.
 * Returns GN_OK (accepted), GN_EREJECTED (theta unchanged; lm->mu is the
 * increased damping), GN_ENONFINITE (non-finite residual at theta), or
 * GN_EINVAL for constants outside the ranges above. */
gn_status gn_step_lm(gn_handle h, double *d_theta, gn_lm *lm, gn_stats *h_stats);

/* Stochastic full-matrix Gauss-Newton step (1D problems).  Paper: Methods,
 * "Second-order Optimizer": G is estimated by an exponential moving average,
 * across iterations, of an unbiased rank-1 estimate from one product with
 * the Jacobian, and the learning rate and momentum are set in closed form each
 * iteration (Martens and Grosse 2015, section 7).  One call:
 *   u = J^T v;  G_ema <- beta G_ema + (1 - beta) u u^T (lower triangle);
 *   if refactor: factor G_ema + gamma I (kept in the handle's workspace);
 *   Delta = -(G_ema + gamma I)^{-1} g,  g = J^T r;
 *   (alpha, mu) minimise M(d) = g^T d + d^T (J^T J + gamma I) d / 2 over
 *   d = alpha Delta + mu d_prev, with J Delta and J d_prev formed exactly
 *   (without momentum, d_prev = 0 or a 2 x 2 determinant at most 1e-12 of
 *   its diagonal product: mu = 0 and alpha alone);
 *   d_prev <- d;  theta <- theta + d.
 * d_G_ema: P x P (ldG >= P), caller-owned state, lower triangle read and
 * written (start from zeros).  d_prev: P, the previous update (zeros at the
 * first step), overwritten with this one.  d_v: gn_num_rows entries with
 * E[v v^T] = I (e.g. random signs), drawn by the caller.  The factor lives in
 * the handle's Gram workspace, so gn_step, gn_step_lm, gn_solve, a batched
 * step or new points discard it: refactor = 0 then returns GN_ESTATE.
 * Synchronises once.  Errors: GN_EINVAL (2D handle, ldG < P, beta outside
 * [0, 1], gamma <= 0, P > 65535), GN_ENOTPD (factorisation failed; theta and
 * d_prev unchanged, G_ema updated), GN_ENONFINITE. */
typedef struct {
    double beta;        /* moving-average decay, 0 <= beta <= 1 */
    double gamma;       /* damping, > 0 */
    int32_t refactor;   /* nonzero: factor G_ema + gamma I on this step */
    int32_t momentum;   /* nonzero: use d_prev in the closed-form coefficients */
} gn_rank1_args;

typedef struct {
    double half_sq_norm;     /* |r|^2 / 2 at the input theta */
    double max_abs_R;        /* max |R_i| over collocation points */
    double max_abs_R_val;    /* max |R| over the validation grid */
    double alpha;            /* learning rate */
    double mu;               /* momentum coefficient */
    double model;            /* M(d), the predicted change of h (<= 0) */
    int64_t chol_info;       /* 0, or 1-based first bad pivot of G_ema + gamma I */
    int32_t used_momentum;   /* 1 if the 2 x 2 system was solved */
    int32_t status;          /* gn_status of the step */
} gn_rank1_stats;

gn_status gn_step_rank1(gn_handle h, double *d_theta, double *d_G_ema, int64_t ldG, double *d_prev,
                        const double *d_v, const gn_rank1_args *args, gn_rank1_stats *h_stats);

/* Fields of a 1D first stage at its collocation points (which = 0, n
 * entries) or validation grid (which = 1, n_val entries): the raw residual
 * R, V = (1+lam) y + U and Theta' (device outputs), for gn_set_stage1.
 * Synchronises.  Errors: GN_EINVAL (2D or second-stage handle), GN_ESTATE. */
gn_status gn_fields(gn_handle h, const double *d_theta, int32_t which, double *d_R, double *d_V, double *d_Ty);

/* Make h (1D, without derivative rows) the second stage of multi-stage
 * training around a fixed first stage.  Paper: Methods, "Multi-stage
 * Training": the solution is Theta_1 + eps Theta_2 and, to first order in
 * eps, Theta_2 solves the equation linearised around Theta_1.  The d0 rows
 * become sqrt(rho_i/N) (R_1 + eps D[Theta_1] Theta_2) with
 * D Phi = -lam Phi + V_1 Phi' + U[Phi] Theta_1' (U[Phi] = H Phi for CCF, Phi
 * for the local variant), the validation max-norm uses the same expression;
 * the normalisation row is unchanged (use c_target = 0: NN_2(q = 1) = 0 keeps
 * the first stage's normalisation).  d_R1, d_V1, d_T1y: the first stage's R,
 * V and Theta' at h's collocation points (n each, from gn_fields on a handle
 * with the same points), d_R1v, d_V1v, d_T1yv at its validation grid (n_val
 * each, required when n_val > 0); copied.  gn_set_points ends the second
 * stage.  Errors: GN_EINVAL (2D, derivative rows, missing arrays, eps not
 * finite), GN_ESTATE, GN_ENOMEM. */
gn_status gn_set_stage1(gn_handle h, double eps, const double *d_R1, const double *d_V1, const double *d_T1y,
                        const double *d_R1v, const double *d_V1v, const double *d_T1yv);

/* Maximum d1 and d2 residuals on the validation grid (1D): *h_max_d1 =
 * max |R'|, *h_max_d2 = max |R''| (raw, unscaled; R', R'' as for
 * gn_set_points_ex).  Paper: Methods, "Validation Metrics for Solutions"
 * (the maximum dn residual).  Synchronises.  Errors: GN_EINVAL (2D handle),
 * GN_ESTATE (no points or no validation grid). */
gn_status gn_eval_derivs(gn_handle h, const double *d_theta, double *h_max_d1, double *h_max_d2);

/* Blow-up rate implied by the profile at the origin (1D CCF).  Paper:
 * Methods, "Identifying Admissible lambda Values" (lambda inference: the
 * derivatives of the self-similar equation at the origin must vanish).  For
 * an even profile R'(0) = 0 identically and R''(0) = Theta''(0)
 * (2 + lam + 2 U'(0)), so *h_lam = -2 (1 + U'(0)), U'(0) = H[Theta'](0) =
 * -(2/pi) int_0^inf Theta'(t)/t dt on the Hilbert nodes (also returned in
 * *h_dU0 when not NULL).  Synchronises.  Errors: GN_EINVAL (not 1D CCF),
 * GN_ESTATE. */
gn_status gn_lambda_estimate(gn_handle h, const double *d_theta, double *h_lam, double *h_dU0);

/* Proxy of funnel inference for a 1D first stage.  Paper: Methods,
 * "Identifying Admissible lambda Values" (funnel inference: near an
 * admissible lam the smallest reachable residual, taken with its sign, is
 * about linear in lam with a zero there; after training at a fixed lam, the
 * proxy r_hat(lam) is the residual of largest magnitude in a small
 * neighbourhood of the origin, and lam is updated by the secant method).
 * Evaluates the raw residual R at theta on the validation grid and returns,
 * over its points with y <= y_max, the value R_i of largest |R_i| (a NaN
 * counts as largest; the smallest index on ties) in *h_r_hat and y_i in
 * *h_y_at (when not NULL).  Synchronises.  Errors: GN_EINVAL (null theta or
 * r_hat, y_max not finite, 2D or second-stage handle), GN_ESTATE (no points,
 * no validation grid, or no validation point with y <= y_max). */
gn_status gn_funnel_residual(gn_handle h, const double *d_theta, double y_max, double *h_r_hat, double *h_y_at);

/* Residual statistics at theta (half_sq_norm, max_abs_R, max_abs_R_val).
 * Synchronises. */
gn_status gn_eval(gn_handle h, const double *d_theta, gn_stats *h_stats);

/* out = J^T v (P) without forming J; activations are recomputed.  The
 * adjoint of gn_residual (backward of a differentiable residual). */
gn_status gn_vjp(gn_handle h, const double *d_theta, const double *d_v, double *d_out);

/* Batches of independent problems (e.g. one profile per blow-up rate lambda)
 * that share the network widths (hence P) and use GN_FP64.  Each handle keeps
 * its own points, lambda and workspace; the batch groups the dense stages of
 * a step: one launch forms the Gram of every instance, each Cholesky panel is
 * one launch over all instances (a workgroup per instance for the diagonal
 * block, batched MFMA GEMMs for the panel and trailing update), and the back
 * substitution and update are batched likewise.  gn_batch_create copies the
 * handle list, reads their workspace layout (after gn_set_points) and
 * allocates the device descriptor arrays.  It does not own the handles, which
 * must outlive it; after gn_set_points on any of them, gn_step_batched returns
 * GN_ESTATE.  Errors: GN_EINVAL (n < 1, NULL handle, mixed P or a GN_SPLIT32
 * handle), GN_ESTATE (points not set), GN_ENOMEM.  All work is enqueued on
 * `stream` (hipStream_t as void*, NULL = default stream). */
typedef struct gn_batch_context *gn_batch;
gn_status gn_batch_create(gn_handle *hs, int32_t n, void *stream, gn_batch *out);
gn_status gn_batch_destroy(gn_batch b);
/* One damped GN step of every instance: d_thetas is a host array of n device
 * pointers (each updated in place, left unchanged on failure).  h_stats (n
 * entries, may be NULL) receives each instance's statistics and status; the
 * call synchronises only to fill it.  Returns GN_OK unless an argument or the
 * runtime fails; per-instance failures are reported in h_stats[i].status. */
gn_status gn_step_batched(gn_batch b, double *const *d_thetas, double mu, gn_stats *h_stats);

/* Measured throughput of the FP64 matrix instructions on the current device
 * (tracing support, not part of the paper's method: the practical ceiling
 * reported beside the published peak).  Every CU runs 32 waves of eight
 * independent v_mfma_f64_16x16x4f64 chains (no memory traffic) for about
 * 30 ms on `stream` (hipStream_t as void*, NULL = default stream);
 * *h_tflops receives 2 x 16 x 16 x 4 flops per instruction over the
 * event-timed span.  Synchronises.  Errors: GN_EINVAL (null pointer),
 * GN_EDEVICE. */
gn_status gn_probe_fp64_mfma(void *stream, double *h_tflops);

/* Phase timing of gn_step with HIP events recorded on the handle's stream
 * (tracing support; not part of the paper's method).  gn_step_batched
 * records its phases on the first handle of the batch (the local Jacobian
 * rows are timed with the forward phase).  Phases: */
typedef enum {
    GN_PHASE_FORWARD = 0,   /* weight transpose, forward jets, residual rows, validation grid */
    GN_PHASE_JLOCAL = 1,    /* per-row reverse sweeps writing the local Jacobian rows */
    GN_PHASE_COUPLING = 2,  /* Hilbert coupling GEMM J[:N] += diag(sc Theta_y) Q B */
    GN_PHASE_GRAM = 3,      /* Gram of [J | r] (lower triangle, FP64 MFMA) and |r|^2 */
    GN_PHASE_CHOLESKY = 4,  /* blocked Cholesky of the bordered matrix */
    GN_PHASE_SOLVE = 5,     /* back substitution, finiteness check, update of theta */
    GN_PHASE_COUNT = 6
} gn_phase;

/* enable = 1: record the phases of the next max_steps calls of gn_step
 * (creates the events here, outside the step path); enable = 0: stop and
 * release them.  Re-enabling restarts the count. */
gn_status gn_profile_enable(gn_handle h, int32_t enable, int32_t max_steps);
/* Synchronises; h_ms[k] = summed duration (ms) of phase k over the recorded
 * steps (n_phases <= GN_PHASE_COUNT entries written); *n_steps = steps
 * recorded. */
gn_status gn_profile_read(gn_handle h, double *h_ms, int32_t n_phases, int32_t *n_steps);

#ifdef __cplusplus
}
#endif
#endif /* GN_H */
