/*
 * Oracle dense linear algebra in plain C, FP64.  TEST INFRASTRUCTURE ONLY:
 * called by tests/, the smoke check and the benchmark's CPU-baseline leg,
 * never by the GPU library.  It shares no code with the GPU path.
 *
 * Paper reference: Methods, "Second-order Optimizer" -- the update
 *   theta <- theta - (G + gamma I)^{-1} grad h,  G = J^T J,  grad h ~ J^T r.
 *
 * - Gram and gradient: every entry is one compensated dot product, Dot2 of
 *   Ogita, Rump and Oishi (SIAM J. Sci. Comput. 26(6), 2005): TwoProduct by
 *   FMA plus TwoSum, so each entry is as accurate as if accumulated in twice
 *   the working precision and then rounded.
 * - Cholesky: unblocked textbook algorithm (Golub and Van Loan, "Matrix
 *   Computations", Cholesky by dot products), lower factor, LAPACK pivot
 *   convention for failures (1-based index of the first non-positive pivot).
 * - Forward and back substitution, plain loops.
 *
 * Storage: row-major; element (i, j) of a matrix with leading dimension ld is
 * a[i * ld + j].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Error-free transformations. */
static inline void two_sum(double a, double b, double *s, double *e) {
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

static inline void two_prod(double a, double b, double *p, double *e) {
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

/* Dot2: compensated dot product of x and y (strides sx, sy). */
static double dot2(const double *x, int64_t sx, const double *y, int64_t sy, int64_t n) {
    double s = 0.0, c = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        double p, ep, t, et;
        two_prod(x[k * sx], y[k * sy], &p, &ep);
        two_sum(s, p, &t, &et);
        s = t;
        c += ep + et;
    }
    return s + c;
}

/* Number of OpenMP threads the oracle runs with (1 without OpenMP). */
int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for later parallel loops (timing on one core or all cores). */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * G = J^T J (full symmetric, both triangles written) with J m x p, row-major,
 * leading dimension ldj.  Columns are first copied to a contiguous
 * column-major buffer so that each entry is one Dot2 over contiguous memory.
 */
int oracle_gram(const double *J, int64_t m, int64_t p, int64_t ldj, double *G, int64_t ldg) {
    double *Jt = (double *)malloc(sizeof(double) * (size_t)m * (size_t)p);
    if (!Jt) return -1;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t a = 0; a < p; ++a) Jt[a * m + i] = J[i * ldj + a];
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t a = 0; a < p; ++a) {
        for (int64_t b = 0; b <= a; ++b) {
            double v = dot2(Jt + a * m, 1, Jt + b * m, 1, m);
            G[a * ldg + b] = v;
            G[b * ldg + a] = v;
        }
    }
    free(Jt);
    return 0;
}

/* Selected entries G[rows[k], cols[k]] = sum_i J[i,rows[k]] J[i,cols[k]]. */
void oracle_gram_entries(const double *J, int64_t m, int64_t ldj, const int64_t *rows,
                         const int64_t *cols, int64_t count, double *out) {
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < count; ++k)
        out[k] = dot2(J + rows[k], ldj, J + cols[k], ldj, m);
}

/* g = J^T r. */
void oracle_gradient(const double *J, int64_t m, int64_t p, int64_t ldj, const double *r, double *g) {
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < p; ++a) g[a] = dot2(J + a, ldj, r, 1, m);
}

/*
 * In-place Cholesky A = L L^T of the lower triangle of the n x n matrix A.
 * Returns 0 on success, otherwise the 1-based index of the first pivot that
 * is not positive (A is then partially overwritten).  The strict upper
 * triangle is not referenced.
 */
int64_t oracle_cholesky(double *A, int64_t n, int64_t lda) {
    for (int64_t j = 0; j < n; ++j) {
        double *rj = A + j * lda;
        double d = rj[j] - dot2(rj, 1, rj, 1, j);
        if (!(d > 0.0)) return j + 1;
        double ljj = sqrt(d);
        rj[j] = ljj;
#pragma omp parallel for schedule(static)
        for (int64_t i = j + 1; i < n; ++i) {
            double *ri = A + i * lda;
            ri[j] = (ri[j] - dot2(ri, 1, rj, 1, j)) / ljj;
        }
    }
    return 0;
}

/* Solve L x = b in place (L lower, unit stride rows). */
void oracle_solve_lower(const double *L, int64_t n, int64_t ldl, double *b) {
    for (int64_t i = 0; i < n; ++i) {
        double s = b[i] - dot2(L + i * ldl, 1, b, 1, i);
        b[i] = s / L[i * ldl + i];
    }
}

/* Solve L^T x = b in place (column i of L^T is row i of L). */
void oracle_solve_lower_t(const double *L, int64_t n, int64_t ldl, double *b) {
    for (int64_t i = n - 1; i >= 0; --i) {
        /* x_i = (b_i - sum_{k>i} L[k,i] x_k) / L[i,i] */
        double s = b[i] - dot2(L + (i + 1) * ldl + i, ldl, b + i + 1, 1, n - 1 - i);
        b[i] = s / L[i * ldl + i];
    }
}

/* y = A x for a symmetric matrix given by its lower triangle (upper ignored). */
void oracle_symv_lower(const double *A, int64_t n, int64_t lda, const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0, c = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            double a = (k <= i) ? A[i * lda + k] : A[k * lda + i];
            double p, ep, t, et;
            two_prod(a, x[k], &p, &ep);
            two_sum(s, p, &t, &et);
            s = t;
            c += ep + et;
        }
        y[i] = s + c;
    }
}
