/*
 * FP64 CPU oracle for core-elements subsampled ALS.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the HIP library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, header, table or helper with the HIP library.
 *
 * What it computes (Xue, Li, Zhang, Meng, "Core-elements Subsampling for
 * Alternating Least Squares"):
 *
 *  - objective f(U, M) with the weighted lambda penalty   (Section 2.1, eq. for f)
 *  - the full-data row update                              (Section 2.1, eq. (U)/(M))
 *  - core-elements subsampling CES: per column of the design matrix X keep the
 *    s = floor(|I_i| r) entries of largest magnitude        (Section 3, Algorithm 1
 *                                                             and the selection rule)
 *  - the core estimator u = (X*^T X + lambda n_i E)^-1 X*^T y
 *                                                          (Section 3, eq. core_ui/core_mj)
 *  - one half-sweep of Core-ALS over all rows              (Section 3, Algorithm 2)
 *  - UNIF, the uniform-subsampling comparator           (Section 5, Tables 1, 2)
 *  - implicit-feedback Core-ALS                          (Section 3, last paragraph)
 *  - the fast variant: CES once per half-sweep on the whole factor matrix of
 *    the other side, each row regressing on that global sketch
 *                                                          (Section 3, the paragraph
 *                                                             after Algorithm 2)
 *
 * Readings where the paper leaves a choice open:
 *  - ties in the top-s are broken by smaller position first;
 *  - s = min(n, max(min_keep, floor(n num / den))) in 64-bit integers;
 *  - an empty row gets the zero vector (counted);
 *  - a core system (s < n) whose partial-pivoting LU meets a pivot with
 *    |pivot| <= n_f 2^-52 max|A| is replaced by the full-data row update
 *    (eq. (U)), solved by Cholesky (counted as a singular fallback); when
 *    s = n the system already is eq. (U), and a singular one gives u = 0
 *    (not counted).
 *
 * All arithmetic is double precision.  Input factor matrices are double
 * (callers widen fp32 arrays exactly).  OpenMP parallelises over rows only;
 * each row's arithmetic is sequential and in the order written here.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_OK 0
#define ORA_E_ARG 1
#define ORA_E_INDEX 2
#define ORA_E_VALUE 3

int ora_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ora_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Problem statement (Section 2.1): every observed index lies inside the
 * matrix, a row lists each column once (ascending here), values are finite. */
int ora_validate(int64_t n_rows, int64_t n_cols, const int64_t *row_ptr,
                 const int32_t *col_idx, const float *val) {
    if (n_rows < 0 || n_cols < 0) return ORA_E_ARG;
    if (row_ptr[0] != 0) return ORA_E_INDEX;
    for (int64_t i = 0; i < n_rows; ++i) {
        if (row_ptr[i + 1] < row_ptr[i]) return ORA_E_INDEX;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            if (col_idx[e] < 0 || col_idx[e] >= n_cols) return ORA_E_INDEX;
            if (e > row_ptr[i] && col_idx[e] <= col_idx[e - 1]) return ORA_E_INDEX;
            if (!isfinite((double)val[e])) return ORA_E_VALUE;
        }
    }
    return ORA_OK;
}

/* Column view of R: the item half-sweep regresses over I_j^M (Section 2.1). */
void ora_transpose(int64_t n_rows, int64_t n_cols, const int64_t *row_ptr,
                   const int32_t *col_idx, const float *val,
                   int64_t *col_ptr, int32_t *row_idx, float *val_t) {
    int64_t *fill = (int64_t *)calloc((size_t)n_cols + 1, sizeof(int64_t));
    for (int64_t j = 0; j <= n_cols; ++j) col_ptr[j] = 0;
    for (int64_t e = 0; e < row_ptr[n_rows]; ++e) col_ptr[col_idx[e] + 1] += 1;
    for (int64_t j = 0; j < n_cols; ++j) col_ptr[j + 1] += col_ptr[j];
    for (int64_t i = 0; i < n_rows; ++i) {
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            int64_t j = col_idx[e];
            int64_t dst = col_ptr[j] + fill[j]++;
            row_idx[dst] = (int32_t)i;
            val_t[dst] = val[e];
        }
    }
    free(fill);
}

/* Budget s = floor(|I_i| r) (Section 3, selection rule), r = num/den,
 * raised to min_keep and capped at n. */
int64_t ora_budget(int64_t n, int64_t num, int64_t den, int64_t min_keep) {
    int64_t s = (n * num) / den;
    if (s < min_keep) s = min_keep;
    if (s > n) s = n;
    if (s < 0) s = 0;
    return s;
}

typedef struct {
    double mag;
    int32_t pos;
} ora_key;

/* larger magnitude first; equal magnitudes: smaller position first */
static int ora_key_cmp(const void *pa, const void *pb) {
    const ora_key *a = (const ora_key *)pa, *b = (const ora_key *)pb;
    if (a->mag > b->mag) return -1;
    if (a->mag < b->mag) return 1;
    return (a->pos > b->pos) - (a->pos < b->pos);
}

static int ora_int_cmp(const void *pa, const void *pb) {
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    return (a > b) - (a < b);
}

/* CES (Algorithm 1) on an n x nf matrix X (row-major): for every column a,
 * the s positions whose |X[k][a]| are largest.  Writes pos[a*s + t], the
 * positions of column a in ascending order. */
void ora_select(int64_t n, int32_t nf, const double *X, int64_t s, int32_t *pos) {
    if (s <= 0) return;
    ora_key *keys = (ora_key *)malloc(sizeof(ora_key) * (size_t)(n > 0 ? n : 1));
    for (int32_t a = 0; a < nf; ++a) {
        for (int64_t k = 0; k < n; ++k) {
            keys[k].mag = fabs(X[k * nf + a]);
            keys[k].pos = (int32_t)k;
        }
        qsort(keys, (size_t)n, sizeof(ora_key), ora_key_cmp);
        for (int64_t t = 0; t < s; ++t) pos[a * s + t] = keys[t].pos;
        qsort(pos + a * s, (size_t)s, sizeof(int32_t), ora_int_cmp);
    }
    free(keys);
}

/* Solve A x = b (n x n, row-major, overwritten) by Gaussian elimination with
 * partial pivoting; the first row of largest |pivot| wins.  Returns 0 on
 * success, 1 if some |pivot| <= tol. */
static int ora_gepp(int32_t n, double *A, double *b, double tol) {
    for (int32_t j = 0; j < n; ++j) {
        int32_t p = j;
        double best = fabs(A[j * n + j]);
        for (int32_t i = j + 1; i < n; ++i) {
            double v = fabs(A[i * n + j]);
            if (v > best) { best = v; p = i; }
        }
        if (!(best > tol)) return 1;
        if (p != j) {
            for (int32_t c = 0; c < n; ++c) {
                double t = A[j * n + c]; A[j * n + c] = A[p * n + c]; A[p * n + c] = t;
            }
            double t = b[j]; b[j] = b[p]; b[p] = t;
        }
        for (int32_t i = j + 1; i < n; ++i) {
            double l = A[i * n + j] / A[j * n + j];
            if (l == 0.0) continue;
            for (int32_t c = j; c < n; ++c) A[i * n + c] -= l * A[j * n + c];
            b[i] -= l * b[j];
        }
    }
    for (int32_t j = n - 1; j >= 0; --j) {
        double acc = b[j];
        for (int32_t c = j + 1; c < n; ++c) acc -= A[j * n + c] * b[c];
        b[j] = acc / A[j * n + j];
    }
    return 0;
}

/* Solve G x = b for symmetric positive definite G by Cholesky G = L L^T.
 * Returns 1 if a pivot d_j (the diagonal before its square root, the pivot an
 * elimination without row exchanges meets) is <= tol. */
static int ora_cholesky_solve(int32_t n, double *G, double *b, double tol) {
    for (int32_t j = 0; j < n; ++j) {
        double d = G[j * n + j];
        for (int32_t c = 0; c < j; ++c) d -= G[j * n + c] * G[j * n + c];
        if (!(d > tol)) return 1;
        d = sqrt(d);
        G[j * n + j] = d;
        for (int32_t i = j + 1; i < n; ++i) {
            double v = G[i * n + j];
            for (int32_t c = 0; c < j; ++c) v -= G[i * n + c] * G[j * n + c];
            G[i * n + j] = v / d;
        }
    }
    for (int32_t j = 0; j < n; ++j) {
        double v = b[j];
        for (int32_t c = 0; c < j; ++c) v -= G[j * n + c] * b[c];
        b[j] = v / G[j * n + j];
    }
    for (int32_t j = n - 1; j >= 0; --j) {
        double v = b[j];
        for (int32_t c = j + 1; c < n; ++c) v -= G[c * n + j] * b[c];
        b[j] = v / G[j * n + j];
    }
    return 0;
}

/* Full-data row update, eq. (U): (X^T X + lambda n E) u = X^T y. */
static int ora_full_row(int64_t n, int32_t nf, const double *X, const double *y,
                        double lam, double *u) {
    double *G = (double *)calloc((size_t)nf * nf, sizeof(double));
    for (int32_t a = 0; a < nf; ++a) {
        for (int32_t c = 0; c < nf; ++c) {
            double acc = 0.0;
            for (int64_t k = 0; k < n; ++k) acc += X[k * nf + a] * X[k * nf + c];
            G[a * nf + c] = acc;
        }
        G[a * nf + a] += lam * (double)n;
        double acc = 0.0;
        for (int64_t k = 0; k < n; ++k) acc += X[k * nf + a] * y[k];
        u[a] = acc;
    }
    /* the singularity rule of the core system: a pivot <= n_f 2^-52 max|G| */
    double gmax = 0.0;
    for (int64_t e = 0; e < (int64_t)nf * nf; ++e) gmax = fmax(gmax, fabs(G[e]));
    int bad = ora_cholesky_solve(nf, G, u, (double)nf * ldexp(1.0, -52) * gmax);
    if (bad) for (int32_t a = 0; a < nf; ++a) u[a] = 0.0;
    free(G);
    return bad;
}

/* One core regression, eq. core_ui: X is n x nf, y has n entries.
 * Returns 0 normal, 1 empty row, 2 singular fallback taken (core rows, s < n),
 * 3 singular full-data system (s = n: the system is eq. (U) itself, so there
 * is nothing to fall back to; u = 0). */
int ora_core_row(int64_t n, int32_t nf, const double *X, const double *y, double lam,
                 int64_t s, double *u) {
    if (n == 0) {
        for (int32_t a = 0; a < nf; ++a) u[a] = 0.0;
        return 1;
    }
    int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)nf * (size_t)(s > 0 ? s : 1));
    ora_select(n, nf, X, s, pos);
    double *A = (double *)calloc((size_t)nf * nf, sizeof(double));
    double *b = (double *)calloc((size_t)nf, sizeof(double));
    /* row a of X*^T X: sum over the kept positions of column a */
    for (int32_t a = 0; a < nf; ++a) {
        for (int64_t t = 0; t < s; ++t) {
            int64_t k = pos[a * s + t];
            double xa = X[k * nf + a];
            for (int32_t c = 0; c < nf; ++c) A[a * nf + c] += xa * X[k * nf + c];
            b[a] += xa * y[k];
        }
        A[a * nf + a] += lam * (double)n;
    }
    double amax = 0.0;
    for (int64_t e = 0; e < (int64_t)nf * nf; ++e) amax = fmax(amax, fabs(A[e]));
    double tol = (double)nf * ldexp(1.0, -52) * amax;
    int status = 0;
    if (ora_gepp(nf, A, b, tol)) {
        if (s < n) {
            ora_full_row(n, nf, X, y, lam, u);
            status = 2;
        } else {
            for (int32_t a = 0; a < nf; ++a) u[a] = 0.0;
            status = 3;
        }
    } else {
        for (int32_t a = 0; a < nf; ++a) u[a] = b[a];
    }
    free(A);
    free(b);
    free(pos);
    return status;
}

/* Gather the design matrix of one row: X[k] = other[col_idx[e_k]] (Section 2.1,
 * the sub-matrix of the other factor whose rows are the observed columns). */
static void ora_gather(int64_t beg, int64_t n, int32_t nf, const int32_t *col_idx,
                       const float *val, const double *other, double *X, double *y) {
    for (int64_t k = 0; k < n; ++k) {
        int64_t j = col_idx[beg + k];
        for (int32_t a = 0; a < nf; ++a) X[k * nf + a] = other[j * nf + a];
        y[k] = (double)val[beg + k];
    }
}

/* One half-sweep of Algorithm 2: every row of a CSR regresses on `other`.
 * out is n_rows x nf.  stats[0] counts empty rows, stats[1] singular fallbacks. */
void ora_half_sweep(int64_t n_rows, int32_t nf, const int64_t *row_ptr,
                    const int32_t *col_idx, const float *val, const double *other,
                    double lam, int64_t num, int64_t den, int64_t min_keep,
                    double *out, int64_t *stats) {
    int64_t n_empty = 0, n_fallback = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : n_empty, n_fallback)
    for (int64_t i = 0; i < n_rows; ++i) {
        int64_t beg = row_ptr[i];
        int64_t n = row_ptr[i + 1] - beg;
        double *X = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * nf);
        double *y = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        ora_gather(beg, n, nf, col_idx, val, other, X, y);
        int64_t s = ora_budget(n, num, den, min_keep);
        int st = ora_core_row(n, nf, X, y, lam, s, out + i * nf);
        if (st == 1) n_empty++;
        if (st == 2) n_fallback++;
        free(X);
        free(y);
    }
    if (stats) {
        stats[0] = n_empty;
        stats[1] = n_fallback;
    }
}

/* Same as ora_half_sweep restricted to the listed rows (for sampled checks
 * at full size); out holds len(rows) x nf. */
void ora_half_sweep_rows(int64_t n_list, const int64_t *rows, int32_t nf,
                         const int64_t *row_ptr, const int32_t *col_idx, const float *val,
                         const double *other, double lam, int64_t num, int64_t den,
                         int64_t min_keep, double *out, int64_t *stats) {
    int64_t n_empty = 0, n_fallback = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : n_empty, n_fallback)
    for (int64_t t = 0; t < n_list; ++t) {
        int64_t i = rows[t];
        int64_t beg = row_ptr[i];
        int64_t n = row_ptr[i + 1] - beg;
        double *X = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * nf);
        double *y = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        ora_gather(beg, n, nf, col_idx, val, other, X, y);
        int64_t s = ora_budget(n, num, den, min_keep);
        int st = ora_core_row(n, nf, X, y, lam, s, out + t * nf);
        if (st == 1) n_empty++;
        if (st == 2) n_fallback++;
        free(X);
        free(y);
    }
    if (stats) {
        stats[0] = n_empty;
        stats[1] = n_fallback;
    }
}

/* CES positions for the listed rows: for row rows[t] with budget s, column a,
 * writes s ascending positions at sel[sel_ptr[t] + a*s ...]. */
void ora_core_select_rows(int64_t n_list, const int64_t *rows, int32_t nf,
                          const int64_t *row_ptr, const int32_t *col_idx,
                          const double *other, int64_t num, int64_t den, int64_t min_keep,
                          const int64_t *sel_ptr, int32_t *sel) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < n_list; ++t) {
        int64_t i = rows[t];
        int64_t beg = row_ptr[i];
        int64_t n = row_ptr[i + 1] - beg;
        double *X = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * nf);
        for (int64_t k = 0; k < n; ++k) {
            int64_t j = col_idx[beg + k];
            for (int32_t a = 0; a < nf; ++a) X[k * nf + a] = other[j * nf + a];
        }
        int64_t s = ora_budget(n, num, den, min_keep);
        ora_select(n, nf, X, s, sel + sel_ptr[t]);
        free(X);
    }
}

/* Objective (Section 2.1): out[0] = f = SSE + lambda (sum_i n_i |u_i|^2 +
 * sum_j n_j |m_j|^2), out[1] = SSE, out[2] = RMSE = sqrt(SSE / nnz),
 * out[3] = ReMSE = sqrt(SSE) / sqrt(sum r^2)  (Section 5.1). */
void ora_objective(int64_t n_u, int64_t n_m, int32_t nf, const int64_t *row_ptr,
                   const int32_t *col_idx, const float *val, const double *U,
                   const double *M, double lam, double *out) {
    double sse = 0.0, rr = 0.0, pen_u = 0.0, pen_m = 0.0;
    int64_t nnz = row_ptr[n_u];
    int64_t *deg_m = (int64_t *)calloc((size_t)n_m + 1, sizeof(int64_t));
    for (int64_t e = 0; e < nnz; ++e) deg_m[col_idx[e]] += 1;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : sse, rr, pen_u)
    for (int64_t i = 0; i < n_u; ++i) {
        double nrm = 0.0;
        for (int32_t a = 0; a < nf; ++a) nrm += U[i * nf + a] * U[i * nf + a];
        pen_u += (double)(row_ptr[i + 1] - row_ptr[i]) * nrm;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            int64_t j = col_idx[e];
            double pred = 0.0;
            for (int32_t a = 0; a < nf; ++a) pred += U[i * nf + a] * M[j * nf + a];
            double r = (double)val[e] - pred;
            sse += r * r;
            rr += (double)val[e] * (double)val[e];
        }
    }
    for (int64_t j = 0; j < n_m; ++j) {
        double nrm = 0.0;
        for (int32_t a = 0; a < nf; ++a) nrm += M[j * nf + a] * M[j * nf + a];
        pen_m += (double)deg_m[j] * nrm;
    }
    free(deg_m);
    out[0] = sse + lam * (pen_u + pen_m);
    out[1] = sse;
    out[2] = nnz > 0 ? sqrt(sse / (double)nnz) : 0.0;
    out[3] = rr > 0.0 ? sqrt(sse) / sqrt(rr) : 0.0;
}

/* ------------------------------------------------------------------------
 * Fast variant of Core-ALS (Section 3, the paragraph and figure after
 * Algorithm 2; its details are in the paper's appendix, which is not part of
 * the text).  Reading: before each half-sweep, CES (Algorithm 1) is applied
 * once to the whole factor matrix of the other side, at the rate r, instead of
 * to every row's slice; each regression then uses the rows of that global
 * sketch, X* = (global mask) applied to the row's design matrix.  The per-row
 * number of kept entries therefore only follows r on average, as the paper
 * says of this variant.
 * ---------------------------------------------------------------------- */

/* keep[j * nf + a] = 1 for the s = budget(n_other) entries of column a with
 * the largest |other[j][a]| (ties: the smaller j), 0 elsewhere. */
void ora_global_select(int64_t n_other, int32_t nf, const double *other, int64_t s, uint8_t *keep) {
    for (int64_t e = 0; e < n_other * (int64_t)nf; ++e) keep[e] = 0;
    if (s <= 0) return;
    int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)nf * (size_t)s);
    ora_select(n_other, nf, other, s, pos);
    for (int32_t a = 0; a < nf; ++a)
        for (int64_t t = 0; t < s; ++t) keep[(int64_t)pos[a * s + t] * nf + a] = 1;
    free(pos);
}

/* One regression with a given sketch mask K (n x nf): (X*^T X + lambda n E) u
 * = X*^T y, X* = K (elementwise) X, the system of eq. core_ui.  Status as
 * ora_core_row: 1 empty row, 2 singular system replaced by eq. (U), 3 singular
 * with every entry kept (the system is eq. (U) itself; u = 0). */
int ora_masked_row(int64_t n, int32_t nf, const double *X, const uint8_t *K, const double *y, double lam,
                   double *u) {
    if (n == 0) {
        for (int32_t a = 0; a < nf; ++a) u[a] = 0.0;
        return 1;
    }
    double *A = (double *)calloc((size_t)nf * nf, sizeof(double));
    double *b = (double *)calloc((size_t)nf, sizeof(double));
    int all_kept = 1;
    for (int32_t a = 0; a < nf; ++a) {
        for (int64_t k = 0; k < n; ++k) {
            if (!K[k * nf + a]) {
                all_kept = 0;
                continue;
            }
            double xa = X[k * nf + a];
            for (int32_t c = 0; c < nf; ++c) A[a * nf + c] += xa * X[k * nf + c];
            b[a] += xa * y[k];
        }
        A[a * nf + a] += lam * (double)n;
    }
    double amax = 0.0;
    for (int64_t e = 0; e < (int64_t)nf * nf; ++e) amax = fmax(amax, fabs(A[e]));
    int status = 0;
    if (ora_gepp(nf, A, b, (double)nf * ldexp(1.0, -52) * amax)) {
        if (!all_kept) {
            ora_full_row(n, nf, X, y, lam, u);
            status = 2;
        } else {
            for (int32_t a = 0; a < nf; ++a) u[a] = 0.0;
            status = 3;
        }
    } else {
        for (int32_t a = 0; a < nf; ++a) u[a] = b[a];
    }
    free(A);
    free(b);
    return status;
}

/* One half-sweep of the fast variant: the global sketch of `other`
 * (n_other x nf) at budget(n_other), then every row's regression on it.
 * stats[0] empty rows, stats[1] singular systems replaced by eq. (U). */
void ora_fast_half_sweep(int64_t n_rows, int32_t nf, const int64_t *row_ptr, const int32_t *col_idx,
                         const float *val, int64_t n_other, const double *other, double lam, int64_t num,
                         int64_t den, int64_t min_keep, double *out, int64_t *stats) {
    uint8_t *keep = (uint8_t *)malloc((size_t)(n_other > 0 ? n_other : 1) * nf);
    ora_global_select(n_other, nf, other, ora_budget(n_other, num, den, min_keep), keep);
    int64_t n_empty = 0, n_fallback = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : n_empty, n_fallback)
    for (int64_t i = 0; i < n_rows; ++i) {
        int64_t beg = row_ptr[i];
        int64_t n = row_ptr[i + 1] - beg;
        double *X = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * nf);
        double *y = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        uint8_t *K = (uint8_t *)malloc((size_t)(n > 0 ? n : 1) * nf);
        ora_gather(beg, n, nf, col_idx, val, other, X, y);
        for (int64_t k = 0; k < n; ++k)
            for (int32_t a = 0; a < nf; ++a) K[k * nf + a] = keep[(int64_t)col_idx[beg + k] * nf + a];
        int st = ora_masked_row(n, nf, X, K, y, lam, out + i * nf);
        if (st == 1) n_empty++;
        if (st == 2) n_fallback++;
        free(X);
        free(y);
        free(K);
    }
    free(keep);
    if (stats) {
        stats[0] = n_empty;
        stats[1] = n_fallback;
    }
}

/* ------------------------------------------------------------------------
 * UNIF, the uniform-subsampling comparator of Section 5 (Table 1 and 2).
 * Reading (the paper names the method and its rate only): each regression
 * draws s = budget(n) of its n observed entries uniformly without
 * replacement and solves the ridge regression of that sample,
 *     (X_S^T X_S + lambda s E) u = X_S^T y_S,
 * the weighted-lambda rule of Section 2.1 applied to the subsample (the same
 * system as the inverse-probability-weighted estimator with lambda n, scaled
 * by s / n).  The draw: the s entries whose key h(seed, row, col) is smallest
 * (ties: smaller position), with h the upper 32 bits of splitmix64 (Steele,
 * Lea and Flood, 2014) at seed * 0x9E3779B97F4A7C15 + row * n_cols + col.
 * ---------------------------------------------------------------------- */

uint64_t ora_splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint32_t ora_unif_key(uint64_t seed, int64_t row, int64_t n_cols, int64_t col) {
    return (uint32_t)(ora_splitmix64(seed * 0x9E3779B97F4A7C15ull + (uint64_t)(row * n_cols + col)) >> 32);
}

typedef struct {
    uint32_t key;
    int32_t pos;
} ora_ukey;

static int ora_ukey_cmp(const void *pa, const void *pb) {
    const ora_ukey *a = (const ora_ukey *)pa, *b = (const ora_ukey *)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return (a->pos > b->pos) - (a->pos < b->pos);
}

/* keep[k] = 1 for the s entries of the row with the smallest keys. */
void ora_unif_select(int64_t n, const int32_t *cols, int64_t row, int64_t n_cols, uint64_t seed, int64_t s,
                     uint8_t *keep) {
    ora_ukey *k = (ora_ukey *)malloc(sizeof(ora_ukey) * (size_t)(n > 0 ? n : 1));
    for (int64_t t = 0; t < n; ++t) {
        k[t].key = ora_unif_key(seed, row, n_cols, cols[t]);
        k[t].pos = (int32_t)t;
        keep[t] = 0;
    }
    qsort(k, (size_t)n, sizeof(ora_ukey), ora_ukey_cmp);
    for (int64_t t = 0; t < s && t < n; ++t) keep[k[t].pos] = 1;
    free(k);
}

/* The subsample's ridge regression; returns 1 for an empty row, 3 when the
 * system is singular (s = 0 at any lambda, or lambda = 0 with a rank-deficient
 * sample): u = 0. */
int ora_unif_row(int64_t n, int32_t nf, const double *X, const uint8_t *keep, const double *y, double lam,
                 int64_t s, double *u) {
    if (n == 0) {
        for (int32_t a = 0; a < nf; ++a) u[a] = 0.0;
        return 1;
    }
    double *G = (double *)calloc((size_t)nf * nf, sizeof(double));
    for (int32_t a = 0; a < nf; ++a) {
        double acc = 0.0;
        for (int64_t k = 0; k < n; ++k)
            if (keep[k]) acc += X[k * nf + a] * y[k];
        u[a] = acc;
        for (int32_t c = 0; c < nf; ++c) {
            double g = 0.0;
            for (int64_t k = 0; k < n; ++k)
                if (keep[k]) g += X[k * nf + a] * X[k * nf + c];
            G[a * nf + c] = g;
        }
        G[a * nf + a] += lam * (double)s;
    }
    double gmax = 0.0;
    for (int64_t e = 0; e < (int64_t)nf * nf; ++e) gmax = fmax(gmax, fabs(G[e]));
    int bad = ora_cholesky_solve(nf, G, u, (double)nf * ldexp(1.0, -52) * gmax);
    if (bad || gmax == 0.0)
        for (int32_t a = 0; a < nf; ++a) u[a] = 0.0;
    free(G);
    return (bad || gmax == 0.0) ? 3 : 0;
}

/* One half-sweep of UNIF.  stats[0] empty rows, stats[1] singular systems. */
void ora_unif_half_sweep(int64_t n_rows, int32_t nf, const int64_t *row_ptr, const int32_t *col_idx,
                         const float *val, int64_t n_cols, const double *other, double lam, int64_t num,
                         int64_t den, int64_t min_keep, uint64_t seed, double *out, int64_t *stats) {
    int64_t n_empty = 0, n_sing = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : n_empty, n_sing)
    for (int64_t i = 0; i < n_rows; ++i) {
        int64_t beg = row_ptr[i];
        int64_t n = row_ptr[i + 1] - beg;
        double *X = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * nf);
        double *y = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        uint8_t *keep = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
        ora_gather(beg, n, nf, col_idx, val, other, X, y);
        int64_t s = ora_budget(n, num, den, min_keep);
        ora_unif_select(n, col_idx + beg, i, n_cols, seed, s, keep);
        int st = ora_unif_row(n, nf, X, keep, y, lam, s, out + i * nf);
        if (st == 1) n_empty++;
        if (st == 3) n_sing++;
        free(X);
        free(y);
        free(keep);
    }
    if (stats) {
        stats[0] = n_empty;
        stats[1] = n_sing;
    }
}

/* ------------------------------------------------------------------------
 * Implicit-feedback Core-ALS (Section 3, last paragraph; the paper defers its
 * form to the appendix, which is not in the text).  Reading: the implicit
 * ALS of Hu, Koren and Volinsky (2008) with the core-elements sketch on the
 * observed part.  Every observed entry is a preference 1 with confidence
 * c = 1 + alpha r; every other entry a preference 0 with confidence 1.  The
 * full-data update of row i, (Y^T C_i Y + lambda E) u = Y^T C_i p_i, splits as
 * Y^T Y + X^T W X with X the row's observed rows of Y and W = diag(alpha r_k);
 * the core version sketches the observed part:
 *     (Y^T Y + X*^T W X + lambda E) u = X*^T (1 + alpha r),
 * X* = CES(X, r) column by column as in Algorithm 1.  At r = 1 it is implicit
 * ALS exactly.
 * ---------------------------------------------------------------------- */

/* G = other^T other (n_other x nf, row-major), the Gram over all rows. */
void ora_global_gram(int64_t n_other, int32_t nf, const double *other, double *G) {
    for (int32_t a = 0; a < nf; ++a)
        for (int32_t c = 0; c < nf; ++c) {
            double acc = 0.0;
            for (int64_t j = 0; j < n_other; ++j) acc += other[j * nf + a] * other[j * nf + c];
            G[a * nf + c] = acc;
        }
}

/* One implicit core regression.  Status: 1 empty row (u = 0: b = 0), 2
 * singular core system replaced by the full-data implicit update, 3 singular
 * with s = n (u = 0). */
int ora_implicit_row(int64_t n, int32_t nf, const double *X, const double *r, const double *G, double lam,
                     double alpha, int64_t s, double *u) {
    if (n == 0) {
        for (int32_t a = 0; a < nf; ++a) u[a] = 0.0;
        return 1;
    }
    int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)nf * (size_t)(s > 0 ? s : 1));
    ora_select(n, nf, X, s, pos);
    double *A = (double *)malloc(sizeof(double) * (size_t)nf * nf);
    double *b = (double *)calloc((size_t)nf, sizeof(double));
    int status = 0;
    for (int attempt = 0; attempt < 2; ++attempt) {
        for (int64_t e = 0; e < (int64_t)nf * nf; ++e) A[e] = G[e];
        for (int32_t a = 0; a < nf; ++a) {
            b[a] = 0.0;
            const int64_t cnt = attempt == 0 ? s : n;
            for (int64_t t = 0; t < cnt; ++t) {
                int64_t k = attempt == 0 ? pos[a * s + t] : t;
                double xa = X[k * nf + a];
                for (int32_t c = 0; c < nf; ++c) A[a * nf + c] += alpha * r[k] * xa * X[k * nf + c];
                b[a] += (1.0 + alpha * r[k]) * xa;
            }
            A[a * nf + a] += lam;
        }
        double amax = 0.0;
        for (int64_t e = 0; e < (int64_t)nf * nf; ++e) amax = fmax(amax, fabs(A[e]));
        if (!ora_gepp(nf, A, b, (double)nf * ldexp(1.0, -52) * amax)) {
            for (int32_t a = 0; a < nf; ++a) u[a] = b[a];
            break;
        }
        if (attempt == 1 || s >= n) {
            for (int32_t a = 0; a < nf; ++a) u[a] = 0.0;
            status = s >= n ? 3 : 2;
            break;
        }
        status = 2;
    }
    free(A);
    free(b);
    free(pos);
    return status;
}

/* One implicit half-sweep: G = other^T other, then every row.  stats[0]
 * empty rows, stats[1] singular core systems replaced by the full data. */
void ora_implicit_half_sweep(int64_t n_rows, int32_t nf, const int64_t *row_ptr, const int32_t *col_idx,
                             const float *val, int64_t n_other, const double *other, double lam, double alpha,
                             int64_t num, int64_t den, int64_t min_keep, double *out, int64_t *stats) {
    double *G = (double *)malloc(sizeof(double) * (size_t)nf * nf);
    ora_global_gram(n_other, nf, other, G);
    int64_t n_empty = 0, n_fallback = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : n_empty, n_fallback)
    for (int64_t i = 0; i < n_rows; ++i) {
        int64_t beg = row_ptr[i];
        int64_t n = row_ptr[i + 1] - beg;
        double *X = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * nf);
        double *y = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        ora_gather(beg, n, nf, col_idx, val, other, X, y);
        int st = ora_implicit_row(n, nf, X, y, G, lam, alpha, ora_budget(n, num, den, min_keep), out + i * nf);
        if (st == 1) n_empty++;
        if (st == 2) n_fallback++;
        free(X);
        free(y);
    }
    free(G);
    if (stats) {
        stats[0] = n_empty;
        stats[1] = n_fallback;
    }
}
