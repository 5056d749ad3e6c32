/*
 * FP64 CPU oracle for the OPEN collaborative-filtering hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load this file's library.  The GPU product path never calls it and
 * shares no code with it.
 *
 * Everything is computed in double precision, straight from the definitions, with no
 * blocking or reordering beyond what the definitions state:
 *
 *   - ridge row solve ("fold-in"): the paper fills a new application's missing entries by
 *     collaborative filtering (Section III-B.2); the completion is weighted-lambda ALS after
 *     the paper's CF reference (Zhou et al. 2008, cited in Section III-B.1).  With the
 *     setting factors F fixed, row i gets
 *         x_i = (sum_{j in O_i} f_j f_j^T + lambda w_i I)^-1 sum_{j in O_i} r_ij f_j,
 *     w_i = |O_i| (weighted) or 1, solved by a textbook Cholesky factorisation.
 *   - ALS-WR fit: alternate the row solve over all rows (against V) and over all columns
 *     (against U), recording the objective after every half-sweep.
 *   - objective  f(U,V) = sum_O (r_ij - u_i.v_j)^2 + lambda (sum_i w_i |u_i|^2 + sum_j w^j |v_j|^2).
 *   - Alg. 2 (Section III-B.3), energy-efficient cap selection on p = u_i . v_s.
 *   - observed-entry RMS residual of a row.
 *
 * Row status codes: 0 ok, 1 empty row (output 0), 2 non-positive pivot (output 0),
 * 3 non-finite input value (output 0).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ROW_OK = 0, ROW_EMPTY = 1, ROW_NONPOS_PIVOT = 2, ROW_NONFINITE = 3 };

void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Solve A x = b for a d x d symmetric positive definite A (row-major, overwritten by its
 * Cholesky factor L in the lower triangle); b is overwritten by x.  Returns 0, or 1 when a
 * pivot is not positive. */
static int cholesky_solve(double *A, double *b, int d) {
  for (int j = 0; j < d; ++j) {
    double s = A[j * d + j];
    for (int q = 0; q < j; ++q) s -= A[j * d + q] * A[j * d + q];
    if (!(s > 0.0)) return 1;
    const double ljj = sqrt(s);
    A[j * d + j] = ljj;
    for (int i = j + 1; i < d; ++i) {
      double t = A[i * d + j];
      for (int q = 0; q < j; ++q) t -= A[i * d + q] * A[j * d + q];
      A[i * d + j] = t / ljj;
    }
  }
  for (int i = 0; i < d; ++i) { /* L y = b */
    double t = b[i];
    for (int q = 0; q < i; ++q) t -= A[i * d + q] * b[q];
    b[i] = t / A[i * d + i];
  }
  for (int i = d - 1; i >= 0; --i) { /* L^T x = y */
    double t = b[i];
    for (int q = i + 1; q < d; ++q) t -= A[q * d + i] * b[q];
    b[i] = t / A[i * d + i];
  }
  return 0;
}

/* One ridge solve per CSR row against fixed factors F (rows of F indexed by idx). */
static int ridge_row(int k, int64_t beg, int64_t end, const int32_t *idx, const double *val,
                     const double *F, double lambda, int weighted, double *x, double *A, double *b) {
  const int64_t cnt = end - beg;
  memset(x, 0, sizeof(double) * (size_t)k);
  if (cnt == 0) return ROW_EMPTY;
  for (int64_t t = beg; t < end; ++t)
    if (!isfinite(val[t])) return ROW_NONFINITE;
  memset(A, 0, sizeof(double) * (size_t)k * (size_t)k);
  memset(b, 0, sizeof(double) * (size_t)k);
  for (int64_t t = beg; t < end; ++t) {
    const double *f = F + (int64_t)idx[t] * k;
    for (int a = 0; a < k; ++a) {
      b[a] += val[t] * f[a];
      for (int c = 0; c < k; ++c) A[a * k + c] += f[a] * f[c];
    }
  }
  const double reg = lambda * (weighted ? (double)cnt : 1.0);
  for (int a = 0; a < k; ++a) A[a * k + a] += reg;
  if (cholesky_solve(A, b, k)) return ROW_NONPOS_PIVOT;
  memcpy(x, b, sizeof(double) * (size_t)k);
  return ROW_OK;
}

/* Ridge solve of every row of a CSR (m rows) against F; X is m x k. status may be NULL.
 * Returns the number of rows whose status is not ok. */
int64_t oracle_ridge_rows(int64_t m, int k, const int64_t *ptr, const int32_t *idx, const double *val,
                          const double *F, double lambda, int weighted, double *X, int32_t *status) {
  int64_t bad = 0;
#pragma omp parallel reduction(+ : bad)
  {
    double *A = (double *)malloc(sizeof(double) * (size_t)k * (size_t)k);
    double *b = (double *)malloc(sizeof(double) * (size_t)k);
#pragma omp for schedule(dynamic, 256)
    for (int64_t i = 0; i < m; ++i) {
      int st = ridge_row(k, ptr[i], ptr[i + 1], idx, val, F, lambda, weighted, X + i * k, A, b);
      if (status) status[i] = st;
      if (st != ROW_OK) ++bad;
    }
    free(A);
    free(b);
  }
  return bad;
}

/* Ridge solve for a subset of rows (rows[t], t < cnt); X is cnt x k. */
int64_t oracle_ridge_subset(int64_t cnt, const int64_t *rows, int k, const int64_t *ptr, const int32_t *idx,
                            const double *val, const double *F, double lambda, int weighted, double *X,
                            int32_t *status) {
  int64_t bad = 0;
#pragma omp parallel reduction(+ : bad)
  {
    double *A = (double *)malloc(sizeof(double) * (size_t)k * (size_t)k);
    double *b = (double *)malloc(sizeof(double) * (size_t)k);
#pragma omp for schedule(dynamic, 64)
    for (int64_t t = 0; t < cnt; ++t) {
      const int64_t i = rows[t];
      int st = ridge_row(k, ptr[i], ptr[i + 1], idx, val, F, lambda, weighted, X + t * k, A, b);
      if (status) status[t] = st;
      if (st != ROW_OK) ++bad;
    }
    free(A);
    free(b);
  }
  return bad;
}

/* Column view of a CSR: col_ptr[n+1], row index and value of every entry, ordered by
 * column and, within a column, by row. */
void oracle_csr_to_csc(int64_t m, int n, const int64_t *row_ptr, const int32_t *col, const double *val,
                       int64_t *col_ptr, int32_t *row_idx, double *cval) {
  const int64_t nnz = row_ptr[m];
  memset(col_ptr, 0, sizeof(int64_t) * (size_t)(n + 1));
  for (int64_t t = 0; t < nnz; ++t) col_ptr[col[t] + 1]++;
  for (int j = 0; j < n; ++j) col_ptr[j + 1] += col_ptr[j];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  memcpy(fill, col_ptr, sizeof(int64_t) * (size_t)n);
  for (int64_t i = 0; i < m; ++i)
    for (int64_t t = row_ptr[i]; t < row_ptr[i + 1]; ++t) {
      const int64_t d = fill[col[t]]++;
      row_idx[d] = (int32_t)i;
      cval[d] = val[t];
    }
  free(fill);
}

double oracle_objective(int64_t m, int n, int k, const int64_t *row_ptr, const int32_t *col, const double *val,
                        const double *U, const double *V, double lambda, int weighted) {
  double loss = 0.0, ru = 0.0, rv = 0.0;
  int64_t *ncol = (int64_t *)calloc((size_t)n, sizeof(int64_t));
  for (int64_t t = 0; t < row_ptr[m]; ++t) ncol[col[t]]++;
#pragma omp parallel for reduction(+ : loss, ru) schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    const double *u = U + i * k;
    for (int64_t t = row_ptr[i]; t < row_ptr[i + 1]; ++t) {
      const double *v = V + (int64_t)col[t] * k;
      double p = 0.0;
      for (int a = 0; a < k; ++a) p += u[a] * v[a];
      loss += (val[t] - p) * (val[t] - p);
    }
    double nu = 0.0;
    for (int a = 0; a < k; ++a) nu += u[a] * u[a];
    ru += (weighted ? (double)(row_ptr[i + 1] - row_ptr[i]) : 1.0) * nu;
  }
  for (int j = 0; j < n; ++j) {
    double nv = 0.0;
    for (int a = 0; a < k; ++a) nv += V[(int64_t)j * k + a] * V[(int64_t)j * k + a];
    rv += (weighted ? (double)ncol[j] : 1.0) * nv;
  }
  free(ncol);
  return loss + lambda * (ru + rv);
}

/* ALS-WR: `sweeps` times (rows against V, then columns against U), starting from the
 * U, V passed in; obj (nullable) receives f after each half-sweep (2*sweeps values). */
int oracle_fit(int64_t m, int n, int k, const int64_t *row_ptr, const int32_t *col, const double *val,
               double lambda, int weighted, int sweeps, double *U, double *V, double *obj) {
  const int64_t nnz = row_ptr[m];
  int64_t *col_ptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int32_t *row_idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  double *cval = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  oracle_csr_to_csc(m, n, row_ptr, col, val, col_ptr, row_idx, cval);
  for (int s = 0; s < sweeps; ++s) {
    oracle_ridge_rows(m, k, row_ptr, col, val, V, lambda, weighted, U, NULL);
    if (obj) obj[2 * s] = oracle_objective(m, n, k, row_ptr, col, val, U, V, lambda, weighted);
    oracle_ridge_rows(n, k, col_ptr, row_idx, cval, U, lambda, weighted, V, NULL);
    if (obj) obj[2 * s + 1] = oracle_objective(m, n, k, row_ptr, col, val, U, V, lambda, weighted);
  }
  free(col_ptr);
  free(row_idx);
  free(cval);
  return 0;
}

/* Alg. 2 (Section III-B.3) for every row i of the predicted matrix p_is = u_i . v_s.
 * Baseline setting `base` = (C_b, G_b); E_base = (C_b + G_b) * 1; a setting is valid when
 * its predicted performance is positive and 1 - p/p_base <= gamma; its energy bound is
 * E = (c + g) / p and its saving (E_base - E) / E_base.  The valid setting with the largest
 * saving wins, the lowest index on ties.  A row whose baseline prediction is not positive
 * returns the baseline with saving 0 and status 2.  P (m x n, nullable) receives p. */
void oracle_predict_select(int64_t m, int n, int k, const double *U, const double *V, const double *cap_c,
                           const double *cap_g, int base, double gamma, double *P, int32_t *best, double *saving,
                           int32_t *status) {
  const double e_base = (cap_c[base] + cap_g[base]) * 1.0;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    const double *u = U + i * k;
    double p_base = 0.0;
    for (int a = 0; a < k; ++a) p_base += u[a] * V[(int64_t)base * k + a];
    int arg = -1;
    double best_saving = 0.0;
    for (int s = 0; s < n; ++s) {
      double p = 0.0;
      for (int a = 0; a < k; ++a) p += u[a] * V[(int64_t)s * k + a];
      if (P) P[i * n + s] = p;
      if (!(p_base > 0.0) || !(p > 0.0)) continue;
      const double loss = 1.0 - p / p_base;
      if (loss <= gamma) {
        const double e = (cap_c[s] + cap_g[s]) / p;
        const double sv = (e_base - e) / e_base;
        if (arg < 0 || sv > best_saving) {
          arg = s;
          best_saving = sv;
        }
      }
    }
    if (!(p_base > 0.0)) {
      best[i] = base;
      saving[i] = 0.0;
      if (status) status[i] = 2;
    } else {
      best[i] = arg;
      saving[i] = best_saving;
      if (status) status[i] = 0;
    }
  }
}

/* rho_i = sqrt(mean over observed j of (r_ij - u_i . v_j)^2); 0 for an empty row. */
void oracle_residual(int64_t m, int k, const int64_t *row_ptr, const int32_t *col, const double *val,
                     const double *U, const double *V, double *rho) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    const int64_t cnt = row_ptr[i + 1] - row_ptr[i];
    double acc = 0.0;
    for (int64_t t = row_ptr[i]; t < row_ptr[i + 1]; ++t) {
      double p = 0.0;
      for (int a = 0; a < k; ++a) p += U[i * k + a] * V[(int64_t)col[t] * k + a];
      acc += (val[t] - p) * (val[t] - p);
    }
    rho[i] = cnt > 0 ? sqrt(acc / (double)cnt) : 0.0;
  }
}
