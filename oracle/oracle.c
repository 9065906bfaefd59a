/*
 * oracle.c -- FP64 CPU reference for the SpMV hot path and the three power
 * iterations built on it.  TEST INFRASTRUCTURE ONLY: it is called by the test
 * suite, by the smoke check and by the benchmark's CPU-baseline leg, never by
 * the library's product path.  It shares no code with the GPU library.
 *
 * Everything is the plain definition, computed in double precision from the
 * same FP32 matrix values and FP32 input vectors the GPU reads (upcast):
 *
 *   SpMV (Appendix B, the product y = A x of an n x m sparse matrix in CSR):
 *     y_i = sum_{k = row_ptr[i]}^{row_ptr[i+1]-1} val[k] * x[col[k]],
 *     each row summed left to right.  Rows are independent, so the OpenMP
 *     split over rows does not change any result.
 *   PageRank (Appendix F, Eq. 6), damping c, p^(0) = 1/n, with the mass of
 *     dangling columns (columns with no entry) spread uniformly:
 *     p' = c (M p + (d/n) 1) + ((1-c)/n) 1,   d = sum of p_j over dangling j.
 *   HITS (Appendix F, Eq. 7-8): x' = B x on the 2n x 2n block matrix, then each
 *     half of x' divided by its own sum; x^(0) = 1/n everywhere.
 *   RWR (Appendix F, Eq. 9): r' = c W r + (1-c) e_s, r^(0) = e_s.
 *   Residual of each iteration: the L1 norm of the change of the iterate.
 *   Reductions run sequentially in index order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

/* y = A x with x given in FP32 (upcast) */
void or_spmv_f32x(int64_t n_rows, const int64_t* row_ptr, const int32_t* col, const float* val,
                  const float* x, double* y) {
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n_rows; ++i) {
    double s = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s += (double)val[k] * (double)x[col[k]];
    y[i] = s;
  }
}

/* y = A x with x in FP64 */
void or_spmv_f64x(int64_t n_rows, const int64_t* row_ptr, const int32_t* col, const float* val,
                  const double* x, double* y) {
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n_rows; ++i) {
    double s = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s += (double)val[k] * x[col[k]];
    y[i] = s;
  }
}

/* |A| |x| row sums (the scale of the rounding error bound); x FP32 */
void or_absmv_f32x(int64_t n_rows, const int64_t* row_ptr, const int32_t* col, const float* val,
                   const float* x, double* y) {
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n_rows; ++i) {
    double s = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s += fabs((double)val[k]) * fabs((double)x[col[k]]);
    y[i] = s;
  }
}

/* Selected rows only: y[t] = row rows[t] of A x  (for sampled checks at full size) */
void or_spmv_rows_f32x(int64_t n_sel, const int64_t* rows, const int64_t* row_ptr, const int32_t* col,
                       const float* val, const float* x, double* y, double* absy) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t t = 0; t < n_sel; ++t) {
    int64_t i = rows[t];
    double s = 0.0, a = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      s += (double)val[k] * (double)x[col[k]];
      a += fabs((double)val[k]) * fabs((double)x[col[k]]);
    }
    y[t] = s;
    absy[t] = a;
  }
}

/* Y = A X, X is n_cols x k row-major FP32, Y n_rows x k row-major FP64 */
void or_spmm_f32x(int64_t n_rows, const int64_t* row_ptr, const int32_t* col, const float* val,
                  const float* X, int64_t k, double* Y) {
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < n_rows; ++i) {
    double* yi = Y + i * k;
    for (int64_t q = 0; q < k; ++q) yi[q] = 0.0;
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      const float* xr = X + (int64_t)col[e] * k;
      double v = (double)val[e];
      for (int64_t q = 0; q < k; ++q) yi[q] += v * (double)xr[q];
    }
  }
}

/* Columns with no stored entry (dangling nodes of M = W^T). */
static char* or_empty_columns(int64_t n_cols, int64_t nnz, const int32_t* col) {
  char* has = (char*)calloc((size_t)n_cols, 1);
  for (int64_t k = 0; k < nnz; ++k) has[col[k]] = 1;
  for (int64_t j = 0; j < n_cols; ++j) has[j] = !has[j];
  return has;
}

/* PageRank power iteration (Eq. 6 with uniform dangling mass).
 * Runs until the L1 change is <= tol (tol <= 0: exactly max_iter iterations).
 * p_out: final iterate; resid_hist[k]: L1 change of iteration k (max_iter entries).
 * Returns the number of iterations run. */
int64_t or_pagerank(int64_t n, const int64_t* row_ptr, const int32_t* col, const float* val,
                    double c, double tol, int64_t max_iter, double* p_out, double* resid_hist) {
  char* dang = or_empty_columns(n, row_ptr[n], col);
  double* p = (double*)malloc((size_t)n * sizeof(double));
  double* y = (double*)malloc((size_t)n * sizeof(double));
  for (int64_t i = 0; i < n; ++i) p[i] = 1.0 / (double)n;
  int64_t it = 0;
  for (; it < max_iter; ++it) {
    double d = 0.0;
    for (int64_t j = 0; j < n; ++j) if (dang[j]) d += p[j];
    or_spmv_f64x(n, row_ptr, col, val, p, y);
    double r = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double pn = c * (y[i] + d / (double)n) + (1.0 - c) / (double)n;
      r += fabs(pn - p[i]);
      p[i] = pn;
    }
    if (resid_hist) resid_hist[it] = r;
    if (tol > 0.0 && r <= tol) { ++it; break; }
  }
  memcpy(p_out, p, (size_t)n * sizeof(double));
  free(dang); free(p); free(y);
  return it;
}

/* HITS on the 2n x 2n block matrix B (Eq. 8).  x_out holds [a; h].
 * Returns iterations run, or -1 if a half sums to zero. */
int64_t or_hits(int64_t n2, const int64_t* row_ptr, const int32_t* col, const float* val,
                double tol, int64_t max_iter, double* x_out, double* resid_hist) {
  int64_t n = n2 / 2;
  double* x = (double*)malloc((size_t)n2 * sizeof(double));
  double* y = (double*)malloc((size_t)n2 * sizeof(double));
  for (int64_t i = 0; i < n2; ++i) x[i] = 1.0 / (double)n;
  int64_t it = 0, ret = 0;
  for (; it < max_iter; ++it) {
    or_spmv_f64x(n2, row_ptr, col, val, x, y);
    double sa = 0.0, sh = 0.0;
    for (int64_t i = 0; i < n; ++i) sa += y[i];
    for (int64_t i = n; i < n2; ++i) sh += y[i];
    if (sa == 0.0 || sh == 0.0) { ret = -1; break; }
    double r = 0.0;
    for (int64_t i = 0; i < n2; ++i) {
      double xn = y[i] / (i < n ? sa : sh);
      r += fabs(xn - x[i]);
      x[i] = xn;
    }
    if (resid_hist) resid_hist[it] = r;
    if (tol > 0.0 && r <= tol) { ++it; break; }
  }
  memcpy(x_out, x, (size_t)n2 * sizeof(double));
  free(x); free(y);
  return ret < 0 ? -1 : it;
}

/* RWR for k seeds (Eq. 9): R is n x k row-major; column q restarts at seeds[q].
 * All columns iterate together until every column's L1 change is <= tol
 * (tol <= 0: exactly max_iter).  resid_hist[it*k + q] per column. */
int64_t or_rwr(int64_t n, const int64_t* row_ptr, const int32_t* col, const float* val,
               const int32_t* seeds, int64_t k, double c, double tol, int64_t max_iter,
               double* R_out, double* resid_hist) {
  double* R = (double*)calloc((size_t)(n * k), sizeof(double));
  double* Y = (double*)malloc((size_t)(n * k) * sizeof(double));
  for (int64_t q = 0; q < k; ++q) R[(int64_t)seeds[q] * k + q] = 1.0;
  int64_t it = 0;
  double* rcol = (double*)malloc((size_t)k * sizeof(double));
  for (; it < max_iter; ++it) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
      double* yi = Y + i * k;
      for (int64_t q = 0; q < k; ++q) yi[q] = 0.0;
      for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        const double* xr = R + (int64_t)col[e] * k;
        double v = (double)val[e];
        for (int64_t q = 0; q < k; ++q) yi[q] += v * xr[q];
      }
    }
    for (int64_t q = 0; q < k; ++q) rcol[q] = 0.0;
    for (int64_t i = 0; i < n; ++i)
      for (int64_t q = 0; q < k; ++q) {
        double rn = c * Y[i * k + q] + (i == seeds[q] ? (1.0 - c) : 0.0);
        rcol[q] += fabs(rn - R[i * k + q]);
        R[i * k + q] = rn;
      }
    double rmax = 0.0;
    for (int64_t q = 0; q < k; ++q) {
      if (resid_hist) resid_hist[it * k + q] = rcol[q];
      if (rcol[q] > rmax) rmax = rcol[q];
    }
    if (tol > 0.0 && rmax <= tol) { ++it; break; }
  }
  memcpy(R_out, R, (size_t)(n * k) * sizeof(double));
  free(R); free(Y); free(rcol);
  return it;
}

int or_num_threads(void) { return omp_get_max_threads(); }
void or_set_threads(int n) { omp_set_num_threads(n); }
