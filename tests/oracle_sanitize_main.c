/* Runs every entry point of oracle/oracle.c on small seeded graphs, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer (host code only;
 * see test_oracle_sanitize.py).  Exits non-zero on a wrong invariant; the
 * sanitizers abort on an invalid access or undefined behaviour. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void or_spmv_f32x(int64_t, const int64_t*, const int32_t*, const float*, const float*, double*);
void or_absmv_f32x(int64_t, const int64_t*, const int32_t*, const float*, const float*, double*);
void or_spmv_rows_f32x(int64_t, const int64_t*, const int64_t*, const int32_t*, const float*, const float*,
                       double*, double*);
void or_spmm_f32x(int64_t, const int64_t*, const int32_t*, const float*, const float*, int64_t, double*);
int64_t or_pagerank(int64_t, const int64_t*, const int32_t*, const float*, double, double, int64_t, double*,
                    double*);
int64_t or_hits(int64_t, const int64_t*, const int32_t*, const float*, double, int64_t, double*, double*);
int64_t or_rwr(int64_t, const int64_t*, const int32_t*, const float*, const int32_t*, int64_t, double, double,
               int64_t, double*, double*);
void or_set_threads(int);

static uint64_t st = 0x9e3779b97f4a7c15ull;
static uint64_t next(void) {
  st ^= st << 13;
  st ^= st >> 7;
  st ^= st << 17;
  return st;
}

/* a random directed graph on n nodes with up to m edges (duplicates kept,
 * some nodes without out-edges), as the column-stochastic PageRank matrix
 * M[v][u] = 1/outdeg(u) in CSR by row v */
static int check_graph(int64_t n, int64_t m) {
  int32_t* src = malloc(sizeof(int32_t) * m);
  int32_t* dst = malloc(sizeof(int32_t) * m);
  int64_t* outdeg = calloc(n, sizeof(int64_t));
  int64_t* rp = calloc(n + 1, sizeof(int64_t));
  for (int64_t e = 0; e < m; ++e) {
    src[e] = (int32_t)(next() % (uint64_t)(n > 1 ? n - 1 : 1));  /* node n-1 never links: dangling */
    dst[e] = (int32_t)(next() % (uint64_t)n);
    outdeg[src[e]]++;
    rp[dst[e] + 1]++;
  }
  for (int64_t i = 0; i < n; ++i) rp[i + 1] += rp[i];
  int32_t* col = malloc(sizeof(int32_t) * (m ? m : 1));
  float* val = malloc(sizeof(float) * (m ? m : 1));
  int64_t* fill = calloc(n, sizeof(int64_t));
  for (int64_t e = 0; e < m; ++e) {
    int64_t k = rp[dst[e]] + fill[dst[e]]++;
    col[k] = src[e];
    val[k] = (float)(1.0 / (double)outdeg[src[e]]);
  }
  float* x = malloc(sizeof(float) * n);
  for (int64_t i = 0; i < n; ++i) x[i] = (float)(next() % 1024) / 1024.0f;
  double* y = malloc(sizeof(double) * n);
  double* a = malloc(sizeof(double) * n);
  or_spmv_f32x(n, rp, col, val, x, y);
  or_absmv_f32x(n, rp, col, val, x, a);
  int bad = 0;
  for (int64_t i = 0; i < n; ++i) bad |= !(fabs(y[i]) <= a[i] + 1e-12);
  int64_t sel[3] = {0, n / 2, n - 1};
  double ys[3], as[3];
  or_spmv_rows_f32x(3, sel, rp, col, val, x, ys, as);
  for (int t = 0; t < 3; ++t) bad |= ys[t] != y[sel[t]];
  const int64_t k = 5;
  float* X = malloc(sizeof(float) * n * k);
  double* Y = malloc(sizeof(double) * n * k);
  for (int64_t i = 0; i < n * k; ++i) X[i] = (float)(next() % 64) / 64.0f;
  or_spmm_f32x(n, rp, col, val, X, k, Y);
  double* p = malloc(sizeof(double) * n);
  double* hist = malloc(sizeof(double) * 40 * k);
  int64_t it = or_pagerank(n, rp, col, val, 0.85, 0.0, 20, p, hist);
  double sp = 0.0;
  for (int64_t i = 0; i < n; ++i) sp += p[i];
  bad |= it != 20 || fabs(sp - 1.0) > 1e-5;  /* FP32 values 1/outdeg: column sums 1 within 2^-24 */
  /* HITS on the 2n block matrix [[0, A^T], [A, 0]] with ones (A: u -> v) */
  int64_t n2 = 2 * n;
  int64_t* rp2 = calloc(n2 + 1, sizeof(int64_t));
  int32_t* col2 = malloc(sizeof(int32_t) * 2 * (m ? m : 1));
  float* val2 = malloc(sizeof(float) * 2 * (m ? m : 1));
  for (int64_t e = 0; e < m; ++e) {
    rp2[dst[e] + 1]++;      /* authority row v: hub column n + u */
    rp2[n + src[e] + 1]++;  /* hub row u: authority column v */
  }
  for (int64_t i = 0; i < n2; ++i) rp2[i + 1] += rp2[i];
  int64_t* f2 = calloc(n2, sizeof(int64_t));
  for (int64_t e = 0; e < m; ++e) {
    int64_t r = dst[e];
    col2[rp2[r] + f2[r]] = (int32_t)(n + src[e]);
    val2[rp2[r] + f2[r]++] = 1.0f;
    r = n + src[e];
    col2[rp2[r] + f2[r]] = dst[e];
    val2[rp2[r] + f2[r]++] = 1.0f;
  }
  double* hx = malloc(sizeof(double) * n2);
  it = or_hits(n2, rp2, col2, val2, 0.0, 10, hx, hist);
  bad |= m > 0 && it != 10;
  int32_t seeds[5] = {0, 1, (int32_t)(n / 3), (int32_t)(n / 2), (int32_t)(n - 1)};
  double* R = malloc(sizeof(double) * n * k);
  it = or_rwr(n, rp, col, val, seeds, k, 0.85, 0.0, 8, R, hist);
  bad |= it != 8;
  free(src); free(dst); free(outdeg); free(rp); free(col); free(val); free(fill); free(x); free(y); free(a);
  free(X); free(Y); free(p); free(hist); free(rp2); free(col2); free(val2); free(f2); free(hx); free(R);
  return bad;
}

int main(void) {
  int bad = 0;
  for (int threads = 1; threads <= 4; threads *= 4) {
    or_set_threads(threads);
    bad |= check_graph(7, 20);
    bad |= check_graph(300, 2500);
    bad |= check_graph(4096, 40000);
  }
  printf(bad ? "oracle sanitizer run: invariant FAILED\n" : "oracle sanitizer run: ok\n");
  return bad;
}
