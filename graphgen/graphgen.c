/*
 * graphgen.c -- seeded synthetic power-law graphs and the sparse matrices the
 * graph-mining problems are posed on.
 *
 * This module is input preparation only.  It is shared by the FP64 oracle side
 * and the GPU side; it computes none of the SpMV method's arithmetic (no
 * tiling, no sorting by degree, no products with vectors).
 *
 * Random numbers: a counter-based generator built from the SplitMix64 output
 * function (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014; constants as published by Vigna).  Draw i of stream
 * s under seed k is mix(k * G + (s << 56) + i * G) where G is the 64-bit golden
 * ratio constant, so every draw is independent of thread count and order.
 *
 * Graphs:
 *   R-MAT (Chakrabarti, Zhan, Faloutsos 2004): 2^scale nodes, m draws; for every
 *     bit level the quadrant probabilities a, b, c, d pick one bit of the source
 *     and one of the destination (most significant bit first).  Exact duplicate
 *     edges are removed, self-loops kept, node ids not relabelled.
 *   Chung-Lu (Chung and Lu 2002): expected-degree model.  Node i has weight
 *     (i+1)^(-1/(gamma-1)), scaled so the weights sum to the target edge count,
 *     capped at `cap` with the remaining weight rescaled to a fixpoint.  In-weights
 *     are the same weights under an independent random permutation.  Sources and
 *     destinations are drawn independently in proportion to the weights (Walker
 *     alias tables, Vose's construction); the
 *     first `target` distinct edges in draw order are kept; finally node ids are
 *     relabelled by a random permutation.
 *
 * Matrices built from an edge list (u -> v):
 *   pagerank:  M = W^T, M[v][u] = fl32(1/outdeg(u))          (column-stochastic)
 *   hits:      B = [[0, A^T], [A, 0]], 2n x 2n, values 1.0f
 *   rwr:       column-normalised adjacency of the symmetrised graph,
 *              S[i][j] = fl32(1/deg(j)) with deg counted on the symmetrised,
 *              deduplicated edge set (self-loops once)
 * All CSR outputs have ascending column ids within each row.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

#define GG_GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t gg_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t gg_draw(uint64_t seed, uint64_t stream, uint64_t i) {
  return gg_mix(seed * GG_GOLDEN + (stream << 56) + (i + 1) * GG_GOLDEN);
}

/* uniform double in [0,1) with 53 random bits */
static inline double gg_unif(uint64_t seed, uint64_t stream, uint64_t i) {
  return (double)(gg_draw(seed, stream, i) >> 11) * (1.0 / 9007199254740992.0);
}

/* ---------------------------------------------------------------- sorting */
/* Stable LSD radix sort of (key, payload) pairs on the low `bits` bits of key.
 * Parallel with per-thread histograms; result independent of thread count. */
static void gg_radix_sort_u64(uint64_t* key, uint32_t* pay, int64_t n, int bits) {
  if (n <= 1 || bits <= 0) return;
  uint64_t* k2 = (uint64_t*)malloc((size_t)n * sizeof(uint64_t));
  uint32_t* p2 = pay ? (uint32_t*)malloc((size_t)n * sizeof(uint32_t)) : NULL;
  const int RB = 11, NB = 1 << RB;
  int nthr = omp_get_max_threads();
  int64_t* hist = (int64_t*)malloc((size_t)nthr * NB * sizeof(int64_t));
  uint64_t *src = key, *dst = k2;
  uint32_t *psrc = pay, *pdst = p2;
  for (int shift = 0; shift < bits; shift += RB) {
    memset(hist, 0, (size_t)nthr * NB * sizeof(int64_t));
#pragma omp parallel num_threads(nthr)
    {
      int t = omp_get_thread_num(), nt = omp_get_num_threads();
      int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
      int64_t* h = hist + (size_t)t * NB;
      for (int64_t i = lo; i < hi; ++i) h[(src[i] >> shift) & (NB - 1)]++;
#pragma omp barrier
#pragma omp single
      {
        int64_t run = 0;
        for (int d = 0; d < NB; ++d)
          for (int tt = 0; tt < nt; ++tt) {
            int64_t c = hist[(size_t)tt * NB + d];
            hist[(size_t)tt * NB + d] = run;
            run += c;
          }
      }
      for (int64_t i = lo; i < hi; ++i) {
        int64_t pos = h[(src[i] >> shift) & (NB - 1)]++;
        dst[pos] = src[i];
        if (psrc) pdst[pos] = psrc[i];
      }
    }
    uint64_t* tk = src; src = dst; dst = tk;
    uint32_t* tp = psrc; psrc = pdst; pdst = tp;
  }
  if (src != key) {
    memcpy(key, src, (size_t)n * sizeof(uint64_t));
    if (pay) memcpy(pay, psrc, (size_t)n * sizeof(uint32_t));
  }
  free(k2); free(p2); free(hist);
}

static int gg_bits_for(uint64_t v) { int b = 0; while (v) { ++b; v >>= 1; } return b; }

/* Sort keys ascending and drop repeats in place; returns the unique count. */
static int64_t gg_sort_unique(uint64_t* key, int64_t n, int bits) {
  gg_radix_sort_u64(key, NULL, n, bits);
  int64_t u = 0;
  for (int64_t i = 0; i < n; ++i)
    if (i == 0 || key[i] != key[i - 1]) key[u++] = key[i];
  return u;
}

/* Random permutation of 0..n-1 (Fisher-Yates driven by the counter stream). */
static void gg_permutation(int64_t n, uint64_t seed, uint64_t stream, int32_t* perm) {
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    uint64_t r = gg_draw(seed, stream, (uint64_t)i);
    int64_t j = (int64_t)(r % (uint64_t)(i + 1));
    int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
  }
}

/* ------------------------------------------------------------------ R-MAT */
/* m draws on 2^scale nodes.  src/dst must hold m entries; the unique edges are
 * written sorted by (src, dst) and their count returned in *n_edges. */
int gg_rmat(int scale, int64_t m, double a, double b, double c, uint64_t seed,
            int32_t* src, int32_t* dst, int64_t* n_edges) {
  if (scale < 1 || scale > 30 || m < 0) return -1;
  uint64_t* key = (uint64_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(uint64_t));
  if (!key) return -2;
  const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    uint64_t s = 0, d = 0;
    for (int l = 0; l < scale; ++l) {
      /* level-major counter: level l of edge e is draw l*m + e */
      double u = gg_unif(seed, 0, (uint64_t)l * (uint64_t)m + (uint64_t)e);
      int sb = 0, db = 0;
      if (u < a) { }
      else if (u < ab) db = 1;
      else if (u < abc) sb = 1;
      else { sb = 1; db = 1; }
      s = (s << 1) | (uint64_t)sb;
      d = (d << 1) | (uint64_t)db;
    }
    key[e] = (s << scale) | d;
  }
  int64_t u = gg_sort_unique(key, m, 2 * scale);
  uint64_t mask = (1ULL << scale) - 1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < u; ++i) {
    src[i] = (int32_t)(key[i] >> scale);
    dst[i] = (int32_t)(key[i] & mask);
  }
  *n_edges = u;
  free(key);
  return 0;
}

/* --------------------------------------------------------------- Chung-Lu */
static void gg_chung_lu_weights(int64_t n, double gamma, double total, double cap, double* w) {
  double ex = -1.0 / (gamma - 1.0);
  for (int64_t i = 0; i < n; ++i) w[i] = pow((double)(i + 1), ex);
  /* scale to `total`, cap, and rescale the uncapped part until no new caps */
  char* capped = (char*)calloc((size_t)n, 1);
  for (int it = 0; it < 100; ++it) {
    double sc = 0.0, su = 0.0;
    int64_t ncap = 0;
    for (int64_t i = 0; i < n; ++i) {
      if (capped[i]) { sc += cap; ++ncap; } else su += w[i];
    }
    double f = (total - sc) / su;
    int changed = 0;
    for (int64_t i = 0; i < n; ++i) {
      if (capped[i]) { w[i] = cap; continue; }
      w[i] *= f;
      if (w[i] > cap) { capped[i] = 1; w[i] = cap; changed = 1; }
    }
    if (!changed) break;
  }
  free(capped);
}

/* Walker alias table (Vose's construction): O(1) sampling in proportion to w. */
static void gg_alias_build(int64_t n, const double* w, double* prob, int32_t* alias) {
  double tot = 0.0;
  for (int64_t i = 0; i < n; ++i) tot += w[i];
  int32_t* small = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int32_t* large = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int64_t ns = 0, nl = 0;
  for (int64_t i = 0; i < n; ++i) {
    prob[i] = w[i] * (double)n / tot;
    alias[i] = (int32_t)i;
    if (prob[i] < 1.0) small[ns++] = (int32_t)i; else large[nl++] = (int32_t)i;
  }
  while (ns > 0 && nl > 0) {
    int32_t s = small[--ns], l = large[--nl];
    alias[s] = l;
    prob[l] = (prob[l] + prob[s]) - 1.0;
    if (prob[l] < 1.0) small[ns++] = l; else large[nl++] = l;
  }
  while (nl > 0) prob[large[--nl]] = 1.0;
  while (ns > 0) prob[small[--ns]] = 1.0;
  free(small); free(large);
}

/* one 53-bit uniform: integer part of u*n picks the column, the fraction the side */
static inline int32_t gg_alias_pick(const double* prob, const int32_t* alias, int64_t n, double u) {
  double t = u * (double)n;
  int64_t i = (int64_t)t;
  if (i >= n) i = n - 1;
  return (t - (double)i) < prob[i] ? (int32_t)i : alias[i];
}

/* 2^log2n nodes, exactly `target` distinct directed edges (if reachable).
 * src/dst must hold `target` entries; output sorted by (src, dst). */
int gg_chung_lu(int log2n, int64_t target, double gamma, double cap, uint64_t seed,
                int32_t* src, int32_t* dst, int64_t* n_edges) {
  if (log2n < 1 || log2n > 30 || target < 0 || gamma <= 1.0) return -1;
  int64_t n = (int64_t)1 << log2n;
  double* w = (double*)malloc((size_t)n * sizeof(double));
  double* w_in = (double*)malloc((size_t)n * sizeof(double));
  double* prob_out = (double*)malloc((size_t)n * sizeof(double));
  double* prob_in = (double*)malloc((size_t)n * sizeof(double));
  int32_t* alias_out = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int32_t* alias_in = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int32_t* sig = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int32_t* pi = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  if (!w || !w_in || !prob_out || !prob_in || !alias_out || !alias_in || !sig || !pi) return -2;
  gg_chung_lu_weights(n, gamma, (double)target, cap, w);
  gg_permutation(n, seed, 1, sig);   /* in-weight of node i is w[sig[i]] */
  gg_permutation(n, seed, 2, pi);    /* final relabelling i -> pi[i] */
  for (int64_t i = 0; i < n; ++i) w_in[i] = w[sig[i]];
  gg_alias_build(n, w, prob_out, alias_out);
  gg_alias_build(n, w_in, prob_in, alias_in);

  int64_t D = target + target / 4 + 1024;
  uint64_t* key = NULL;
  uint32_t* idx = NULL;
  int64_t uniq = 0;
  const int kb = 2 * log2n;
  for (int round = 0; round < 16; ++round) {
    key = (uint64_t*)realloc(key, (size_t)D * sizeof(uint64_t));
    idx = (uint32_t*)realloc(idx, (size_t)D * sizeof(uint32_t));
    if (!key || !idx) return -2;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < D; ++i) {
      int32_t s = gg_alias_pick(prob_out, alias_out, n, gg_unif(seed, 3, 2 * (uint64_t)i));
      int32_t d = gg_alias_pick(prob_in, alias_in, n, gg_unif(seed, 3, 2 * (uint64_t)i + 1));
      key[i] = ((uint64_t)s << log2n) | (uint64_t)d;
      idx[i] = (uint32_t)i;
    }
    /* stable sort keeps draw order inside each run of equal keys */
    gg_radix_sort_u64(key, idx, D, kb);
    uniq = 0;
    for (int64_t i = 0; i < D; ++i)
      if (i == 0 || key[i] != key[i - 1]) ++uniq;
    if (uniq >= target || D > ((int64_t)1 << 32) - 1) break;
    D = D + 2 * (target - uniq) + 1024;
  }
  /* keep the first `target` distinct edges in draw order */
  char* first = (char*)calloc((size_t)D, 1);
  uint64_t* kfirst = (uint64_t*)malloc((size_t)D * sizeof(uint64_t));
  for (int64_t i = 0; i < D; ++i)
    if (i == 0 || key[i] != key[i - 1]) { first[idx[i]] = 1; kfirst[idx[i]] = key[i]; }
  int64_t kept = 0;
  for (int64_t i = 0; i < D && kept < target; ++i)
    if (first[i]) key[kept++] = kfirst[i];
  free(first); free(kfirst); free(idx);
  /* relabel and sort by (src, dst) */
  uint64_t mask = ((uint64_t)1 << log2n) - 1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < kept; ++i) {
    uint64_t s = (uint64_t)pi[key[i] >> log2n], d = (uint64_t)pi[key[i] & mask];
    key[i] = (s << log2n) | d;
  }
  gg_radix_sort_u64(key, NULL, kept, kb);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < kept; ++i) {
    src[i] = (int32_t)(key[i] >> log2n);
    dst[i] = (int32_t)(key[i] & mask);
  }
  *n_edges = kept;
  free(key); free(w); free(w_in); free(prob_out); free(prob_in); free(alias_out); free(alias_in);
  free(sig); free(pi);
  return 0;
}

/* ------------------------------------------------------------ matrices */
/* Stable counting sort of entries by row: entries arrive in the caller's order
 * and keep it inside each row. */
static void gg_rows_to_csr(int64_t n_rows, int64_t nnz, const int32_t* row, const int32_t* col,
                           int64_t* row_ptr, int32_t* col_out, int64_t* pos_out) {
  memset(row_ptr, 0, (size_t)(n_rows + 1) * sizeof(int64_t));
  for (int64_t k = 0; k < nnz; ++k) row_ptr[row[k] + 1]++;
  for (int64_t i = 0; i < n_rows; ++i) row_ptr[i + 1] += row_ptr[i];
  int64_t* fill = (int64_t*)malloc((size_t)(n_rows + 1) * sizeof(int64_t));
  memcpy(fill, row_ptr, (size_t)(n_rows + 1) * sizeof(int64_t));
  for (int64_t k = 0; k < nnz; ++k) {
    int64_t p = fill[row[k]]++;
    col_out[p] = col[k];
    if (pos_out) pos_out[p] = k;
  }
  free(fill);
}

/* M[v][u] = fl32(1/outdeg(u)) for every edge u -> v.  Edges must be sorted by
 * (src, dst) so rows come out with ascending column ids. */
int gg_pagerank_csr(int64_t n, int64_t nnz, const int32_t* src, const int32_t* dst,
                    int64_t* row_ptr, int32_t* col, float* val) {
  int32_t* outdeg = (int32_t*)calloc((size_t)n, sizeof(int32_t));
  if (!outdeg) return -2;
  for (int64_t k = 0; k < nnz; ++k) {
    if (src[k] < 0 || src[k] >= n || dst[k] < 0 || dst[k] >= n) { free(outdeg); return -1; }
    outdeg[src[k]]++;
  }
  gg_rows_to_csr(n, nnz, dst, src, row_ptr, col, NULL);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < nnz; ++k) val[k] = 1.0f / (float)outdeg[col[k]];
  free(outdeg);
  return 0;
}

/* B = [[0, A^T], [A, 0]] with A[u][v] = 1 for edge u -> v:
 *   row v     (authority part) holds column n + u,
 *   row n + u (hub part)       holds column v. */
int gg_hits_csr(int64_t n, int64_t nnz, const int32_t* src, const int32_t* dst,
                int64_t* row_ptr, int32_t* col, float* val) {
  int64_t m = 2 * nnz;
  int32_t* r = (int32_t*)malloc((size_t)m * sizeof(int32_t));
  int32_t* c = (int32_t*)malloc((size_t)m * sizeof(int32_t));
  if (!r || !c) return -2;
  /* A^T block first (columns n+u ascend because edges are sorted by src),
   * then the A block (columns v ascend inside each src). */
  for (int64_t k = 0; k < nnz; ++k) { r[k] = dst[k]; c[k] = (int32_t)(n + src[k]); }
  for (int64_t k = 0; k < nnz; ++k) { r[nnz + k] = (int32_t)(n + src[k]); c[nnz + k] = dst[k]; }
  gg_rows_to_csr(2 * n, m, r, c, row_ptr, col, NULL);
  for (int64_t k = 0; k < m; ++k) val[k] = 1.0f;
  free(r); free(c);
  return 0;
}

/* Symmetrised, deduplicated adjacency, column-normalised.  col/val must hold
 * 2*nnz entries; the entry count is returned in *nnz_out. */
int gg_rwr_csr(int64_t n, int64_t nnz, const int32_t* src, const int32_t* dst,
               int64_t* row_ptr, int32_t* col, float* val, int64_t* nnz_out) {
  int lb = gg_bits_for((uint64_t)(n > 1 ? n - 1 : 1));
  uint64_t* key = (uint64_t*)malloc((size_t)(2 * nnz + 1) * sizeof(uint64_t));
  if (!key) return -2;
  for (int64_t k = 0; k < nnz; ++k) {
    key[2 * k] = ((uint64_t)dst[k] << lb) | (uint64_t)src[k];
    key[2 * k + 1] = ((uint64_t)src[k] << lb) | (uint64_t)dst[k];
  }
  int64_t u = gg_sort_unique(key, 2 * nnz, 2 * lb);
  int32_t* deg = (int32_t*)calloc((size_t)n, sizeof(int32_t));
  uint64_t mask = ((uint64_t)1 << lb) - 1;
  memset(row_ptr, 0, (size_t)(n + 1) * sizeof(int64_t));
  for (int64_t k = 0; k < u; ++k) {
    int32_t i = (int32_t)(key[k] >> lb), j = (int32_t)(key[k] & mask);
    col[k] = j;
    row_ptr[i + 1]++;
    deg[j]++;
  }
  for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] += row_ptr[i];
  for (int64_t k = 0; k < u; ++k) val[k] = 1.0f / (float)deg[col[k]];
  *nnz_out = u;
  free(key); free(deg);
  return 0;
}

/* x[i] uniform in [0,1): 24 random bits, exactly representable in FP32. */
void gg_uniform_f32(int64_t n, uint64_t seed, float* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    out[i] = (float)(gg_draw(seed, 4, (uint64_t)i) >> 40) * (1.0f / 16777216.0f);
}

/* Uniform integers in [0, bound). */
void gg_uniform_int(int64_t n, uint64_t seed, int64_t bound, int64_t* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = (int64_t)(gg_draw(seed, 5, (uint64_t)i) % (uint64_t)bound);
}

/* Random permutation (exported for seed selection in callers). */
void gg_random_permutation(int64_t n, uint64_t seed, int32_t* perm) {
  gg_permutation(n, seed, 6, perm);
}
