/*
 * tcspmv.h -- tiled composite sparse matrix-vector products for power-law
 * graph matrices on AMD Instinct MI355X (gfx950), and the PageRank, HITS and
 * Random Walk with Restart power iterations built on them.
 *
 * Method: Yang, Parthasarathy, Sadayappan, "Fast Sparse Matrix-Vector
 * Multiplication on GPUs: Implications for Graph Mining" (arXiv 1103.2405).
 *   - columns reordered by decreasing length and the long ones cut into column
 *     tiles so each tile reads one segment of x (Section 3.1, Solutions 1-2);
 *   - inside each tile, rows sorted by length and packed into balanced
 *     workloads, row-major when at least as wide as tall, else column-major,
 *     padded to the wavefront width (Solution 3); the remaining short columns
 *     form one more such tile;
 *   - the number of tiles and each tile's workload size chosen by Algorithms
 *     1-3 and the performance model of Eq. 1-5 (Section 3.3, Appendix E).
 *
 * Conventions for every call below:
 *   - Matrices are given in CSR with 64-bit row offsets, 32-bit column ids and
 *     FP32 values; vectors are FP32.  Pointers named d_* or documented as
 *     "device" are device memory owned by the caller; they must stay valid
 *     until the work queued on `stream` has finished.
 *   - Every call is asynchronous on `stream` (a hipStream_t) unless it says it
 *     synchronises.  Calls on one handle must not overlap on different streams.
 *   - Errors: every call returns a tc_status; on anything but TC_OK,
 *     tc_last_error() gives a message (per thread).  No call aborts the process.
 *   - Index space: tc_spmv / tc_spmm take x and return y in the caller's own
 *     row and column ids; the *_internal variants and the drivers' inner loops
 *     work in the handle's relabelled ids (columns sorted by length; for a
 *     square matrix rows carry the same relabelling).
 */
#ifndef TCSPMV_H
#define TCSPMV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* identical to hipStream_t */
typedef struct ihipStream_t* tc_stream_t;

typedef enum {
  TC_OK = 0,
  TC_EINVAL = 1,        /* invalid argument or invalid CSR */
  TC_ENOMEM = 2,        /* a device allocation failed */
  TC_EHIP = 3,          /* a HIP runtime call failed */
  TC_ENOTCONV = 4,      /* a driver did not reach its tolerance in max_iter */
  TC_EUNSUPPORTED = 5   /* valid but not supported (e.g. nnz >= 2^31) */
} tc_status;

typedef struct tc_handle tc_handle;

/* A sparse matrix in CSR form, all arrays in device memory, read only.
 *   row_ptr: n_rows + 1 offsets, row_ptr[0] = 0, non-decreasing, row_ptr[n_rows] = nnz
 *   col_idx: nnz column ids in [0, n_cols)
 *   val:     nnz values (finite: a stored 0 times inf would not be 0) */
typedef struct {
  int64_t n_rows, n_cols, nnz;
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const float* val;
} tc_csr;

/* Build options (tc_build_opts_default fills the defaults). */
typedef struct {
  int32_t tile_width;         /* W, columns per dense tile (Solution 1); 0 = 2^23 (32 MB of x,
                                 measured best on MI355X for power-law graphs up to 2^23 nodes)
                                 without row panels, and with automatic panels the largest power
                                 of two of columns whose x fills at most half of one XCD's L2
                                 (2^19 with MI355X's 4 MB) */
  int32_t n_tiles;            /* -1: Algorithm 1 decides; >= 0: that many dense tiles (clipped) */
  int32_t wl_policy;          /* 0: Algorithm 2 per tile; 1: wl_per_tile; 2: wl_all for every tile */
  int32_t wl_all;             /* workload size for wl_policy 2 */
  const int32_t* wl_per_tile; /* host array, one size per tile (dense tiles, then the sparse
                                 tile), at least as long as the number of tiles built */
  int32_t n_wl_per_tile;      /* length of wl_per_tile */
  int32_t wave;               /* padding multiple S of workloads; 0 = 64 (the wavefront width) */
  int32_t split_len;          /* rows longer than this many entries in a tile are split
                                 across wavefronts in chunks of this size; 0 = never
                                 (the paper's rule); -1 = automatic per tile (default):
                                 the tile's nnz per resident wavefront, rounded up to a
                                 multiple of the wave width, within [wave, 8192] */
  int32_t camping_pad;        /* 1: 64 pad elements after workloads whose size is a multiple
                                 of 512 (Solution 3, partition camping); default 0 */
  int32_t relabel;            /* -1: relabel rows like columns when square; 0: keep row ids */
  int32_t max_act_warp;       /* resident wavefronts assumed by the model (Eq. 1); 0 = 8192 */
  int32_t xcd_groups;         /* 0: tiles of Algorithm 1 run one after the other (default);
                                 G > 0: MI355X schedule -- tile 0 = columns [0, W), then G
                                 column ranges holding equal numbers of entries, run together
                                 with range g pinned to XCD g-1 and summed afterwards */
  int32_t kernel;             /* 0: TILE-COMPOSITE (padded row-major / column-major workloads,
                                 Solution 3; default).  1: TILE-COO -- each tile's entries in
                                 coordinate form, equal intervals per wavefront and a segmented
                                 sum (Section 3.1, Observation 3); the composite workloads are
                                 still built (SpMM and the metadata use them) */
  int32_t value_map;          /* 1: keep, for every padded slot, the CSR entry it holds (4 bytes
                                 per slot on the device), so tc_refresh_values can put new values
                                 of the same pattern in place without a rebuild.  Composite
                                 kernel only; default 0 */
  int32_t slices;             /* row slices per workload of the single-vector tile kernels: 0 =
                                 automatic (4 on tiles of at least 4096 workloads of at least
                                 1024 entries, else 1); 1, 2, 4 or 8 = that count on every
                                 tile.  Each row is summed whole, in the same order, by one lane
                                 or one wavefront, so the result does not depend on it */
  const int32_t* tile_bounds; /* host array of n_tile_bounds increasing internal column ids in
                                 (0, n_cols]: dense tiles [0, b0), [b0, b1), ... [b_{k-2}, b_{k-1}),
                                 then the sparse tile [b_{k-1}, n_cols) when b_{k-1} < n_cols.
                                 Tiles of different widths (Solution 1 with one width per cache
                                 level); tile_width and n_tiles are then not used.  NULL = none */
  int32_t n_tile_bounds;      /* length of tile_bounds (0 = none) */
  int32_t lds_stage;          /* 0 (default): a tile no wider than one workgroup's LDS (160 KB,
                                 40960 columns) with at least 8 entries per float staged has its
                                 x segment staged in LDS by a persistent kernel, so its gathers
                                 are LDS reads; 1: every tile that fits is staged; -1: every
                                 tile gathers x through the caches */
  int32_t panels;             /* row panels (MI355X reading of Section 3.2's row partition, applied
                                 to the workgroups of one GPU): 0 (default) = none; P > 0 = P
                                 panels; -1 = automatic: min(compute units, ceil(n_rows / 2048))
                                 panels of up to 17/16 of an even share of rows (rounded up to 64)
                                 unless panel_rows is given, and, unless tile_bounds is given, a
                                 head tile of the columns that fit in the LDS left behind y (a
                                 multiple of 1024, staged in LDS), then tiles of tile_width
                                 (default: half an XCD's L2 of x) columns by Algorithm 1's rule, then the sparse
                                 tile; with wl_policy 0 and split_len -1 the panel tiles then
                                 take workloads of 512 entries and split rows longer than 1024
                                 (measured best here for a build and 100 products: Algorithm
                                 2's sizes save 1% of each product but cost 7 ms of build
                                 over the thousands of panel tiles).  Internal rows are cut into contiguous panels of at
                                 most panel_rows rows holding about equal numbers of the entries
                                 that stay with their row (a segment longer than its column
                                 tile's split length is chunked and belongs to no panel); every
                                 (panel, column tile) pair is a tile of the format, panel-major.
                                 One workgroup per panel keeps the panel's y in LDS and sweeps
                                 the column tiles in order.  Not with xcd_groups or kernel = 1 */
  int32_t panel_rows;         /* most rows of a panel; 0 = half the LDS of a compute unit, in
                                 floats (20480 on gfx950); at most one workgroup's LDS */
  int32_t panel_waves;        /* wavefronts of a panel's workgroup (4, 8 or 16; 0 = 16), also the
                                 resident wavefronts of Eq. 1 when Algorithm 2 sizes the
                                 workloads of a panel's tile */
  const char* perf_table;     /* path of a throughput table for the model; NULL = built-in */
  /* optional device allocator for the handle's buffers; NULL = hipMalloc / hipFree */
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* alloc_ctx;
} tc_build_opts;

/* Sizes and parameters of a built handle (host struct filled by tc_handle_info). */
typedef struct {
  int64_t n_rows, n_cols, nnz;
  int32_t tile_width, wave, split_len, relabel;  /* split_len as given (-1 = automatic) */
  int32_t xcd_groups, kernel;
  int32_t n_dense_tiles;      /* T of Algorithm 1 */
  int32_t n_tiles;            /* T plus one if a sparse tile exists */
  int64_t n_workloads;
  int64_t nnz_pad;            /* stored elements, pads included */
  int64_t n_rowid;            /* stored row ids */
  int64_t n_rows_sorted;      /* sum over tiles of the tile's non-empty rows */
  int64_t n_split_rows;       /* heavy rows split across wavefronts */
  int64_t n_partials;         /* chunks of split rows */
  int64_t n_dangling;         /* empty columns; internal ids n_cols - n_dangling .. n_cols-1 */
  int64_t device_bytes;       /* device memory held by the handle */
  double build_us;            /* wall time of tc_build_tiled */
  double model_us;            /* Eq. 1-5 prediction for one product with the built workload sizes, summed
                                 over tiles (microseconds; the throughput table is in entries per us) */
  int32_t n_panels;           /* row panels (0 = none); tile g is panel g / n_col_tiles, column
                                 tile g % n_col_tiles */
  int32_t n_col_tiles;        /* column tiles (dense tiles plus the sparse tile) */
  int32_t panel_rows;         /* most rows per panel used by the build (0 without panels) */
  int32_t panel_waves;        /* wavefronts per panel workgroup (0 without panels) */
} tc_info;

/* Host copies of the whole format, for checking it entry by entry.  The caller
 * allocates every array (sizes from tc_info; a NULL pointer skips that array). */
typedef struct {
  int32_t* cperm;             /* [n_cols]  internal column -> original column */
  int32_t* rowmap;            /* [n_rows]  original row -> internal row */
  int64_t* tile_col_begin;    /* [n_tiles] first internal column of each tile */
  int64_t* tile_col_end;      /* [n_tiles] one past the last */
  int64_t* tile_nnz;          /* [n_tiles] */
  int64_t* tile_wl;           /* [n_tiles] workload size used */
  int64_t* tile_split;        /* [n_tiles] split length used (0 = none) */
  int64_t* tile_row_off;      /* [n_tiles + 1] offsets into rows_sorted */
  int32_t* rows_sorted;       /* [n_rows_sorted] each tile's rows by decreasing length */
  int32_t* rows_len;          /* [n_rows_sorted] the row's entries in that tile */
  int32_t* wl_tile;           /* [n_workloads] ... one entry per workload ... */
  int32_t* wl_layout;         /* 0 row-major, 1 column-major (a split chunk is row-major) */
  int32_t* wl_w;              /* width of the first row (chunk: the chunk's length) */
  int32_t* wl_w_pad;          /* stored row length (RM) or w (CM) */
  int32_t* wl_h_pad;          /* stored rows: h (RM), padded rows (CM), 1 (chunk) */
  int32_t* wl_row_begin;      /* index of the first row in rows_sorted */
  int32_t* wl_n_rows;         /* real rows */
  int32_t* wl_chunk;          /* chunk index of a split row, -1 otherwise */
  int32_t* wl_n_chunks;       /* chunks of that split row in this tile, 0 otherwise */
  int64_t* wl_data_off;       /* first element in idx / val */
  int64_t* wl_rowid_off;      /* first entry in rowid */
  int32_t* idx;               /* [nnz_pad] internal column id; pads: the tile's first column */
  float* val;                 /* [nnz_pad] value; pads: +0.0 */
  int32_t* rowid;             /* [n_rowid] internal row id; pad rows: -1 */
  /* TILE-COO handles only ([nnz], tile t at offset sum of tile_nnz before t): */
  int32_t* coo_row;           /* internal row id, bit 30 set when an earlier tile holds the row */
  int32_t* coo_col;           /* internal column id */
  float* coo_val;             /* value */
  /* handles built with row panels only: */
  int64_t* panel_begin;       /* [n_panels + 1] first internal row of each panel, then n_rows */
} tc_format_view;

/* Accumulated time of the tile kernels when timing is enabled (tc_set_timing). */
typedef struct {
  double tile_kernel_ms;      /* sum of per-launch durations (HIP events) */
  int64_t tile_launches;
  int64_t spmv_calls;         /* products run (each = one pass over all tiles) */
} tc_timing;

void tc_build_opts_default(tc_build_opts* opts);

/* Build the tiled composite format of `A` on the GPU (Section 3.1 Solutions
 * 1-3; Section 3.3 and Algorithms 1-3 for the tile count and workload sizes).
 * Steps: column lengths, columns sorted by decreasing length (ties by id),
 * tile count, entries bucketed by tile, each tile's rows sorted by decreasing
 * length (ties by internal row id), workloads chosen and packed.  The handle
 * owns all its device memory; A may be freed once this call returns.
 * Synchronises `stream`.  Errors: TC_EINVAL for a NULL argument, negative
 * sizes, a non-monotone row_ptr, row_ptr[n_rows] != nnz, a column id out of
 * range or an unusable option; TC_EUNSUPPORTED for nnz >= 2^31, n_rows >= 2^30 or
 * n_cols >= 2^31 - 1; TC_ENOMEM; TC_EHIP.  The per-tile host work runs on a
 * pool of up to 16 threads kept for the life of the process; TC_HOST_THREADS=n
 * in the environment (read when the pool starts) sets its size, 1 keeping all
 * of it on the calling thread. */
tc_status tc_build_tiled(const tc_csr* A, const tc_build_opts* opts, tc_stream_t stream,
                         tc_handle** out);

/* y := A x (overwrite) in the caller's index space (Appendix B: y = A x for an
 * n x m sparse A).  d_x: n_cols floats, d_y: n_rows floats, device, must not
 * alias.  Tiles are applied in order, dense tiles first, then the sparse tile;
 * each row's sum is formed in FP64 and added to y in FP32 once per tile. */
tc_status tc_spmv(const tc_handle* h, const float* d_x, float* d_y, tc_stream_t stream);

/* y := A x with x and y in the handle's internal ids (no permutation). */
tc_status tc_spmv_internal(const tc_handle* h, const float* d_x, float* d_y, tc_stream_t stream);

/* As tc_spmv_internal, but always one launch per tile in tile order (the
 * paper's scheme of one kernel per tile, Section 3.1), also for a handle built
 * with row panels, whose products otherwise run as one row-panel launch.  Both
 * orders add each row's per-tile sums in the same order, so for a panel handle
 * the two give the same bits; this call exists to check that.  Same arguments,
 * ownership and errors as tc_spmv_internal. */
tc_status tc_spmv_tiles(const tc_handle* h, const float* d_x, float* d_y, tc_stream_t stream);

/* Y := A X for k right-hand sides: X is n_cols x k and Y n_rows x k, both
 * row-major, device, caller's index space; 1 <= k <= 256. */
tc_status tc_spmm(const tc_handle* h, const float* d_X, float* d_Y, int32_t k, tc_stream_t stream);

/* Y := A X like tc_spmm, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): X (n_cols x k) and Y (n_rows x k) are row-major in the
 * handle's internal ids (row i of X is the caller's row cperm[i], see
 * tc_export_format; Y's row rowmap[r] is the caller's row r), so no staging
 * copies are needed, and the split rows' partial sums go to a file-scope
 * device array of 16 MiB per GPU (held until the process ends) instead of
 * the handle's pool.  The call allocates nothing and is not timed by
 * tc_set_timing.  Calls that overlap on one GPU share that array and race.
 * Same kernels and order as tc_spmm, so the same bits.  Errors: TC_EINVAL for
 * NULL arguments, k outside [1, 256], X == Y, or partial sums larger than the
 * array (n_partials * pieces * k doubles); TC_EHIP. */
tc_status tc_spmm_internal_noalloc(const tc_handle* h, const float* d_X, float* d_Y, int32_t k, tc_stream_t stream);

/* PageRank (Appendix F, Eq. 6): M must be the handle of the column-stochastic
 * matrix W^T (M[v][u] = 1/outdeg(u)); empty columns are dangling nodes whose
 * mass is spread uniformly.  p^(0) = 1/n;
 *   p' = c (M p + (d/n) 1) + ((1-c)/n) 1,  d = sum of p over dangling nodes.
 * Stops when the L1 change is <= tol, checked every check_every iterations
 * (that check synchronises); tol <= 0 runs exactly max_iter iterations with no
 * synchronisation until the end.  d_p_out: n floats (device, caller's ids).
 * *iters: iterations run; *resid: L1 change of the last iteration (FP64
 * reduction).  TC_ENOTCONV if tol > 0 was not reached (p_out still written). */
tc_status tc_pagerank(const tc_handle* M, float c, float tol, int32_t max_iter, int32_t check_every,
                      float* d_p_out, int32_t* iters, double* resid, tc_stream_t stream);

/* HITS (Appendix F, Eq. 7-8): B must be the handle of the 2n x 2n matrix
 * [[0, A^T], [A, 0]].  x^(0) = 1/n everywhere; each iteration x' = B x, then
 * the authority half (ids < n) and the hub half (ids >= n) are each divided by
 * their own sum.  d_auth, d_hub: n floats each (device).  Convergence as in
 * tc_pagerank on the L1 change of the 2n vector.  TC_EINVAL if a half sums to
 * zero (a graph without edges). */
tc_status tc_hits(const tc_handle* B, float tol, int32_t max_iter, int32_t check_every, float* d_auth,
                  float* d_hub, int32_t* iters, double* resid, tc_stream_t stream);

/* Random walk with restart (Appendix F, Eq. 9) for k query nodes at once:
 * r' = c W r + (1-c) e_s, r^(0) = e_s, W the handle of the column-normalised
 * adjacency (of the symmetrised graph for the paper's undirected setting).
 * seeds: host array of k node ids (caller's ids).  d_R: n x k row-major
 * (device).  Stops when every column's L1 change is <= tol (check as above);
 * *resid is the largest column change of the last iteration. */
tc_status tc_rwr(const tc_handle* W, const int32_t* seeds, int32_t k, float c, float tol,
                 int32_t max_iter, int32_t check_every, float* d_R, int32_t* iters, double* resid,
                 tc_stream_t stream);

/* RWR (Appendix F, Eq. 9) on many graphs at once, one query per graph.
 * handles[g] is built from graph g's matrix as for tc_rwr; seeds[g] is its
 * restart node (original id, host array); d_R[g] (host array of device
 * pointers) receives its n_g scores in original ids.  Every launch covers all
 * graphs: tile t of each, the split rows of each, then the update of each, so
 * small graphs share the GPU.  Stopping as in tc_rwr with the largest per-graph
 * L1 change; resid (host array of n_graphs, may be NULL) gets each graph's last
 * change.  flags bit 0: capture the iterations between checks in a HIP graph
 * once and replay it (kernels only; results are identical to eager launches).
 * Handles built with the XCD schedule are rejected (TC_EUNSUPPORTED).  The
 * call synchronises `stream`. */
tc_status tc_rwr_multi(tc_handle* const* handles, int32_t n_graphs, const int32_t* seeds, float c, float tol,
                       int32_t max_iter, int32_t check_every, int32_t flags, float* const* d_R, int32_t* iters,
                       double* resid, tc_stream_t stream);

/* ---- Differentiable RWR: learned edge weights (Appendix F, Eq. 9) ----------
 * For a square pattern A (n x n, entries e = (i, j), CSR rp/col on the device)
 * with nf features per entry (d_feats, nnz x nf row-major):
 *   z_e = theta . f_e,  w_e = softplus(z_e),  W_e = w_e / S_j  (S_j: sum of w over column j),
 *   r^0 = e_s,  r^{k+1} = c W r^k + (1 - c) e_s.
 * The gradient of a loss on r^K runs back through the iteration:
 *   g^k = c W^T g^{k+1}   (tiled SpMV on a build of W^T),
 *   dL/dW_e = c sum_k g^{k+1}_i r^k_j,
 * then through the normalisation and the softplus to theta.  Vectors are in
 * the caller's ids; every FP64 sum below has a fixed order. */

/* CSR of A^T (n_cols x n_rows): d_rpT (n_cols + 1), d_colT and d_valT (nnz)
 * and d_permT (nnz; entry e' of A^T is entry d_permT[e'] of A).  Each row of
 * A^T lists its entries by increasing row of A.  d_colT, d_valT and d_permT
 * may be NULL.  Validates A like tc_build_tiled.  Synchronous. */
tc_status tc_csr_transpose(const tc_csr* A, int64_t* d_rpT, int32_t* d_colT, float* d_valT, int32_t* d_permT,
                           tc_stream_t stream);

/* Row gather: row q of d_dst (n rows of `width` floats) is row d_idx[q] of
 * d_src (n_src rows).  Puts the per-entry features of the learned weights
 * into A^T's order (d_idx = d_permT of tc_csr_transpose).  Indices outside
 * [0, n_src) give TC_EINVAL before anything is written.  Synchronous. */
tc_status tc_gather_rows(const float* d_src, int64_t n_src, const int32_t* d_idx, int64_t n, int32_t width,
                         float* d_dst, tc_stream_t stream);

/* Learned edge weights (Appendix F, Eq. 9, with w = softplus(theta . f)):
 * for theta (host, nf <= 16 doubles) computes z and w (FP64, nnz, in A^T's
 * order), the column sums S (FP64, n_cols) and the FP32 values of W in A's
 * order (d_val) and in A^T's order (d_valT), bit-identical entry by entry.
 * d_feats holds nf floats per entry in A's order, d_featsT the same rows in
 * A^T's order (tc_gather_rows); d_col is A's column array and d_rpT A^T's
 * row pointers (tc_csr_transpose).  Synchronous. */
tc_status tc_rwr_edge_weights(int64_t n_cols, int64_t nnz, const int32_t* d_col, const int64_t* d_rpT, int32_t nf,
                              const float* d_feats, const float* d_featsT, const double* theta, double* d_zT,
                              double* d_wT, double* d_S, float* d_val, float* d_valT, tc_stream_t stream);

/* K RWR iterations on the handle of W from e_seed; d_rK receives r^K and
 * d_ckpt (ceil(K / every) x n) the checkpoints r^0, r^every, ...  Each step
 * rounds like tc_rwr, so r^K equals tc_rwr's with k = 1. */
tc_status tc_rwr_iterates(const tc_handle* W, int32_t seed, float c, int32_t K, int32_t every, float* d_ckpt,
                          float* d_rK, tc_stream_t stream);

/* Adjoint pass from d_gK = dL/dr^K: recomputes the iterates between
 * checkpoints (every x n scratch), and returns, for every entry (i, j) of A in
 * A^T's order, d_G = sum_k g^{k+1}_i r^k_j (FP64, nnz; dL/dW = c G) and, if
 * d_g0 is not NULL, g^0.  Wt is the handle built from A^T with W's values
 * (d_rpT, d_colT and d_valT); the sum of each entry runs latest step first,
 * so the result does not depend on `every`. */
tc_status tc_rwr_adjoint(const tc_handle* W, const tc_handle* Wt, const int64_t* d_rpT, const int32_t* d_colT,
                         int32_t seed, float c, int32_t K, int32_t every, const float* d_ckpt, const float* d_gK,
                         double* d_G, float* d_g0, tc_stream_t stream);

/* dL/dtheta (host, nf doubles) from d_G of tc_rwr_adjoint and the A^T-order
 * d_featsT, z, w and S of tc_rwr_edge_weights: through the column
 * normalisation and the softplus.  Synchronous. */
tc_status tc_rwr_theta_grad(int64_t n_cols, int64_t nnz, const int64_t* d_rpT, int32_t nf, const float* d_featsT,
                            const double* d_zT, const double* d_wT, const double* d_S, const double* d_G, float c,
                            double* dtheta, tc_stream_t stream);

/* Plain CSR SpMV, the baseline the tiled kernels are compared with: the
 * CSR-vector kernel of Appendix B (one wavefront per row, FP64 partial sums
 * reduced across it; Section 3.1, Observation 4).  y := A x in the caller's
 * ids, no handle; d_x and d_y are device arrays of n_cols and n_rows floats. */
tc_status tc_csr_spmv(const tc_csr* A, const float* d_x, float* d_y, tc_stream_t stream);

/* Measurement of the streaming-read rate the product kernels can reach (the
 * attainable side of the roofline, next to the nominal HBM peak): reads the n
 * floats of d_buf once, 16 bytes per load with the non-temporal loads of the
 * tile kernels, four loads in flight per thread, 8192 workgroups of 256
 * threads; each thread's sum is written to d_sink, which must hold
 * 8192 * 256 floats (device).  n must be a multiple of 4 and d_buf 16-byte
 * aligned (TC_EINVAL otherwise).  Asynchronous on `stream`; the caller times
 * it with events on that stream. */
tc_status tc_stream_read(const float* d_buf, int64_t n, float* d_sink, tc_stream_t stream);

/* Measurement of the random-gather rate the product kernels can reach (the
 * other attainable limit of the panel pass, whose x gathers cannot be
 * coalesced; Section 3.1 on the cost of gathering x): for each of the n
 * entries, reads d_idx[e] and d_val[e] (int32 and float, device) in coalesced
 * groups of 64 as a column-major workload does, then gathers d_x[d_idx[e]]
 * (d_x: n_x floats, device; by buffer loads with 32-bit offsets as the panel
 * pass does, when n_x <= 2^29); eight entries per lane in flight, 8192
 * workgroups of 256 threads, each thread's sum written to d_sink (8192 * 256
 * floats, device).  An index outside [0, n_x) reads d_x[0].  n must be a
 * multiple of 512 and n_x at least 1 (TC_EINVAL otherwise).  Asynchronous on
 * `stream`; the caller times it with events on that stream. */
tc_status tc_gather_read(const float* d_x, int64_t n_x, const int32_t* d_idx, const float* d_val, int64_t n,
                         float* d_sink, tc_stream_t stream);

/* Sizes and parameters of a handle (host, no GPU work). */
tc_status tc_handle_info(const tc_handle* h, tc_info* info);

/* New values for the pattern the handle was built from: d_val holds nnz
 * floats in the order of that CSR's entries (device).  The format's values
 * become exactly what a build from the same CSR with these values would hold;
 * nothing else changes.  Needs a handle built with value_map = 1 (else
 * TC_EINVAL).  Asynchronous on the stream; d_val may be released once the
 * stream reaches this point. */
tc_status tc_refresh_values(tc_handle* h, const float* d_val, tc_stream_t stream);

/* Copy the format to host arrays (synchronous). */
tc_status tc_export_format(const tc_handle* h, tc_format_view* view);

/* Time every tile-kernel launch with HIP events (enable = 1) or stop (0);
 * enabling also clears the totals. */
tc_status tc_set_timing(tc_handle* h, int32_t enable);
/* Read the totals (synchronises the handle's pending events). */
tc_status tc_get_timing(tc_handle* h, tc_timing* t);

/* Release the handle and all its device memory (waits for the device).  The
 * memory goes back to the library's device pool, where later builds on the
 * same device reuse it. */
void tc_destroy(tc_handle* h);

/* Return every block cached in the library's device pool to HIP (all
 * devices; synchronous), and free the host blocks the builder keeps for reuse
 * (page-locked transfer buffers, workload lists of destroyed handles).
 * Handles still alive keep their memory.  Returns the number of bytes
 * released, device and host together.  Setting TC_POOL=0 in the environment
 * before the first call disables both pools (every release then goes straight
 * to hipFree or free). */
size_t tc_release_cached_memory(void);

/* Message of the last failing call on this thread ("" if none). */
const char* tc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TCSPMV_H */
