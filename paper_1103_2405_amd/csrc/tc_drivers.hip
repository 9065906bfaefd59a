// The power iterations on a built handle (Appendix F): PageRank (Eq. 6), HITS
// (Eq. 7-8) and RWR (Eq. 9), with their vector updates, reductions in FP64
// and, on iterations whose convergence measure is not read, the update fused
// into the product.
#include <algorithm>
#include <cmath>
#include <vector>

#include "tc_host.h"

namespace tc {

namespace {

// The tile kernel with the fused PageRank update (PrX); d = *dmass, the
// dangling mass of x.
template <int S>
__global__ void __launch_bounds__(kB) k_tile_spmv_pr(const Wl* __restrict__ wl, int64_t n_wl,
                                                     const int32_t* __restrict__ idx, const float* __restrict__ val,
                                                     const int32_t* __restrict__ rowid, const float* __restrict__ x,
                                                     float* __restrict__ pn, double* __restrict__ partial, double c,
                                                     const double* __restrict__ dmass, int64_t n) {
  const int lane = lane_id();
  const int64_t w = (int64_t)blockIdx.x * kWpb + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (w >= n_wl * S) return;
  const Wl d = wl[w / S];
  run_workload<S>(d, lane, idx, val, rowid, PrX{x, c, *dmass / (double)n, (1.0 - c) / (double)n}, pn, partial,
                  (int32_t)(w % S));
}

// The tile kernel with the fused restart of a one-query RWR (RwrX); the seed
// is an internal id on the device.
template <int S>
__global__ void __launch_bounds__(kB) k_tile_spmv_rwr(const Wl* __restrict__ wl, int64_t n_wl,
                                                      const int32_t* __restrict__ idx, const float* __restrict__ val,
                                                      const int32_t* __restrict__ rowid, const float* __restrict__ x,
                                                      float* __restrict__ rn, double* __restrict__ partial, double c,
                                                      const int32_t* __restrict__ seed) {
  const int lane = lane_id();
  const int64_t w = (int64_t)blockIdx.x * kWpb + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (w >= n_wl * S) return;
  const Wl d = wl[w / S];
  run_workload<S>(d, lane, idx, val, rowid, RwrX{x, c, *seed}, rn, partial, (int32_t)(w % S));
}

// PageRank update (Eq. 6 with uniform dangling mass), fused with the L1
// change and the dangling mass of the new iterate:
//   p'_i = c (y_i + d/n) + (1-c)/n
// (ypriv, G): private copies of y of the XCD schedule still to be added, in
// g order, to y (G = 0 when there are none).
__global__ void __launch_bounds__(kB) k_pr_update(const float* __restrict__ y, const float* __restrict__ ypriv,
                                                  int32_t G, float* __restrict__ p, int64_t n, int64_t dang_begin,
                                                  double c, const double* __restrict__ dmass,
                                                  double* __restrict__ parts) {
  const double dn = *dmass / (double)n;
  const double tele = (1.0 - c) / (double)n;
  double v[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
    float yi = y[i];
    if (G > 0) {
      double s = (double)yi;
      for (int32_t g = 0; g < G; ++g) s += (double)ypriv[(int64_t)g * n + i];
      yi = (float)s;
    }
    const float pn = (float)(c * ((double)yi + dn) + tele);
    v[0] += fabs((double)pn - (double)p[i]);
    if (i >= dang_begin) v[1] += (double)pn;
    p[i] = pn;
  }
  block_sum_store<2>(v, parts + blockIdx.x, gridDim.x);
}

// sum of p over the dangling range (first iteration)
__global__ void __launch_bounds__(kB) k_range_sum(const float* __restrict__ p, int64_t b, int64_t e,
                                                  double* __restrict__ parts) {
  double v[1] = {0.0};
  for (int64_t i = b + (int64_t)blockIdx.x * kB + threadIdx.x; i < e; i += (int64_t)gridDim.x * kB) v[0] += (double)p[i];
  block_sum_store<1>(v, parts + blockIdx.x, gridDim.x);
}

// HITS: sums of the two halves of y
__global__ void __launch_bounds__(kB) k_hits_sums(const float* __restrict__ y, const int32_t* __restrict__ rowinv,
                                                  int64_t n2, int64_t n, double* __restrict__ parts) {
  double v[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n2; i += (int64_t)gridDim.x * kB)
  {
    if (rowinv[i] >= n)
      v[1] += (double)y[i];
    else
      v[0] += (double)y[i];
  }
  block_sum_store<2>(v, parts + blockIdx.x, gridDim.x);
}

// HITS: x' = y / (sum of its half), L1 change
__global__ void __launch_bounds__(kB) k_hits_update(const float* __restrict__ y, float* __restrict__ x,
                                                    const int32_t* __restrict__ rowinv, int64_t n2, int64_t n,
                                                    const double* __restrict__ sums, double* __restrict__ parts,
                                                    int* __restrict__ err) {
  const double sa = sums[0], sh = sums[1];
  if (blockIdx.x == 0 && threadIdx.x == 0 && (sa == 0.0 || sh == 0.0)) *err = 1;
  double v[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n2; i += (int64_t)gridDim.x * kB) {
    const double s = rowinv[i] >= n ? sh : sa;
    const float xn = s != 0.0 ? (float)((double)y[i] / s) : 0.0f;
    v[0] += fabs((double)xn - (double)x[i]);
    x[i] = xn;
  }
  block_sum_store<1>(v, parts + blockIdx.x, gridDim.x);
}

// Fused PageRank step, the rows the tile kernel does not write: split rows
// (their chunks' sums) and rows without entries (y = 0), same formula as PrX.
__global__ void k_pr_split_empty(const SplitRow* __restrict__ sr, int64_t n_split, const double* __restrict__ partial,
                                 const int32_t* __restrict__ empty, int64_t n_empty, float* __restrict__ pn, double c,
                                 const double* __restrict__ dmass, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double dn = *dmass / (double)n, tele = (1.0 - c) / (double)n;
  if (t < n_split) {
    const SplitRow s = sr[t];
    const double acc = sum_slots(partial + s.slot_begin, s.n_slots);
    pn[s.row] = (float)(c * ((double)(float)acc + dn) + tele);
  } else if (t < n_split + n_empty) {
    pn[empty[t - n_split]] = (float)(c * ((double)0.0f + dn) + tele);
  }
}

// Fused PageRank step with row panels, the split rows: their unsplit
// segments' sum (yraw, from the panel pass) plus their chunks, then the same
// formula as the panel pass; the rows without entries were written by it.
__global__ void __launch_bounds__(kB) k_pr_split_panel(const SplitRow* __restrict__ sr, int64_t n_split,
                                                        const double* __restrict__ partial,
                                                        const float* __restrict__ yraw, float* __restrict__ pn,
                                                        double c, const double* __restrict__ dmass, int64_t n) {
  // one wavefront per split row
  const int lane = lane_id();
  const int64_t t = (int64_t)blockIdx.x * kWpb + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (t >= n_split) return;
  __shared__ double buf[kWpb][4 * kWave];
  const SplitRow s = sr[t];
  const double acc = sum_slots_wave(partial + s.slot_begin, s.n_slots, lane, buf[threadIdx.x / kWave]);
  if (lane == 0) {
    const double dn = *dmass / (double)n, tele = (1.0 - c) / (double)n;
    const float yv = (float)((double)yraw[t] + acc);
    pn[s.row] = (float)(c * ((double)yv + dn) + tele);
  }
}

// Fused one-query RWR step, the rows the tile kernel does not write: split
// rows (their chunks' sums) and, when `empty` is given, rows without entries
// (y = 0), same formula as RwrX.
__global__ void k_rwr1_split_empty(const SplitRow* __restrict__ sr, int64_t n_split, const double* __restrict__ partial,
                                   const int32_t* __restrict__ empty, int64_t n_empty, float* __restrict__ rn,
                                   double c, const int32_t* __restrict__ seed) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t sd = *seed;
  if (t < n_split) {
    const SplitRow s = sr[t];
    const double acc = sum_slots(partial + s.slot_begin, s.n_slots);
    rn[s.row] = (float)(c * (double)(float)acc + (s.row == sd ? 1.0 - c : 0.0));
  } else if (empty && t < n_split + n_empty) {
    const int32_t row = empty[t - n_split];
    rn[row] = (float)(c * (double)0.0f + (row == sd ? 1.0 - c : 0.0));
  }
}

// Dangling mass of p, split over blocks exactly as k_pr_update splits it
// (same elements per thread, same order), into parts[blockIdx.x]
__global__ void __launch_bounds__(kB) k_dang_sum(const float* __restrict__ p, int64_t n, int64_t dang_begin,
                                                 double* __restrict__ parts) {
  const int64_t base = (int64_t)blockIdx.x * kB + threadIdx.x, stride = (int64_t)gridDim.x * kB;
  const int64_t i0 = base >= dang_begin ? base : base + (dang_begin - base + stride - 1) / stride * stride;
  double v[1] = {0.0};
  for (int64_t i = i0; i < n; i += stride) v[0] += (double)p[i];
  block_sum_store<1>(v, parts + blockIdx.x, gridDim.x);
}

// RWR: R' = c Y + (1-c) E, per-column L1 change (nq columns of k at q0)
__global__ void __launch_bounds__(kB) k_rwr_update(const float* __restrict__ Y, float* __restrict__ R, int64_t n,
                                                   int32_t k, double c, const int32_t* __restrict__ seeds,
                                                   double* __restrict__ parts, int nblocks) {
  // thread layout: each thread owns one column q (threadIdx.x % k) of rows
  // spaced by the grid; k <= 256
  const int32_t q = threadIdx.x % k;
  const int32_t rpb = kB / k;  // rows per block step
  const int32_t rr = threadIdx.x / k;
  __shared__ double sm[kB];
  double s = 0.0;
  if (rr < rpb) {
    const int32_t seed = seeds[q];
    const int64_t step = (int64_t)gridDim.x * rpb;
    for (int64_t i0 = (int64_t)blockIdx.x * rpb + rr; i0 < n; i0 += 4 * step) {
      float y[4], r[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {  // four rows' loads together (past n: row i0, not used)
        const int64_t e = (i0 + u * step < n ? i0 + u * step : i0) * k + q;
        y[u] = Y[e];
        r[u] = R[e];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t i = i0 + u * step;
        if (i < n) {
          const float rn = (float)(c * (double)y[u] + (i == seed ? (1.0 - c) : 0.0));
          s += fabs((double)rn - (double)r[u]);
          R[i * k + q] = rn;
        }
      }
    }
  }
  sm[threadIdx.x] = s;
  __syncthreads();
  if ((int32_t)threadIdx.x < k) {
    double t = 0.0;
    for (int32_t u = 0; u < rpb; ++u) t += sm[u * k + threadIdx.x];
    parts[(int64_t)threadIdx.x * nblocks + blockIdx.x] = t;
  }
}

__global__ void k_rwr_init(float* __restrict__ R, int64_t n, int32_t k, const int32_t* __restrict__ seeds) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * k) return;
  const int64_t i = t / k;
  const int32_t q = (int32_t)(t % k);
  R[t] = (i == seeds[q]) ? 1.0f : 0.0f;
}

__global__ void k_map_ids(const int32_t* __restrict__ ids, const int32_t* __restrict__ map, int32_t k,
                          int32_t* __restrict__ out) {
  for (int32_t q = threadIdx.x; q < k; q += blockDim.x) out[q] = map[ids[q]];
}

__global__ void k_max_of(const double* __restrict__ v, int n, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double m = 0.0;
    for (int i = 0; i < n; ++i) m = fmax(m, v[i]);
    *out = m;
  }
}

}  // namespace
}  // namespace tc

using namespace tc;

extern "C" tc_status tc_pagerank(const tc_handle* hc, float c, float tol, int32_t max_iter, int32_t check_every,
                                 float* p_out, int32_t* iters, double* resid, tc_stream_t stream) {
  return guarded("tc_pagerank", [&]() -> tc_status {
    if (!hc || (!p_out && hc->n_rows > 0)) throw Err{TC_EINVAL, "NULL argument"};
    if (!(c >= 0.0f && c <= 1.0f) || max_iter < 0) throw Err{TC_EINVAL, "need 0 <= c <= 1 and max_iter >= 0"};
    need_square(hc, "tc_pagerank");
    tc_handle* h = const_cast<tc_handle*>(hc);
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = h->n_rows;
    if (check_every < 1) check_every = 1;
    float* p = h->d_xbuf;
    float* y = h->d_ybuf;
    double* parts = h->d_red;                  // 2 * kRedBlocks
    double* res = h->d_red + 2 * kRedBlocks;   // [resid, dangling mass]
    int32_t it = 0;
    double r = 0.0;
    bool conv = false;
    if (n > 0) {
      hipLaunchKernelGGL(k_fill_f32, dim3(nblk(n, kB)), dim3(kB), 0, st, p, n, (float)(1.0 / (double)n));
      HIPC(hipGetLastError());
      hipLaunchKernelGGL(k_range_sum, dim3(kRedBlocks), dim3(kB), 0, st, (const float*)p, n - h->n_dangling, n,
                         parts + kRedBlocks);
      HIPC(hipGetLastError());
      hipLaunchKernelGGL(k_finish, dim3(1), dim3(kB), 0, st, (const double*)(parts + kRedBlocks), kRedBlocks, 1,
                         res + 1);
      HIPC(hipGetLastError());
      const bool xcd = h->xcd_groups > 0 && h->n_tiles > 1;
      const int32_t G = xcd ? h->n_tiles - 1 : 0;
      // Iterations whose L1 change is not read run the update fused into the
      // product, into the other buffer (one tile, composite kernel); their
      // dangling mass comes from a pass over the dangling range alone.  The
      // others run the product into the other buffer, then the update in place.
      const bool fuse = !xcd && h->n_tiles == 1 && h->kernel == 0;
      const bool fuse_panel = h->n_panels > 0 && h->kernel == 0;
      float* buf[2] = {p, y};
      bool zero_rows[2] = {false, false};  // the buffer's rows without entries hold 0
      int cur = 0;
      for (it = 0; it < max_iter;) {
        const bool need_res = it + 1 == max_iter || (tol > 0.0f && (it + 1) % check_every == 0);
        float* pc = buf[cur];
        float* pn = buf[1 - cur];
        if (fuse_panel && !need_res) {
          const PanelPr pr{(double)c, (const double*)(res + 1), n, (const int64_t*)h->d_panel_split_begin,
                           (const SplitRow*)h->d_split, h->d_panel_yraw};
          panel_pass(h, pc, pn, st, &pr);
          if (h->n_split_rows > 0) {
            hipLaunchKernelGGL(k_pr_split_panel, dim3(nblk(h->n_split_rows, kWpb)), dim3(kB), 0, st, h->d_split,
                               h->n_split_rows, (const double*)h->d_partial, (const float*)h->d_panel_yraw, pn,
                               (double)c, (const double*)(res + 1), n);
            HIPC(hipGetLastError());
          }
          hipLaunchKernelGGL(k_dang_sum, dim3(kRedBlocks), dim3(kB), 0, st, (const float*)pn, n, n - h->n_dangling,
                             parts + kRedBlocks);
          HIPC(hipGetLastError());
          hipLaunchKernelGGL(k_finish, dim3(1), dim3(kB), 0, st, (const double*)(parts + kRedBlocks), kRedBlocks, 1,
                             res + 1);
          HIPC(hipGetLastError());
          h->spmv_calls++;
          zero_rows[1 - cur] = false;
          cur = 1 - cur;
        } else if (fuse && !need_res) {
          const int64_t b = h->tile_wl_begin[0], e = h->tile_wl_begin[1];
          if (e > b)
            launch_tile(h,
                        pick_slices(tile_slices(h, 0, e - b), k_tile_spmv_pr<1>, k_tile_spmv_pr<2>,
                                    k_tile_spmv_pr<4>, k_tile_spmv_pr<8>),
                        dim3(nblk((e - b) * tile_slices(h, 0, e - b), kWpb)), dim3(kB), 0, st, (const Wl*)(h->d_wl + b),
                        (int64_t)(e - b), (const int32_t*)h->d_idx, (const float*)h->d_val,
                        (const int32_t*)h->d_rowid, (const float*)pc, pn, h->d_partial, (double)c,
                        (const double*)(res + 1), n);
          if (h->n_split_rows + h->n_empty > 0) {
            hipLaunchKernelGGL(k_pr_split_empty, dim3(nblk(h->n_split_rows + h->n_empty, kB)), dim3(kB), 0, st,
                               h->d_split, h->n_split_rows, (const double*)h->d_partial,
                               (const int32_t*)h->d_empty, h->n_empty, pn, (double)c, (const double*)(res + 1), n);
            HIPC(hipGetLastError());
          }
          hipLaunchKernelGGL(k_dang_sum, dim3(kRedBlocks), dim3(kB), 0, st, (const float*)pn, n, n - h->n_dangling,
                             parts + kRedBlocks);
          HIPC(hipGetLastError());
          hipLaunchKernelGGL(k_finish, dim3(1), dim3(kB), 0, st, (const double*)(parts + kRedBlocks), kRedBlocks, 1,
                             res + 1);
          HIPC(hipGetLastError());
          h->spmv_calls++;
          zero_rows[1 - cur] = false;
          cur = 1 - cur;
        } else {
          spmv_internal(h, pc, pn, st, xcd, zero_rows[1 - cur]);
          zero_rows[1 - cur] = true;
          hipLaunchKernelGGL(k_pr_update, dim3(kRedBlocks), dim3(kB), 0, st, (const float*)pn,
                             (const float*)h->d_ypriv, G, pc, n, n - h->n_dangling, (double)c,
                             (const double*)(res + 1), parts);
          HIPC(hipGetLastError());
          zero_rows[cur] = false;
          hipLaunchKernelGGL(k_finish, dim3(1), dim3(kB), 0, st, (const double*)parts, kRedBlocks, 2, res);
          HIPC(hipGetLastError());
        }
        ++it;
        if (tol > 0.0f && (it % check_every == 0 || it == max_iter)) {
          r = read_f64(res, st);
          if (r <= (double)tol) {
            conv = true;
            break;
          }
        }
      }
      if (it > 0) r = read_f64(res, st);
      gather_rows(buf[cur], h->d_rowmap, n, 1, p_out, st);
    }
    if (iters) *iters = it;
    if (resid) *resid = r;
    if (tol > 0.0f && !conv && n > 0) {
      set_error("tc_pagerank: tolerance not reached in max_iter iterations");
      return TC_ENOTCONV;
    }
    return TC_OK;
  });
}

extern "C" tc_status tc_hits(const tc_handle* hc, float tol, int32_t max_iter, int32_t check_every, float* auth,
                             float* hub, int32_t* iters, double* resid, tc_stream_t stream) {
  return guarded("tc_hits", [&]() -> tc_status {
    if (!hc || ((!auth || !hub) && hc->n_rows > 0)) throw Err{TC_EINVAL, "NULL argument"};
    if (max_iter < 0) throw Err{TC_EINVAL, "max_iter < 0"};
    need_square(hc, "tc_hits");
    if (hc->n_rows % 2) throw Err{TC_EINVAL, "the HITS matrix must be 2n x 2n"};
    tc_handle* h = const_cast<tc_handle*>(hc);
    hipStream_t st = (hipStream_t)stream;
    const int64_t n2 = h->n_rows, n = n2 / 2;
    if (check_every < 1) check_every = 1;
    float* x = h->d_xbuf;
    float* y = h->d_ybuf;
    double* parts = h->d_red;
    double* sums = h->d_red + 2 * kRedBlocks;       // [s_a, s_h]
    double* res = h->d_red + 2 * kRedBlocks + 2;    // resid
    int* err = (int*)workspace(h, 256, st);
    int32_t it = 0;
    double r = 0.0;
    bool conv = false;
    if (n2 > 0) {
      HIPC(hipMemsetAsync(err, 0, sizeof(int), st));
      hipLaunchKernelGGL(k_fill_f32, dim3(nblk(n2, kB)), dim3(kB), 0, st, x, n2, (float)(1.0 / (double)n));
      HIPC(hipGetLastError());
      for (it = 0; it < max_iter;) {
        spmv_internal(h, x, y, st);
        hipLaunchKernelGGL(k_hits_sums, dim3(kRedBlocks), dim3(kB), 0, st, (const float*)y,
                           (const int32_t*)h->d_rowinv, n2, n, parts);
        HIPC(hipGetLastError());
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(kB), 0, st, (const double*)parts, kRedBlocks, 2, sums);
        HIPC(hipGetLastError());
        hipLaunchKernelGGL(k_hits_update, dim3(kRedBlocks), dim3(kB), 0, st, (const float*)y, x,
                           (const int32_t*)h->d_rowinv, n2, n, (const double*)sums, parts, err);
        HIPC(hipGetLastError());
        hipLaunchKernelGGL(k_finish, dim3(1), dim3(kB), 0, st, (const double*)parts, kRedBlocks, 1, res);
        HIPC(hipGetLastError());
        ++it;
        if (tol > 0.0f && (it % check_every == 0 || it == max_iter)) {
          r = read_f64(res, st);
          if (r <= (double)tol) {
            conv = true;
            break;
          }
        }
      }
      int herr = 0;
      HIPC(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPC(hipStreamSynchronize(st));
      if (herr) throw Err{TC_EINVAL, "a half of the iterate sums to zero (graph without edges?)"};
      if (it > 0) r = read_f64(res, st);
      gather_rows(x, h->d_rowmap, n, 1, auth, st);
      gather_rows(x, h->d_rowmap + n, n, 1, hub, st);
    }
    if (iters) *iters = it;
    if (resid) *resid = r;
    if (tol > 0.0f && !conv && n2 > 0) {
      set_error("tc_hits: tolerance not reached in max_iter iterations");
      return TC_ENOTCONV;
    }
    return TC_OK;
  });
}

extern "C" tc_status tc_rwr(const tc_handle* hc, const int32_t* seeds, int32_t k, float c, float tol,
                            int32_t max_iter, int32_t check_every, float* R_out, int32_t* iters, double* resid,
                            tc_stream_t stream) {
  return guarded("tc_rwr", [&]() -> tc_status {
    if (!hc || !seeds || (!R_out && hc->n_rows > 0)) throw Err{TC_EINVAL, "NULL argument"};
    if (k < 1 || k > 256) throw Err{TC_EINVAL, "k must be in [1, 256]"};
    if (!(c >= 0.0f && c <= 1.0f) || max_iter < 0) throw Err{TC_EINVAL, "need 0 <= c <= 1 and max_iter >= 0"};
    need_square(hc, "tc_rwr");
    tc_handle* h = const_cast<tc_handle*>(hc);
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = h->n_rows;
    for (int32_t q = 0; q < k; ++q)
      if (seeds[q] < 0 || seeds[q] >= n) throw Err{TC_EINVAL, "seed out of range"};
    if (check_every < 1) check_every = 1;
    const int nb = 2048;  // update blocks (one partial per block and column)
    const size_t vb = ((sizeof(float) * (size_t)n * k + 255) / 256) * 256;
    const size_t need = 2 * vb + sizeof(double) * ((size_t)nb * k + k + 8) + 2 * sizeof(int32_t) * k;
    char* ws = (char*)workspace(h, need, st);
    float* Rm = (float*)ws;
    float* Ym = (float*)(ws + vb);
    double* parts = (double*)(ws + 2 * vb);
    double* colres = parts + (size_t)nb * k;
    double* mx = colres + k;
    int32_t* rawseeds = (int32_t*)(mx + 8);
    int32_t* dseeds = rawseeds + k;
    // internal ids of the seeds
    HIPC(hipMemcpyAsync(rawseeds, seeds, sizeof(int32_t) * k, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_map_ids, dim3(1), dim3(kB), 0, st, (const int32_t*)rawseeds, (const int32_t*)h->d_rowmap, k,
                       dseeds);
    HIPC(hipGetLastError());
    int32_t it = 0;
    double r = 0.0;
    bool conv = false;
    if (n > 0) {
      hipLaunchKernelGGL(k_rwr_init, dim3(nblk(n * k, kB)), dim3(kB), 0, st, Rm, n, k, (const int32_t*)dseeds);
      HIPC(hipGetLastError());
      // Iterations whose L1 change is not read run the restart fused into the
      // product, into the other buffer (one tile, k > 1); the others run the
      // product and then the update with its per-column change.
      const bool fuse = k > 1 && h->n_tiles == 1 && h->xcd_groups == 0;
      const bool fuse1 = k == 1 && h->n_tiles == 1 && h->xcd_groups == 0 && h->kernel == 0;
      const RwrEpi epi{(double)c, dseeds};
      // what the rows without entries hold in each buffer (they change only
      // between 0, for a product, and their restart values)
      enum { kUnknown, kZero, kRestart };
      float* buf[2] = {Rm, Ym};
      int held[2] = {kUnknown, kUnknown};
      int cur = 0;
      for (it = 0; it < max_iter;) {
        const bool need_res = it + 1 == max_iter || (tol > 0.0f && (it + 1) % check_every == 0);
        float* Rcur = buf[cur];
        float* Yb = buf[1 - cur];
        if (fuse && !need_res) {
          spmm_internal(h, Rcur, Yb, k, st, held[1 - cur] == kRestart, &epi);
          held[1 - cur] = kRestart;
          cur = 1 - cur;
        } else if (fuse1 && !need_res) {
          const int64_t b = h->tile_wl_begin[0], e = h->tile_wl_begin[1];
          if (e > b)
            launch_tile(h,
                        pick_slices(tile_slices(h, 0, e - b), k_tile_spmv_rwr<1>, k_tile_spmv_rwr<2>,
                                    k_tile_spmv_rwr<4>, k_tile_spmv_rwr<8>),
                        dim3(nblk((e - b) * tile_slices(h, 0, e - b), kWpb)), dim3(kB), 0, st, (const Wl*)(h->d_wl + b),
                        (int64_t)(e - b), (const int32_t*)h->d_idx, (const float*)h->d_val,
                        (const int32_t*)h->d_rowid, (const float*)Rcur, Yb, h->d_partial, (double)c,
                        (const int32_t*)dseeds);
          const int64_t ne = held[1 - cur] == kRestart ? 0 : h->n_empty;
          if (h->n_split_rows + ne > 0) {
            hipLaunchKernelGGL(k_rwr1_split_empty, dim3(nblk(h->n_split_rows + ne, kB)), dim3(kB), 0, st,
                               h->d_split, h->n_split_rows, (const double*)h->d_partial,
                               ne ? (const int32_t*)h->d_empty : nullptr, ne, Yb, (double)c, (const int32_t*)dseeds);
            HIPC(hipGetLastError());
          }
          h->spmv_calls++;
          held[1 - cur] = kRestart;
          cur = 1 - cur;
        } else {
          if (k == 1)
            spmv_internal(h, Rcur, Yb, st, false, held[1 - cur] == kZero);
          else
            spmm_internal(h, Rcur, Yb, k, st, held[1 - cur] == kZero);
          held[1 - cur] = kZero;
          hipLaunchKernelGGL(k_rwr_update, dim3(nb), dim3(kB), 0, st, (const float*)Yb, Rcur, n, k, (double)c,
                             (const int32_t*)dseeds, parts, nb);
          HIPC(hipGetLastError());
          held[cur] = kRestart;  // the update wrote every row of R
          hipLaunchKernelGGL(k_finish, dim3(nblk(k, kWpb)), dim3(kB), 0, st, (const double*)parts, nb, k, colres);
          HIPC(hipGetLastError());
          hipLaunchKernelGGL(k_max_of, dim3(1), dim3(64), 0, st, (const double*)colres, k, mx);
          HIPC(hipGetLastError());
        }
        ++it;
        if (tol > 0.0f && (it % check_every == 0 || it == max_iter)) {
          r = read_f64(mx, st);
          if (r <= (double)tol) {
            conv = true;
            break;
          }
        }
      }
      if (it > 0) r = read_f64(mx, st);
      gather_rows(buf[cur], h->d_rowmap, n, k, R_out, st);
    }
    if (iters) *iters = it;
    if (resid) *resid = r;
    if (tol > 0.0f && !conv && n > 0) {
      set_error("tc_rwr: tolerance not reached in max_iter iterations");
      return TC_ENOTCONV;
    }
    return TC_OK;
  });
}
