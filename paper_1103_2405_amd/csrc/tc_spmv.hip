// Single-vector products with a built handle: y = A x (Appendix B) by the
// tiled composite kernels, the TILE-COO kernels and the plain CSR baseline.
//
// Tiles run in order, one launch each (dense tiles, then the sparse tile), so
// every row's y entry is read-modified-written at most once per tile and
// never by two wavefronts at once (Section 3.1: a kernel per tile).
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "tc_host.h"

namespace tc {

namespace {

// S wavefronts per workload of the tile (row slices; grid = workloads * S / 4).
template <int S>
__global__ void __launch_bounds__(kB) k_tile_spmv(const Wl* __restrict__ wl, int64_t n_wl,
                                                  const int32_t* __restrict__ idx, const float* __restrict__ val,
                                                  const int32_t* __restrict__ rowid, const float* __restrict__ x,
                                                  float* __restrict__ y, double* __restrict__ partial) {
  const int lane = lane_id();
  const int64_t w = (int64_t)blockIdx.x * kWpb + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (w >= n_wl * S) return;
  const Wl d = wl[w / S];
  run_workload<S>(d, lane, idx, val, rowid, GlobalX{x}, y, partial, (int32_t)(w % S));
}

// x of a tile whose whole column range sits in LDS (a tile no wider than the
// LDS of one workgroup): every gather of the tile is an LDS read.
struct LdsX {
  const float* xs;  // LDS copy of x[cb, cb + width)
  int32_t cb;
  __device__ float operator()(int32_t i) const { return xs[i - cb]; }
  __device__ void addy(float* y, int32_t rid, double s) const { addy_first_touch(y, rid, s); }
};

// Tile pass with the tile's x segment staged in LDS (Section 3.1, Solution 1:
// the segment of x a tile reads is kept in the nearest memory; on gfx950 that
// is the 160 KB LDS of a compute unit).  Persistent: each workgroup copies
// x[cb, cb + lw) into LDS once, then its wavefronts take the work items
// (workload slices) w = global wavefront id, + total wavefronts, ... until
// none is left, so every wavefront ends after a bounded number of items.
constexpr int kLdsB = 1024;  // threads of an LDS-tile workgroup
template <int S>
__global__ void __launch_bounds__(kLdsB) k_tile_lds(const Wl* __restrict__ wl, int64_t n_wl,
                                                    const int32_t* __restrict__ idx, const float* __restrict__ val,
                                                    const int32_t* __restrict__ rowid, const float* __restrict__ x,
                                                    int32_t cb, int32_t lw, float* __restrict__ y,
                                                    double* __restrict__ partial) {
  extern __shared__ float xs[];
  const float* xsrc = x + cb;
  if (((uintptr_t)xsrc & 15) == 0 && (lw & 3) == 0) {
    for (int32_t k = 4 * (int32_t)threadIdx.x; k < lw; k += 4 * kLdsB)
      *(float4*)(xs + k) = *(const float4*)(xsrc + k);
  } else {
    for (int32_t k = threadIdx.x; k < lw; k += kLdsB) xs[k] = xsrc[k];
  }
  __syncthreads();
  const int lane = lane_id();
  const int64_t waves = (int64_t)gridDim.x * (kLdsB / kWave);
  const int64_t items = n_wl * S;
  const LdsX xg{xs, cb};
  for (int64_t w = (int64_t)blockIdx.x * (kLdsB / kWave) + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
       w < items; w += waves) {
    const Wl d = wl[w / S];
    run_workload<S>(d, lane, idx, val, rowid, xg, y, partial, (int32_t)(w % S));
  }
}

// x of a row panel: gathers through the caches; the panel's rows of y sit in
// LDS (ys[row - base]) and every tile adds its row sums there.  A panel row
// is in at most one workload of a tile, and tiles are separated by barriers,
// so each row's adds happen in tile order, as the first-touch product does
// them (an add to the zeroed LDS row gives fl32(s), the first tile's store).
template <bool Buf>
struct PanelX {
  const float* __restrict__ x;
  float* ys;
  int32_t base;
  __device__ float operator()(int32_t i) const {
    if constexpr (Buf)
      return ld_buf(x, i);
    else
      return x[i];
  }
  __device__ void addy(float*, int32_t rid, double s) const {
    float* q = ys + ((rid & ~kAddFlag) - base);
    *q = (float)((double)*q + s);
  }
};

// ... and column tile 0 of a panel handle with its x segment staged in LDS
// (behind the panel's rows of y): its gathers are LDS reads.
struct PanelLdsX {
  const float* xs;
  float* ys;
  int32_t base;
  __device__ float operator()(int32_t i) const { return xs[i]; }
  __device__ void addy(float*, int32_t rid, double s) const {
    float* q = ys + ((rid & ~kAddFlag) - base);
    *q = (float)((double)*q + s);
  }
};

// The workloads of column tile t for workgroup p: the tile's own workloads
// that are not split chunks, then every np-th chunk workload of column tile t
// over all panels (chunk sums go to partial slots, so any workgroup may run
// them).
template <int NW, class G>
__device__ inline void panel_tile(const G& xg, int64_t g, int32_t t, int32_t p, int32_t np, int32_t wv, int lane,
                                  const Wl* __restrict__ wl, const int64_t* __restrict__ wl_begin,
                                  const int64_t* __restrict__ ncb, const int64_t* __restrict__ chunks,
                                  const int64_t* __restrict__ cb, const int32_t* __restrict__ idx,
                                  const float* __restrict__ val, const int32_t* __restrict__ rowid, float* y,
                                  double* __restrict__ partial) {
  // each wavefront's next descriptor is read while it runs the current one
  const int64_t e = wl_begin[g + 1];
  int64_t j = ncb[g] + wv;
  if (j < e) {
    Wl d = wl[j];
    for (;;) {
      const int64_t jn = j + NW;
      const Wl dn = wl[jn < e ? jn : j];
      run_workload<1>(d, lane, idx, val, rowid, xg, y, partial);
      if (jn >= e) break;
      d = dn;
      j = jn;
    }
  }
  const int64_t ce = cb[t + 1];
  int64_t k = cb[t] + p + (int64_t)wv * np;
  if (k < ce) {
    Wl d = wl[chunks[k]];
    for (;;) {
      const int64_t kn = k + (int64_t)NW * np;
      const Wl dn = wl[chunks[kn < ce ? kn : k]];
      run_workload<1>(d, lane, idx, val, rowid, xg, y, partial);
      if (kn >= ce) break;
      d = dn;
      k = kn;
    }
  }
}

// Row-panel pass (one launch per product).  Workgroup p owns internal rows
// [pb[p], pb[p+1]) and keeps their y in LDS while it sweeps the column tiles
// in order, a barrier after each.  All workgroups walk the column tiles in the
// same order, so the x segment of the current tile is what the L2s hold; with
// w0 > 0 column tile 0 (internal columns [0, w0), the hottest) is first copied
// into LDS behind y (rows_cap floats in).  At the end the panel's y is stored
// once, coalesced (PR: as the PageRank update of it).
// BufX: x gathered by buffer loads (n_cols <= kBufMaxFloats).
template <int NW, bool PR, bool BufX>
__global__ void __launch_bounds__(NW * kWave) k_panel_spmv(const Wl* __restrict__ wl,
                                                           const int64_t* __restrict__ wl_begin,
                                                           const int64_t* __restrict__ ncb,
                                                           const int64_t* __restrict__ chunks,
                                                           const int64_t* __restrict__ cb, int32_t nct, int32_t np,
                                                           const int32_t* __restrict__ pb, int32_t rows_cap,
                                                           int32_t w0, const int32_t* __restrict__ idx,
                                                           const float* __restrict__ val,
                                                           const int32_t* __restrict__ rowid,
                                                           const float* __restrict__ x, float* __restrict__ y,
                                                           double* __restrict__ partial, PanelPr pr) {
  extern __shared__ float ys[];
  const int32_t p = blockIdx.x;
  const int32_t r0 = pb[p], nr = pb[p + 1] - r0;
  for (int32_t i = threadIdx.x; i < nr; i += NW * kWave) ys[i] = 0.0f;
  float* xs = ys + rows_cap;  // rows_cap is a multiple of 4: 16-byte aligned
  if (w0 > 0) {
    const int32_t w4 = ((uintptr_t)x & 15) == 0 ? w0 & ~3 : 0;
    for (int32_t k = 4 * (int32_t)threadIdx.x; k < w4; k += 4 * NW * kWave)
      *(float4*)(xs + k) = *(const float4*)(x + k);
    for (int32_t k = w4 + (int32_t)threadIdx.x; k < w0; k += NW * kWave) xs[k] = x[k];
  }
  __syncthreads();
  const int lane = lane_id();
  const int32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  int32_t t = 0;
  if (w0 > 0 && nct > 0) {
    panel_tile<NW>(PanelLdsX{xs, ys, r0}, (int64_t)p * nct, 0, p, np, wv, lane, wl, wl_begin, ncb, chunks, cb, idx,
                   val, rowid, y, partial);
    __syncthreads();
    t = 1;
  }
  const PanelX<BufX> xg{x, ys, r0};
  for (; t < nct; ++t) {
    panel_tile<NW>(xg, (int64_t)p * nct + t, t, p, np, wv, lane, wl, wl_begin, ncb, chunks, cb, idx, val, rowid, y,
                   partial);
    __syncthreads();
  }
  if (PR) {
    const double dn = *pr.dmass / (double)pr.n, tele = (1.0 - pr.c) / (double)pr.n;
    for (int32_t i = threadIdx.x; i < nr; i += NW * kWave) y[r0 + i] = (float)(pr.c * ((double)ys[i] + dn) + tele);
    const int64_t se = pr.psb[p + 1];
    for (int64_t q = pr.psb[p] + threadIdx.x; q < se; q += NW * kWave) pr.yraw[q] = ys[pr.split[q].row - r0];
  } else {
    for (int32_t i = threadIdx.x; i < nr; i += NW * kWave) y[r0 + i] = ys[i];
  }
}

// Concurrent pass over tiles 1..G of the XCD schedule.  Workgroups are
// dispatched round-robin over the 8 XCDs, so block b runs on XCD b % 8: tile
// 1 + (b % G) takes blocks b with that residue, and its x range stays in one
// XCD's L2.  Each tile writes its own copy of y (ypriv + g * n_rows).
__global__ void __launch_bounds__(kB) k_tile_xcd(const Wl* __restrict__ wl, const int64_t* __restrict__ wl_begin,
                                                 int32_t G, const int32_t* __restrict__ idx,
                                                 const float* __restrict__ val, const int32_t* __restrict__ rowid,
                                                 const float* __restrict__ x, float* __restrict__ ypriv, int64_t n_rows,
                                                 double* __restrict__ partial) {
  const int lane = lane_id();
  const int32_t g = blockIdx.x % G;
  const int64_t jb = blockIdx.x / G;
  const int64_t b = wl_begin[g], e = wl_begin[g + 1];
  const int64_t j = b + jb * kWpb + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (j >= e) return;
  const Wl d = wl[j];
  run_workload(d, lane, idx, val, rowid, PrivX{x}, ypriv + (int64_t)g * n_rows, partial);
}

// y[r] += sum over g of ypriv[g][r], in g order (rows tile 0 did not write were zeroed).
__global__ void k_combine_priv(float* __restrict__ y, const float* __restrict__ ypriv, int64_t n, int32_t G) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double s = (double)y[r];
  for (int32_t g = 0; g < G; ++g) s += (double)ypriv[(int64_t)g * n + r];
  y[r] = (float)s;
}

// Sum of every split row's chunks in (tile, chunk) order, added to y (or
// stored when no tile wrote the row); one wavefront per split row.
__global__ void __launch_bounds__(kB) k_split_combine(const SplitRow* __restrict__ sr, int64_t n,
                                                      const double* __restrict__ partial, float* __restrict__ y,
                                                      int force_add) {
  const int lane = lane_id();
  const int64_t i = (int64_t)blockIdx.x * kWpb + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (i >= n) return;
  __shared__ double buf[kWpb][4 * kWave];
  const SplitRow s = sr[i];
  const double acc = sum_slots_wave(partial + s.slot_begin, s.n_slots, lane, buf[threadIdx.x / kWave]);
  if (lane != 0) return;
  if (s.store && !force_add)
    y[s.row] = (float)acc;
  else
    add_to_y(y, s.row, acc);
}

// Start of a product: zero the rows no tile writes, reset the tile counters.
__global__ void k_begin_spmv(float* __restrict__ y, const int32_t* __restrict__ empty, int64_t n_empty,
                             unsigned long long* __restrict__ counters, int32_t nt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_empty) y[empty[i]] = 0.0f;
  if (i < nt) counters[i] = 0ull;
}

// ---- streaming read (measurement): every 16-byte word of the buffer read
// once with the tile kernels' non-temporal loads, four per thread in flight;
// the per-thread sums go to sink so the loads cannot be dropped.
__global__ void __launch_bounds__(kB) k_stream_read(const v4f* __restrict__ a, int64_t n4, float* __restrict__ sink) {
  const int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x;
  const int64_t T = (int64_t)gridDim.x * kB;
  float s = 0.0f;
  int64_t i = t;
  for (; i + 3 * T < n4; i += 4 * T) {
    const v4f v0 = __builtin_nontemporal_load(a + i), v1 = __builtin_nontemporal_load(a + i + T);
    const v4f v2 = __builtin_nontemporal_load(a + i + 2 * T), v3 = __builtin_nontemporal_load(a + i + 3 * T);
    s += ((v0.x + v0.y) + (v0.z + v0.w)) + ((v1.x + v1.y) + (v1.z + v1.w)) + ((v2.x + v2.y) + (v2.z + v2.w)) +
         ((v3.x + v3.y) + (v3.z + v3.w));
  }
  for (; i < n4; i += T) {
    const v4f v = __builtin_nontemporal_load(a + i);
    s += (v.x + v.y) + (v.z + v.w);
  }
  sink[t] = s;
}
constexpr int kStreamBlocks = 8192;

// Measurement of the random-gather rate: coalesced index and value streams
// with one gather of x per entry, the access pattern of a column-major
// workload (lane l of a group of 64 takes entry g*64 + l), eight entries per
// lane in flight; the same grid as k_stream_read, each thread's sum to sink.
// An index outside [0, n_x) reads x[0].
constexpr int kGatherPer = 8;
template <bool Buf>
__global__ void __launch_bounds__(kB) k_gather_read(const float* __restrict__ x, int64_t n_x,
                                                    const int32_t* __restrict__ idx, const float* __restrict__ val,
                                                    int64_t n_chunks, float* __restrict__ sink) {
  const int lane = lane_id();
  const int64_t t = (int64_t)blockIdx.x * kB + threadIdx.x;
  const int64_t W = (int64_t)gridDim.x * kWpb;
  float s = 0.0f;
  for (int64_t c = t / kWave; c < n_chunks; c += W) {
    const int64_t base = c * (kGatherPer * kWave) + lane;
    int32_t id[kGatherPer];
    float v[kGatherPer];
#pragma unroll
    for (int u = 0; u < kGatherPer; ++u) {
      id[u] = __builtin_nontemporal_load(idx + base + u * kWave);
      v[u] = __builtin_nontemporal_load(val + base + u * kWave);
    }
#pragma unroll
    for (int u = 0; u < kGatherPer; ++u) {
      const int32_t i = (uint64_t)(uint32_t)id[u] < (uint64_t)n_x ? id[u] : 0;
      if constexpr (Buf)
        s += v[u] * ld_buf(x, i);
      else
        s += v[u] * x[i];
    }
  }
  sink[t] = s;
}

// ---- plain CSR baseline: the CSR-vector kernel of Appendix B and Section 3.1
// (Observation 4), one wavefront per row.  The lanes stride the row with
// four loads in flight each, keep FP64 partial sums and reduce them across
// the wavefront.  On a power-law matrix one wavefront walks each long row
// alone, which is the imbalance the tiled format removes.
__global__ void __launch_bounds__(kB) k_csr_vector(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                   const float* __restrict__ val, int64_t n_rows,
                                                   const float* __restrict__ x, float* __restrict__ y) {
  const int lane = lane_id();
  const int64_t r = (int64_t)blockIdx.x * kWpb + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (r >= n_rows) return;
  const int64_t e = rp[r + 1];
  double acc = 0.0;
  int64_t k = rp[r] + lane;
  for (; k + 3 * kWave < e; k += 4 * kWave) {
    int32_t c[4];
    float v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      c[u] = col[k + u * kWave];
      v[u] = val[k + u * kWave];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = fma((double)v[u], (double)x[c[u]], acc);
  }
  for (; k < e; k += kWave) acc = fma((double)val[k], (double)x[col[k]], acc);
  acc = wave_sum(acc);
  if (lane == 0) y[r] = (float)acc;
}

// ---- TILE-COO (Section 3.1, Observation 3)
//
// A tile's entries, sorted by row, are cut into intervals of kCooIv entries,
// one per wavefront, whatever the row lengths.  Lane l takes kCooPer
// consecutive entries and sums them row by row: rows that start and end in
// its run are written at once; its first and last row go to a segmented scan
// across the lanes (pairs (a, g): out_l = a_l + g_l out_{l-1}, g = 1 when the
// lane holds a single row continuing the previous lane's last one).  A row
// that crosses an interval boundary leaves partial sums in a per-wavefront
// record; a fix-up pass adds them in interval order.  All sums are FP64 in a
// fixed order; y gets fl32 once per row and tile (store, or add when an
// earlier tile holds the row).
constexpr int kCooPer = 8;
constexpr int kCooIv = kWave * kCooPer;

struct CooCarry {
  int32_t row0, row1;  // first and last row of the interval (flagged ids)
  int32_t flags;       // 1: row0 started before the interval, 2: row1 continues after it, 4: single row
  int32_t pad;
  double p0, p1;       // this interval's partial sums of row0 and row1
};

__device__ inline void coo_write(float* __restrict__ y, int32_t rf, double s) {
  const int32_t r = rf & ~kAddFlag;
  if (rf & kAddFlag)
    y[r] = (float)((double)y[r] + s);
  else
    y[r] = (float)s;
}

__global__ void __launch_bounds__(kB) k_tile_coo(const int32_t* __restrict__ crow, const int32_t* __restrict__ ccol,
                                                 const float* __restrict__ cval, int64_t n,
                                                 const float* __restrict__ x, float* __restrict__ y,
                                                 CooCarry* __restrict__ carry) {
  const int lane = lane_id();
  const int64_t w = (int64_t)blockIdx.x * kWpb + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t b = w * kCooIv;
  if (b >= n) return;
  const int64_t e = min(n, b + (int64_t)kCooIv);
  const int last = (int)((e - b - 1) / kCooPer);  // last lane holding entries
  const int64_t s0 = b + (int64_t)lane * kCooPer;
  const int cnt = lane <= last ? (int)min<int64_t>(kCooPer, e - s0) : 0;
  int32_t rr[kCooPer];
  double pp[kCooPer];
  // every load on every lane (past the lane's entries: its last one, or the
  // interval's first), so the loads and gathers go out together
  const int64_t qlast = cnt > 0 ? s0 + cnt - 1 : b;
#pragma unroll
  for (int j = 0; j < kCooPer; ++j) {
    const int64_t q = min(s0 + j, qlast);
    const int32_t rv = crow[q];
    const float vv = cval[q];
    const float xv = x[ccol[q]];
    rr[j] = j < cnt ? rv : 0;
    pp[j] = j < cnt ? (double)vv * (double)xv : 0.0;
  }
  // lane pass
  const int32_t first = rr[0];
  int32_t cur = first;
  double acc = 0.0, head = 0.0;
  bool multi = false;
#pragma unroll
  for (int j = 0; j < kCooPer; ++j) {
    if (j < cnt) {
      if (rr[j] != cur) {
        if (!multi) {
          head = acc;
          multi = true;
        } else {
          coo_write(y, cur, acc);  // a row inside this lane's run
        }
        cur = rr[j];
        acc = 0.0;
      }
      acc += pp[j];
    }
  }
  const int32_t tail_row = cur;
  // scan over lanes
  const int32_t prev_tail = __shfl_up(tail_row, 1, kWave);
  const bool cont = lane > 0 && lane <= last && first == prev_tail;  // first row continues lane l-1's last
  double a = lane <= last ? acc : 0.0;
  int g = (lane <= last && !multi && cont) ? 1 : 0;
  for (int o = 1; o < kWave; o <<= 1) {
    const double au = __shfl_up(a, o, kWave);
    const int gu = __shfl_up(g, o, kWave);
    if (lane >= o) {
      if (g) a += au;
      g = g & gu;
    }
  }
  const double out_prev = __shfl_up(a, 1, kWave);
  const double c_in = cont ? out_prev : 0.0;
  // interval boundary rows
  const int32_t R0 = __shfl(first, 0, kWave), R1 = __shfl(tail_row, last, kWave);
  const bool cont_in = b > 0 && crow[b - 1] == R0;
  const bool cont_out = e < n && crow[e] == R1;
  const bool single = R0 == R1;
  // completion of the lane's first row (multi-row lanes)
  if (lane <= last && multi) {
    const double t = head + c_in;
    if (first == R0 && cont_in)
      carry[w].p0 = t;
    else
      coo_write(y, first, t);
  }
  // completion of the lane's last row
  const int32_t next_first = __shfl_down(first, 1, kWave);
  if (lane <= last) {
    const bool ends_here = lane < last ? next_first != tail_row : !cont_out;
    if (lane == last && cont_out) {
      carry[w].p1 = a;
      if (single) carry[w].p0 = a;
    } else if (ends_here) {
      if (tail_row == R0 && cont_in)
        carry[w].p0 = a;
      else
        coo_write(y, tail_row, a);
    }
  }
  if (lane == 0) {
    carry[w].row0 = R0;
    carry[w].row1 = R1;
    carry[w].flags = (cont_in ? 1 : 0) | (cont_out ? 2 : 0) | (single ? 4 : 0);
  }
}

// rows crossing interval boundaries: the interval where such a row starts
// adds the partial sums of the following intervals, in order, and writes it
__global__ void k_coo_fixup(const CooCarry* __restrict__ carry, int64_t nw, float* __restrict__ y) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nw) return;
  const CooCarry c = carry[w];
  if (!(c.flags & 2) || ((c.flags & 4) && (c.flags & 1))) return;
  double t = c.p1;
  for (int64_t v = w + 1; v < nw; ++v) {
    const CooCarry d = carry[v];
    t += d.p0;
    if (!((d.flags & 4) && (d.flags & 2))) break;
  }
  coo_write(y, c.row1, t);
}

}  // namespace

void* workspace(tc_handle* h, size_t bytes, hipStream_t st) {
  if (bytes <= h->ws_bytes) return h->d_ws;
  if (h->d_ws) pool_free(h->d_ws, st, false);
  h->d_ws = nullptr;
  h->ws_bytes = 0;
  if (!(h->d_ws = pool_alloc(bytes, st)))
    throw Err{TC_ENOMEM, "workspace allocation of " + std::to_string(bytes) + " bytes failed"};
  h->ws_bytes = bytes;
  return h->d_ws;
}

hipEvent_t next_event(tc_handle* h) {
  if (h->ev_used == h->ev_pool.size()) {
    hipEvent_t e;
    HIPC(hipEventCreate(&e));
    h->ev_pool.push_back(e);
  }
  return h->ev_pool[h->ev_used++];
}

// Row slices: S wavefronts share each workload, slice s taking every S-th
// 64-row block (column-major) or row (row-major).  Each row is still summed
// whole by one lane or one wavefront in the same order, so the result does not
// depend on S.  It evens out the tail of the launch: on a 2^27-entry Chung-Lu
// matrix (WL 8183) the product takes 1064 / 1032 / 998 / 1325 us with
// S = 1 / 2 / 4 / 8.  Slices pay where workloads are large and many, so
// without a given count a tile of fewer than kSliceMinWl workloads, or with a
// workload size below kSliceMinSize entries, runs one slice per workload
// (R-MAT 20 at WL 512: 85 us with one slice, 90 us with four; 32 small R-MAT
// graphs at WL 128-256, one after another: 13.1 ms with one, 15.3 ms with
// four; at WL 1984 four slices win, 98 against 104 us).  The build option
// `slices` (1, 2, 4 or 8) applies one count to every tile instead.
constexpr int64_t kSliceMinWl = 4096;
constexpr int64_t kSliceMinSize = 1024;
constexpr int32_t kSlicesDefault = 4;
int32_t tile_slices(const tc_handle* h, int t, int64_t n_wl) {
  if (h->slices > 0) return h->slices;
  return n_wl >= kSliceMinWl && h->tile_wl[t] >= kSliceMinSize ? kSlicesDefault : 1;
}

// LDS staging of a tile's x segment: the tile must fit the LDS of one
// workgroup, and carry enough entries for the copy (lw floats into every
// resident workgroup) to be a small part of its traffic: at least
// kLdsMinReuse gathers per staged float.  Returns the width to stage, or 0.
constexpr int64_t kLdsMinReuse = 8;
int64_t lds_tile_width(const tc_handle* h, int t) {
  if (!h->lds_tiles || h->lds_floats <= 0) return 0;
  const int64_t lw = h->tile_col_end[t] - h->tile_col_begin[t];
  if (lw <= 0 || lw > h->lds_floats) return 0;
  if (h->lds_tiles == 1 && h->tile_nnz[t] < kLdsMinReuse * lw * lds_tile_blocks(h, lw)) return 0;
  return lw;
}

// Resident workgroups of the LDS tile kernel for a segment of lw floats (one
// grid of them covers the GPU once).
int64_t lds_tile_blocks(const tc_handle* h, int64_t lw) {
  const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(2, h->lds_cu_bytes / std::max<int64_t>(4 * lw, 1)));
  return per_cu * h->n_cu;
}

// Floats of x that the row-panel pass stages in LDS (column tile 0, when it
// fits behind the panel's rows of y and staging is not turned off), else 0.
int64_t panel_stage_width(const tc_handle* h) {
  if (h->n_panels <= 0 || h->lds_tiles == 0 || h->n_col_tiles < 1) return 0;
  const int64_t rows_cap = (h->panel_rows + 3) & ~3;
  const int64_t w0 = h->tile_col_end[0] - h->tile_col_begin[0];
  return rows_cap + w0 <= h->lds_floats ? w0 : 0;
}

// One launch of the row-panel pass: every row of y is stored by its panel
// (with pr: the fused PageRank update of it).
void panel_pass(tc_handle* h, const float* x, float* y, hipStream_t st, const PanelPr* pr) {
  if (h->n_panels <= 0 || h->n_wl == 0) return;
  const int64_t rows_cap = (h->panel_rows + 3) & ~3;
  const int64_t w0 = panel_stage_width(h);
  const uint32_t lds = (uint32_t)(4 * (rows_cap + w0));
  const bool bx = h->n_cols <= kBufMaxFloats;
  auto kern = pr ? (bx ? (h->panel_waves == 4   ? k_panel_spmv<4, true, true>
                          : h->panel_waves == 8 ? k_panel_spmv<8, true, true>
                                                : k_panel_spmv<16, true, true>)
                       : (h->panel_waves == 4   ? k_panel_spmv<4, true, false>
                          : h->panel_waves == 8 ? k_panel_spmv<8, true, false>
                                                : k_panel_spmv<16, true, false>))
                 : (bx ? (h->panel_waves == 4   ? k_panel_spmv<4, false, true>
                          : h->panel_waves == 8 ? k_panel_spmv<8, false, true>
                                                : k_panel_spmv<16, false, true>)
                       : (h->panel_waves == 4   ? k_panel_spmv<4, false, false>
                          : h->panel_waves == 8 ? k_panel_spmv<8, false, false>
                                                : k_panel_spmv<16, false, false>));
  const PanelPr none{0.0, nullptr, 0, nullptr, nullptr, nullptr};
  if (lds > 65536) HIPC(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  launch_tile(h, kern, dim3((unsigned)h->n_panels), dim3((unsigned)(h->panel_waves * kWave)), lds, st,
              (const Wl*)h->d_wl, (const int64_t*)h->d_tile_wl_begin, (const int64_t*)h->d_panel_ncb,
              (const int64_t*)h->d_panel_chunks, (const int64_t*)h->d_panel_cb, (int32_t)h->n_col_tiles,
              (int32_t)h->n_panels, (const int32_t*)h->d_panel_begin, (int32_t)rows_cap, (int32_t)w0,
              (const int32_t*)h->d_idx, (const float*)h->d_val, (const int32_t*)h->d_rowid, x, y, h->d_partial,
              pr ? *pr : none);
}

void spmv_internal(tc_handle* h, const float* x, float* y, hipStream_t st, bool fuse_combine, bool skip_zero,
                   bool tilewise) {
  if (h->n_panels > 0 && !tilewise) {
    panel_pass(h, x, y, st, nullptr);
    if (h->n_split_rows > 0) {
      hipLaunchKernelGGL(k_split_combine, dim3(nblk(h->n_split_rows, kWpb)), dim3(kB), 0, st, h->d_split,
                         h->n_split_rows, h->d_partial, y, 0);
      HIPC(hipGetLastError());
    }
    h->spmv_calls++;
    return;
  }
  const bool xcd = h->xcd_groups > 0 && h->n_tiles > 1;
  const int64_t nzero = xcd ? h->n_zero0 : h->n_empty;
  const int64_t nz = std::max<int64_t>(nzero, h->n_tiles);
  if (nz > 0 && !(skip_zero && !xcd)) {
    hipLaunchKernelGGL(k_begin_spmv, dim3(nblk(nz, kB)), dim3(kB), 0, st, y,
                       (const int32_t*)(xcd ? h->d_zero0 : h->d_empty), nzero, h->d_counters, (int32_t)h->n_tiles);
    HIPC(hipGetLastError());
  }
  if (h->kernel == 1) {  // TILE-COO: tiles in order, each an interval pass and its fix-up
    int64_t maxw = 0;
    for (int t = 0; t < h->n_tiles; ++t)
      maxw = std::max<int64_t>(maxw, (h->tile_coo_off[t + 1] - h->tile_coo_off[t] + kCooIv - 1) / kCooIv);
    if (maxw > h->coo_carry_n) {
      if (h->d_coo_carry) pool_free(h->d_coo_carry, st, false);
      h->d_coo_carry = pool_alloc(sizeof(CooCarry) * maxw, st);
      h->coo_carry_n = h->d_coo_carry ? maxw : 0;
      if (!h->d_coo_carry) throw Err{TC_ENOMEM, "TILE-COO carry records: allocation failed"};
    }
    for (int t = 0; t < h->n_tiles; ++t) {
      const int64_t o = h->tile_coo_off[t], nt = h->tile_coo_off[t + 1] - o;
      if (nt == 0) continue;
      const int64_t nw = (nt + kCooIv - 1) / kCooIv;
      launch_tile(h, k_tile_coo, dim3(nblk(nw, kWpb)), dim3(kB), 0, st, (const int32_t*)(h->d_coo_row + o),
                  (const int32_t*)(h->d_coo_col + o), (const float*)(h->d_coo_val + o), nt, x, y,
                  (CooCarry*)h->d_coo_carry);
      hipLaunchKernelGGL(k_coo_fixup, dim3(nblk(nw, kB)), dim3(kB), 0, st, (const CooCarry*)h->d_coo_carry, nw, y);
      HIPC(hipGetLastError());
    }
    h->spmv_calls++;
    return;
  }
  for (int t = 0; t < (xcd ? 1 : h->n_tiles); ++t) {
    const int64_t b = h->tile_wl_begin[t], e = h->tile_wl_begin[t + 1];
    if (e == b) continue;
    const int32_t S = tile_slices(h, t, e - b);
    const int64_t lw = lds_tile_width(h, t);
    if (lw > 0) {
      auto kern = pick_slices(S, k_tile_lds<1>, k_tile_lds<2>, k_tile_lds<4>, k_tile_lds<8>);
      if (lw * 4 > 65536) HIPC(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                    (int)(lw * 4)));
      const unsigned grid = (unsigned)std::min<int64_t>(lds_tile_blocks(h, lw), nblk((e - b) * S, kLdsB / kWave));
      launch_tile(h, kern, dim3(grid), dim3(kLdsB), (uint32_t)(lw * 4), st, (const Wl*)(h->d_wl + b),
                  (int64_t)(e - b), (const int32_t*)h->d_idx, (const float*)h->d_val, (const int32_t*)h->d_rowid, x,
                  (int32_t)h->tile_col_begin[t], (int32_t)lw, y, h->d_partial);
      continue;
    }
    launch_tile(h, pick_slices(S, k_tile_spmv<1>, k_tile_spmv<2>, k_tile_spmv<4>, k_tile_spmv<8>),
                dim3(nblk((e - b) * S, kWpb)), dim3(kB), 0, st, (const Wl*)(h->d_wl + b), (int64_t)(e - b),
                (const int32_t*)h->d_idx, (const float*)h->d_val, (const int32_t*)h->d_rowid, x, y, h->d_partial);
  }
  if (xcd) {
    const int32_t G = h->n_tiles - 1;
    int64_t maxb = 0;
    for (int g = 1; g <= G; ++g)
      maxb = std::max<int64_t>(maxb, (h->tile_wl_begin[g + 1] - h->tile_wl_begin[g] + kWpb - 1) / kWpb);
    if (maxb > 0)
      launch_tile(h, k_tile_xcd, dim3((unsigned)(maxb * G)), dim3(kB), 0, st, (const Wl*)h->d_wl,
                  (const int64_t*)(h->d_tile_wl_begin + 1), G, (const int32_t*)h->d_idx, (const float*)h->d_val,
                  (const int32_t*)h->d_rowid, x, h->d_ypriv, h->n_rows, h->d_partial);
    if (h->n_rows > 0 && !fuse_combine) {
      hipLaunchKernelGGL(k_combine_priv, dim3(nblk(h->n_rows, kB)), dim3(kB), 0, st, y, (const float*)h->d_ypriv,
                         h->n_rows, G);
      HIPC(hipGetLastError());
    }
  }
  if (h->n_split_rows > 0) {
    hipLaunchKernelGGL(k_split_combine, dim3(nblk(h->n_split_rows, kWpb)), dim3(kB), 0, st, h->d_split,
                       h->n_split_rows, h->d_partial, y, xcd ? 1 : 0);
    HIPC(hipGetLastError());
  }
  h->spmv_calls++;
}

void gather_rows(const float* in, const int32_t* perm, int64_t n, int32_t w, float* out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gather_rows, dim3(nblk(n * w, kB)), dim3(kB), 0, st, in, perm, n, w, out);
  HIPC(hipGetLastError());
}

double read_f64(const double* d, hipStream_t st) {
  double v = 0.0;
  HIPC(hipMemcpyAsync(&v, d, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  return v;
}

void need_square(const tc_handle* h, const char* who) {
  if (!h->relabel || h->n_rows != h->n_cols)
    throw Err{TC_EINVAL, std::string(who) + ": needs a square matrix built with row relabelling"};
}

}  // namespace tc

using namespace tc;


extern "C" tc_status tc_spmv_internal(const tc_handle* hc, const float* x, float* y, tc_stream_t stream) {
  return guarded("tc_spmv_internal", [&]() -> tc_status {
    if (!hc || (!x && hc->n_cols > 0) || (!y && hc->n_rows > 0)) throw Err{TC_EINVAL, "NULL argument"};
    if ((const void*)x == (const void*)y && hc->n_rows > 0) throw Err{TC_EINVAL, "x and y must not alias"};
    spmv_internal(const_cast<tc_handle*>(hc), x, y, (hipStream_t)stream);
    return TC_OK;
  });
}

extern "C" tc_status tc_spmv_tiles(const tc_handle* hc, const float* x, float* y, tc_stream_t stream) {
  return guarded("tc_spmv_tiles", [&]() -> tc_status {
    if (!hc || (!x && hc->n_cols > 0) || (!y && hc->n_rows > 0)) throw Err{TC_EINVAL, "NULL argument"};
    if ((const void*)x == (const void*)y && hc->n_rows > 0) throw Err{TC_EINVAL, "x and y must not alias"};
    spmv_internal(const_cast<tc_handle*>(hc), x, y, (hipStream_t)stream, false, false, true);
    return TC_OK;
  });
}

extern "C" tc_status tc_spmv(const tc_handle* hc, const float* x, float* y, tc_stream_t stream) {
  return guarded("tc_spmv", [&]() -> tc_status {
    if (!hc || (!x && hc->n_cols > 0) || (!y && hc->n_rows > 0)) throw Err{TC_EINVAL, "NULL argument"};
    if ((const void*)x == (const void*)y && hc->n_rows > 0) throw Err{TC_EINVAL, "x and y must not alias"};
    tc_handle* h = const_cast<tc_handle*>(hc);
    hipStream_t st = (hipStream_t)stream;
    gather_rows(x, h->d_cperm, h->n_cols, 1, h->d_xbuf, st);
    if (h->relabel) {
      spmv_internal(h, h->d_xbuf, h->d_ybuf, st);
      gather_rows(h->d_ybuf, h->d_rowmap, h->n_rows, 1, y, st);
    } else {
      spmv_internal(h, h->d_xbuf, y, st);
    }
    return TC_OK;
  });
}

extern "C" tc_status tc_csr_spmv(const tc_csr* A, const float* x, float* y, tc_stream_t stream) {
  return guarded("tc_csr_spmv", [&]() -> tc_status {
    if (!A || !A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->val)) || (!x && A->n_cols > 0) ||
        (!y && A->n_rows > 0))
      throw Err{TC_EINVAL, "NULL argument"};
    if (A->n_rows < 0 || A->n_cols < 0 || A->nnz < 0) throw Err{TC_EINVAL, "negative size"};
    if (A->n_rows > 0) {
      hipLaunchKernelGGL(k_csr_vector, dim3(nblk(A->n_rows, kWpb)), dim3(kB), 0, (hipStream_t)stream, A->row_ptr,
                         A->col_idx, A->val, A->n_rows, x, y);
      HIPC(hipGetLastError());
    }
    return TC_OK;
  });
}

extern "C" tc_status tc_gather_read(const float* d_x, int64_t n_x, const int32_t* d_idx, const float* d_val, int64_t n,
                                   float* d_sink, tc_stream_t stream) {
  return guarded("tc_gather_read", [&]() -> tc_status {
    if (!d_sink || (n > 0 && (!d_x || !d_idx || !d_val))) throw Err{TC_EINVAL, "NULL argument"};
    if (n < 0 || n % (kGatherPer * kWave) || n_x < 1)
      throw Err{TC_EINVAL, "n must be a multiple of 512 and n_x positive"};
    auto kern = n_x <= kBufMaxFloats ? k_gather_read<true> : k_gather_read<false>;
    hipLaunchKernelGGL(kern, dim3(kStreamBlocks), dim3(kB), 0, (hipStream_t)stream, d_x, n_x, d_idx, d_val,
                       n / (kGatherPer * kWave), d_sink);
    HIPC(hipGetLastError());
    return TC_OK;
  });
}

extern "C" tc_status tc_stream_read(const float* d_buf, int64_t n, float* d_sink, tc_stream_t stream) {
  return guarded("tc_stream_read", [&]() -> tc_status {
    if ((!d_buf && n > 0) || !d_sink) throw Err{TC_EINVAL, "NULL argument"};
    if (n < 0 || (n & 3) || ((uintptr_t)d_buf & 15)) throw Err{TC_EINVAL, "n must be a multiple of 4 and the buffer 16-byte aligned"};
    hipLaunchKernelGGL(k_stream_read, dim3(kStreamBlocks), dim3(kB), 0, (hipStream_t)stream, (const v4f*)d_buf, n / 4,
                       d_sink);
    HIPC(hipGetLastError());
    return TC_OK;
  });
}
