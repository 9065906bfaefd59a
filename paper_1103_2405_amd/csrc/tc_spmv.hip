// Products with a built handle and the power iterations on top of them.
//
// Tile pass (Section 3.1, Solution 3): one wavefront per workload.
//   row-major:    the wavefront walks one row at a time, lanes striding the
//                 padded row, then a cross-lane sum; lane 0 updates y.
//   column-major: lane r owns row r of the rectangle and walks its columns;
//                 consecutive lanes read consecutive addresses.
//   chunk:        one piece of a split heavy row; its sum goes to a partial
//                 slot that is added to y after the last tile.
// Tiles run in order, one launch each (dense tiles, then the sparse tile), so
// every row's y entry is read-modified-written at most once per tile and
// never by two wavefronts at once (Section 3.1: a kernel per tile).  Products
// are exact in FP64 and each row's per-tile sum is accumulated in FP64, then
// added to the FP32 y once per tile.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <type_traits>

#include "tc_internal.h"

namespace tc {

namespace {

constexpr int kB = 256;
constexpr int kWpb = kB / kWave;  // workloads per block

inline unsigned nblk(int64_t n, int64_t per) { return (unsigned)((n + per - 1) / per); }

__device__ inline int lane_id() { return (int)__lane_id(); }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

__device__ inline void add_to_y(float* y, int32_t row, double s) { y[row] = (float)((double)y[row] + s); }

typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Streams of the matrix are read once per product: non-temporal loads keep
// them from evicting x and y from the caches.
__device__ inline int32_t ld_nt(const int32_t* p) { return __builtin_nontemporal_load(p); }
__device__ inline float ld_nt(const float* p) { return __builtin_nontemporal_load(p); }
__device__ inline v4i ld_nt4(const int32_t* p) { return __builtin_nontemporal_load((const v4i*)p); }
__device__ inline v4f ld_nt4(const float* p) { return __builtin_nontemporal_load((const v4f*)p); }

// Cross-lane moves of a double through DPP (two 32-bit halves).  Lanes whose
// source is outside the row read 0 (bound_ctrl), rows outside ROWMASK add 0.
template <int CTRL, int ROWMASK = 0xf>
__device__ inline double dpp_f64(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int l2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWMASK, 0xf, true);
  const int h2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWMASK, 0xf, true);
  return __hiloint2double(h2, l2);
}

// Sum over each DPP row of 16 lanes; the total lands in the row's lane 15.
__device__ inline double row16_sum(double v) {
  v += dpp_f64<0x111>(v);  // row_shr:1
  v += dpp_f64<0x112>(v);  // row_shr:2
  v += dpp_f64<0x114>(v);  // row_shr:4
  v += dpp_f64<0x118>(v);  // row_shr:8
  return v;
}
// ... over 32 lanes (total in lanes 31 and 63)
__device__ inline double row32_sum(double v) {
  v = row16_sum(v);
  return v + dpp_f64<0x142, 0xa>(v);
}
// ... over the wavefront (total in lane 63)
__device__ inline double wave_total(double v) {
  v = row16_sum(v);
  v += dpp_f64<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

template <class G>
__device__ inline double dot4(v4i i, v4f v, const G& xg) {
  const float x0 = xg(i.x), x1 = xg(i.y), x2 = xg(i.z), x3 = xg(i.w);
  double s = (double)v.x * (double)x0;
  s = fma((double)v.y, (double)x1, s);
  s = fma((double)v.z, (double)x2, s);
  return fma((double)v.w, (double)x3, s);
}

// Row-major rectangle with 64-element-aligned rows (S a multiple of 64):
// every lane reads 4 consecutive entries (16 bytes) per 256-entry chunk.
//   w_pad = 64:  a chunk holds 4 rows, 16 lanes each -> sums per DPP row
//   w_pad = 128: a chunk holds 2 rows, 32 lanes each
//   otherwise:   one row at a time, chunks of 256 (last one masked)
// Two chunks are in flight per iteration (8 gathers per lane).
template <int S, class G>
__device__ inline void rm_wide(const Wl& d, int lane, const int32_t* __restrict__ idx,
                               const float* __restrict__ val, const int32_t* __restrict__ rowid,
                               const G& x, float* __restrict__ y, double* __restrict__ partial,
                               bool chunk, int32_t sl) {
  const int64_t off = d.data_off;
  const int32_t wp = d.w_pad, nr = d.n_rows;
  if (wp == 64 || wp == 128) {
    const int lpr = wp >> 2;             // lanes per row
    const int rpc = kWave / lpr;         // rows per chunk
    const int my = lane / lpr;           // my row inside the chunk
    const int nchunk = (nr + rpc - 1) / rpc;
    for (int q = 2 * sl; q < nchunk; q += 2 * S) {
      const int ra = q * rpc + my, rb = (q + 1) * rpc + my;
      const bool oka = ra < nr, okb = rb < nr;
      double sa = 0.0, sb = 0.0;
      v4i ia, ib;
      v4f va, vb;
      if (oka) {
        ia = ld_nt4(idx + off + (int64_t)q * 256 + 4 * lane);
        va = ld_nt4(val + off + (int64_t)q * 256 + 4 * lane);
      }
      if (okb) {
        ib = ld_nt4(idx + off + (int64_t)(q + 1) * 256 + 4 * lane);
        vb = ld_nt4(val + off + (int64_t)(q + 1) * 256 + 4 * lane);
      }
      if (oka) sa = dot4(ia, va, x);
      if (okb) sb = dot4(ib, vb, x);
      if (wp == 64) {
        sa = row16_sum(sa);
        sb = row16_sum(sb);
      } else {
        sa = row32_sum(sa);
        sb = row32_sum(sb);
      }
      if ((lane % lpr) == lpr - 1) {
        if (chunk) {
          if (oka) partial[d.info >> 2] = sa;
        } else {
          if (oka) x.addy(y, ld_nt(rowid + d.rowid_off + ra), sa);
          if (okb) x.addy(y, ld_nt(rowid + d.rowid_off + rb), sb);
        }
      }
    }
    return;
  }
  for (int32_t r = sl; r < nr; r += S) {
    const int64_t base = off + (int64_t)r * wp;
    double acc = 0.0;
    int32_t c = 4 * lane;
    for (; c + 256 < wp; c += 512) {
      const v4i ia = ld_nt4(idx + base + c), ib = ld_nt4(idx + base + c + 256);
      const v4f va = ld_nt4(val + base + c), vb = ld_nt4(val + base + c + 256);
      acc += dot4(ia, va, x) + dot4(ib, vb, x);
    }
    if (c < wp) acc += dot4(ld_nt4(idx + base + c), ld_nt4(val + base + c), x);
    acc = wave_total(acc);
    if (lane == kWave - 1) {
      if (chunk)
        partial[d.info >> 2] = acc;
      else
        x.addy(y, ld_nt(rowid + d.rowid_off + r), acc);
    }
  }
}

// Column-major rectangle: lane owns rows r = 64 u + lane; U row blocks and C
// columns are in flight together (U * C independent gathers per lane).  Every
// load runs on every lane: a lane past the last row reads the workload's first
// entry and takes index 0 and value 0 instead (its sum is never stored).  A
// load under a per-lane branch would end its branch with a wait for it, so
// the loads would go out one at a time.
template <int U, int C, int S, class G>
__device__ inline void cm_rows(const Wl& d, int lane, const int32_t* __restrict__ idx,
                               const float* __restrict__ val, const int32_t* __restrict__ rowid,
                               const G& x, float* __restrict__ y, int32_t sl) {
  const int64_t off = d.data_off, hp = d.h_pad;
  const int32_t w = d.w_pad, nr = d.n_rows;
  // slice sl of S takes the 64-row blocks sl, sl + S, ..., U of them at a time
  for (int32_t r0 = sl * kWave; r0 < nr; r0 += U * S * kWave) {
    double acc[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc[u] = 0.0;
      ok[u] = r0 + u * S * kWave + lane < nr;
    }
    int32_t c = 0;
    for (; c + C <= w; c += C) {
      int32_t ii[U][C];
      float vv[U][C], xv[U][C];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < C; ++k) {
          const int64_t e = ok[u] ? off + (int64_t)(c + k) * hp + r0 + u * S * kWave + lane : off;
          const int32_t ti = ld_nt(idx + e);
          const float tv = ld_nt(val + e);
          ii[u][k] = ok[u] ? ti : 0;
          vv[u][k] = ok[u] ? tv : 0.0f;
        }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < C; ++k) xv[u][k] = x(ii[u][k]);
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < C; ++k) acc[u] = fma((double)vv[u][k], (double)xv[u][k], acc[u]);
    }
    for (; c < w; ++c) {
      int32_t ii[U];
      float vv[U], xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t e = ok[u] ? off + (int64_t)c * hp + r0 + u * S * kWave + lane : off;
        const int32_t ti = ld_nt(idx + e);
        const float tv = ld_nt(val + e);
        ii[u] = ok[u] ? ti : 0;
        vv[u] = ok[u] ? tv : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) xv[u] = x(ii[u]);
#pragma unroll
      for (int u = 0; u < U; ++u) acc[u] = fma((double)vv[u], (double)xv[u], acc[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (ok[u]) x.addy(y, ld_nt(rowid + d.rowid_off + r0 + u * S * kWave + lane), acc[u]);
  }
}

// Any layout, any padding (used when the rectangle is not 64-aligned).
template <int S, class G>
__device__ inline void generic_wl(const Wl& d, int lane, int layout, const int32_t* __restrict__ idx,
                                  const float* __restrict__ val, const int32_t* __restrict__ rowid,
                                  const G& x, float* __restrict__ y, double* __restrict__ partial,
                                  int32_t sl) {
  if (layout == kCM) {
    const int64_t hp = d.h_pad;
    for (int32_t r = sl * kWave + lane; r < d.n_rows; r += kWave * S) {
      double acc = 0.0;
      for (int32_t c = 0; c < d.w_pad; ++c) {
        const int64_t e = d.data_off + (int64_t)c * hp + r;
        acc = fma((double)val[e], (double)x(idx[e]), acc);
      }
      x.addy(y, rowid[d.rowid_off + r], acc);
    }
    return;
  }
  const int64_t wp = d.w_pad;
  for (int32_t r = sl; r < d.n_rows; r += S) {
    const int64_t base = d.data_off + r * wp;
    double acc = 0.0;
    for (int64_t c = lane; c < wp; c += kWave) acc = fma((double)val[base + c], (double)x(idx[base + c]), acc);
    acc = wave_total(acc);
    if (lane == kWave - 1) {
      if (layout == kChunk)
        partial[d.info >> 2] = acc;
      else
        x.addy(y, rowid[d.rowid_off + r], acc);
    }
  }
}

// y update of one row by a tile: the row's first writer stores fl32(s); a
// later tile (kAddFlag in the row id) stores fl32(y + s).  With NT the
// accesses are non-temporal.
template <bool NT>
__device__ inline void addy_policy(float* y, int32_t rid, double s) {
  if (rid & kAddFlag) {
    const int32_t row = rid & ~kAddFlag;
    if (NT) {
      const float o = __builtin_nontemporal_load(y + row);
      __builtin_nontemporal_store((float)((double)o + s), y + row);
    } else {
      y[row] = (float)((double)y[row] + s);
    }
  } else {
    if (NT)
      __builtin_nontemporal_store((float)s, y + rid);
    else
      y[rid] = (float)s;
  }
}

// x as read by a tile: straight from global memory (through L1/L2) ...
template <bool NT>
struct GlobalX {
  const float* __restrict__ x;
  __device__ float operator()(int32_t i) const { return x[i]; }
  __device__ void addy(float* y, int32_t row, double s) const { addy_policy<NT>(y, row, s); }
};
// ... or with the tile's first `lw` columns staged in LDS (the hottest ones:
// columns are sorted by decreasing length, so a tile's head carries most of
// its entries).
struct StagedX {
  const float* __restrict__ x;
  const float* xs;
  int32_t cb, lw;
  __device__ float operator()(int32_t i) const {
    const uint32_t k = (uint32_t)(i - cb);
    return k < (uint32_t)lw ? xs[k] : x[i];
  }
  __device__ void addy(float* y, int32_t row, double s) const { addy_policy<true>(y, row, s); }
};

// ... or with the PageRank update fused into the row writes (one tile: each
// row's value is final where it is written):
//   p'[row] = fl32(c (fl32(s) + d/n) + (1 - c)/n),
// the rounding of the separate update after a stored y.
struct PrX {
  const float* __restrict__ x;
  double c, dn, tele;
  __device__ float operator()(int32_t i) const { return x[i]; }
  __device__ void addy(float* y, int32_t rid, double s) const {
    y[rid & ~kAddFlag] = (float)(c * ((double)(float)s + dn) + tele);
  }
};

// ... or with the RWR restart of one query fused in (one tile):
//   r'[row] = fl32(c fl32(s) + (1 - c) [row == seed]),
// the rounding of the separate update after a stored y.
struct RwrX {
  const float* __restrict__ x;
  double c;
  int32_t seed;
  __device__ float operator()(int32_t i) const { return x[i]; }
  __device__ void addy(float* y, int32_t rid, double s) const {
    const int32_t row = rid & ~kAddFlag;
    y[row] = (float)(c * (double)(float)s + (row == seed ? 1.0 - c : 0.0));
  }
};

// ... or writing a private copy of y: every row of a tile is written once,
// so the copy is stored whatever the first-writer flag says.
struct PrivX {
  const float* __restrict__ x;
  __device__ float operator()(int32_t i) const { return x[i]; }
  __device__ void addy(float* y, int32_t rid, double s) const { y[rid & ~kAddFlag] = (float)s; }
};

template <int S = 1, class G>
__device__ __attribute__((always_inline)) inline void run_workload(const Wl& d, int lane, const int32_t* __restrict__ idx,
                                    const float* __restrict__ val, const int32_t* __restrict__ rowid, const G& x,
                                    float* __restrict__ y, double* __restrict__ partial, int32_t sl = 0) {
  const int layout = d.info & 3;
  const bool aligned = (d.data_off & 3) == 0;
  if (layout == kCM && (d.h_pad & 63) == 0) {
    // row blocks of this slice
    const int32_t blocks = ((d.n_rows + kWave - 1) / kWave - sl + S - 1) / S;
    if (blocks >= 8)
      cm_rows<8, 1, S>(d, lane, idx, val, rowid, x, y, sl);
    else if (blocks >= 4)
      cm_rows<4, 2, S>(d, lane, idx, val, rowid, x, y, sl);
    else if (blocks >= 2)
      cm_rows<2, 4, S>(d, lane, idx, val, rowid, x, y, sl);
    else
      cm_rows<1, 8, S>(d, lane, idx, val, rowid, x, y, sl);
  } else if (layout != kCM && aligned && (d.w_pad & 63) == 0) {
    rm_wide<S>(d, lane, idx, val, rowid, x, y, partial, layout == kChunk, sl);
  } else {
    generic_wl<S>(d, lane, layout, idx, val, rowid, x, y, partial, sl);
  }
}

// S wavefronts per workload of the tile (row slices; grid = workloads * S / 4).
template <bool YNT, int S>
__global__ void __launch_bounds__(kB) k_tile_spmv(const Wl* __restrict__ wl, int64_t n_wl,
                                                  const int32_t* __restrict__ idx, const float* __restrict__ val,
                                                  const int32_t* __restrict__ rowid, const float* __restrict__ x,
                                                  float* __restrict__ y, double* __restrict__ partial) {
  const int lane = lane_id();
  const int64_t w = (int64_t)blockIdx.x * kWpb + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (w >= n_wl * S) return;
  const Wl d = wl[w / S];
  run_workload<S>(d, lane, idx, val, rowid, GlobalX<YNT>{x}, y, partial, (int32_t)(w % S));
}

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

// Persistent tile pass: a few workgroups per CU stage the tile's hot x head
// [cb, cb + lw) in LDS, then every wavefront takes workloads from the tile's
// counter until none is left (each wavefront leaves once the counter passes
// n_wl, so the grid always drains).  The counter must be 0 at launch.
constexpr int kPB = 1024;  // threads of a persistent workgroup
__global__ void __launch_bounds__(kPB) k_tile_persist(const Wl* __restrict__ wl, int64_t n_wl,
                                                      const int32_t* __restrict__ idx, const float* __restrict__ val,
                                                      const int32_t* __restrict__ rowid, const float* __restrict__ x,
                                                      float* __restrict__ y, double* __restrict__ partial,
                                                      int32_t cb, int32_t lw, unsigned long long* __restrict__ counter) {
  extern __shared__ float xs[];
  for (int32_t k = threadIdx.x; k < lw; k += blockDim.x) xs[k] = x[cb + k];
  __syncthreads();
  const int lane = lane_id();
  const StagedX xg{x, xs, cb, lw};
  for (;;) {
    unsigned long long jj = 0;
    if (lane == 0) jj = atomicAdd(counter, 1ull);
    const int64_t j = (int64_t)__shfl(jj, 0, kWave);
    if (j >= n_wl) break;
    const Wl d = wl[j];
    run_workload(d, lane, idx, val, rowid, xg, y, partial);
  }
}

// p[0] + p[s] + ... + p[(n-1) s], added in that order; eight loads go out
// together (a split row can have dozens of chunks, summed by one thread)
__device__ inline double sum_slots(const double* __restrict__ p, int64_t n, int64_t s = 1) {
  double acc = 0.0;
  int64_t q = 0;
  for (; q + 8 <= n; q += 8) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = p[(q + u) * s];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += t[u];
  }
  for (; q < n; ++q) acc += p[q * s];
  return acc;
}

// Sum of every split row's chunks in (tile, chunk) order, added to y (or
// stored when no tile wrote the row).
__global__ void k_split_combine(const SplitRow* __restrict__ sr, int64_t n, const double* __restrict__ partial,
                                float* __restrict__ y, int force_add) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const SplitRow s = sr[i];
  const double acc = sum_slots(partial + s.slot_begin, s.n_slots);
  if (s.store && !force_add)
    y[s.row] = (float)acc;
  else
    add_to_y(y, s.row, acc);
}

// ---- multiple right-hand sides.  Pad entries (value 0) are skipped.
//
// SpMM, Y := A X with X row-major n_cols x k.  Each lane owns V consecutive
// right-hand sides (V = 4 when k is a multiple of 4 and X, Y are 16-byte
// aligned: one 16-byte load per gathered X row and lane).  A wavefront holds
// 64 / kg lane groups of kg lanes (kg = ceil(k / V) rounded up to a power of
// two, at most 64); lane q of a group owns right-hand sides
// V * (q + 64 * blockIdx.y) ... + V - 1, so every gathered X row is one
// coalesced access and one load instruction serves 64 / kg entries.
template <int V>
struct Vec {
  double a[V];
  __device__ void zero() {
#pragma unroll
    for (int i = 0; i < V; ++i) a[i] = 0.0;
  }
};

// Branch-free: an inactive lane (pad entry, or right-hand sides past k) reads
// X[0 .. V) and takes zeros.  A load under a branch would end its branch with
// a wait for that load (the conversions to double sink into it), so a step's
// gathers would go out one at a time instead of all together.
template <int V>
__device__ inline void load_x(const float* __restrict__ X, int64_t row, int32_t k, int32_t col, bool act, float* xv) {
  const int64_t o = act ? row * k + col : 0;
  if constexpr (V == 4) {
    const float4 t = *(const float4*)(X + o);
    xv[0] = act ? t.x : 0.0f;
    xv[1] = act ? t.y : 0.0f;
    xv[2] = act ? t.z : 0.0f;
    xv[3] = act ? t.w : 0.0f;
  } else {
    const float t = X[o];
    xv[0] = act ? t : 0.0f;
  }
}

template <int V>
__device__ inline void fma_vec(Vec<V>& acc, float v, const float* xv) {
#pragma unroll
  for (int i = 0; i < V; ++i) acc.a[i] = fma((double)v, (double)xv[i], acc.a[i]);
}

template <int V>
__device__ inline void add_y(float* __restrict__ Y, int32_t rid, int32_t k, int32_t col, const Vec<V>& s) {
  const bool add = (rid & kAddFlag) != 0;
  float* p = Y + (int64_t)(rid & ~kAddFlag) * k + col;
  if constexpr (V == 4) {
    float4 o;
    if (add) {
      const float4 t = *(const float4*)p;
      o = make_float4((float)((double)t.x + s.a[0]), (float)((double)t.y + s.a[1]), (float)((double)t.z + s.a[2]),
                      (float)((double)t.w + s.a[3]));
    } else {
      o = make_float4((float)s.a[0], (float)s.a[1], (float)s.a[2], (float)s.a[3]);
    }
    *(float4*)p = o;
  } else {
    *p = add ? (float)((double)*p + s.a[0]) : (float)s.a[0];
  }
}

// RWR restart fused into the product (one tile: each row's value is final
// where it is written): R'[row][q] = fl32(c fl32(y) + (1 - c) [row == seed_q]),
// the same rounding as the separate update after a stored y.
struct RwrEpi {
  double c;
  const int32_t* seeds;  // internal ids, one per right-hand side
};

__device__ inline float rwr_restart(double c, float y, bool is_seed) {
  return (float)(c * (double)y + (is_seed ? 1.0 - c : 0.0));
}

template <int V>
__device__ inline void rwr_y(float* __restrict__ Y, int32_t rid, int32_t k, int32_t col, const Vec<V>& s,
                             const RwrEpi& epi, const int32_t* seeds_lds) {
  const int32_t* sd = seeds_lds + col;
  const int32_t row = rid & ~kAddFlag;
  float* p = Y + (int64_t)row * k + col;
  float o[V];
#pragma unroll
  for (int i = 0; i < V; ++i) o[i] = rwr_restart(epi.c, (float)s.a[i], row == sd[i]);
  if constexpr (V == 4)
    *(float4*)p = make_float4(o[0], o[1], o[2], o[3]);
  else
    *p = o[0];
}

// Cross-group sum of a row-major row: the groups took interleaved entries,
// and an xor tree over the group bits of the lane id adds their sums.
template <int V>
__device__ inline void group_sum(Vec<V>& s, int kg) {
  for (int o = kg; o < kWave; o <<= 1)
#pragma unroll
    for (int i = 0; i < V; ++i) s.a[i] += __shfl_xor(s.a[i], o, kWave);
}

// One step over RS consecutive matrix slots: lane l < RS loads slot l with one
// coalesced load (value and index), then in sub-step u (u < RS / groups) lane
// group g takes slot u * groups + g by a lane shuffle and gathers that X row.
// So the wavefront issues two matrix loads per RS entries instead of two per
// sub-step.
template <int V, int SUB = 8>
__device__ inline void step_gather(float vl, int32_t il, int subs, int groups, int g, const float* __restrict__ X,
                                   int32_t k, int32_t col, bool act, float* v, float (*xv)[V]) {
  int32_t ii[SUB];
#pragma unroll
  for (int u = 0; u < SUB; ++u) {
    if (u < subs) {
      const int src = u * groups + g;
      v[u] = __shfl(vl, src, kWave);
      ii[u] = __shfl(il, src, kWave);
    } else {
      v[u] = 0.0f;
      ii[u] = 0;
    }
  }
#pragma unroll
  for (int u = 0; u < SUB; ++u) load_x<V>(X, ii[u], k, col, act && v[u] != 0.0f, xv[u]);
}

// entries [lo, hi) of the row-major row at `base`; slot u * groups + g of each
// step goes to group g, so this lane's sums cover the entries c with
// (c - lo) mod 64 in its group's residues, in increasing c
template <int V>
__device__ inline Vec<V> rm_range(const int32_t* __restrict__ idx, const float* __restrict__ val,
                                  const float* __restrict__ X, int64_t base, int64_t lo, int64_t hi, int32_t k,
                                  int32_t col, bool act, int g, int groups, int lane) {
  const int rs = min(kWave, groups * 8), subs = rs / groups;
  Vec<V> acc;
  acc.zero();
  for (int64_t c0 = lo; c0 < hi; c0 += rs) {
    const bool in = lane < rs && c0 + lane < hi;
    const float vl = in ? ld_nt(val + base + c0 + lane) : 0.0f;
    const int32_t il = in ? ld_nt(idx + base + c0 + lane) : 0;
    float v[8], xv[8][V];
    step_gather<V>(vl, il, subs, groups, g, X, k, col, act, v, xv);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (v[u] != 0.0f) fma_vec<V>(acc, v[u], xv[u]);
  }
  return acc;
}

// Every workload but the leading chunk workloads of a tile (those go to
// k_spmm_chunks); `pieces` = slots per chunk in `partial` (1 when a chunk
// shows up here: it is then done whole, as one piece).
// SUB: rows summed per lane group in one column step (accumulators per lane).
// `slices` wavefronts share a workload, slice s taking every slices-th step.
// RWR: rows are written through the fused restart (epi) instead of stored.
template <int V, int SUB, bool RWR = false>
__global__ void __launch_bounds__(kB) k_tile_spmm(const Wl* __restrict__ wl, int64_t n_wl, int32_t slices,
                                                  const int32_t* __restrict__ idx,
                                                  const float* __restrict__ val, const int32_t* __restrict__ rowid,
                                                  const float* __restrict__ X, float* __restrict__ Y, int32_t k,
                                                  int32_t kg, double* __restrict__ partial, RwrEpi epi) {
  // fused restart: the seeds (k <= kB) in LDS, read only where rows are written
  __shared__ int32_t sd[RWR ? kB : 1];
  if constexpr (RWR) {
    if ((int32_t)threadIdx.x < k) sd[threadIdx.x] = epi.seeds[threadIdx.x];
    __syncthreads();
  }
  const int lane = lane_id();
  const int64_t w = (int64_t)blockIdx.x * kWpb + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (w >= n_wl * slices) return;
  const int64_t j = w / slices;
  const int32_t sl = (int32_t)(w % slices);
  const int groups = kWave / kg;
  const int g = lane / kg;
  const int32_t col = ((int32_t)blockIdx.y * kg + lane % kg) * V;
  const bool act = col < k;
  const Wl d = wl[j];
  const int layout = d.info & 3;
  const int64_t off = d.data_off;
  if (layout == kCM) {
    // RS rows per step: lane l loads row r0 + l's entry of column c, and row
    // r0 + u * groups + g is summed by group g in sub-step u, in column order
    const int rs = min(kWave, groups * SUB), subs = rs / groups;
    const int64_t hp = d.h_pad;
    for (int32_t r0 = sl * rs; r0 < d.n_rows; r0 += rs * slices) {
      const bool okl = lane < rs && r0 + lane < d.n_rows;
      Vec<V> a[SUB];
#pragma unroll
      for (int u = 0; u < SUB; ++u) a[u].zero();
      // column c + 1's entries are loaded while column c's X rows are in
      // flight (a lane past the rows reads the workload's first entry)
      const int64_t eb = okl ? off + r0 + lane : off;
      const int64_t es = okl ? hp : 0;
      float nv = ld_nt(val + eb);
      int32_t ni = ld_nt(idx + eb);
      for (int32_t c = 0; c < d.w_pad; ++c) {
        const float vl = okl ? nv : 0.0f;
        const int32_t il = okl ? ni : 0;
        float v[SUB], xv[SUB][V];
        step_gather<V, SUB>(vl, il, subs, groups, g, X, k, col, act, v, xv);
        const int64_t en = eb + (c + 1 < d.w_pad ? (int64_t)(c + 1) * es : 0);
        nv = ld_nt(val + en);
        ni = ld_nt(idx + en);
#pragma unroll
        for (int u = 0; u < SUB; ++u)
          if (v[u] != 0.0f) fma_vec<V>(a[u], v[u], xv[u]);
      }
      if (act) {
#pragma unroll
        for (int u = 0; u < SUB; ++u) {
          const int32_t r = r0 + u * groups + g;
          if (u < subs && r < d.n_rows) {
            if constexpr (RWR)
              rwr_y<V>(Y, ld_nt(rowid + d.rowid_off + r), k, col, a[u], epi, sd);
            else
              add_y<V>(Y, ld_nt(rowid + d.rowid_off + r), k, col, a[u]);
          }
        }
      }
    }
  } else {
    const int64_t wp = d.w_pad;
    for (int32_t r = sl; r < d.n_rows; r += slices) {
      Vec<V> acc = rm_range<V>(idx, val, X, off + (int64_t)r * wp, 0, wp, k, col, act, g, groups, lane);
      group_sum<V>(acc, kg);
      if (act && g == 0) {
        if (layout == kChunk) {
#pragma unroll
          for (int i = 0; i < V; ++i) partial[(int64_t)(d.info >> 2) * k + col + i] = acc.a[i];
        } else {
          if constexpr (RWR)
            rwr_y<V>(Y, ld_nt(rowid + d.rowid_off + r), k, col, acc, epi, sd);
          else
            add_y<V>(Y, ld_nt(rowid + d.rowid_off + r), k, col, acc);
        }
      }
    }
  }
}

// Chunk workloads of one tile (a split row's pieces of w_pad entries): wave
// w takes entries [p*kPiece, (p+1)*kPiece) of chunk w / pieces, p = w % pieces,
// and writes its sums to slot (chunk slot * pieces + p) of `partial`.
constexpr int kPiece = 512;
template <int V>
__global__ void __launch_bounds__(kB) k_spmm_chunks(const Wl* __restrict__ wl, int64_t n_wl, int32_t pieces,
                                                    const int32_t* __restrict__ idx, const float* __restrict__ val,
                                                    const float* __restrict__ X, int32_t k, int32_t kg,
                                                    double* __restrict__ partial) {
  const int lane = lane_id();
  const int64_t w = (int64_t)blockIdx.x * kWpb + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (w >= n_wl * pieces) return;
  const int64_t j = w / pieces;
  const int32_t p = (int32_t)(w % pieces);
  const int groups = kWave / kg;
  const int g = lane / kg;
  const int32_t col = ((int32_t)blockIdx.y * kg + lane % kg) * V;
  const bool act = col < k;
  const Wl d = wl[j];
  const int64_t lo = min<int64_t>((int64_t)p * kPiece, d.w_pad), hi = min<int64_t>(lo + kPiece, d.w_pad);
  Vec<V> acc = rm_range<V>(idx, val, X, d.data_off, lo, hi, k, col, act, g, groups, lane);
  group_sum<V>(acc, kg);
  if (act && g == 0)
#pragma unroll
    for (int i = 0; i < V; ++i) partial[((int64_t)(d.info >> 2) * pieces + p) * k + col + i] = acc.a[i];
}

// Zero the rows no workload writes: block b takes rows b * rpb ..., thread
// (r, q) of the block row r's entries q, q + kk, ... (kk = min(k, kB))
// (with the fused restart, epi.seeds != NULL: the rows' restart values)
__global__ void k_begin_spmm(float* __restrict__ Y, const int32_t* __restrict__ empty, int64_t n_empty, int32_t k,
                             RwrEpi epi) {
  const int32_t kk = min(k, kB), rpb = kB / kk;
  const int32_t r = threadIdx.x / kk, q0 = threadIdx.x % kk;
  if (r >= rpb) return;
  for (int64_t i = (int64_t)blockIdx.x * rpb + r; i < n_empty; i += (int64_t)gridDim.x * rpb) {
    const int32_t e = empty[i];
    float* row = Y + (int64_t)e * k;
    for (int32_t q = q0; q < k; q += kk) row[q] = epi.seeds ? rwr_restart(epi.c, 0.0f, e == epi.seeds[q]) : 0.0f;
  }
}

__global__ void k_split_combine_mm(const SplitRow* __restrict__ sr, int64_t n, const double* __restrict__ partial,
                                   int32_t pieces, float* __restrict__ Y, int32_t k, RwrEpi epi) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * k) return;
  const int64_t i = t / k;
  const int32_t q = (int32_t)(t % k);
  const SplitRow s = sr[i];
  const int64_t u0 = (int64_t)s.slot_begin * pieces;
  const double acc = sum_slots(partial + u0 * k + q, (int64_t)s.n_slots * pieces, k);
  if (epi.seeds)  // fused restart (one tile: the chunks are all of the row)
    Y[(int64_t)s.row * k + q] = rwr_restart(epi.c, (float)acc, s.row == epi.seeds[q]);
  else if (s.store)
    Y[(int64_t)s.row * k + q] = (float)acc;
  else
    add_to_y(Y + (int64_t)s.row * k, q, acc);
}

// ---- plain CSR baseline: one thread per row (FP64 accumulation)
__global__ void k_csr_scalar(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                             const float* __restrict__ val, int64_t n_rows, const float* __restrict__ x,
                             float* __restrict__ y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_rows) return;
  double acc = 0.0;
  for (int64_t k = rp[i]; k < rp[i + 1]; ++k) acc = fma((double)val[k], (double)x[col[k]], acc);
  y[i] = (float)acc;
}

// ---- vector kernels
__global__ void k_fill_f32(float* __restrict__ a, int64_t n, float v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// out[k*row_stride + q] = in[perm[k]*row_stride + q]   (rows gathered)
__global__ void k_gather_rows(const float* __restrict__ in, const int32_t* __restrict__ perm, int64_t n, int32_t w,
                              float* __restrict__ out) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * w) return;
  const int64_t k = t / w;
  const int32_t q = (int32_t)(t % w);
  out[t] = in[(int64_t)perm[k] * w + q];
}

template <int NV>
__device__ inline void block_sum_store(double (&v)[NV], double* out_base, int64_t stride) {
  __shared__ double sm[NV][kB / kWave];
  const int lane = lane_id(), wv = threadIdx.x / kWave;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = wave_sum(v[q]);
    if (lane == 0) sm[q][wv] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double s = 0.0;
      for (int w = 0; w < kB / kWave; ++w) s += sm[q][w];
      out_base[q * stride] = s;
    }
  }
}

constexpr int kRedBlocks = 1024;

// Sum of nparts consecutive partials for each of nv quantities, fixed order:
// one wavefront per quantity (lane-strided sums, then the wavefront's tree),
// quantities spread over the wavefronts of the grid.
__global__ void k_finish(const double* __restrict__ parts, int nparts, int nv, double* __restrict__ out) {
  const int lane = lane_id();
  for (int q = blockIdx.x * kWpb + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave); q < nv;
       q += gridDim.x * kWpb) {
    const double* pq = parts + (int64_t)q * nparts;
    double s = 0.0;
    for (int i0 = lane; i0 < nparts; i0 += 8 * kWave) {  // eight loads in flight (past the end: pq[0], not added)
      double t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = pq[i0 + u * kWave < nparts ? i0 + u * kWave : 0];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += i0 + u * kWave < nparts ? t[u] : 0.0;
    }
    s = wave_sum(s);
    if (lane == 0) out[q] = s;
  }
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

// ---- several graphs per launch (batched RWR over many small graphs)
//
// One launch runs tile t of every graph.  A segment is one graph's tile t:
// its workloads, matrix arrays and vectors; `begin` is the number of
// workloads of the launch before it, so wavefront j belongs to the last
// segment with begin <= j.
struct MultiSeg {
  const Wl* wl;
  int64_t begin;
  const int32_t* idx;
  const float* val;
  const int32_t* rowid;
  const float* x;
  float* y;
  double* partial;
  int64_t seed;  // internal id of the graph's restart node (fused RWR step)
};

// last i in [0, n) with key(i) <= j (keys increasing, key(0) = 0)
template <class K>
__device__ inline int last_le(int n, int64_t j, K key) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (key(mid) <= j) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// MultiSeg as the kernel reads it: the same layout with every pointer typed
// as device global memory.  A plain pointer read from memory is generic to the
// compiler, and every access through it would be a flat (not global) access.
#define TC_GLOBAL __attribute__((address_space(1)))
struct MultiSegG {
  const Wl* wl;  // one record per wavefront: left generic
  int64_t begin;
  const TC_GLOBAL int32_t* idx;
  const TC_GLOBAL float* val;
  const TC_GLOBAL int32_t* rowid;
  const TC_GLOBAL float* x;
  TC_GLOBAL float* y;
  TC_GLOBAL double* partial;
  int64_t seed;
};
#undef TC_GLOBAL
static_assert(sizeof(MultiSegG) == sizeof(MultiSeg), "MultiSegG mirrors MultiSeg");

// the same with the RWR restart of each graph fused into its row writes
__global__ void __launch_bounds__(kB) k_tile_spmv_multi_rwr(const MultiSeg* __restrict__ segs, int32_t n_segs,
                                                            int64_t total, double c) {
  const int lane = lane_id();
  const int64_t j = (int64_t)blockIdx.x * kWpb + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (j >= total) return;
  const int i = __builtin_amdgcn_readfirstlane(last_le(n_segs, j, [&](int m) { return segs[m].begin; }));
  const MultiSegG s = ((const MultiSegG*)segs)[i];
  run_workload(s.wl[j - s.begin], lane, (const int32_t*)s.idx, (const float*)s.val, (const int32_t*)s.rowid,
               RwrX{(const float*)s.x, c, (int32_t)s.seed}, (float*)s.y, (double*)s.partial);
}

__global__ void __launch_bounds__(kB) k_tile_spmv_multi(const MultiSeg* __restrict__ segs, int32_t n_segs,
                                                        int64_t total) {
  const int lane = lane_id();
  const int64_t j = (int64_t)blockIdx.x * kWpb + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (j >= total) return;
  const int i = __builtin_amdgcn_readfirstlane(last_le(n_segs, j, [&](int m) { return segs[m].begin; }));
  const MultiSegG s = ((const MultiSegG*)segs)[i];
  run_workload(s.wl[j - s.begin], lane, (const int32_t*)s.idx, (const float*)s.val, (const int32_t*)s.rowid,
               GlobalX<false>{(const float*)s.x}, (float*)s.y, (double*)s.partial);
}

// Per-graph element ranges: [begin, begin + n) of the launch's index space.
struct MultiVec {
  int64_t begin, n;
  const int32_t* list;      // empty rows / split rows
  const SplitRow* split;
  const double* partial;
  float* y;                 // product of the graph
  float* r;                 // iterate of the graph (RWR)
  int32_t seed;             // internal id of the restart node
};

__global__ void k_begin_multi(const MultiVec* __restrict__ v, int32_t nv, int64_t total) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const MultiVec m = v[last_le(nv, t, [&](int q) { return v[q].begin; })];
  m.y[m.list[t - m.begin]] = 0.0f;
}

__global__ void k_split_combine_multi(const MultiVec* __restrict__ v, int32_t nv, int64_t total) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const MultiVec m = v[last_le(nv, t, [&](int q) { return v[q].begin; })];
  const SplitRow s = m.split[t - m.begin];
  const double acc = sum_slots(m.partial + s.slot_begin, s.n_slots);
  if (s.store)
    m.y[s.row] = (float)acc;
  else
    add_to_y(m.y, s.row, acc);
}

// Fused RWR step of every graph, the rows the tile kernel does not write:
// split rows (index space [0, s_tot) of spl) and rows without entries
// ([s_tot, s_tot + e_tot), of emp), same formula as RwrX.
__global__ void k_rwr_rest_multi(const MultiVec* __restrict__ spl, const MultiVec* __restrict__ emp, int32_t nv,
                                 int64_t s_tot, int64_t e_tot, double c) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < s_tot) {
    const MultiVec m = spl[last_le(nv, t, [&](int q) { return spl[q].begin; })];
    const SplitRow s = m.split[t - m.begin];
    const double acc = sum_slots(m.partial + s.slot_begin, s.n_slots);
    m.y[s.row] = (float)(c * (double)(float)acc + (s.row == m.seed ? 1.0 - c : 0.0));
  } else if (t < s_tot + e_tot) {
    const int64_t u = t - s_tot;
    const MultiVec m = emp[last_le(nv, u, [&](int q) { return emp[q].begin; })];
    const int32_t row = m.list[u - m.begin];
    m.y[row] = (float)(c * (double)0.0f + (row == m.seed ? 1.0 - c : 0.0));
  }
}

// RWR step of every graph, r <- c y + (1 - c) e_seed, with the L1 change.
// Blocks never straddle graphs: block b works on graph g's elements
// [(b - bbeg_g) * kB * kMultiPer, ...) and writes its partial change to parts[b].
constexpr int kMultiPer = 16;
__global__ void __launch_bounds__(kB) k_rwr_update_multi(const MultiVec* __restrict__ v,
                                                         const int32_t* __restrict__ block_graph,
                                                         const int64_t* __restrict__ block_first, double c,
                                                         double* __restrict__ parts) {
  const int b = blockIdx.x;
  const MultiVec m = v[block_graph[b]];
  const int64_t lo = block_first[b] * (int64_t)kB * kMultiPer;
  const int64_t hi = min(m.n, lo + (int64_t)kB * kMultiPer);
  double d[1] = {0.0};
  for (int64_t i = lo + threadIdx.x; i < hi; i += kB) {
    const float rn = (float)(c * (double)m.y[i] + (i == m.seed ? 1.0 - c : 0.0));
    d[0] += fabs((double)rn - (double)m.r[i]);
    m.r[i] = rn;
  }
  block_sum_store<1>(d, parts + b, 0);
}

// per graph: sum of its blocks' changes (in block order); then the largest
__global__ void k_multi_resid(const int64_t* __restrict__ graph_blocks, int32_t ng, const double* __restrict__ parts,
                              double* __restrict__ resid, double* __restrict__ mx) {
  __shared__ double sm[kB];
  double m = 0.0;
  for (int g = threadIdx.x; g < ng; g += kB) {
    double s = 0.0;
    for (int64_t b = graph_blocks[g]; b < graph_blocks[g + 1]; ++b) s += parts[b];
    resid[g] = s;
    m = fmax(m, s);
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < kB; ++i) t = fmax(t, sm[i]);
    *mx = t;
  }
}

__global__ void k_rwr_init_multi(const MultiVec* __restrict__ v, int32_t nv, int64_t total) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const MultiVec m = v[last_le(nv, t, [&](int q) { return v[q].begin; })];
  const int64_t i = t - m.begin;
  m.r[i] = i == m.seed ? 1.0f : 0.0f;
}

__global__ void k_map_ids_multi(const int32_t* const* __restrict__ maps, const int32_t* __restrict__ ids, int32_t n,
                                int32_t* __restrict__ out) {
  for (int32_t g = threadIdx.x; g < n; g += blockDim.x) out[g] = maps[g][ids[g]];
}

// ---- differentiable RWR: learned edge weights (Appendix F, Eq. 9)
//
// z_e = theta . f_e, w_e = softplus(z_e), W_e = w_e / S_j with S_j the sum of
// w over column j.  The per-entry arrays of the gradient (features, z, w, G)
// are kept in the order of A^T's CSR (the columns of A, each by increasing
// row), so every column quantity is a contiguous segmented pass; the values
// of W in A's own order are computed from A's copy of the features.
__device__ inline double softplus_d(double z) { return fmax(z, 0.0) + log1p(exp(-fabs(z))); }

// w of one entry; the same arithmetic in both orders, so W and W^T get
// bit-identical values
__device__ inline double edge_w(const float* __restrict__ f, const double* __restrict__ theta, int32_t nf,
                                double* z_out) {
  double a = 0.0;
  for (int32_t d = 0; d < nf; ++d) a = fma((double)f[d], theta[d], a);
  if (z_out) *z_out = a;
  return softplus_d(a);
}

__global__ void k_edge_softplus(const float* __restrict__ featsT, int64_t nnz, int32_t nf,
                                const double* __restrict__ theta, double* __restrict__ zT, double* __restrict__ wT) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nnz) return;
  double z;
  wT[q] = edge_w(featsT + q * nf, theta, nf, &z);
  zT[q] = z;
}

// W in A's order: val_e = fl32(w_e / S_col(e))
__global__ void k_edge_values(const float* __restrict__ feats, const int32_t* __restrict__ col, int64_t nnz,
                              int32_t nf, const double* __restrict__ theta, const double* __restrict__ S,
                              float* __restrict__ val) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) val[e] = (float)(edge_w(feats + e * nf, theta, nf, nullptr) / S[col[e]]);
}

// Column sums over A^T's CSR: one wavefront per kColLanes-column group, a
// group of kColLanes lanes per column, and a column of more than kColLong
// entries by the whole wavefront (with more loads in flight).  Every lane
// loads (a lane past the column's end at the column's first entry) and adds
// only its own entries.  The per-entry passes that need a column's sum are
// flat passes over the entries (the column of entry q: rowT[q]).
constexpr int kColLanes = 8;
constexpr int kColLong = 512;
constexpr int kGradBlocks = 1024;
constexpr int kMaxFeat = 16;

// sum over each aligned group of kColLanes lanes (every lane gets the same bits)
__device__ inline double group_sum8(double v) {
  v += __shfl_xor(v, 1, kWave);
  v += __shfl_xor(v, 2, kWave);
  v += __shfl_xor(v, 4, kWave);
  return v;
}

// this lane's part of the sum over q in [a, b) of f(q): LANES lanes from
// offset gl, U loads in flight
template <int LANES, int U, class F>
__device__ inline double seg_part(int64_t a, int64_t b, int gl, F f) {
  double s = 0.0;
  for (int64_t q0 = a + gl; q0 < b; q0 += U * LANES) {
    double t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t q = q0 + u * LANES;
      t[u] = f(q < b ? q : a);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) s += q0 + u * LANES < b ? t[u] : 0.0;
  }
  return s;
}

// out[j] = post(j, sum over column j's entries q of f(q))
template <class F, class P>
__device__ inline void col_sums(const int64_t* __restrict__ rpT, int64_t n_cols, F f, P post,
                                double* __restrict__ out) {
  const int lane = lane_id(), gl = lane % kColLanes;
  const int64_t cg = (int64_t)blockIdx.x * kWpb + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t j0 = cg * (kWave / kColLanes);
  if (j0 >= n_cols) return;
  const int64_t j = j0 + lane / kColLanes;
  int64_t a = 0, b = 0;
  if (j < n_cols) {
    a = rpT[j];
    b = rpT[j + 1];
  }
  const bool lng = b - a > kColLong;
  const double s = group_sum8(lng || j >= n_cols ? 0.0 : seg_part<kColLanes, 4>(a, b, gl, f));
  if (!lng && j < n_cols && gl == 0) out[j] = post(j, s);
  for (uint64_t m = __ballot(lng && gl == 0); m; m &= m - 1) {
    const int src = __ffsll((unsigned long long)m) - 1;
    const int64_t jj = j0 + src / kColLanes;
    const int64_t aa = __shfl(a, src, kWave), bb = __shfl(b, src, kWave);
    const double t = wave_sum(seg_part<kWave, 16>(aa, bb, lane, f));
    if (lane == 0) out[jj] = post(jj, t);
  }
}

// S_j = sum of w over column j
__global__ void __launch_bounds__(kB) k_col_norm(const int64_t* __restrict__ rpT, int64_t n_cols,
                                                 const double* __restrict__ wT, double* __restrict__ S) {
  col_sums(
      rpT, n_cols, [&](int64_t q) { return wT[q]; }, [](int64_t, double s) { return s; }, S);
}

// W^T's values fl32(w / S_j)
__global__ void k_values_T(const int32_t* __restrict__ rowT, int64_t nnz, const double* __restrict__ wT,
                           const double* __restrict__ S, float* __restrict__ valT) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nnz) valT[q] = (float)(wT[q] / S[rowT[q]]);
}

// r_next = fl32(c y + (1 - c) [i == seed]) (the same rounding as k_rwr_update)
__global__ void k_rwr_step(const float* __restrict__ y, float* __restrict__ r, int64_t n, int32_t seed, double c) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) r[i] = (float)(c * (double)y[i] + (i == seed ? 1.0 - c : 0.0));
}

__global__ void k_scale(const float* __restrict__ y, float* __restrict__ g, int64_t n, double c) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) g[i] = (float)(c * (double)y[i]);
}

// G_q += sum over the steps of one checkpoint segment, latest step first, of
// g^{k+1}_i r^k_j for the entry q = (i, j) of A (row j of A^T, column i of
// A^T: gidx = A^T's column array, ridx = A^T's row of every entry).  gi and ri
// hold g^{k+1} and r^k of the segment's m steps k = k0 + t interleaved by node
// (node i's m values at i * m), so an entry reads its values from one or two
// cache lines.
__global__ void k_edge_accum_seg(const int32_t* __restrict__ gidx, const int32_t* __restrict__ ridx, int64_t nnz,
                                 const float* __restrict__ gi, const float* __restrict__ ri, int32_t m,
                                 double* __restrict__ G) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nnz) return;
  const float* gp = gi + (int64_t)gidx[q] * m;
  const float* rp = ri + (int64_t)ridx[q] * m;
  double acc = G[q];
  for (int32_t t = m - 1; t >= 0; --t) acc = fma((double)gp[t], (double)rp[t], acc);
  G[q] = acc;
}

// dst[i * m + t] = src[t * n + i]: m vectors of n, interleaved by index
__global__ void k_interleave(const float* __restrict__ src, int32_t m, int64_t n, float* __restrict__ dst) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n * m) return;
  dst[x] = src[(x % m) * n + x / m];
}


// row index of every entry: short rows by their thread, long rows (> 64
// entries) by the whole wavefront in turn
__global__ void k_rows_of(const int64_t* __restrict__ rp, int64_t n_rows, int32_t* __restrict__ row_of) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = lane_id();
  int64_t a = 0, b = 0;
  if (i < n_rows) {
    a = rp[i];
    b = rp[i + 1];
  }
  const bool longrow = (b - a) > kWave;
  if (!longrow)
    for (int64_t e = a; e < b; ++e) row_of[e] = (int32_t)i;
  uint64_t m = __ballot(longrow);
  while (m) {
    const int src = __ffsll((unsigned long long)m) - 1;
    m &= m - 1;
    const int64_t aa = __shfl(a, src, kWave), bb = __shfl(b, src, kWave);
    const int32_t r = (int32_t)__shfl((int64_t)i, src, kWave);
    for (int64_t e = aa + lane; e < bb; e += kWave) row_of[e] = r;
  }
}

__global__ void k_onehot(float* __restrict__ r, int64_t n, int32_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) r[i] = i == seed ? 1.0f : 0.0f;
}

// per column j: cs_j = sum over its entries of dL/dW W, with dL/dW = c G and
// W = w / S_j, taken as (c / S_j) sum G w
__global__ void __launch_bounds__(kB) k_col_dot(const int64_t* __restrict__ rpT, int64_t n_cols,
                                                const double* __restrict__ GT, const double* __restrict__ wT,
                                                const double* __restrict__ S, double c, double* __restrict__ cs) {
  col_sums(
      rpT, n_cols, [&](int64_t q) { return GT[q] * wT[q]; }, [&](int64_t j, double s) { return c / S[j] * s; },
      cs);
}

// dL/dz = (c G - cs_j) / S_j * sigmoid(z) per entry (column j = rowT[q]);
// per-block partial sums of dL/dz f (nf of them), combined afterwards in
// block order
__global__ void __launch_bounds__(kB) k_theta_grad(const int32_t* __restrict__ rowT, int64_t nnz, int32_t nf,
                                                   const float* __restrict__ featsT, const double* __restrict__ zT,
                                                   const double* __restrict__ S, const double* __restrict__ GT,
                                                   const double* __restrict__ cs, double c,
                                                   double* __restrict__ parts) {
  double acc[kMaxFeat];
#pragma unroll
  for (int d = 0; d < kMaxFeat; ++d) acc[d] = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * kB + threadIdx.x; q < nnz; q += (int64_t)gridDim.x * kB) {
    const int32_t j = rowT[q];
    const double dz = (c * GT[q] - cs[j]) / S[j] / (1.0 + exp(-zT[q]));
#pragma unroll
    for (int d = 0; d < kMaxFeat; ++d)
      if (d < nf) acc[d] = fma(dz, (double)featsT[q * nf + d], acc[d]);
  }
  __shared__ double sm[kMaxFeat][kB / kWave];
  const int lane = lane_id(), wv = threadIdx.x / kWave;
#pragma unroll
  for (int d = 0; d < kMaxFeat; ++d) {
    const double t = wave_sum(acc[d]);
    if (lane == 0) sm[d][wv] = t;
  }
  __syncthreads();
  if ((int32_t)threadIdx.x < nf) {
    double t = 0.0;
    for (int q = 0; q < kB / kWave; ++q) t += sm[threadIdx.x][q];
    parts[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
  }
}

// ------------------------------------------------------------ host side
struct Err {
  tc_status st;
  std::string msg;
};

#define HIPC(call)                                                          \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) throw Err{TC_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

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

template <typename... KArgs, typename... Args>
void launch_tile(tc_handle* h, void (*kern)(KArgs...), dim3 grid, dim3 block, uint32_t shmem, hipStream_t st,
                 Args... args) {
  if (h->timing) {
    hipEvent_t a = next_event(h), b = next_event(h);
    hipExtLaunchKernelGGL(kern, grid, block, shmem, st, a, b, 0, args...);
    h->tile_launches++;
  } else {
    hipLaunchKernelGGL(kern, grid, block, shmem, st, args...);
  }
  HIPC(hipGetLastError());
}

// Start of a product: zero the rows no tile writes, reset the tile counters.
__global__ void k_begin_spmv(float* __restrict__ y, const int32_t* __restrict__ empty, int64_t n_empty,
                             unsigned long long* __restrict__ counters, int32_t nt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_empty) y[empty[i]] = 0.0f;
  if (i < nt) counters[i] = 0ull;
}

// Launch shape of the tile passes (defaults from measurement; the
// environment variables TC_LDS_FLOATS and TC_PERSIST override them).
struct TileConfig {
  int persist = 0;
  int lds_floats = 32768;
  int y_nt = 0;
  // row slices: S wavefronts share each workload of the single-vector tile
  // kernels, slice s taking every S-th 64-row block (column-major) or row
  // (row-major). Each row is still summed whole by one lane or one wavefront
  // in the same order, so the result does not depend on S. It evens out the
  // tail of the launch; on a 2^27-entry Chung-Lu matrix (WL 8183) the
  // product takes 1064 / 1032 / 998 / 1325 us with S = 1 / 2 / 4 / 8.
  int slices = 4;
};
TileConfig tile_config() {
  static TileConfig cfg = [] {
    TileConfig c;
    if (const char* e = getenv("TC_PERSIST")) c.persist = atoi(e);
    if (const char* e = getenv("TC_LDS_FLOATS")) c.lds_floats = atoi(e);
    if (const char* e = getenv("TC_Y_NT")) c.y_nt = atoi(e);
    if (const char* e = getenv("TC_TILE_SLICES")) c.slices = atoi(e) >= 8 ? 8 : atoi(e) >= 4 ? 4 : atoi(e) >= 2 ? 2 : 1;
    int dev = 0, maxsh = 65536;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&maxsh, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) maxsh = 65536;
    c.lds_floats = std::max(0, std::min(c.lds_floats, maxsh / 4));
    return c;
  }();
  return cfg;
}

// the instance of a tile kernel for the configured number of row slices
// Slices pay where workloads are large and many. A tile of fewer than
// kSliceMinWl workloads, or with a workload size below kSliceMinSize entries,
// runs one slice per workload: there the extra wavefronts cost more than they
// balance (R-MAT 20 at WL 512: 85 us with one slice, 90 us with four; 32
// small R-MAT graphs at WL 128-256, one after another: 13.1 ms with one,
// 15.3 ms with four; at WL 1984 four slices win, 98 against 104 us).
constexpr int64_t kSliceMinWl = 4096;
constexpr int64_t kSliceMinSize = 1024;
int32_t tile_slices(const tc_handle* h, int t, int64_t n_wl) {
  return n_wl >= kSliceMinWl && h->tile_wl[t] >= kSliceMinSize ? tile_config().slices : 1;
}
template <class K>
K pick_slices(int32_t s, K s1, K s2, K s4, K s8) {
  return s == 8 ? s8 : s == 4 ? s4 : s == 2 ? s2 : s1;
}

// y := A x in internal ids (x: n_cols, y: n_rows)
// fuse_combine: in the XCD schedule, leave y without the private copies (the
// caller adds them in its own pass); split rows are then added to y first.
// skip_zero: y's empty rows are still zero from an earlier product into the
// same y (nothing else writes them), so the zeroing launch can be left out
// (one-tile-order schedule without the persistent variant only).
void spmv_internal(tc_handle* h, const float* x, float* y, hipStream_t st, bool fuse_combine = false,
                   bool skip_zero = false) {
  const TileConfig cfg = tile_config();
  const bool xcd = h->xcd_groups > 0 && h->n_tiles > 1;
  const int64_t nzero = xcd ? h->n_zero0 : h->n_empty;
  const int64_t nz = std::max<int64_t>(nzero, h->n_tiles);
  if (nz > 0 && !(skip_zero && !xcd && !cfg.persist)) {
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
    if (cfg.persist) {
      const int32_t cb = (int32_t)h->tile_col_begin[t];
      const int32_t lw = (int32_t)std::min<int64_t>(cfg.lds_floats, h->tile_col_end[t] - cb);
      const int64_t wpb = kPB / kWave;
      const int64_t grid = std::min<int64_t>((int64_t)h->n_cu, (e - b + wpb - 1) / wpb);
      if (lw > 32768 / 2) HIPC(hipFuncSetAttribute((const void*)k_tile_persist,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, lw * 4));
      launch_tile(h, k_tile_persist, dim3((unsigned)grid), dim3(kPB), (uint32_t)(lw * 4), st,
                  (const Wl*)(h->d_wl + b), (int64_t)(e - b), (const int32_t*)h->d_idx, (const float*)h->d_val,
                  (const int32_t*)h->d_rowid, x, y, h->d_partial, cb, lw, h->d_counters + t);
    } else {
      const int32_t S = tile_slices(h, t, e - b);
      launch_tile(h, pick_slices(S, cfg.y_nt ? k_tile_spmv<true, 1> : k_tile_spmv<false, 1>,
                                 cfg.y_nt ? k_tile_spmv<true, 2> : k_tile_spmv<false, 2>,
                                 cfg.y_nt ? k_tile_spmv<true, 4> : k_tile_spmv<false, 4>,
                                 cfg.y_nt ? k_tile_spmv<true, 8> : k_tile_spmv<false, 8>),
                  dim3(nblk((e - b) * S, kWpb)), dim3(kB), 0, st, (const Wl*)(h->d_wl + b), (int64_t)(e - b),
                  (const int32_t*)h->d_idx, (const float*)h->d_val,
                  (const int32_t*)h->d_rowid, x, y, h->d_partial);
    }
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
    hipLaunchKernelGGL(k_split_combine, dim3(nblk(h->n_split_rows, kB)), dim3(kB), 0, st, h->d_split,
                       h->n_split_rows, h->d_partial, y, xcd ? 1 : 0);
    HIPC(hipGetLastError());
  }
  h->spmv_calls++;
}

// Leading chunk workloads of every tile, found once per handle from the host
// workload list.  pieces = 1 when some tile has a chunk after a non-chunk
// workload (those chunks are then done whole by k_tile_spmm).
void spmm_plan(tc_handle* h) {
  if (h->mm_planned) return;
  h->mm_lead.assign(h->n_tiles, 0);
  int64_t max_wpad = 0;
  bool lead_only = true;
  for (int t = 0; t < h->n_tiles; ++t) {
    const int64_t b = h->tile_wl_begin[t], e = h->tile_wl_begin[t + 1];
    int64_t i = b;
    while (i < e && h->wls[i].layout == kChunk) max_wpad = std::max<int64_t>(max_wpad, h->wls[i++].w_pad);
    h->mm_lead[t] = i - b;
    for (; i < e; ++i)
      if (h->wls[i].layout == kChunk) lead_only = false;
  }
  h->mm_pieces = lead_only && max_wpad > 0 ? (int32_t)((max_wpad + kPiece - 1) / kPiece) : 1;
  if (!lead_only) h->mm_lead.assign(h->n_tiles, 0);
  h->mm_planned = true;
}

// epi (one tile, k <= kB): write the RWR restart of every row instead of
// the product.  skip_empty: the rows no workload writes already hold what
// this call would write there (0, or with epi their restart values).
void spmm_internal(tc_handle* h, const float* X, float* Y, int32_t k, hipStream_t st, bool skip_empty = false,
                   const RwrEpi* epi = nullptr) {
  if (epi && !(h->n_tiles == 1 && h->xcd_groups == 0 && k <= kB))
    throw Err{TC_EINVAL, "fused restart needs one tile and k <= 256"};
  const RwrEpi ep = epi ? *epi : RwrEpi{0.0, nullptr};
  // four right-hand sides per lane when the rows allow 16-byte accesses
  const bool v4 = k % 4 == 0 && ((uintptr_t)X % 16) == 0 && ((uintptr_t)Y % 16) == 0;
  const int32_t V = v4 ? 4 : 1;
  const int32_t kq = (k + V - 1) / V;
  // one pass (grid row) covers at most 32 right-hand sides: 128 bytes of each
  // X row, one cache line per gather. Wider passes spread the gathers over
  // n * 4k bytes, past the 256 MB MALL at a million rows and k = 64 (measured
  // on a 31M-entry power-law matrix, 1M rows: k = 64 1262 -> 1152 us, k = 128
  // 2718 -> 2244 us per product; 16 per pass slows k = 32 by 40%)
  int32_t kg = 1;
  while (kg < kq && kg < 32 / V) kg <<= 1;
  spmm_plan(h);
  const int32_t pieces = h->mm_pieces;
  const int kchunks = (kq + kg - 1) / kg;
  // 4-wide lanes: four rows per sub-step group (fewer registers, more
  // wavefronts resident) and each workload cut into four row slices
  // (measured on a 31M-entry power-law matrix at k = 32: 25% over one slice,
  // and within 2% of two columns per step or eight rows per group)
  const int32_t slices = v4 ? 4 : 1;
  double* partial = nullptr;
  if (h->n_slots > 0) {
    const size_t need = sizeof(double) * (size_t)h->n_slots * pieces * k;
    if (need > h->mm_partial_bytes) {
      if (h->d_mm_partial) pool_free(h->d_mm_partial, st, false);
      h->d_mm_partial = nullptr;
      h->mm_partial_bytes = 0;
      if (!(h->d_mm_partial = (double*)pool_alloc(need, st)))
        throw Err{TC_ENOMEM, "SpMM partial sums: allocation of " + std::to_string(need) + " bytes failed"};
      h->mm_partial_bytes = need;
    }
    partial = h->d_mm_partial;
  }
  if (h->n_empty > 0 && !skip_empty) {
    const int64_t rpb = kB / std::min(k, kB);
    hipLaunchKernelGGL(k_begin_spmm, dim3((unsigned)std::min<int64_t>(nblk(h->n_empty, rpb), 1 << 16)), dim3(kB), 0,
                       st, Y, (const int32_t*)h->d_empty, h->n_empty, k, ep);
    HIPC(hipGetLastError());
  }
  for (int t = 0; t < h->n_tiles; ++t) {
    const int64_t b = h->tile_wl_begin[t], e = h->tile_wl_begin[t + 1];
    const int64_t lead = h->mm_lead[t];
    if (lead > 0)
      launch_tile(h, v4 ? k_spmm_chunks<4> : k_spmm_chunks<1>, dim3(nblk(lead * pieces, kWpb), kchunks), dim3(kB), 0,
                  st, (const Wl*)(h->d_wl + b), lead, pieces, (const int32_t*)h->d_idx, (const float*)h->d_val, X, k,
                  kg, partial);
    if (e > b + lead)
      launch_tile(h,
                  epi ? (v4 ? k_tile_spmm<4, 4, true> : k_tile_spmm<1, 8, true>)
                      : (v4 ? k_tile_spmm<4, 4> : k_tile_spmm<1, 8>),
                  dim3(nblk((e - b - lead) * slices, kWpb), kchunks), dim3(kB), 0, st,
                  (const Wl*)(h->d_wl + b + lead), (int64_t)(e - b - lead), slices, (const int32_t*)h->d_idx,
                  (const float*)h->d_val, (const int32_t*)h->d_rowid, X, Y, k, kg, partial, ep);
  }
  if (h->n_split_rows > 0) {
    hipLaunchKernelGGL(k_split_combine_mm, dim3(nblk(h->n_split_rows * k, kB)), dim3(kB), 0, st, h->d_split,
                       h->n_split_rows, (const double*)partial, pieces, Y, k, ep);
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

template <class F>
tc_status guarded(const char* who, F&& f) {
  try {
    return f();
  } catch (const Err& e) {
    set_error(std::string(who) + ": " + e.msg);
    return e.st;
  } catch (const std::bad_alloc&) {
    set_error(std::string(who) + ": host allocation failed");
    return TC_ENOMEM;
  }
}

}  // namespace
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

extern "C" tc_status tc_spmm(const tc_handle* hc, const float* X, float* Y, int32_t k, tc_stream_t stream) {
  return guarded("tc_spmm", [&]() -> tc_status {
    if (!hc || (!X && hc->n_cols > 0) || (!Y && hc->n_rows > 0)) throw Err{TC_EINVAL, "NULL argument"};
    if (k < 1 || k > 256) throw Err{TC_EINVAL, "k must be in [1, 256]"};
    if ((const void*)X == (const void*)Y && hc->n_rows > 0) throw Err{TC_EINVAL, "X and Y must not alias"};
    tc_handle* h = const_cast<tc_handle*>(hc);
    hipStream_t st = (hipStream_t)stream;
    const size_t xb = sizeof(float) * (size_t)h->n_cols * k, yb = sizeof(float) * (size_t)h->n_rows * k;
    char* ws = (char*)workspace(h, ((xb + 255) / 256) * 256 + yb, st);
    float* Xi = (float*)ws;
    float* Yi = (float*)(ws + ((xb + 255) / 256) * 256);
    gather_rows(X, h->d_cperm, h->n_cols, k, Xi, st);
    if (h->relabel) {
      spmm_internal(h, Xi, Yi, k, st);
      gather_rows(Yi, h->d_rowmap, h->n_rows, k, Y, st);
    } else {
      spmm_internal(h, Xi, Y, k, st);
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
      hipLaunchKernelGGL(k_csr_scalar, dim3(nblk(A->n_rows, kB)), dim3(kB), 0, (hipStream_t)stream, A->row_ptr,
                         A->col_idx, A->val, A->n_rows, x, y);
      HIPC(hipGetLastError());
    }
    return TC_OK;
  });
}

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
      const bool fuse = !xcd && h->n_tiles == 1 && h->kernel == 0 && !tile_config().persist;
      float* buf[2] = {p, y};
      bool zero_rows[2] = {false, false};  // the buffer's rows without entries hold 0
      int cur = 0;
      for (it = 0; it < max_iter;) {
        const bool need_res = it + 1 == max_iter || (tol > 0.0f && (it + 1) % check_every == 0);
        float* pc = buf[cur];
        float* pn = buf[1 - cur];
        if (fuse && !need_res) {
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
      const bool fuse1 = k == 1 && h->n_tiles == 1 && h->xcd_groups == 0 && h->kernel == 0 && !tile_config().persist;
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

// Batched RWR over many graphs: every launch covers all graphs (tile t of
// each, then the split rows, then the update), so small graphs share the GPU
// instead of leaving it idle one after another.
extern "C" tc_status tc_rwr_multi(tc_handle* const* hs, int32_t n_graphs, const int32_t* seeds, float c, float tol,
                                  int32_t max_iter, int32_t check_every, int32_t flags, float* const* R_out,
                                  int32_t* iters, double* resid, tc_stream_t stream) {
  return guarded("tc_rwr_multi", [&]() -> tc_status {
    if (n_graphs < 0 || (n_graphs > 0 && (!hs || !seeds || !R_out))) throw Err{TC_EINVAL, "NULL argument"};
    if (!(c >= 0.0f && c <= 1.0f) || max_iter < 0) throw Err{TC_EINVAL, "need 0 <= c <= 1 and max_iter >= 0"};
    if (check_every < 1) check_every = 1;
    hipStream_t st = (hipStream_t)stream;
    int max_tiles = 0;
    int64_t nv_total = 0;
    for (int32_t g = 0; g < n_graphs; ++g) {
      const tc_handle* h = hs[g];
      if (!h) throw Err{TC_EINVAL, "NULL handle"};
      need_square(h, "tc_rwr_multi");
      if (h->xcd_groups > 0 && h->n_tiles > 1) throw Err{TC_EUNSUPPORTED, "handles built with the XCD schedule"};
      if (seeds[g] < 0 || seeds[g] >= h->n_rows) throw Err{TC_EINVAL, "seed out of range"};
      if (h->n_rows > 0 && !R_out[g]) throw Err{TC_EINVAL, "NULL output"};
      max_tiles = std::max(max_tiles, h->n_tiles);
      nv_total += h->n_rows;
    }
    // host tables, two sets: with parity p the iterate of every graph is in
    // buffer p (R for 0, Y for 1) and the product goes to the other one
    std::vector<std::vector<MultiSeg>> segs[2];
    std::vector<std::vector<int32_t>> seg_graph(max_tiles);
    segs[0].resize(max_tiles);
    segs[1].resize(max_tiles);
    std::vector<int64_t> seg_total(max_tiles, 0);
    std::vector<MultiVec> vec[2], emp[2], spl[2];
    for (int q = 0; q < 2; ++q) {
      vec[q].resize(n_graphs);
      emp[q].resize(n_graphs);
      spl[q].resize(n_graphs);
    }
    std::vector<int32_t> block_graph;
    std::vector<int64_t> block_first, graph_blocks(n_graphs + 1, 0);
    int64_t off = 0, e_tot = 0, s_tot = 0;
    const size_t vbytes = sizeof(float) * (size_t)std::max<int64_t>(nv_total, 1);
    float* R = (float*)pool_alloc(vbytes, st);
    float* Y = (float*)pool_alloc(vbytes, st);
    if (!R || !Y) {
      if (R) pool_free(R, st, false);
      if (Y) pool_free(Y, st, false);
      throw Err{TC_ENOMEM, "tc_rwr_multi: vector allocation failed"};
    }
    float* buf[2] = {R, Y};
    for (int32_t g = 0; g < n_graphs; ++g) {
      const tc_handle* h = hs[g];
      for (int t = 0; t < h->n_tiles; ++t) {
        const int64_t b = h->tile_wl_begin[t], e = h->tile_wl_begin[t + 1];
        if (e == b) continue;
        for (int q = 0; q < 2; ++q)
          segs[q][t].push_back(MultiSeg{h->d_wl + b, seg_total[t], h->d_idx, h->d_val, h->d_rowid, buf[q] + off,
                                        buf[1 - q] + off, h->d_partial, -1});
        seg_graph[t].push_back(g);
        seg_total[t] += e - b;
      }
      for (int q = 0; q < 2; ++q) {
        vec[q][g] = MultiVec{off, h->n_rows, nullptr, nullptr, nullptr, buf[1 - q] + off, buf[q] + off, -1};
        emp[q][g] = MultiVec{e_tot, h->n_empty, h->d_empty, nullptr, nullptr, buf[1 - q] + off, nullptr, -1};
        spl[q][g] = MultiVec{s_tot, h->n_split_rows, nullptr, h->d_split, h->d_partial, buf[1 - q] + off, nullptr, -1};
      }
      e_tot += h->n_empty;
      s_tot += h->n_split_rows;
      const int64_t nb = (h->n_rows + (int64_t)kB * kMultiPer - 1) / ((int64_t)kB * kMultiPer);
      for (int64_t q = 0; q < nb; ++q) {
        block_graph.push_back(g);
        block_first.push_back(q);
      }
      graph_blocks[g + 1] = graph_blocks[g] + nb;
      off += h->n_rows;
    }
    // device tables in one pool block
    size_t bytes = 0;
    auto reserve = [&](size_t n) { const size_t at = bytes; bytes += (n + 255) / 256 * 256; return at; };
    std::vector<size_t> seg_at[2];
    size_t vec_at[2], emp_at[2], spl_at[2];
    for (int q = 0; q < 2; ++q) {
      seg_at[q].resize(max_tiles);
      for (int t = 0; t < max_tiles; ++t) seg_at[q][t] = reserve(sizeof(MultiSeg) * segs[q][t].size());
      vec_at[q] = reserve(sizeof(MultiVec) * n_graphs);
      emp_at[q] = reserve(sizeof(MultiVec) * n_graphs);
      spl_at[q] = reserve(sizeof(MultiVec) * n_graphs);
    }
    const size_t bg_at = reserve(sizeof(int32_t) * block_graph.size()),
                 bf_at = reserve(sizeof(int64_t) * block_first.size()),
                 gb_at = reserve(sizeof(int64_t) * graph_blocks.size()),
                 parts_at = reserve(sizeof(double) * block_graph.size()),
                 res_at = reserve(sizeof(double) * (n_graphs + 1)), seeds_at = reserve(sizeof(int32_t) * n_graphs),
                 maps_at = reserve(sizeof(int32_t*) * n_graphs);
    char* tab = (char*)pool_alloc(std::max<size_t>(bytes, 256), st);
    if (!tab) {
      pool_free(R, st, false);
      pool_free(Y, st, false);
      throw Err{TC_ENOMEM, "tc_rwr_multi: table allocation failed"};
    }
    struct Release {
      void* a; void* b; void* c; hipStream_t s;
      ~Release() { pool_free(a, s, false); pool_free(b, s, false); pool_free(c, s, false); }
    } rel{R, Y, tab, st};
    auto up = [&](size_t at, const void* src, size_t n) {
      if (n) HIPC(hipMemcpyAsync(tab + at, src, n, hipMemcpyHostToDevice, st));
    };
    // internal seed ids: seed_int = rowmap[seed] read on the device
    {
      std::vector<const int32_t*> maps(n_graphs);
      for (int32_t g = 0; g < n_graphs; ++g) maps[g] = hs[g]->d_rowmap;
      up(maps_at, maps.data(), sizeof(int32_t*) * n_graphs);
      up(seeds_at, seeds, sizeof(int32_t) * n_graphs);
      std::vector<int32_t> sint(n_graphs, 0);
      if (n_graphs > 0) {
        hipLaunchKernelGGL(k_map_ids_multi, dim3(1), dim3(kB), 0, st, (const int32_t* const*)(tab + maps_at),
                           (const int32_t*)(tab + seeds_at), n_graphs, (int32_t*)(tab + seeds_at));
        HIPC(hipGetLastError());
        HIPC(hipMemcpyAsync(sint.data(), tab + seeds_at, sizeof(int32_t) * n_graphs, hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
      }
      for (int q = 0; q < 2; ++q) {
        for (int32_t g = 0; g < n_graphs; ++g) vec[q][g].seed = emp[q][g].seed = spl[q][g].seed = sint[g];
        for (int t = 0; t < max_tiles; ++t)
          for (size_t i = 0; i < segs[q][t].size(); ++i) segs[q][t][i].seed = sint[seg_graph[t][i]];
      }
    }
    for (int q = 0; q < 2; ++q) {
      for (int t = 0; t < max_tiles; ++t) up(seg_at[q][t], segs[q][t].data(), sizeof(MultiSeg) * segs[q][t].size());
      up(vec_at[q], vec[q].data(), sizeof(MultiVec) * n_graphs);
      up(emp_at[q], emp[q].data(), sizeof(MultiVec) * n_graphs);
      up(spl_at[q], spl[q].data(), sizeof(MultiVec) * n_graphs);
    }
    up(bg_at, block_graph.data(), sizeof(int32_t) * block_graph.size());
    up(bf_at, block_first.data(), sizeof(int64_t) * block_first.size());
    up(gb_at, graph_blocks.data(), sizeof(int64_t) * graph_blocks.size());
    double* d_parts = (double*)(tab + parts_at);
    double* d_res = (double*)(tab + res_at);
    const int64_t nblocks = (int64_t)block_graph.size();

    // Iterations whose L1 change is not read run the restart fused into the
    // products (every graph one tile), into the other buffer: parity flips.
    // The others run the products into the other buffer, then the update of
    // the iterate in place, with its change.
    const bool fuse = max_tiles <= 1;
    auto iteration = [&](hipStream_t s2, int par, bool fused) {
      if (fused) {
        if (max_tiles == 1 && seg_total[0] > 0) {
          hipLaunchKernelGGL(k_tile_spmv_multi_rwr, dim3(nblk(seg_total[0], kWpb)), dim3(kB), 0, s2,
                             (const MultiSeg*)(tab + seg_at[par][0]), (int32_t)segs[par][0].size(), seg_total[0],
                             (double)c);
          HIPC(hipGetLastError());
        }
        if (s_tot + e_tot > 0) {
          hipLaunchKernelGGL(k_rwr_rest_multi, dim3(nblk(s_tot + e_tot, kB)), dim3(kB), 0, s2,
                             (const MultiVec*)(tab + spl_at[par]), (const MultiVec*)(tab + emp_at[par]), n_graphs,
                             s_tot, e_tot, (double)c);
          HIPC(hipGetLastError());
        }
        return;
      }
      if (e_tot > 0) {
        hipLaunchKernelGGL(k_begin_multi, dim3(nblk(e_tot, kB)), dim3(kB), 0, s2,
                           (const MultiVec*)(tab + emp_at[par]), n_graphs, e_tot);
        HIPC(hipGetLastError());
      }
      for (int t = 0; t < max_tiles; ++t) {
        if (seg_total[t] == 0) continue;
        hipLaunchKernelGGL(k_tile_spmv_multi, dim3(nblk(seg_total[t], kWpb)), dim3(kB), 0, s2,
                           (const MultiSeg*)(tab + seg_at[par][t]), (int32_t)segs[par][t].size(), seg_total[t]);
        HIPC(hipGetLastError());
      }
      if (s_tot > 0) {
        hipLaunchKernelGGL(k_split_combine_multi, dim3(nblk(s_tot, kB)), dim3(kB), 0, s2,
                           (const MultiVec*)(tab + spl_at[par]), n_graphs, s_tot);
        HIPC(hipGetLastError());
      }
      if (nblocks > 0) {
        hipLaunchKernelGGL(k_rwr_update_multi, dim3((unsigned)nblocks), dim3(kB), 0, s2,
                           (const MultiVec*)(tab + vec_at[par]), (const int32_t*)(tab + bg_at),
                           (const int64_t*)(tab + bf_at), (double)c, d_parts);
        HIPC(hipGetLastError());
        hipLaunchKernelGGL(k_multi_resid, dim3(1), dim3(kB), 0, s2, (const int64_t*)(tab + gb_at), n_graphs,
                           (const double*)d_parts, d_res, d_res + n_graphs);
        HIPC(hipGetLastError());
      }
    };
    // iterations [it0, it0 + n) from parity par; returns the parity after them
    auto run = [&](hipStream_t s2, int32_t it0, int32_t n, int par) {
      for (int32_t q = it0; q < it0 + n; ++q) {
        const bool need_res = q + 1 == max_iter || (tol > 0.0f && (q + 1) % check_every == 0);
        const bool fused = fuse && !need_res;
        iteration(s2, par, fused);
        if (fused) par = 1 - par;
      }
      return par;
    };

    int32_t it = 0;
    int par = 0;
    double r = 0.0;
    bool conv = false;
    if (nv_total > 0) {
      hipLaunchKernelGGL(k_rwr_init_multi, dim3(nblk(nv_total, kB)), dim3(kB), 0, st,
                         (const MultiVec*)(tab + vec_at[0]), n_graphs, nv_total);
      HIPC(hipGetLastError());
      const int32_t chunk = tol > 0.0f ? check_every : std::max(max_iter, 1);
      // one captured chunk per starting parity (a chunk of full length starts
      // at a multiple of chunk, so its fused steps are the same every time)
      hipGraphExec_t exec[2] = {nullptr, nullptr};
      hipGraph_t graph[2] = {nullptr, nullptr};
      int par_after[2] = {0, 1};
      hipStream_t cap = nullptr;
      struct GraphRelease {
        hipGraphExec_t* e; hipGraph_t* g; hipStream_t* s;
        ~GraphRelease() {
          for (int q = 0; q < 2; ++q) {
            if (e[q]) (void)hipGraphExecDestroy(e[q]);
            if (g[q]) (void)hipGraphDestroy(g[q]);
          }
          if (*s) (void)hipStreamDestroy(*s);
        }
      } grel{exec, graph, &cap};
      const bool use_graph = (flags & 1) && max_iter > 0;
      while (it < max_iter) {
        const int32_t step = std::min(chunk, max_iter - it);
        if (use_graph && step == chunk) {
          if (!exec[par]) {
            if (!cap) HIPC(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            HIPC(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
            par_after[par] = run(cap, it, step, par);
            HIPC(hipStreamEndCapture(cap, &graph[par]));
            HIPC(hipGraphInstantiate(&exec[par], graph[par], nullptr, nullptr, 0));
          }
          HIPC(hipGraphLaunch(exec[par], st));
          par = par_after[par];
        } else {
          par = run(st, it, step, par);
        }
        it += step;
        if (tol > 0.0f) {
          r = read_f64(d_res + n_graphs, st);
          if (r <= (double)tol) {
            conv = true;
            break;
          }
        }
      }
      if (it > 0) r = read_f64(d_res + n_graphs, st);
      off = 0;
      for (int32_t g = 0; g < n_graphs; ++g) {
        gather_rows(buf[par] + off, hs[g]->d_rowmap, hs[g]->n_rows, 1, R_out[g], st);
        off += hs[g]->n_rows;
      }
      if (resid && n_graphs > 0) HIPC(hipMemcpyAsync(resid, d_res, sizeof(double) * n_graphs, hipMemcpyDeviceToHost, st));
      HIPC(hipStreamSynchronize(st));
    } else if (resid) {
      for (int32_t g = 0; g < n_graphs; ++g) resid[g] = 0.0;
    }
    if (iters) *iters = it;
    if (tol > 0.0f && !conv && nv_total > 0) {
      set_error("tc_rwr_multi: tolerance not reached in max_iter iterations");
      return TC_ENOTCONV;
    }
    return TC_OK;
  });
}

// ---- differentiable RWR (host)
namespace tc {
namespace {
// y := A x in the caller's ids (as tc_spmv)
void spmv_user(tc_handle* h, const float* x, float* y, hipStream_t st) {
  gather_rows(x, h->d_cperm, h->n_cols, 1, h->d_xbuf, st);
  if (h->relabel) {
    spmv_internal(h, h->d_xbuf, h->d_ybuf, st);
    gather_rows(h->d_ybuf, h->d_rowmap, h->n_rows, 1, y, st);
  } else {
    spmv_internal(h, h->d_xbuf, y, st);
  }
}

struct PoolBuf {
  void* p = nullptr;
  hipStream_t st;
  PoolBuf(size_t bytes, hipStream_t s) : st(s) {
    p = pool_alloc(bytes ? bytes : 1, s);
    if (!p) throw Err{TC_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
  }
  ~PoolBuf() { pool_free(p, st, false); }
  template <class T>
  T* as() const { return (T*)p; }
};

int32_t n_checkpoints(int32_t K, int32_t every) { return K <= 0 ? 0 : (K + every - 1) / every; }
}  // namespace
}  // namespace tc

extern "C" tc_status tc_rwr_edge_weights(int64_t n_cols, int64_t nnz, const int32_t* d_col, const int64_t* d_rpT,
                                         int32_t nf, const float* d_feats, const float* d_featsT, const double* theta,
                                         double* d_zT, double* d_wT, double* d_S, float* d_val, float* d_valT,
                                         tc_stream_t stream) {
  return guarded("tc_rwr_edge_weights", [&]() -> tc_status {
    if (n_cols < 0 || nnz < 0 || nf < 1 || nf > kMaxFeat) throw Err{TC_EINVAL, "need sizes >= 0 and 1 <= nf <= 16"};
    if (!theta || !d_rpT || !d_S ||
        (nnz > 0 && (!d_col || !d_feats || !d_featsT || !d_zT || !d_wT || !d_val || !d_valT)))
      throw Err{TC_EINVAL, "NULL argument"};
    hipStream_t st = (hipStream_t)stream;
    PoolBuf th(sizeof(double) * nf, st);
    HIPC(hipMemcpyAsync(th.p, theta, sizeof(double) * nf, hipMemcpyHostToDevice, st));
    if (nnz > 0) {
      hipLaunchKernelGGL(k_edge_softplus, dim3(nblk(nnz, kB)), dim3(kB), 0, st, d_featsT, nnz, nf,
                         th.as<const double>(), d_zT, d_wT);
      HIPC(hipGetLastError());
    }
    if (n_cols > 0) {
      hipLaunchKernelGGL(k_col_norm, dim3(nblk(nblk(n_cols, kWave / kColLanes), kWpb)), dim3(kB), 0, st, d_rpT,
                         n_cols, (const double*)d_wT, d_S);
      HIPC(hipGetLastError());
    }
    if (nnz > 0) {
      PoolBuf rowT(sizeof(int32_t) * (size_t)nnz, st);
      hipLaunchKernelGGL(k_rows_of, dim3(nblk(n_cols, kB)), dim3(kB), 0, st, d_rpT, n_cols, rowT.as<int32_t>());
      HIPC(hipGetLastError());
      hipLaunchKernelGGL(k_values_T, dim3(nblk(nnz, kB)), dim3(kB), 0, st, rowT.as<const int32_t>(), nnz,
                         (const double*)d_wT, (const double*)d_S, d_valT);
      HIPC(hipGetLastError());
      hipLaunchKernelGGL(k_edge_values, dim3(nblk(nnz, kB)), dim3(kB), 0, st, d_feats, d_col, nnz, nf,
                         th.as<const double>(), (const double*)d_S, d_val);
      HIPC(hipGetLastError());
      HIPC(hipStreamSynchronize(st));  // before rowT goes back to the pool
    }
    HIPC(hipStreamSynchronize(st));  // theta's staging copy is released below
    return TC_OK;
  });
}

extern "C" tc_status tc_rwr_iterates(const tc_handle* hc, int32_t seed, float c, int32_t K, int32_t every,
                                     float* d_ckpt, float* d_rK, tc_stream_t stream) {
  return guarded("tc_rwr_iterates", [&]() -> tc_status {
    if (!hc || (!d_rK && hc->n_rows > 0)) throw Err{TC_EINVAL, "NULL argument"};
    need_square(hc, "tc_rwr_iterates");
    if (K < 0 || every < 1 || !(c >= 0.0f && c <= 1.0f)) throw Err{TC_EINVAL, "need K >= 0, every >= 1, 0 <= c <= 1"};
    if (seed < 0 || seed >= hc->n_rows) throw Err{TC_EINVAL, "seed out of range"};
    if (K > 0 && !d_ckpt) throw Err{TC_EINVAL, "NULL checkpoint array"};
    tc_handle* h = const_cast<tc_handle*>(hc);
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = h->n_rows;
    PoolBuf y(sizeof(float) * n, st);
    hipLaunchKernelGGL(k_onehot, dim3(nblk(n, kB)), dim3(kB), 0, st, d_rK, n, seed);
    HIPC(hipGetLastError());
    for (int32_t k = 0; k < K; ++k) {
      if (k % every == 0)
        HIPC(hipMemcpyAsync(d_ckpt + (int64_t)(k / every) * n, d_rK, sizeof(float) * n, hipMemcpyDeviceToDevice,
                            st));
      spmv_user(h, d_rK, y.as<float>(), st);
      hipLaunchKernelGGL(k_rwr_step, dim3(nblk(n, kB)), dim3(kB), 0, st, y.as<const float>(), d_rK, n, seed,
                         (double)c);
      HIPC(hipGetLastError());
    }
    return TC_OK;
  });
}

extern "C" tc_status tc_rwr_adjoint(const tc_handle* hc, const tc_handle* htc, const int64_t* d_rpT,
                                    const int32_t* d_colT, int32_t seed, float c, int32_t K, int32_t every,
                                    const float* d_ckpt, const float* d_gK, double* d_G, float* d_g0,
                                    tc_stream_t stream) {
  return guarded("tc_rwr_adjoint", [&]() -> tc_status {
    if (!hc || !htc || !d_rpT || (hc->n_rows > 0 && !d_gK)) throw Err{TC_EINVAL, "NULL argument"};
    need_square(hc, "tc_rwr_adjoint");
    need_square(htc, "tc_rwr_adjoint");
    if (htc->n_rows != hc->n_rows || htc->nnz != hc->nnz) throw Err{TC_EINVAL, "the second handle must hold A^T"};
    if (K < 0 || every < 1 || !(c >= 0.0f && c <= 1.0f)) throw Err{TC_EINVAL, "need K >= 0, every >= 1, 0 <= c <= 1"};
    if (seed < 0 || seed >= hc->n_rows) throw Err{TC_EINVAL, "seed out of range"};
    const int64_t n = hc->n_rows, nnz = hc->nnz;
    if (nnz > 0 && (!d_colT || !d_G)) throw Err{TC_EINVAL, "NULL argument"};
    if (K > 0 && !d_ckpt) throw Err{TC_EINVAL, "NULL checkpoint array"};
    tc_handle* h = const_cast<tc_handle*>(hc);
    tc_handle* ht = const_cast<tc_handle*>(htc);
    hipStream_t st = (hipStream_t)stream;
    const int32_t seglen = std::min(every, std::max(K, 1));
    PoolBuf seg(sizeof(float) * (size_t)n * seglen, st), gseg(sizeof(float) * (size_t)n * seglen, st),
        segi(sizeof(float) * (size_t)n * seglen, st), gsegi(sizeof(float) * (size_t)n * seglen, st),
        g(sizeof(float) * n, st), tmp(sizeof(float) * n, st),
        rows(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1), st);
    if (nnz > 0) {
      HIPC(hipMemsetAsync(d_G, 0, sizeof(double) * nnz, st));
      hipLaunchKernelGGL(k_rows_of, dim3(nblk(n, kB)), dim3(kB), 0, st, d_rpT, n, rows.as<int32_t>());
      HIPC(hipGetLastError());
    }
    if (n > 0) HIPC(hipMemcpyAsync(g.p, d_gK, sizeof(float) * n, hipMemcpyDeviceToDevice, st));
    float* S = seg.as<float>();
    for (int32_t q = n_checkpoints(K, every) - 1; q >= 0; --q) {
      const int32_t k0 = q * every, k1 = std::min(K, k0 + every);
      // recompute r^{k0} .. r^{k1-1} from the checkpoint
      HIPC(hipMemcpyAsync(S, d_ckpt + (int64_t)q * n, sizeof(float) * n, hipMemcpyDeviceToDevice, st));
      for (int32_t t = 1; t < k1 - k0; ++t) {
        spmv_user(h, S + (int64_t)(t - 1) * n, tmp.as<float>(), st);
        hipLaunchKernelGGL(k_rwr_step, dim3(nblk(n, kB)), dim3(kB), 0, st, tmp.as<const float>(), S + (int64_t)t * n,
                           n, seed, (double)c);
        HIPC(hipGetLastError());
      }
      // adjoint vectors g^{k+1} of the segment, latest first, kept for one
      // pass over the entries (which then reads them per step)
      float* GS = gseg.as<float>();
      for (int32_t k = k1 - 1; k >= k0; --k) {
        if (n > 0)
          HIPC(hipMemcpyAsync(GS + (int64_t)(k - k0) * n, g.p, sizeof(float) * n, hipMemcpyDeviceToDevice, st));
        spmv_user(ht, g.as<const float>(), tmp.as<float>(), st);
        hipLaunchKernelGGL(k_scale, dim3(nblk(n, kB)), dim3(kB), 0, st, tmp.as<const float>(), g.as<float>(), n,
                           (double)c);
        HIPC(hipGetLastError());
      }
      if (nnz > 0) {
        const int32_t m = k1 - k0;
        hipLaunchKernelGGL(k_interleave, dim3(nblk(n * m, kB)), dim3(kB), 0, st, (const float*)GS, m, n,
                           gsegi.as<float>());
        HIPC(hipGetLastError());
        hipLaunchKernelGGL(k_interleave, dim3(nblk(n * m, kB)), dim3(kB), 0, st, (const float*)S, m, n,
                           segi.as<float>());
        HIPC(hipGetLastError());
        hipLaunchKernelGGL(k_edge_accum_seg, dim3(nblk(nnz, kB)), dim3(kB), 0, st, d_colT, rows.as<const int32_t>(),
                           nnz, gsegi.as<const float>(), segi.as<const float>(), m, d_G);
        HIPC(hipGetLastError());
      }
    }
    if (d_g0 && n > 0) HIPC(hipMemcpyAsync(d_g0, g.p, sizeof(float) * n, hipMemcpyDeviceToDevice, st));
    return TC_OK;
  });
}

extern "C" tc_status tc_rwr_theta_grad(int64_t n_cols, int64_t nnz, const int64_t* d_rpT, int32_t nf,
                                       const float* d_featsT, const double* d_zT, const double* d_wT,
                                       const double* d_S, const double* d_G, float c, double* dtheta,
                                       tc_stream_t stream) {
  return guarded("tc_rwr_theta_grad", [&]() -> tc_status {
    if (n_cols < 0 || nnz < 0 || nf < 1 || nf > kMaxFeat) throw Err{TC_EINVAL, "need sizes >= 0 and 1 <= nf <= 16"};
    if (!dtheta || !d_rpT || !d_S || (nnz > 0 && (!d_featsT || !d_zT || !d_wT || !d_G)))
      throw Err{TC_EINVAL, "NULL argument"};
    hipStream_t st = (hipStream_t)stream;
    PoolBuf cs(sizeof(double) * (size_t)std::max<int64_t>(n_cols, 1), st),
        rowT(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1), st),
        parts(sizeof(double) * (size_t)kGradBlocks * nf, st), out(sizeof(double) * nf, st);
    if (n_cols > 0) {
      hipLaunchKernelGGL(k_col_dot, dim3(nblk(nblk(n_cols, kWave / kColLanes), kWpb)), dim3(kB), 0, st, d_rpT,
                         n_cols, d_G, d_wT, d_S, (double)c, cs.as<double>());
      HIPC(hipGetLastError());
      hipLaunchKernelGGL(k_rows_of, dim3(nblk(n_cols, kB)), dim3(kB), 0, st, d_rpT, n_cols, rowT.as<int32_t>());
      HIPC(hipGetLastError());
    }
    hipLaunchKernelGGL(k_theta_grad, dim3(kGradBlocks), dim3(kB), 0, st, rowT.as<const int32_t>(), nnz, nf, d_featsT,
                       d_zT, d_S, d_G, cs.as<const double>(), (double)c, parts.as<double>());
    HIPC(hipGetLastError());
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kB), 0, st, parts.as<const double>(), kGradBlocks, nf,
                       out.as<double>());
    HIPC(hipGetLastError());
    HIPC(hipMemcpyAsync(dtheta, out.p, sizeof(double) * nf, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    return TC_OK;
  });
}

// dst row q = src row idx[q] (rows of `width` floats); idx is checked against
// the source's n_src rows first
__global__ void k_idx_check(const int32_t* __restrict__ idx, int64_t n, int64_t n_src, int32_t* __restrict__ bad) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n && (idx[q] < 0 || idx[q] >= n_src)) atomicOr(bad, 1);
}

extern "C" tc_status tc_gather_rows(const float* d_src, int64_t n_src, const int32_t* d_idx, int64_t n, int32_t width,
                                    float* d_dst, tc_stream_t stream) {
  return guarded("tc_gather_rows", [&]() -> tc_status {
    if (n < 0 || n_src < 0 || width < 1) throw Err{TC_EINVAL, "need n, n_src >= 0 and width >= 1"};
    if (n == 0) return TC_OK;
    if (!d_src || !d_idx || !d_dst) throw Err{TC_EINVAL, "NULL argument"};
    hipStream_t st = (hipStream_t)stream;
    PoolBuf bad(sizeof(int32_t), st);
    HIPC(hipMemsetAsync(bad.p, 0, sizeof(int32_t), st));
    hipLaunchKernelGGL(k_idx_check, dim3(nblk(n, kB)), dim3(kB), 0, st, d_idx, n, n_src, bad.as<int32_t>());
    HIPC(hipGetLastError());
    int32_t hbad = 0;
    HIPC(hipMemcpyAsync(&hbad, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    if (hbad) throw Err{TC_EINVAL, "row index out of range"};
    hipLaunchKernelGGL(k_gather_rows, dim3(nblk(n * width, kB)), dim3(kB), 0, st, d_src, d_idx, n, width, d_dst);
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(st));
    return TC_OK;
  });
}
