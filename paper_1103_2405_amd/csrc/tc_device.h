// Device-side building blocks shared by the library's product kernels: the
// tile pass over one workload (Section 3.1, Solution 3), wavefront sums, the
// sum of a split row's partial slots and a few small vector kernels.
//
// Tile pass: one wavefront per workload (or per row slice of a workload).
//   row-major:    the wavefront walks one row at a time, lanes striding the
//                 padded row, then a cross-lane sum; the last lane updates y.
//   column-major: lane r owns row r of the rectangle and walks its columns;
//                 consecutive lanes read consecutive addresses.
//   chunk:        one piece of a split heavy row; its sum goes to a partial
//                 slot that is added to y after the last tile.
// Products are exact in FP64 and each row's per-tile sum is accumulated in
// FP64, then added to the FP32 y once per tile.
#pragma once

#include "tc_internal.h"

namespace tc {

// RWR restart fused into the product (one tile: each row's value is final
// where it is written): R'[row][q] = fl32(c fl32(y) + (1 - c) [row == seed_q]),
// the same rounding as the separate update after a stored y.
struct RwrEpi {
  double c;
  const int32_t* seeds;  // internal ids, one per right-hand side
};

// PageRank update fused into the row-panel pass (Eq. 6): every row is
// written as p' = fl32(c (fl32(y) + d/n) + (1 - c)/n), the separate update's
// rounding; a split row's sum over its unsplit segments also goes to yraw (in
// the order of the split-row list), for the pass that adds its chunks.
struct PanelPr {
  double c;
  const double* dmass;    // dangling mass of the iterate the product reads
  int64_t n;
  const int64_t* psb;     // [panels + 1] split rows of each panel
  const SplitRow* split;  // split rows, increasing row
  float* yraw;
};

__device__ inline float rwr_restart(double c, float y, bool is_seed) {
  return (float)(c * (double)y + (is_seed ? 1.0 - c : 0.0));
}

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

// x[i] by a raw buffer load: a 32-bit byte offset from one scalar base, so a
// gather needs no 64-bit address per lane (about 1% faster on the panel
// pass).  Same value and cache policy as x[i]; x must hold at most
// kBufMaxFloats floats, so that 4 i fits the signed offset.  The descriptor
// covers the whole 32-bit range (no record limit); its word 3 is the CDNA
// raw-dword format.
constexpr int64_t kBufMaxFloats = (int64_t)1 << 29;
__device__ inline float ld_buf(const float* x, int32_t i) {
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void*)x, (short)0, -1, 0x00020000);
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, i * 4, 0, 0));
}

// Cross-lane moves of a double through DPP (two 32-bit halves).  Lanes whose
// source is outside the row read 0 (bound_ctrl), rows outside ROWMASK add 0.
template <int CTRL, int ROWMASK = 0xf>
__device__ inline double dpp_f64(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int l2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWMASK, 0xf, true);
  const int h2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWMASK, 0xf, true);
  return __hiloint2double(h2, l2);
}

// Sum over each 8-lane half of a DPP row; the totals land in lanes 7 and 15
// of the row (the first three steps of the row's running sum).
__device__ inline double row8_sum(double v) {
  v += dpp_f64<0x111>(v);  // row_shr:1
  v += dpp_f64<0x112>(v);  // row_shr:2
  v += dpp_f64<0x114>(v);  // row_shr:4
  return v;
}
// Sum over each DPP row of 16 lanes; the total lands in the row's lane 15.
__device__ inline double row16_sum(double v) {
  v = row8_sum(v);
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

// Row-major rectangle with 64-element-aligned rows (S a multiple of 64), or
// rows padded to 32: every lane reads 4 consecutive entries (16 bytes) per
// 256-entry chunk.
//   w_pad = 32:  a chunk holds 8 rows, 8 lanes each -> sums per half DPP row
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
  if (wp == 32 || wp == 64 || wp == 128) {
    const int lpr = wp >> 2;             // lanes per row
    const int rpc = kWave / lpr;         // rows per chunk
    const int my = lane / lpr;           // my row inside the chunk
    const int nchunk = (nr + rpc - 1) / rpc;
    for (int q = 2 * sl; q < nchunk; q += 2 * S) {
      const int ra = q * rpc + my, rb = (q + 1) * rpc + my;
      const bool oka = ra < nr, okb = rb < nr;
      // row ids read with the matrix loads (clamped to a valid entry; chunks have none to write)
      const int32_t ida = chunk ? 0 : ld_nt(rowid + d.rowid_off + (oka ? ra : 0));
      const int32_t idb = chunk ? 0 : ld_nt(rowid + d.rowid_off + (okb ? rb : 0));
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
      if (wp == 32) {
        sa = row8_sum(sa);
        sb = row8_sum(sb);
      } else if (wp == 64) {
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
          if (oka) x.addy(y, ida, sa);
          if (okb) x.addy(y, idb, sb);
        }
      }
    }
    return;
  }
  for (int32_t r = sl; r < nr; r += S) {
    const int64_t base = off + (int64_t)r * wp;
    const int32_t idr = chunk ? 0 : ld_nt(rowid + d.rowid_off + r);
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
        x.addy(y, idr, acc);
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
    int32_t rid[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc[u] = 0.0;
      ok[u] = r0 + u * S * kWave + lane < nr;
    }
    // the rows' ids go out with the first matrix loads (a lane past the last
    // row reads the workload's first id and never uses it)
#pragma unroll
    for (int u = 0; u < U; ++u) rid[u] = ld_nt(rowid + d.rowid_off + (ok[u] ? r0 + u * S * kWave + lane : 0));
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
      if (ok[u]) x.addy(y, rid[u], acc[u]);
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
// later tile (kAddFlag in the row id) stores fl32(y + s).
__device__ inline void addy_first_touch(float* y, int32_t rid, double s) {
  if (rid & kAddFlag) {
    const int32_t row = rid & ~kAddFlag;
    y[row] = (float)((double)y[row] + s);
  } else {
    y[rid] = (float)s;
  }
}

// x as read by a tile: straight from global memory (through L1/L2) ...
struct GlobalX {
  const float* __restrict__ x;
  __device__ float operator()(int32_t i) const { return x[i]; }
  __device__ void addy(float* y, int32_t row, double s) const { addy_first_touch(y, row, s); }
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
  } else if (layout != kCM && aligned && ((d.w_pad & 63) == 0 || (d.w_pad == 32 && layout == kRM))) {
    rm_wide<S>(d, lane, idx, val, rowid, x, y, partial, layout == kChunk, sl);
  } else {
    generic_wl<S>(d, lane, layout, idx, val, rowid, x, y, partial, sl);
  }
}

// p[0] + p[s] + ... + p[(n-1) s], added in that order; 32 loads go out
// together, then 8 (a split row can have hundreds of chunks, summed by one
// thread: the loads in flight set its time)
__device__ inline double sum_slots(const double* __restrict__ p, int64_t n, int64_t s = 1) {
  double acc = 0.0;
  int64_t q = 0;
  for (; q + 32 <= n; q += 32) {
    double t[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) t[u] = p[(q + u) * s];
#pragma unroll
    for (int u = 0; u < 32; ++u) acc += t[u];
  }
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

// The same sum as sum_slots (left to right from 0.0, so the same bits) by a
// whole wavefront: each round the lanes copy 256 slots at once into the
// wavefront's LDS buffer `buf` (256 doubles), then lane 0 adds them in slot
// order from LDS.  A row of hundreds of chunks then costs a few global load
// latencies instead of one per 32 slots.  The sum is valid in lane 0.
__device__ inline double sum_slots_wave(const double* __restrict__ p, int64_t n, int lane, double* buf) {
  double acc = 0.0;
  for (int64_t q = 0; q < n; q += 4 * kWave) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = q + u * kWave + lane;
      buf[u * kWave + lane] = i < n ? p[i] : 0.0;
    }
    __builtin_amdgcn_wave_barrier();
    const int m = (int)(n - q < 4 * kWave ? n - q : 4 * kWave);
    if (lane == 0) {
      int k = 0;
      for (; k + 8 <= m; k += 8) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = buf[k + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += t[u];
      }
      for (; k < m; ++k) acc += buf[k];
    }
    __builtin_amdgcn_wave_barrier();
  }
  return acc;
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

}  // namespace
}  // namespace tc
