// Multi-right-hand-side products Y = A X on the tiled composite format (the
// batched queries of Appendix F, Eq. 9, many restart vectors at once).
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>

#include "tc_host.h"

namespace tc {

namespace {

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

}  // namespace

// epi (one tile, k <= kB): write the RWR restart of every row instead of
// the product.  skip_empty: the rows no workload writes already hold what
// this call would write there (0, or with epi their restart values).
size_t spmm_partial_doubles(tc_handle* h, int32_t k) {
  spmm_plan(h);
  return (size_t)h->n_slots * h->mm_pieces * k;
}

void spmm_internal(tc_handle* h, const float* X, float* Y, int32_t k, hipStream_t st, bool skip_empty,
                   const RwrEpi* epi, double* partial_ext) {
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
  if (partial_ext) {
    partial = partial_ext;
  } else if (h->n_slots > 0) {
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
  const bool timing = h->timing;
  if (partial_ext) h->timing = false;  // event creation is not for callers that cannot allocate
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
  h->timing = timing;
  h->spmv_calls++;
}

}  // namespace tc

using namespace tc;

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

// ---- SpMM for callers that cannot allocate (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc): the split-row partial sums
// live in this file-scope device array instead of the handle's pool buffer.
// Every call on a device shares that device's copy (calls that overlap on one
// GPU race); nothing in it needs clearing, each product writes every slot it
// reads.  The array's address on each device comes from hipGetSymbolAddress
// on the first call with that device current.
namespace {
constexpr size_t kScratchDoubles = (size_t)1 << 21;  // 16 MiB per device
__device__ __align__(256) double scratch[kScratchDoubles];
std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_ptr;

double* scratch_on_current_device() {
  int dev = 0;
  HIPC(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  double* p = nullptr;
  HIPC(hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch)));
  g_scratch_ptr[dev] = p;
  return p;
}
}  // namespace

extern "C" tc_status tc_spmm_internal_noalloc(const tc_handle* hc, const float* X, float* Y, int32_t k,
                                              tc_stream_t stream) {
  return guarded("tc_spmm_internal_noalloc", [&]() -> tc_status {
    if (!hc || (!X && hc->n_cols > 0) || (!Y && hc->n_rows > 0)) throw Err{TC_EINVAL, "NULL argument"};
    if (k < 1 || k > 256) throw Err{TC_EINVAL, "k must be in [1, 256]"};
    if ((const void*)X == (const void*)Y && hc->n_rows > 0) throw Err{TC_EINVAL, "X and Y must not alias"};
    tc_handle* h = const_cast<tc_handle*>(hc);
    const size_t need = spmm_partial_doubles(h, k);
    if (need > kScratchDoubles)
      throw Err{TC_EINVAL, "split-row partial sums need " + std::to_string(need * sizeof(double)) +
                               " bytes, more than the " + std::to_string(kScratchDoubles * sizeof(double)) +
                               "-byte scratch of this call"};
    double* ptr = scratch_on_current_device();
    spmm_internal(h, X, Y, k, (hipStream_t)stream, false, nullptr, ptr);
    return TC_OK;
  });
}
