// Format builder on the GPU (Section 3.1 Solutions 1-3, Section 3.3,
// Algorithms 1-3).  Steps, in order:
//   a1  column lengths (entries per column)
//   a2  columns sorted by decreasing length, ties by increasing id (stable
//       LSD counting sort); square matrices relabel rows the same way
//   a3  number of dense tiles (Algorithm 1, on the host from W-strided
//       samples of the sorted lengths)
//   a4  entries bucketed by tile, keeping the input order inside each tile
//   a5  each tile's rows sorted by decreasing length, ties by internal row id
//   a6  workload size per tile (Algorithm 2 with the model of Algorithm 3) and
//       the greedy partition into workloads (host, from length histograms)
//   a7  pack: padded row-major / column-major rectangles, row ids, descriptors
// Every sort is a chain of stable counting-sort passes, so the format is a
// pure function of the input and the options.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>

#include "tc_prims.h"

namespace tc {
const char* get_error();

namespace {

constexpr int kB = 256;

inline unsigned nblk(int64_t n, int64_t per) { return (unsigned)((n + per - 1) / per); }

int bits_for(uint64_t v) {
  int b = 0;
  while (v) {
    ++b;
    v >>= 1;
  }
  return b;
}

struct Fail {
  tc_status st;
  std::string msg;
};

#define HIPX(call)                                                                   \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      throw Fail{TC_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)};        \
  } while (0)

// Temporary device buffers of one build, freed when the build ends.
// Temporary device arrays of one build, taken from the library's pool on the
// build stream and handed back (stream-ordered) when released or at the end.
struct Tmp {
  hipStream_t st;
  std::vector<void*> bufs;
  explicit Tmp(hipStream_t s) : st(s) {}
  template <class T>
  T* get(int64_t n) {
    size_t bytes = (size_t)std::max<int64_t>(n, 1) * sizeof(T);
    void* p = pool_alloc(bytes, st);
    if (!p) throw Fail{TC_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
    bufs.push_back(p);
    return (T*)p;
  }
  void release(void* p) {
    for (auto& b : bufs)
      if (b == p) {
        pool_free(b, st, false);
        b = nullptr;
      }
  }
  ~Tmp() {
    for (void* p : bufs)
      if (p) pool_free(p, st, false);
  }
};

template <class T>
T* hold(tc_handle* h, int64_t n) {
  size_t bytes = (size_t)std::max<int64_t>(n, 1) * sizeof(T);
  void* p = nullptr;
  if (h->alloc) {
    p = h->alloc(bytes, h->alloc_ctx);
    if (!p) throw Fail{TC_ENOMEM, "allocator callback returned NULL for " + std::to_string(bytes) + " bytes"};
  } else if (!(p = pool_alloc(bytes, h->stream))) {
    throw Fail{TC_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
  }
  h->owned.push_back(p);
  return (T*)p;
}

// ----------------------------------------------------------------- kernels
__global__ void k_validate_rows(const int64_t* __restrict__ rp, int64_t n_rows, int64_t nnz, int* flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n_rows) return;
  int64_t a = rp[i];
  bool bad = (i == 0 && a != 0) || (i == n_rows && a != nnz) || (i < n_rows && rp[i + 1] < a);
  if (bad) atomicOr(flag, 1);
}

__global__ void k_validate_cols(const int32_t* __restrict__ col, int64_t nnz, int64_t n_cols, int* flag) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nnz && (col[k] < 0 || (int64_t)col[k] >= n_cols)) atomicOr(flag, 2);
}

__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_iota(int32_t* a, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = (int32_t)i;
}

// a1: column lengths.  A power-law column can hold 10^5-10^6 entries, and
// atomics on one address serialise, so the hottest columns (found from a
// 1/64 sample) are counted in a per-block LDS hash table and flushed once per
// block; every other entry adds to its column directly.
constexpr int kHotCap = 4096;           // hot columns counted in LDS
constexpr int kHotSlots = 2 * kHotCap;  // open-addressing table (load <= 1/2)
constexpr int kSampleStep = 64;

__global__ void k_col_sample(const int32_t* __restrict__ col, int64_t nnz, int32_t* __restrict__ samp) {
  const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kSampleStep;
  if (k < nnz) atomicAdd(&samp[col[k]], 1);
}

// number of columns whose sampled count is >= 2^b, for b = 0..31:
// grid-stride, per-wave ballot counts summed in LDS, one atomic per block and b
__global__ void __launch_bounds__(256) k_sample_hist(const int32_t* __restrict__ samp, int64_t n,
                                                     unsigned long long* __restrict__ ge) {
  __shared__ unsigned int bc[32];
  if (threadIdx.x < 32) bc[threadIdx.x] = 0;
  __syncthreads();
  unsigned int acc[31];
#pragma unroll
  for (int b = 0; b < 31; ++b) acc[b] = 0;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < n; i0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = i0 + threadIdx.x;
    const int32_t v = i < n ? samp[i] : 0;
#pragma unroll
    for (int b = 0; b < 31; ++b) acc[b] += (unsigned int)__popcll(__ballot(v >= (1 << b)));
  }
  if (lane_id() == 0)
    for (int b = 0; b < 31; ++b)
      if (acc[b]) atomicAdd(&bc[b], acc[b]);
  __syncthreads();
  if (threadIdx.x < 31 && bc[threadIdx.x]) atomicAdd(&ge[threadIdx.x], (unsigned long long)bc[threadIdx.x]);
}

__global__ void k_ge_flags(const int32_t* __restrict__ samp, int64_t n, int32_t thr, int32_t* __restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flags[i] = samp[i] >= thr;
}

__global__ void k_compact_idx(const int32_t* __restrict__ flags, const int32_t* __restrict__ pos, int64_t n,
                              int32_t* __restrict__ out);

__device__ inline uint32_t hot_hash(int32_t c) { return ((uint32_t)c * 2654435761u) >> 19; }  // 13 bits

__global__ void __launch_bounds__(256) k_col_count_hot(const int32_t* __restrict__ col, int64_t nnz,
                                                       const int32_t* __restrict__ hot, int32_t n_hot,
                                                       int32_t* __restrict__ clen) {
  __shared__ int32_t key[kHotSlots];
  __shared__ int32_t cnt[kHotSlots];
  for (int i = threadIdx.x; i < kHotSlots; i += blockDim.x) {
    key[i] = -1;
    cnt[i] = 0;
  }
  __syncthreads();
  for (int32_t h = threadIdx.x; h < n_hot; h += blockDim.x) {  // keys are distinct
    uint32_t s = hot_hash(hot[h]) & (kHotSlots - 1);
    while (atomicCAS(&key[s], -1, hot[h]) != -1) s = (s + 1) & (kHotSlots - 1);
  }
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += stride) {
    const int32_t c = col[k];
    uint32_t s = hot_hash(c) & (kHotSlots - 1);
    int32_t kk;
    while ((kk = key[s]) != c && kk != -1) s = (s + 1) & (kHotSlots - 1);
    if (kk == c)
      atomicAdd(&cnt[s], 1);
    else
      atomicAdd(&clen[c], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kHotSlots; i += blockDim.x)
    if (key[i] != -1 && cnt[i]) atomicAdd(&clen[key[i]], cnt[i]);
}

// a1, bucketed: a counting-sort pass groups the column ids by their high
// bits, then each block counts one window of kCntWin columns of one bucket
// (a slice of its ids) in LDS and writes the window's lengths: plain stores
// when the bucket is one slice, atomics on the few buckets that need several.
constexpr int kCntWin = 32768;  // 128 KB of LDS counters
constexpr int kCntBlock = 1024;
constexpr int64_t kCntSlice = 1 << 20;

struct ColBucketOp {
  const int32_t* cin;
  int32_t* cout;
  int shift;
  using Item = int32_t;
  __device__ Item load(int64_t k) const { return cin[k]; }
  __device__ uint32_t bucket_of(Item c) const { return (uint32_t)c >> shift; }
  __device__ void store(int64_t p, Item c) const { cout[p] = c; }
};

struct CntTask {
  int64_t begin, end;  // slice of the bucketed ids
  int32_t base;        // first column of the window
  int32_t atomic;      // several slices share the window
};

__global__ void __launch_bounds__(kCntBlock) k_col_count_lds(const int32_t* __restrict__ bcol,
                                                             const CntTask* __restrict__ tasks, int64_t n_cols,
                                                             int32_t* __restrict__ clen) {
  extern __shared__ int32_t cnt_lds[];
  const CntTask t = tasks[blockIdx.x];
  for (int i = threadIdx.x; i < kCntWin; i += kCntBlock) cnt_lds[i] = 0;
  __syncthreads();
  int64_t k = t.begin + threadIdx.x;
  for (; k + 7 * kCntBlock < t.end; k += 8 * kCntBlock) {  // eight loads in flight
    int32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = bcol[k + u * kCntBlock];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint32_t c = (uint32_t)(v[u] - t.base);
      if (c < (uint32_t)kCntWin) atomicAdd(&cnt_lds[c], 1);
    }
  }
  for (; k < t.end; k += kCntBlock) {
    const uint32_t c = (uint32_t)(bcol[k] - t.base);
    if (c < (uint32_t)kCntWin) atomicAdd(&cnt_lds[c], 1);
  }
  __syncthreads();
  const int64_t lim = min<int64_t>(kCntWin, n_cols - t.base);
  for (int i = threadIdx.x; i < lim; i += kCntBlock) {
    const int32_t v = cnt_lds[i];
    if (t.atomic) {
      if (v) atomicAdd(&clen[t.base + i], v);
    } else {
      clen[t.base + i] = v;
    }
  }
}

// maximum of a non-negative array: grid-stride, one atomic per block
__global__ void __launch_bounds__(256) k_max_i32(const int32_t* __restrict__ a, int64_t n, int32_t* out) {
  __shared__ int32_t wm[256 / kWave];
  int32_t v = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v = max(v, a[i]);
  for (int d = 32; d > 0; d >>= 1) v = max(v, __shfl_xor(v, d, kWave));
  if (lane_id() == 0) wm[threadIdx.x / kWave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 256 / kWave; ++w) v = max(v, wm[w]);
    atomicMax(out, v);
  }
}

__global__ void k_count_eq(const int32_t* __restrict__ a, int64_t n, int32_t v, unsigned long long* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool e = i < n && a[i] == v;
  uint64_t m = __ballot(e);
  if (lane_id() == 0 && m) atomicAdd(out, (unsigned long long)__popcll(m));
}

__global__ void k_desc_keys(const int32_t* __restrict__ len, int64_t n, int32_t maxv, uint32_t* __restrict__ keys,
                            int32_t* __restrict__ vals) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    keys[i] = (uint32_t)(maxv - len[i]);
    vals[i] = (int32_t)i;
  }
}

__global__ void k_cols_finish(const uint32_t* __restrict__ keys, const int32_t* __restrict__ vals, int64_t n,
                              int32_t maxv, int32_t* __restrict__ cperm, int32_t* __restrict__ cpos,
                              int32_t* __restrict__ clen_sorted) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) {
    int32_t j = vals[k];
    cperm[k] = j;
    cpos[j] = (int32_t)k;
    clen_sorted[k] = maxv - (int32_t)keys[k];
  }
}

__global__ void k_rowmap(const int32_t* __restrict__ cpos, int64_t n_rows, int relabel, int32_t* __restrict__ rowmap,
                         int32_t* __restrict__ rowinv) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_rows) {
    int32_t r = relabel ? cpos[i] : (int32_t)i;
    rowmap[i] = r;
    rowinv[r] = (int32_t)i;
  }
}

// smallest i in [0, n) with a[i] >= key[g] (a non-decreasing), for g = 1..G-1
__global__ void k_lower_bound(const int64_t* __restrict__ a, int64_t n, const int64_t* __restrict__ key, int G,
                              int64_t* __restrict__ out) {
  const int g = threadIdx.x;
  if (g < 1 || g >= G) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < key[g]) lo = mid + 1; else hi = mid;
  }
  out[g] = lo;
}

__global__ void k_strided(const int32_t* __restrict__ a, int64_t stride, int64_t cnt, int32_t* __restrict__ out) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < cnt) out[t] = a[t * stride];
}

// Row id of every entry: lanes write their own short rows, the whole
// wavefront writes each long row.
// out[i] = a[i * stride] for i < n
__global__ void k_strided64(const int64_t* __restrict__ a, int64_t stride, int64_t n, int64_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i * stride];
}

__global__ void k_expand_rows(const int64_t* __restrict__ rp, int64_t n_rows, int32_t* __restrict__ row_of) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = lane_id();
  int64_t a = 0, b = 0;
  if (i < n_rows) {
    a = rp[i];
    b = rp[i + 1];
  }
  const bool longrow = (b - a) > kWave;
  if (!longrow)
    for (int64_t k = a; k < b; ++k) row_of[k] = (int32_t)i;
  uint64_t m = __ballot(longrow);
  while (m) {
    const int src = __ffsll((unsigned long long)m) - 1;
    m &= m - 1;
    const int64_t aa = __shfl(a, src, kWave), bb = __shfl(b, src, kWave);
    const int32_t r = (int32_t)__shfl((int64_t)i, src, kWave);
    for (int64_t k = aa + lane; k < bb; k += kWave) row_of[k] = r;
  }
}

__global__ void k_icol(const int32_t* __restrict__ col, const int32_t* __restrict__ cpos, int64_t nnz,
                       int32_t* __restrict__ icol) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nnz) icol[k] = cpos[col[k]];
}

// Entries in internal-row order.  k_irow_len: each internal row's length and
// the start of its CSR range; iptr is their scan.  k_perm_entries: output
// position p lies in internal row irow[p] (expanded from iptr) and takes the
// entry of the same rank in that row's CSR range, so a row keeps its entries
// in CSR order.  Written: the internal column, the value and the internal
// row.
__global__ void k_irow_len(const int64_t* __restrict__ rp, const int32_t* __restrict__ rowinv, int64_t n_rows,
                           int32_t* __restrict__ ilen, int64_t* __restrict__ istart) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n_rows) {
    const int32_t o = rowinv[r];
    const int64_t a = rp[o];
    ilen[r] = (int32_t)(rp[o + 1] - a);
    istart[r] = a;
  }
}

// One block of kPermBlock threads per kPermBlock positions.  With hist, the
// block also counts its positions' tiles (bucket (tile >> 0) & 255 of TileMap
// tm, nbuckets buckets) into hist[bucket * nchunks + block]: the first tile
// pass's histogram when that pass's chunks are kPermBlock items.
constexpr int kPermBlock = 1024;
template <class TM>
__global__ void __launch_bounds__(kPermBlock)
    k_perm_entries(const int32_t* __restrict__ irow, const int64_t* __restrict__ iptr,
                   const int64_t* __restrict__ istart, const int32_t* __restrict__ col,
                   const int32_t* __restrict__ cpos, const float* __restrict__ val, int64_t nnz,
                   int32_t* __restrict__ icol, float* __restrict__ pval, int32_t* __restrict__ prow, TM tm,
                   int32_t nbuckets, int64_t nchunks, int32_t* __restrict__ hist) {
  extern __shared__ int32_t pcnt[];
  if (hist) {
    for (int i = threadIdx.x; i < nbuckets; i += kPermBlock) pcnt[i] = 0;
    __syncthreads();
  }
  const int64_t p = (int64_t)blockIdx.x * kPermBlock + threadIdx.x;
  if (p < nnz) {
    const int32_t r = irow[p];
    const int64_t e = istart[r] + (p - iptr[r]);
    const int32_t c = cpos[col[e]];
    icol[p] = c;
    pval[p] = val[e];
    prow[p] = r;
    if (hist) atomicAdd(&pcnt[(uint32_t)tm(c) & 255u], 1);
  }
  if (hist) {
    __syncthreads();
    for (int i = threadIdx.x; i < nbuckets; i += kPermBlock) hist[(int64_t)i * nchunks + blockIdx.x] = pcnt[i];
  }
}

// Tile of an internal column: fixed-width tiles (icol / W, the columns past
// the T dense tiles forming tile T) or explicit tile starts (tiles 1..ns).
struct TileMap {
  int32_t W, T;
  const int32_t* starts;  // NULL for fixed width
  int32_t ns;
  // starts[i] = s0 + i * W for every i (the automatic panels' head tile, then
  // tiles of W columns): the tile is arithmetic, with a shift when W is a
  // power of two (wshift >= 0), instead of a search over the starts
  int32_t uniform = 0, s0 = 0, wshift = -1;
  __device__ int32_t operator()(int32_t icol) const {
    if (!starts) return min(icol / W, T);
    if (uniform) {
      if (icol < s0) return 0;
      const int32_t q = wshift >= 0 ? (icol - s0) >> wshift : (icol - s0) / W;
      return min(1 + q, ns);
    }
    int32_t lo = 0, hi = ns;  // number of starts <= icol
    while (lo < hi) {
      const int32_t mid = (lo + hi) >> 1;
      if (starts[mid] <= icol) lo = mid + 1; else hi = mid;
    }
    return lo;
  }
};

// first position of each tile in the bucketed entries (tile ids are sorted)
__global__ void k_tile_bounds(const int32_t* __restrict__ b_icol, int64_t nnz, TileMap tm, int32_t ntiles,
                              int64_t* __restrict__ tstart) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > ntiles) return;
  int64_t lo = 0, hi = nnz;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (tm(b_icol[mid]) < t) lo = mid + 1; else hi = mid;
  }
  tstart[t] = lo;
}

// a5: segment heads, the first entry of each (tile, row) pair.  The entries
// are bucketed by tile, so a head is the first entry, a row change, or the
// first entry of a tile (tstart: the ntiles tile starts).  Bit i of the
// result: entry base + i is a head, for the kScanPer entries of one thread
// in the scan layout; rows receives their rows.
__device__ inline uint32_t seg_head_bits(const int32_t* __restrict__ b_row, int64_t nnz,
                                         const int64_t* __restrict__ tstart, int32_t ntiles, int64_t base,
                                         int32_t* rows) {
  int32_t prev = base > 0 && base <= nnz ? b_row[base - 1] : -1;
  load_run(b_row, base, nnz, *reinterpret_cast<int32_t(*)[kScanPer]>(rows));
  int32_t lo = 0, hi = ntiles;  // first tile starting at or after base
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (tstart[mid] < base) lo = mid + 1; else hi = mid;
  }
  // that tile's start, read again only when the run passes it
  int64_t nxt = lo < ntiles ? tstart[lo] : INT64_MAX;
  uint32_t m = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    const int64_t k = base + i;
    bool h = k == 0 || rows[i] != prev;
    while (nxt < k) nxt = ++lo < ntiles ? tstart[lo] : INT64_MAX;
    if (nxt == k) h = true;
    if (k < nnz && h) m |= 1u << i;
    prev = rows[i];
  }
  return m;
}

// heads per scan block (block_sums[b]), for the scan of their positions
__global__ void __launch_bounds__(kScanBlock) k_seghead_count(const int32_t* __restrict__ b_row, int64_t nnz,
                                                              const int64_t* __restrict__ tstart, int32_t ntiles,
                                                              int64_t* __restrict__ block_sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  int32_t rows[kScanPer];
  const uint32_t m = seg_head_bits(b_row, nnz, tstart, ntiles, base, rows);
  int64_t tot;
  block_excl_scan<int64_t>((int64_t)__popc(m), &tot);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// every head's segment at its position: start entry, internal row (b_row
// holds the caller's rows when rowmap is given, else internal rows), tile
__global__ void __launch_bounds__(kScanBlock) k_seghead_emit(const int32_t* __restrict__ b_row,
                                                             const int32_t* __restrict__ b_icol,
                                                             const int32_t* __restrict__ rowmap, int64_t nnz,
                                                             const int64_t* __restrict__ tstart, int32_t ntiles,
                                                             TileMap tm, const int64_t* __restrict__ block_off,
                                                             int32_t* __restrict__ seg_start,
                                                             int32_t* __restrict__ seg_row,
                                                             int32_t* __restrict__ seg_tile) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  int32_t rows[kScanPer], cols[kScanPer];
  const uint32_t m = seg_head_bits(b_row, nnz, tstart, ntiles, base, rows);
  load_run(b_icol, base, nnz, cols);  // read whole, not under the per-head branch
  int64_t tot;
  int64_t off = block_excl_scan<int64_t>((int64_t)__popc(m), &tot) + block_off[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    if (!((m >> i) & 1u)) continue;
    const int64_t k = base + i;
    seg_start[off] = (int32_t)k;
    seg_row[off] = rowmap ? rowmap[rows[i]] : rows[i];
    seg_tile[off] = tm(cols[i]);
    ++off;
  }
}

// a5 with one tile: internal row i is a segment if its original row is non-empty
__global__ void k_rowseg_flags(const int64_t* __restrict__ rp, const int32_t* __restrict__ rowinv, int64_t n_rows,
                               int32_t* __restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_rows) return;
  const int32_t o = rowinv[i];
  flags[i] = rp[o + 1] > rp[o];
}

__global__ void k_rowseg_emit(const int32_t* __restrict__ flags, const int32_t* __restrict__ pos,
                              const int64_t* __restrict__ rp, const int32_t* __restrict__ rowinv, int64_t n_rows,
                              int32_t* __restrict__ seg_start, int32_t* __restrict__ seg_row,
                              int32_t* __restrict__ seg_tile, int32_t* __restrict__ seg_len) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_rows || !flags[i]) return;
  const int32_t s = pos[i], o = rowinv[i];
  const int64_t a = rp[o];
  seg_start[s] = (int32_t)a;
  seg_row[s] = (int32_t)i;
  seg_tile[s] = 0;
  seg_len[s] = (int32_t)(rp[o + 1] - a);
}

__global__ void k_seg_len(const int32_t* __restrict__ seg_start, int64_t nseg, int64_t nnz, int32_t* __restrict__ seg_len) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nseg) seg_len[s] = (int32_t)((s + 1 < nseg ? (int64_t)seg_start[s + 1] : nnz) - seg_start[s]);
}

__global__ void k_seg_keys(const int32_t* __restrict__ seg_tile, const int32_t* __restrict__ seg_len,
                           const int32_t* __restrict__ seg_row, const int32_t* __restrict__ seg_start, int64_t nseg,
                           int32_t maxlen, int lb, int rb, uint64_t* __restrict__ keys, int32_t* __restrict__ vals) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  keys[s] = ((uint64_t)seg_tile[s] << (lb + rb)) | ((uint64_t)(maxlen - seg_len[s]) << rb) | (uint64_t)seg_row[s];
  vals[s] = seg_start[s];
}

// sorted segments: row and length back from the key, start from the value
__global__ void k_seg_decode(const uint64_t* __restrict__ keys, const int32_t* __restrict__ vals, int64_t nseg,
                             int32_t maxlen, int lb, int rb, int32_t* __restrict__ rows_sorted,
                             int32_t* __restrict__ rows_len, int32_t* __restrict__ srt_start) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nseg) return;
  const uint64_t k = keys[i];
  rows_sorted[i] = (int32_t)(k & (((uint64_t)1 << rb) - 1));
  rows_len[i] = maxlen - (int32_t)((k >> rb) & (((uint64_t)1 << lb) - 1));
  srt_start[i] = vals[i];
}

// start of each tile in the sorted segment keys (tile in the top bits)
__global__ void k_key_bounds(const uint64_t* __restrict__ keys, int64_t nseg, int shift, int32_t ntiles,
                             int64_t* __restrict__ off) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > ntiles) return;
  int64_t lo = 0, hi = nseg;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if ((int64_t)(keys[mid] >> shift) < t) lo = mid + 1; else hi = mid;
  }
  off[t] = lo;
}

// run heads of (tile, length) in the sorted segment keys
__global__ void k_run_flags(const uint64_t* __restrict__ keys, int64_t nseg, int rb, int32_t* __restrict__ flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nseg) flags[i] = i == 0 || (keys[i] >> rb) != (keys[i - 1] >> rb);
}

__global__ void k_run_emit(const int32_t* __restrict__ flags, const int32_t* __restrict__ pos,
                           const int32_t* __restrict__ rows_len, int64_t nseg, int64_t* __restrict__ run_pos,
                           int32_t* __restrict__ run_len) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nseg && flags[i]) {
    run_pos[pos[i]] = i;
    run_len[pos[i]] = rows_len[i];
  }
}

// (length, rows) of every run: a run ends where the next begins, or at nseg
__global__ void k_run_pairs(const int64_t* __restrict__ run_pos, const int32_t* __restrict__ run_len, int64_t nruns,
                            int64_t nseg, LenRun* __restrict__ runs) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nruns) runs[r] = LenRun{run_len[r], (r + 1 < nruns ? run_pos[r + 1] : nseg) - run_pos[r]};
}

// rows of the split rows' chunks (sorted-row positions at) and each row's first tile
__global__ void k_chunk_rows(const int32_t* __restrict__ rows_sorted, const int32_t* __restrict__ first,
                             const int32_t* __restrict__ at, int64_t nc, int32_t* __restrict__ row,
                             int32_t* __restrict__ row_first) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nc) return;
  const int32_t r = rows_sorted[at[q]];
  row[q] = r;
  row_first[q] = first[r];
}

// first tile in which each row sits in a workload that is not a split chunk
__global__ void k_first_touch(const int32_t* __restrict__ seg_tile, const int32_t* __restrict__ seg_len,
                              const int32_t* __restrict__ seg_row, int64_t nseg, const int64_t* __restrict__ split_t,
                              int32_t* __restrict__ first, int32_t* __restrict__ touched) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  const int32_t t = seg_tile[s], r = seg_row[s];
  touched[r] = 1;
  const int64_t sp = split_t[t];
  if (!(sp > 0 && (int64_t)seg_len[s] > sp)) atomicMin(&first[r], t);
}

// Row panels: entries of each row that stay with the row (segments no
// longer than their column tile's split length; longer ones become chunks).
__global__ void k_panel_weight(const int32_t* __restrict__ seg_tile, const int32_t* __restrict__ seg_len,
                               const int32_t* __restrict__ seg_row, int64_t nseg, const int64_t* __restrict__ split_t,
                               int32_t* __restrict__ w) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  const int64_t sp = split_t[seg_tile[s]];
  if (!(sp > 0 && (int64_t)seg_len[s] > sp)) atomicAdd(&w[seg_row[s]], seg_len[s]);
}

// first i in [0, n] with pre[i] >= tgt[p] (pre non-decreasing, n + 1 entries)
__global__ void k_lower_bound_pre(const int64_t* __restrict__ pre, int64_t n, const int64_t* __restrict__ tgt, int P,
                                  int64_t* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (pre[mid] < tgt[p]) lo = mid + 1; else hi = mid;
  }
  out[p] = lo;
}

// Row panels: the segment's tile becomes panel * nct + column tile (the
// panel bounds pb staged in LDS when lds_pb), then the row's first-touch
// tile and touched flag as in k_first_touch (split lengths per column tile).
__global__ void k_seg_panel_touch(int32_t* __restrict__ seg_tile, const int32_t* __restrict__ seg_row,
                                  const int32_t* __restrict__ seg_len, int64_t nseg, const int32_t* __restrict__ pb,
                                  int32_t np, int32_t nct, int lds_pb, const int64_t* __restrict__ split_col,
                                  int32_t* __restrict__ first, int32_t* __restrict__ touched) {
  extern __shared__ int32_t spb[];
  if (lds_pb) {
    for (int i = threadIdx.x; i <= np; i += blockDim.x) spb[i] = pb[i];
    __syncthreads();
  }
  const int32_t* b = lds_pb ? spb : pb;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  const int32_t r = seg_row[s], ct = seg_tile[s];
  int32_t lo = 0, hi = np - 1;  // last panel with pb[p] <= r
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (b[mid] <= r) lo = mid; else hi = mid - 1;
  }
  const int32_t t = lo * nct + ct;
  seg_tile[s] = t;
  touched[r] = 1;
  const int64_t sp = split_col[ct];
  if (!(sp > 0 && (int64_t)seg_len[s] > sp)) atomicMin(&first[r], t);
}

__global__ void k_tile_entries(const int64_t* __restrict__ pre, const int64_t* __restrict__ off, int32_t ntiles,
                               int64_t* __restrict__ tnnz) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < ntiles) tnnz[g] = pre[off[g + 1]] - pre[off[g]];
}

__global__ void k_ne(const int32_t* __restrict__ a, int64_t n, int32_t v, int32_t* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] != v;
}

__global__ void k_not(const int32_t* __restrict__ a, int64_t n, int32_t* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] ? 0 : 1;
}

__global__ void k_compact_idx(const int32_t* __restrict__ flags, const int32_t* __restrict__ pos, int64_t n,
                              int32_t* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flags[i]) out[pos[i]] = (int32_t)i;
}

// what the pack needs of a workload beyond its device descriptor
struct PackX {
  int32_t row_begin;  // first sorted row (a chunk: its row)
  int32_t chunk_off;  // a chunk: its first entry within the row, else -1
  int32_t chunk_len;  // a chunk: its real entries
  int32_t tile;
};

// a7: one wavefront per workload writes its rectangle, its pads and row ids.
constexpr int kPackSlices = 4;
__global__ void __launch_bounds__(kB) k_pack(const Wl* __restrict__ dwl, const PackX* __restrict__ pxs,
                                             int64_t n_wl, const int32_t* __restrict__ tile_first, int camping,
                                             const int32_t* __restrict__ srt_start,
                                             const int32_t* __restrict__ rows_len,
                                             const int32_t* __restrict__ rows_sorted,
                                             const int32_t* __restrict__ b_icol, const float* __restrict__ b_val,
                                             const int32_t* __restrict__ first, int32_t* __restrict__ idx,
                                             float* __restrict__ val, int32_t* __restrict__ rowid, float pad) {
  // kPackSlices wavefronts per workload, slice sl taking every kPackSlices-th
  // row (RM), row block of 64 (CM) or 64-entry block (chunk).  Four positions'
  // loads go out together, then their stores: a position past its row's L
  // real entries reloads the row's last entry (entry 0 of the bucketed arrays
  // for a row with none) and stores the pad.
  const int lane = lane_id();
  const int64_t w = (int64_t)blockIdx.x * (kB / kWave) + threadIdx.x / kWave;
  if (w >= n_wl * kPackSlices) return;
  const int64_t j = w / kPackSlices;
  const int sl = (int)(w % kPackSlices);
  const Wl wd = dwl[j];
  const PackX x = pxs[j];
  struct {
    int64_t data_off, rowid_off;
    int32_t w_pad, h_pad, n_rows, layout, row_begin, tile, tile_first, extra;
  } d;
  d.data_off = wd.data_off;
  d.rowid_off = wd.rowid_off;
  d.w_pad = wd.w_pad;
  d.h_pad = wd.h_pad;
  d.n_rows = wd.n_rows;
  d.layout = wd.info & 3;
  d.row_begin = x.row_begin;
  d.tile = x.tile;
  d.tile_first = tile_first[x.tile];
  const int64_t area = (int64_t)wd.w_pad * wd.h_pad;
  d.extra = (camping && area % 512 == 0) ? 64 : 0;  // the camping pad after the rectangle
  const int64_t off = d.data_off;
  if (x.chunk_off >= 0) {
    const int32_t s = d.row_begin;
    const int64_t st = (int64_t)srt_start[s] + x.chunk_off;
    const int64_t L = x.chunk_len;
    const int64_t step = (int64_t)kWave * kPackSlices;
    for (int64_t c0 = lane + (int64_t)sl * kWave; c0 < d.w_pad; c0 += 4 * step) {
      int32_t ti[4];
      float tv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t q = L > 0 ? st + min(c0 + u * step, L - 1) : 0;
        ti[u] = b_icol[q];
        tv[u] = b_val[q];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t c = c0 + u * step;
        if (c < d.w_pad) {
          idx[off + c] = c < L ? ti[u] : d.tile_first;
          val[off + c] = c < L ? tv[u] : pad;
        }
      }
    }
    if (lane == 0 && sl == 0) rowid[d.rowid_off] = rows_sorted[s];
  } else if (d.layout == kRM) {
    for (int32_t r = sl; r < d.n_rows; r += kPackSlices) {
      const int32_t s = d.row_begin + r;
      const int64_t st = srt_start[s];
      const int32_t L = rows_len[s];
      const int64_t base = off + (int64_t)r * d.w_pad;
      for (int64_t c0 = lane; c0 < d.w_pad; c0 += 4 * kWave) {
        int32_t ti[4];
        float tv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t q = L > 0 ? st + min<int64_t>(c0 + u * kWave, L - 1) : 0;
          ti[u] = b_icol[q];
          tv[u] = b_val[q];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t c = c0 + u * kWave;
          if (c < d.w_pad) {
            idx[base + c] = c < L ? ti[u] : d.tile_first;
            val[base + c] = c < L ? tv[u] : pad;
          }
        }
      }
      if (lane == 0) {
        const int32_t row = rows_sorted[s];
        rowid[d.rowid_off + r] = row | (first[row] == d.tile ? 0 : kAddFlag);
      }
    }
  } else {
    for (int32_t r = lane + sl * kWave; r < d.h_pad; r += kWave * kPackSlices) {
      int64_t st = 0;
      int32_t L = 0, row = -1;
      if (r < d.n_rows) {
        const int32_t s = d.row_begin + r;
        st = srt_start[s];
        L = rows_len[s];
        row = rows_sorted[s];
      }
      rowid[d.rowid_off + r] = row < 0 ? row : (row | (first[row] == d.tile ? 0 : kAddFlag));
      for (int32_t c0 = 0; c0 < d.w_pad; c0 += 4) {
        int32_t ti[4];
        float tv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t q = L > 0 ? st + min(c0 + u, L - 1) : 0;
          ti[u] = b_icol[q];
          tv[u] = b_val[q];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int32_t c = c0 + u;
          if (c < d.w_pad) {
            const int64_t e = off + (int64_t)c * d.h_pad + r;
            idx[e] = c < L ? ti[u] : d.tile_first;
            val[e] = c < L ? tv[u] : pad;
          }
        }
      }
    }
  }
  const int64_t end = off + (int64_t)d.w_pad * d.h_pad;
  if (sl == 0)
    for (int32_t c = lane; c < d.extra; c += kWave) {
      idx[end + c] = d.tile_first;
      val[end + c] = pad;
    }
}

// the bit pattern of int32 -1 as a float (the value map's pad mark)
float pad_minus_one() {
  const int32_t m = -1;
  float f;
  std::memcpy(&f, &m, sizeof f);
  return f;
}

// Value map: the build carries every entry's CSR index in place of its value
// (bit pattern) and marks pads with -1; this keeps the map and puts the
// values in.
__global__ void k_iota_i32(int32_t* __restrict__ a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = (int32_t)i;
}

__global__ void k_vmap_finish(float* __restrict__ val, int64_t n, const float* __restrict__ src,
                              int32_t* __restrict__ vmap) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t e = __float_as_int(val[i]);
  vmap[i] = e;
  val[i] = e >= 0 ? src[e] : 0.0f;
}

__global__ void k_refresh_vals(const int32_t* __restrict__ vmap, int64_t n, const float* __restrict__ src,
                               float* __restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t e = vmap[i];
  const float v = src[e >= 0 ? e : 0];  // a pad reads entry 0 and stores 0
  val[i] = e >= 0 ? v : 0.0f;
}

// ------------------------------------------------------ counting-sort ops
template <typename K>
struct KeyVal {
  K key;
  int32_t v;
};

template <typename K>
struct RadixOp {
  const K* kin;
  const int32_t* vin;
  K* kout;
  int32_t* vout;
  int shift;
  using Item = KeyVal<K>;
  __device__ Item load(int64_t k) const { return {kin[k], vin[k]}; }
  __device__ uint32_t bucket_of(const Item& it) const { return (uint32_t)(it.key >> shift) & 255u; }
  __device__ void store(int64_t p, const Item& it) const {
    kout[p] = it.key;
    vout[p] = it.v;
  }
};
using RadixU32Op = RadixOp<uint32_t>;
using RadixU64Op = RadixOp<uint64_t>;

struct TileItem {
  int32_t icol;
  float val;
  int32_t row;
};

struct TileOp {
  const int32_t* icol_in;
  const float* val_in;
  const int32_t* row_in;
  int32_t* icol_out;
  float* val_out;
  int32_t* row_out;
  TileMap tm;
  int shift;
  using Item = TileItem;
  __device__ Item load(int64_t k) const { return {icol_in[k], val_in[k], row_in[k]}; }
  __device__ uint32_t bucket_of(const Item& it) const { return ((uint32_t)tm(it.icol) >> shift) & 255u; }
  __device__ void store(int64_t p, const Item& it) const {
    icol_out[p] = it.icol;
    val_out[p] = it.val;
    row_out[p] = it.row;
  }
};

// ------------------------------------------------------------ host helpers
template <typename In, typename Out>
void excl_scan_async(const In* in, int64_t n, Out* out, int64_t* bs, int64_t nb, hipStream_t st) {
  if (n > 0) {
    hipLaunchKernelGGL((k_scan_reduce<In>), dim3((unsigned)nb), dim3(kScanBlock), 0, st, in, n, bs);
    HIPX(hipGetLastError());
  } else {
    HIPX(hipMemsetAsync(bs, 0, sizeof(int64_t), st));
  }
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kScanBlock), 0, st, bs, nb, bs + nb);
  HIPX(hipGetLastError());
  if (n > 0) {
    hipLaunchKernelGGL((k_scan_down<In, Out>), dim3((unsigned)nb), dim3(kScanBlock), 0, st, in, n, bs, out);
    HIPX(hipGetLastError());
  }
}

// exclusive scan; returns the total (which waits for the stream)
template <typename In, typename Out>
int64_t excl_scan(const In* in, int64_t n, Out* out, Tmp& tmp, hipStream_t st) {
  const int64_t nb = std::max<int64_t>(1, (n + kScanTile - 1) / kScanTile);
  int64_t* bs = tmp.get<int64_t>(nb + 1);
  excl_scan_async(in, n, out, bs, nb, st);
  int64_t total = 0;
  HIPX(hipMemcpyAsync(&total, bs + nb, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIPX(hipStreamSynchronize(st));
  tmp.release(bs);
  return total;
}

// One stable counting-sort pass over `nbits` bits of the key (stream
// ordered, no host wait).  The scatter stages each chunk in LDS, so the
// chunk is sized to keep one block's staging within 80 KB (two blocks per
// compute unit).
constexpr size_t kCsStageBytes = (size_t)80 << 10;
struct CsPlan {
  int nbuckets;
  int64_t chunk, nchunks;
};
template <class Item>
CsPlan cs_plan(int64_t n, int nbits) {
  CsPlan c;
  c.nbuckets = std::max(kWave, 1 << nbits);  // the staged scatter takes multiples of 64
  c.chunk = 4096;
  while (c.chunk > 256 &&
         (size_t)kCsWaves * ((size_t)c.chunk * sizeof(Item) + 16 * (size_t)c.nbuckets) > kCsStageBytes)
    c.chunk /= 2;
  c.nchunks = (n + c.chunk - 1) / c.chunk;
  return c;
}

// pre_hist: the pass's (bucket, chunk) counts, already made by the caller
// with the chunking of cs_plan (owned by the caller)
template <class Op>
void cs_pass(const Op& op, int64_t n, int nbits, Tmp& tmp, hipStream_t st, int32_t* pre_hist = nullptr) {
  if (n <= 0) return;
  using Item = typename Op::Item;
  const CsPlan pl = cs_plan<Item>(n, nbits);
  const int nbuckets = pl.nbuckets;
  const int64_t chunk = pl.chunk, nchunks = pl.nchunks;
  const unsigned grid = (unsigned)((nchunks + kCsWaves - 1) / kCsWaves);
  const int64_t nh = (int64_t)nbuckets * nchunks;
  int32_t* hist = pre_hist ? pre_hist : tmp.get<int32_t>(nh);
  int64_t* offs = tmp.get<int64_t>(nh);
  const int64_t nsb = std::max<int64_t>(1, (nh + kScanTile - 1) / kScanTile);
  int64_t* bs = tmp.get<int64_t>(nsb + 1);
  if (!pre_hist) {
    hipLaunchKernelGGL((k_cs_hist<Op>), dim3(grid), dim3(kCsBlock), kCsWaves * nbuckets * sizeof(int32_t), st, op,
                       n, nbuckets, chunk, nchunks, hist);
    HIPX(hipGetLastError());
  }
  excl_scan_async<int32_t, int64_t>(hist, nh, offs, bs, nsb, st);
  const size_t stage = (size_t)kCsWaves * ((size_t)chunk * sizeof(Item) + 16 * (size_t)nbuckets);
  HIPX(hipFuncSetAttribute((const void*)k_cs_scatter_staged<Op>, hipFuncAttributeMaxDynamicSharedMemorySize,
                           (int)stage));
  hipLaunchKernelGGL((k_cs_scatter_staged<Op>), dim3(grid), dim3(kCsBlock), stage, st, op, n, nbuckets, nbits, chunk,
                     nchunks, (const int64_t*)offs, (const int32_t*)hist);
  HIPX(hipGetLastError());
  if (!pre_hist) tmp.release(hist);
  tmp.release(offs);
  tmp.release(bs);
}

int32_t dev_max(const int32_t* a, int64_t n, Tmp& tmp, hipStream_t st) {
  int32_t* d = tmp.get<int32_t>(1);
  HIPX(hipMemsetAsync(d, 0, sizeof(int32_t), st));
  if (n > 0) hipLaunchKernelGGL(k_max_i32, dim3((unsigned)std::min<int64_t>(1024, nblk(n, kB))), dim3(kB), 0, st, a, n, d);
  HIPX(hipGetLastError());
  int32_t v = 0;
  HIPX(hipMemcpyAsync(&v, d, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPX(hipStreamSynchronize(st));
  tmp.release(d);
  return v;
}

// a1 for small inputs and very wide matrices: global atomics, with the
// hottest columns (found from a 1/64 sample) counted in a per-block LDS table.
void col_count_atomic(const int32_t* col_idx, int64_t nnz, int64_t n_cols, int32_t* clen, Tmp& tmp, hipStream_t st) {
  int32_t n_hot = 0;
  int32_t* hot = nullptr;
  if (nnz >= (int64_t)kSampleStep * 1024) {
    int32_t* samp = tmp.get<int32_t>(n_cols);
    unsigned long long* ge = tmp.get<unsigned long long>(32);
    HIPX(hipMemsetAsync(samp, 0, sizeof(int32_t) * n_cols, st));
    HIPX(hipMemsetAsync(ge, 0, sizeof(unsigned long long) * 32, st));
    const int64_t ns = (nnz + kSampleStep - 1) / kSampleStep;
    hipLaunchKernelGGL(k_col_sample, dim3(nblk(ns, kB)), dim3(kB), 0, st, col_idx, nnz, samp);
    hipLaunchKernelGGL(k_sample_hist, dim3((unsigned)std::min<int64_t>(1024, nblk(n_cols, 256))), dim3(256), 0, st,
                       (const int32_t*)samp, n_cols, ge);
    HIPX(hipGetLastError());
    unsigned long long hge[32];
    HIPX(hipMemcpyAsync(hge, ge, sizeof(hge), hipMemcpyDeviceToHost, st));
    HIPX(hipStreamSynchronize(st));
    int b = 2;  // at least 4 sampled hits (about 256 entries) to be worth a slot
    while (b < 31 && hge[b] > (unsigned long long)kHotCap) ++b;
    if (b < 31 && hge[b] > 0) {
      int32_t* fl = tmp.get<int32_t>(n_cols);
      int32_t* ps = tmp.get<int32_t>(n_cols);
      hipLaunchKernelGGL(k_ge_flags, dim3(nblk(n_cols, kB)), dim3(kB), 0, st, (const int32_t*)samp, n_cols,
                         (int32_t)1 << b, fl);
      HIPX(hipGetLastError());
      n_hot = (int32_t)excl_scan<int32_t, int32_t>(fl, n_cols, ps, tmp, st);
      hot = tmp.get<int32_t>(n_hot);
      hipLaunchKernelGGL(k_compact_idx, dim3(nblk(n_cols, kB)), dim3(kB), 0, st, (const int32_t*)fl,
                         (const int32_t*)ps, n_cols, hot);
      HIPX(hipGetLastError());
    }
  }
  if (nnz > 0) {
    const unsigned grid = (unsigned)std::min<int64_t>(2048, nblk(nnz, kB));
    hipLaunchKernelGGL(k_col_count_hot, dim3(grid), dim3(256), 0, st, col_idx, nnz, (const int32_t*)hot, n_hot, clen);
    HIPX(hipGetLastError());
  }
}

// a1 for everything else: see k_col_count_lds
void col_count_bucketed(const int32_t* col, int64_t nnz, int64_t n_cols, int cshift, int64_t windows, int32_t* clen,
                        Tmp& tmp, hipStream_t st) {
  const int nbits = 8, nb = 1 << nbits;
  const int64_t chunk = 4096;
  const int64_t nchunks = (nnz + chunk - 1) / chunk;
  const unsigned grid = (unsigned)((nchunks + kCsWaves - 1) / kCsWaves);
  int32_t* bcol = tmp.get<int32_t>(nnz);
  int32_t* hist = tmp.get<int32_t>((int64_t)nb * nchunks);
  int64_t* offs = tmp.get<int64_t>((int64_t)nb * nchunks + 1);
  const ColBucketOp op{col, bcol, cshift};
  hipLaunchKernelGGL((k_cs_hist<ColBucketOp>), dim3(grid), dim3(kCsBlock), kCsWaves * nb * sizeof(int32_t), st, op, nnz,
                     nb, chunk, nchunks, hist);
  HIPX(hipGetLastError());
  excl_scan<int32_t, int64_t>(hist, (int64_t)nb * nchunks, offs, tmp, st);
  // staged in LDS, so each bucket's run of a chunk is written coalesced
  const size_t stage = (size_t)kCsWaves * (chunk * sizeof(ColBucketOp::Item) + 16 * (size_t)nb);
  HIPX(hipFuncSetAttribute((const void*)k_cs_scatter_staged<ColBucketOp>, hipFuncAttributeMaxDynamicSharedMemorySize,
                           (int)stage));
  hipLaunchKernelGGL((k_cs_scatter_staged<ColBucketOp>), dim3(grid), dim3(kCsBlock), stage, st, op, nnz, nb, nbits,
                     chunk, nchunks, (const int64_t*)offs, (const int32_t*)hist);
  HIPX(hipGetLastError());
  // bucket starts: offs[b * nchunks]
  int64_t* d_bs = tmp.get<int64_t>(nb);
  hipLaunchKernelGGL(k_strided64, dim3(1), dim3(nb), 0, st, (const int64_t*)offs, nchunks, (int64_t)nb, d_bs);
  HIPX(hipGetLastError());
  std::vector<int64_t> bs(nb + 1);
  HIPX(hipMemcpyAsync(bs.data(), d_bs, sizeof(int64_t) * nb, hipMemcpyDeviceToHost, st));
  HIPX(hipStreamSynchronize(st));
  bs[nb] = nnz;
  std::vector<CntTask> tasks;
  for (int b = 0; b < nb; ++b) {
    const int64_t len = bs[b + 1] - bs[b];
    if (len == 0) continue;
    const int64_t ns = (len + kCntSlice - 1) / kCntSlice;
    for (int64_t w = 0; w < windows; ++w) {
      const int64_t base = ((int64_t)b << cshift) + w * kCntWin;
      if (base >= n_cols) break;
      for (int64_t j = 0; j < ns; ++j)
        tasks.push_back(CntTask{bs[b] + len * j / ns, bs[b] + len * (j + 1) / ns, (int32_t)base, ns > 1 ? 1 : 0});
    }
  }
  if (tasks.empty()) return;
  CntTask* d_tasks = tmp.get<CntTask>((int64_t)tasks.size());
  HIPX(hipMemcpyAsync(d_tasks, tasks.data(), sizeof(CntTask) * tasks.size(), hipMemcpyHostToDevice, st));
  HIPX(hipFuncSetAttribute((const void*)k_col_count_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                           kCntWin * (int)sizeof(int32_t)));
  hipLaunchKernelGGL(k_col_count_lds, dim3((unsigned)tasks.size()), dim3(kCntBlock), kCntWin * sizeof(int32_t), st,
                     (const int32_t*)bcol, (const CntTask*)d_tasks, n_cols, clen);
  HIPX(hipGetLastError());
  // the task list is host memory: finish before it goes out of scope
  HIPX(hipStreamSynchronize(st));
}

// transpose: entry e' of A^T is entry v[e'] of A
__global__ void k_transpose_gather(const int32_t* __restrict__ v, const int32_t* __restrict__ row_of,
                                   const float* __restrict__ val, int64_t n, int32_t* __restrict__ colT,
                                   float* __restrict__ valT, int32_t* __restrict__ permT) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t e = v[i];
  if (colT) colT[i] = row_of[e];
  if (valT) valT[i] = val[e];
  if (permT) permT[i] = e;
}

// CSR of A^T: column counts, their scan, and a stable sort of the entries by
// column (LSD counting-sort passes that carry the entry index), so each row of
// A^T lists its entries by increasing row of A.
void transpose(const tc_csr* A, int64_t* rpT, int32_t* colT, float* valT, int32_t* permT, hipStream_t st) {
  const int64_t n_rows = A->n_rows, n_cols = A->n_cols, nnz = A->nnz;
  Tmp tmp(st);
  {
    int* flag = tmp.get<int>(1);
    HIPX(hipMemsetAsync(flag, 0, sizeof(int), st));
    hipLaunchKernelGGL(k_validate_rows, dim3(nblk(n_rows + 1, kB)), dim3(kB), 0, st, A->row_ptr, n_rows, nnz, flag);
    if (nnz > 0) hipLaunchKernelGGL(k_validate_cols, dim3(nblk(nnz, kB)), dim3(kB), 0, st, A->col_idx, nnz, n_cols, flag);
    HIPX(hipGetLastError());
    int f = 0;
    HIPX(hipMemcpyAsync(&f, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPX(hipStreamSynchronize(st));
    if (f & 1) throw Fail{TC_EINVAL, "invalid CSR: row_ptr must start at 0, not decrease and end at nnz"};
    if (f & 2) throw Fail{TC_EINVAL, "invalid CSR: a column id is outside [0, n_cols)"};
  }
  int32_t* clen = tmp.get<int32_t>(n_cols);
  if (n_cols > 0) HIPX(hipMemsetAsync(clen, 0, sizeof(int32_t) * n_cols, st));
  const int cbits = bits_for((uint64_t)(n_cols > 1 ? n_cols - 1 : 0));
  const int cshift = std::max(15, cbits - 8);
  const int64_t windows = (int64_t)1 << (cshift - 15);
  if (nnz >= 4096 && windows <= 4)
    col_count_bucketed(A->col_idx, nnz, n_cols, cshift, windows, clen, tmp, st);
  else if (n_cols > 0 && nnz > 0)
    col_count_atomic(A->col_idx, nnz, n_cols, clen, tmp, st);
  const int64_t total = n_cols > 0 ? excl_scan<int32_t, int64_t>(clen, n_cols, rpT, tmp, st) : 0;
  HIPX(hipMemcpyAsync(rpT + n_cols, &total, sizeof(int64_t), hipMemcpyHostToDevice, st));
  if (nnz > 0) {
    int32_t* row_of = tmp.get<int32_t>(nnz);
    hipLaunchKernelGGL(k_expand_rows, dim3(nblk(n_rows, kB)), dim3(kB), 0, st, A->row_ptr, n_rows, row_of);
    uint32_t* k0 = tmp.get<uint32_t>(nnz);
    uint32_t* k1 = tmp.get<uint32_t>(nnz);
    int32_t* v0 = tmp.get<int32_t>(nnz);
    int32_t* v1 = tmp.get<int32_t>(nnz);
    HIPX(hipMemcpyAsync(k0, A->col_idx, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_iota, dim3(nblk(nnz, kB)), dim3(kB), 0, st, v0, nnz);
    HIPX(hipGetLastError());
    for (int sh = 0; sh < cbits; sh += 8) {
      cs_pass(RadixU32Op{k0, v0, k1, v1, sh}, nnz, 8, tmp, st);
      std::swap(k0, k1);
      std::swap(v0, v1);
    }
    hipLaunchKernelGGL(k_transpose_gather, dim3(nblk(nnz, kB)), dim3(kB), 0, st, (const int32_t*)v0,
                       (const int32_t*)row_of, A->val, nnz, colT, valT, permT);
    HIPX(hipGetLastError());
  }
  HIPX(hipStreamSynchronize(st));  // the host total above is read by the copy
}

// TILE-COO: first tile holding each row (tiles ascend in the bucketed order)
__global__ void k_coo_first(const int32_t* __restrict__ rows, const int64_t* __restrict__ tstart, int32_t ntiles,
                            const int32_t* __restrict__ rowmap, int64_t nnz, int32_t* __restrict__ first) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  int32_t lo = 0, hi = ntiles - 1;  // tile of entry e: last t with tstart[t] <= e
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (tstart[mid] <= e) lo = mid; else hi = mid - 1;
  }
  atomicMin(&first[rowmap[rows[e]]], lo);
}

__global__ void k_coo_pack(const int32_t* __restrict__ rows, const int32_t* __restrict__ icol,
                           const float* __restrict__ val, const int64_t* __restrict__ tstart, int32_t ntiles,
                           const int32_t* __restrict__ rowmap, const int32_t* __restrict__ first, int64_t nnz,
                           int32_t* __restrict__ crow, int32_t* __restrict__ ccol, float* __restrict__ cval) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  int32_t lo = 0, hi = ntiles - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (tstart[mid] <= e) lo = mid; else hi = mid - 1;
  }
  const int32_t r = rowmap[rows[e]];
  crow[e] = r | (first ? (first[r] == lo ? 0 : kAddFlag) : 0);
  ccol[e] = icol[e];
  cval[e] = val[e];
}

// TC_BUILD_TRACE=1: synchronise after every phase and print its wall time
struct PhaseClock {
  hipStream_t st;
  bool on;
  std::chrono::steady_clock::time_point t;
  explicit PhaseClock(hipStream_t s)
      : st(s), on(std::getenv("TC_BUILD_TRACE") != nullptr), t(std::chrono::steady_clock::now()) {}
  void mark(const char* what) {
    if (!on) return;
    (void)hipStreamSynchronize(st);
    const auto n = std::chrono::steady_clock::now();
    std::fprintf(stderr, "tc build: %-24s %9.3f ms\n", what, std::chrono::duration<double, std::milli>(n - t).count());
    t = n;
  }
};

// Every device descriptor must address only its own part of the packed
// arrays before any kernel is launched on it: rows within the stored rows,
// elements within [0, nnz_pad), row ids within [0, n_rowid), chunk slots
// within [0, n_slots), and its rows within its tile's sorted rows.  The
// offsets come from a running sum, so a violation is a bug in the partition;
// it is reported instead of handing a kernel an address outside a buffer.
inline bool descriptor_ok(const Wl& d, const HostWl& w, int64_t tile, int64_t row_lo, int64_t row_hi,
                          int64_t n_slots, int64_t nnz_pad, int64_t n_rowid) {
  const int layout = d.info & 3;
  bool ok = d.w_pad >= 0 && d.h_pad >= 1 && d.n_rows >= 1 && d.n_rows <= d.h_pad && d.data_off >= 0 &&
            d.rowid_off >= 0 && d.data_off + (int64_t)d.w_pad * d.h_pad <= nnz_pad &&
            d.rowid_off + d.h_pad <= n_rowid && layout <= kChunk && w.tile == tile;
  if (ok && layout == kChunk) ok = d.n_rows == 1 && d.h_pad == 1 && (d.info >> 2) < n_slots;
  if (ok) ok = (int64_t)w.row_begin >= row_lo && (int64_t)w.row_begin + (layout == kChunk ? 1 : w.n_rows) <= row_hi;
  return ok;
}

// Workload size of the automatic row panels (see tc_build_tiled).
constexpr int64_t kPanelWl = 512;

// Host threads for the builder's per-tile loops: started on first use and
// kept for the life of the process, so a build pays no thread start-up.  One
// loop runs on them at a time; a loop issued while another runs (builds on two
// host threads at once) runs on its calling thread alone.
class HostPool {
 public:
  static HostPool& get() {
    static HostPool* p = new HostPool();  // never destroyed: idle threads end with the process
    return *p;
  }
  // f(i) for i in [0, n) on the pool and the calling thread; false if the
  // pool is busy or empty (nothing was run)
  bool run(int64_t n, const std::function<void(int64_t)>& f) {
    std::unique_lock<std::mutex> busy(busy_, std::try_to_lock);
    if (!busy.owns_lock() || th_.empty()) return false;
    {
      std::lock_guard<std::mutex> g(m_);
      f_ = &f;
      n_ = n;
      next_.store(0);
      pending_ = (int)th_.size();
      ++gen_;
    }
    wake_.notify_all();
    work();
    std::unique_lock<std::mutex> g(m_);
    done_.wait(g, [&] { return pending_ == 0; });
    f_ = nullptr;
    return true;
  }

 private:
  // TC_HOST_THREADS=n in the environment: n threads in all (the caller's
  // included; 1 runs every loop on the calling thread); default up to 16
  HostPool() {
    int n = (int)std::min<unsigned>(16, std::max(1u, std::thread::hardware_concurrency()));
    if (const char* e = std::getenv("TC_HOST_THREADS")) n = std::max(1, std::min(256, std::atoi(e)));
    const int k = n - 1;
    for (int i = 0; i < k; ++i) th_.emplace_back([this] { loop(); });
  }
  void work() {
    for (int64_t i; (i = next_.fetch_add(1)) < n_;) (*f_)(i);
  }
  void loop() {
    uint64_t seen = 0;
    std::unique_lock<std::mutex> g(m_);
    for (;;) {
      wake_.wait(g, [&] { return gen_ != seen; });
      seen = gen_;
      g.unlock();
      work();
      g.lock();
      if (--pending_ == 0) done_.notify_one();
    }
  }
  std::mutex busy_, m_;
  std::condition_variable wake_, done_;
  const std::function<void(int64_t)>* f_ = nullptr;
  int64_t n_ = 0;
  std::atomic<int64_t> next_{0};
  int pending_ = 0;
  uint64_t gen_ = 0;
  std::vector<std::thread> th_;
};

// f(i) for i in [0, n) on the host pool when there are at least `min_par`
// items (each i touches only its own outputs), else on this thread.
template <class F>
void parallel_for(int64_t n, int64_t min_par, F&& f) {
  if (n >= min_par) {
    const std::function<void(int64_t)> fn = [&](int64_t i) { f(i); };
    if (HostPool::get().run(n, fn)) return;
  }
  for (int64_t i = 0; i < n; ++i) f(i);
}

// n items of T in a page-locked host block from the library's host pool, for
// the life of one build step.  The block goes back to the pool when its
// holder ends, after the build stream has finished every copy that may still
// read or write it.
template <class T>
struct Staged {
  HostBlock b;
  hipStream_t st;
  T* p;
  Staged(int64_t n, hipStream_t s)
      : b(host_take(sizeof(T) * (size_t)std::max<int64_t>(n, 1), true)), st(s), p((T*)b.p) {}
  ~Staged() {
    (void)hipStreamSynchronize(st);
    host_give(b);
  }
  Staged(const Staged&) = delete;
  Staged& operator=(const Staged&) = delete;
  T& operator[](int64_t i) { return p[i]; }
};

// what a build needs to know of a device
struct DeviceLimits {
  int32_t n_cu = 0;
  int64_t lds_cu_bytes = 0, lds_floats = 0, l2_bytes = 0;
};

// compute units, LDS and L2 of device dev, queried once per process (some
// attributes take milliseconds to read, and every build needs them)
DeviceLimits query_limits(int dev) {
  DeviceLimits L;
  int cus = 0;
  HIPX(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  L.n_cu = cus > 0 ? cus : 256;
  // LDS a workgroup may use (the opt-in limit) and LDS per compute unit
  int blk = 0, optin = 0, per_cu = 0, l2 = 0;
  if (hipDeviceGetAttribute(&blk, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) blk = 65536;
  if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess) optin = 0;
  if (hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess)
    per_cu = 0;
  if (hipDeviceGetAttribute(&l2, hipDeviceAttributeL2CacheSize, dev) != hipSuccess) l2 = 0;
  (void)hipGetLastError();
  const int64_t wg = std::max(blk, optin);
  L.lds_cu_bytes = per_cu > 0 ? per_cu : wg;
  L.lds_floats = std::min<int64_t>(std::min<int64_t>(wg, L.lds_cu_bytes) / 4, kLdsMaxFloats);
  L.l2_bytes = l2 > 0 ? l2 : ((int64_t)4 << 20);
  return L;
}

// compute units, LDS and L2 of the current device
void device_limits(tc_handle* h) {
  static std::mutex mu;
  static std::map<int, DeviceLimits> known;
  int dev = 0;
  HIPX(hipGetDevice(&dev));
  DeviceLimits L;
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = known.find(dev);
    if (it != known.end()) L = it->second;
  }
  if (L.n_cu == 0) {
    L = query_limits(dev);
    std::lock_guard<std::mutex> g(mu);
    known[dev] = L;
  }
  h->n_cu = L.n_cu;
  h->lds_cu_bytes = L.lds_cu_bytes;
  h->lds_floats = L.lds_floats;
  h->l2_bytes = L.l2_bytes;
}

// Row panels (MI355X reading of the row partition of Section 3.2, with the
// workgroups of one GPU in place of GPUs).  Given the (column tile, row)
// segments: each row's weight is its entries in segments that are not split
// into chunks; panel p ends at the first row where the running weight reaches
// ceil((p + 1) total / P), holding at least one and at most `rows` rows, and
// rows left after P panels go into further panels of `rows`.  Returns the
// panel bounds, and in *d_pb_out a device copy (int32).
std::vector<int64_t> make_panels(const int32_t* seg_tile, const int32_t* seg_row, const int32_t* seg_len,
                                 int64_t nseg, int64_t n_rows, const int64_t* d_split_col, int32_t P, int64_t rows,
                                 int32_t nct, Tmp& tmp, hipStream_t st, int32_t** d_pb_out) {
  std::vector<int64_t> pb{0};
  if (n_rows == 0) return pb;
  int32_t* w = tmp.get<int32_t>(n_rows);
  HIPX(hipMemsetAsync(w, 0, sizeof(int32_t) * n_rows, st));
  if (nseg > 0) {
    hipLaunchKernelGGL(k_panel_weight, dim3(nblk(nseg, kB)), dim3(kB), 0, st, seg_tile, seg_len, seg_row, nseg,
                       d_split_col, w);
    HIPX(hipGetLastError());
  }
  int64_t* pre = tmp.get<int64_t>(n_rows + 1);
  const int64_t total = excl_scan<int32_t, int64_t>(w, n_rows, pre, tmp, st);
  HIPX(hipMemcpyAsync(pre + n_rows, &total, sizeof(int64_t), hipMemcpyHostToDevice, st));
  std::vector<int64_t> tgt(P), lb(P);
  for (int32_t p = 0; p < P; ++p) tgt[p] = ((int64_t)(p + 1) * total + P - 1) / P;
  int64_t* d_tgt = tmp.get<int64_t>(P);
  int64_t* d_lb = tmp.get<int64_t>(P);
  HIPX(hipMemcpyAsync(d_tgt, tgt.data(), sizeof(int64_t) * P, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_lower_bound_pre, dim3(nblk(P, kB)), dim3(kB), 0, st, (const int64_t*)pre, n_rows,
                     (const int64_t*)d_tgt, P, d_lb);
  HIPX(hipGetLastError());
  HIPX(hipMemcpyAsync(lb.data(), d_lb, sizeof(int64_t) * P, hipMemcpyDeviceToHost, st));
  HIPX(hipStreamSynchronize(st));
  for (int32_t p = 0; p < P && pb.back() < n_rows; ++p)
    pb.push_back(std::min(std::min(std::max(lb[p], pb.back() + 1), pb.back() + rows), n_rows));
  while (pb.back() < n_rows) pb.push_back(std::min(pb.back() + rows, n_rows));
  const int32_t np = (int32_t)pb.size() - 1;
  if ((int64_t)np * nct >= ((int64_t)1 << 24)) throw Fail{TC_EUNSUPPORTED, "too many (panel, column tile) tiles"};
  std::vector<int32_t> pb32(pb.begin(), pb.end());
  int32_t* d_pb = tmp.get<int32_t>(np + 1);
  HIPX(hipMemcpyAsync(d_pb, pb32.data(), sizeof(int32_t) * (np + 1), hipMemcpyHostToDevice, st));
  HIPX(hipStreamSynchronize(st));  // pb32 goes out of scope
  *d_pb_out = d_pb;
  return pb;
}

void build(const tc_csr* A, const tc_build_opts* o, hipStream_t st, tc_handle* h) {
  PhaseClock clk(st);
  device_limits(h);
  if (h->W == 0) {
    // automatic panels: column tiles whose x segment fills at most half of
    // one XCD's L2 (the rest holds the matrix streams passing through), a
    // power of two of at least 2^16 columns.  All workgroups sweep the
    // column tiles in the same order, so the current tile's x is what every
    // L2 holds (Section 3.1, Solution 1, with the L2 in place of the texture
    // cache).
    int64_t w = (int64_t)1 << 16;
    while (w * 2 * (int64_t)sizeof(float) * 2 <= h->l2_bytes && w < ((int64_t)1 << 30)) w *= 2;
    h->W = (int32_t)w;
  }
  int64_t panel_head = 0;  // automatic panels: width of the LDS-staged head tile
  if (h->n_panels != 0) {
    const int64_t wg_floats = h->lds_floats;
    if (h->panel_rows > wg_floats)
      throw Fail{TC_EINVAL, "panel_rows exceeds the LDS of one workgroup (" + std::to_string(wg_floats) + " floats)"};
    if (h->n_panels < 0) {
      // automatic: one 16-wavefront workgroup per compute unit (fewer for
      // matrices of under 2048 rows per compute unit), each panel sized for
      // a sixteenth more rows than an even share (room for the weights to
      // move the bounds; more slack shrinks the head tile, less unbalances
      // the panels); the LDS left behind y holds the head tile (a multiple
      // of 1024 columns, at least 1024).  More panels than compute units
      // only when the rows do not fit.
      int64_t P = std::max<int64_t>(1, std::min<int64_t>(h->n_cu, (A->n_rows + 2047) / 2048));
      int64_t R = ((17 * ((A->n_rows + P - 1) / P) + 15) / 16 + 63) / 64 * 64;
      if (R > wg_floats - 1024) {
        R = (wg_floats - 1024) / 64 * 64;
        P = (17 * A->n_rows / 16 + R - 1) / R;
      }
      h->n_panels = (int32_t)std::max<int64_t>(1, P);
      if (h->panel_rows == 0) h->panel_rows = (int32_t)std::max<int64_t>(64, R);
      const int64_t head = (wg_floats - ((h->panel_rows + 3) & ~3)) / 1024 * 1024;
      panel_head = head >= 1024 && o->n_tile_bounds == 0 ? std::min<int64_t>(head, A->n_cols) : 0;
    }
    if (h->panel_rows == 0) h->panel_rows = (int32_t)std::min<int64_t>(wg_floats, h->lds_cu_bytes / 8);
  }
  const int64_t n_rows = A->n_rows, n_cols = A->n_cols, nnz = A->nnz;
  Tmp tmp(st);
  h->stream = st;

  // ---- validation
  {
    int* flag = tmp.get<int>(1);
    HIPX(hipMemsetAsync(flag, 0, sizeof(int), st));
    hipLaunchKernelGGL(k_validate_rows, dim3(nblk(n_rows + 1, kB)), dim3(kB), 0, st, A->row_ptr, n_rows, nnz, flag);
    HIPX(hipGetLastError());
    if (nnz > 0) hipLaunchKernelGGL(k_validate_cols, dim3(nblk(nnz, kB)), dim3(kB), 0, st, A->col_idx, nnz, n_cols, flag);
    HIPX(hipGetLastError());
    int f = 0;
    HIPX(hipMemcpyAsync(&f, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPX(hipStreamSynchronize(st));
    if (f & 1) throw Fail{TC_EINVAL, "invalid CSR: row_ptr must start at 0, not decrease and end at nnz"};
    if (f & 2) throw Fail{TC_EINVAL, "invalid CSR: a column id is outside [0, n_cols)"};
  }

  clk.mark("validation");
  // ---- a1: column lengths
  int32_t* clen = hold<int32_t>(h, n_cols);
  h->d_clen = clen;
  if (n_cols > 0) HIPX(hipMemsetAsync(clen, 0, sizeof(int32_t) * n_cols, st));
  const int cbits = bits_for((uint64_t)(n_cols > 1 ? n_cols - 1 : 0));
  const int cshift = std::max(15, cbits - 8);  // bucket = column >> cshift (at most 256 buckets)
  const int64_t windows = (int64_t)1 << (cshift - 15);
  if (nnz >= 4096 && windows <= 4) {
    col_count_bucketed(A->col_idx, nnz, n_cols, cshift, windows, clen, tmp, st);
  } else if (n_cols > 0) {
    col_count_atomic(A->col_idx, nnz, n_cols, clen, tmp, st);
  }
  const int32_t maxclen = dev_max(clen, n_cols, tmp, st);

  clk.mark("a1 column lengths");
  // ---- a2: stable sort of columns by decreasing length
  int32_t* cperm = hold<int32_t>(h, n_cols);
  int32_t* cpos = hold<int32_t>(h, n_cols);
  int32_t* clen_sorted = tmp.get<int32_t>(n_cols);
  h->d_cperm = cperm;
  h->d_cpos = cpos;
  if (n_cols > 0) {
    uint32_t* k0 = tmp.get<uint32_t>(n_cols);
    uint32_t* k1 = tmp.get<uint32_t>(n_cols);
    int32_t* v0 = tmp.get<int32_t>(n_cols);
    int32_t* v1 = tmp.get<int32_t>(n_cols);
    hipLaunchKernelGGL(k_desc_keys, dim3(nblk(n_cols, kB)), dim3(kB), 0, st, clen, n_cols, maxclen, k0, v0);
    HIPX(hipGetLastError());
    const int kb = bits_for((uint64_t)maxclen);
    for (int sh = 0; sh < kb; sh += 8) {
      cs_pass(RadixU32Op{k0, v0, k1, v1, sh}, n_cols, 8, tmp, st);
      std::swap(k0, k1);
      std::swap(v0, v1);
    }
    hipLaunchKernelGGL(k_cols_finish, dim3(nblk(n_cols, kB)), dim3(kB), 0, st, k0, v0, n_cols, maxclen, cperm, cpos,
                       clen_sorted);
    HIPX(hipGetLastError());
    unsigned long long* cnt = tmp.get<unsigned long long>(1);
    HIPX(hipMemsetAsync(cnt, 0, sizeof(*cnt), st));
    hipLaunchKernelGGL(k_count_eq, dim3(nblk(n_cols, kB)), dim3(kB), 0, st, clen_sorted, n_cols, 0, cnt);
    HIPX(hipGetLastError());
    unsigned long long nd = 0;
    HIPX(hipMemcpyAsync(&nd, cnt, sizeof(nd), hipMemcpyDeviceToHost, st));
    HIPX(hipStreamSynchronize(st));
    h->n_dangling = (int64_t)nd;
  }
  int32_t* rowmap = hold<int32_t>(h, n_rows);
  int32_t* rowinv = hold<int32_t>(h, n_rows);
  h->d_rowmap = rowmap;
  h->d_rowinv = rowinv;
  if (n_rows > 0) {
    hipLaunchKernelGGL(k_rowmap, dim3(nblk(n_rows, kB)), dim3(kB), 0, st, cpos, n_rows, h->relabel ? 1 : 0, rowmap,
                       rowinv);
    HIPX(hipGetLastError());
  }

  clk.mark("a2 column sort");
  // ---- a3: Algorithm 1 (or the XCD schedule's column ranges)
  const int32_t W = h->W;
  const int64_t NT = (n_cols + W - 1) / W;
  int32_t T = 0;
  int32_t ntiles = 0;
  std::vector<int32_t> starts;  // tiles 1..ntiles-1
  if (h->xcd_groups > 0 && n_cols > 0) {
    // head tile [0, min(W, n_cols)), then xcd_groups ranges of equal entries
    const int64_t head = std::min<int64_t>(W, n_cols);
    const int64_t m = n_cols - head;
    int64_t* pre = tmp.get<int64_t>(m + 1);
    const int64_t rest = excl_scan<int32_t, int64_t>(clen_sorted + head, m, pre, tmp, st);
    HIPX(hipMemcpyAsync(pre + m, &rest, sizeof(int64_t), hipMemcpyHostToDevice, st));
    const int G = h->xcd_groups;
    int64_t* need = tmp.get<int64_t>(G);
    int64_t* cut = tmp.get<int64_t>(G);
    std::vector<int64_t> hneed(G, 0), hcut(G, 0);
    for (int g = 1; g < G; ++g) hneed[g] = (g * rest + G - 1) / G;
    HIPX(hipMemcpyAsync(need, hneed.data(), sizeof(int64_t) * G, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_lower_bound, dim3(1), dim3(64), 0, st, (const int64_t*)pre, m + 1, (const int64_t*)need, G,
                       cut);
    HIPX(hipGetLastError());
    HIPX(hipMemcpyAsync(hcut.data(), cut, sizeof(int64_t) * G, hipMemcpyDeviceToHost, st));
    HIPX(hipStreamSynchronize(st));
    starts.push_back((int32_t)head);
    for (int g = 1; g < G; ++g) starts.push_back((int32_t)std::max<int64_t>(head + hcut[g], starts.back()));
    T = 1;
    ntiles = 1 + G;
  } else if (panel_head > 0) {
    // automatic row panels: the head tile [0, head) staged in LDS, then tiles
    // of W columns while the first column of the next one holds at least two
    // entries (Algorithm 1's rule), then the sparse tile
    T = 1;
    if (panel_head < n_cols) {
      starts.push_back((int32_t)panel_head);
      const int64_t NTr = (n_cols - panel_head + W - 1) / W;
      int32_t* samp = tmp.get<int32_t>(NTr);
      hipLaunchKernelGGL(k_strided, dim3(nblk(NTr, kB)), dim3(kB), 0, st, clen_sorted + panel_head, (int64_t)W, NTr,
                         samp);
      HIPX(hipGetLastError());
      std::vector<int32_t> hs(NTr);
      HIPX(hipMemcpyAsync(hs.data(), samp, sizeof(int32_t) * NTr, hipMemcpyDeviceToHost, st));
      HIPX(hipStreamSynchronize(st));
      int64_t k = 0;
      while (k < NTr && hs[k] >= 2) {
        ++k;
        if (panel_head + k * W < n_cols) starts.push_back((int32_t)(panel_head + k * W));
      }
      T = (int32_t)(1 + k);
    }
    ntiles = (int32_t)starts.size() + 1;
  } else if (o->n_tile_bounds > 0) {

    // given tile boundaries: dense tiles up to the last bound, then the
    // sparse tile if columns remain
    for (int i = 0; i < o->n_tile_bounds; ++i)
      if (o->tile_bounds[i] < n_cols) starts.push_back(o->tile_bounds[i]);
    T = o->n_tile_bounds;
    ntiles = (int32_t)starts.size() + 1;
  } else {
    if (o->n_tiles >= 0) {
      T = (int32_t)std::min<int64_t>(o->n_tiles, NT);
    } else if (NT > 0) {
      int32_t* samp = tmp.get<int32_t>(NT);
      hipLaunchKernelGGL(k_strided, dim3(nblk(NT, kB)), dim3(kB), 0, st, clen_sorted, (int64_t)W, NT, samp);
      HIPX(hipGetLastError());
      std::vector<int32_t> hs(NT);
      HIPX(hipMemcpyAsync(hs.data(), samp, sizeof(int32_t) * NT, hipMemcpyDeviceToHost, st));
      HIPX(hipStreamSynchronize(st));
      while (T < NT && hs[T] >= 2) ++T;
    }
    ntiles = (int32_t)(T + ((int64_t)T * W < n_cols ? 1 : 0));
    for (int t = 1; t < ntiles; ++t) starts.push_back((int32_t)std::min<int64_t>((int64_t)t * W, n_cols));
  }
  h->T = T;
  h->n_tiles = ntiles;
  h->tile_col_begin.resize(ntiles);
  h->tile_col_end.resize(ntiles);
  for (int t = 0; t < ntiles; ++t) {
    h->tile_col_begin[t] = t == 0 ? 0 : starts[t - 1];
    h->tile_col_end[t] = t + 1 < ntiles ? starts[t] : n_cols;
  }
  TileMap tmap{W, T, nullptr, 0};
  if ((h->xcd_groups > 0 || o->n_tile_bounds > 0 || panel_head > 0) && ntiles > 1) {
    int32_t* d_starts = tmp.get<int32_t>(ntiles - 1);
    HIPX(hipMemcpyAsync(d_starts, starts.data(), sizeof(int32_t) * (ntiles - 1), hipMemcpyHostToDevice, st));
    tmap = TileMap{W, T, d_starts, ntiles - 1};
    bool uni = W > 0;
    for (int i = 0; i < ntiles - 1 && uni; ++i) uni = (int64_t)starts[i] == (int64_t)starts[0] + (int64_t)i * W;
    if (uni) {
      tmap.uniform = 1;
      tmap.s0 = starts[0];
      if ((W & (W - 1)) == 0) tmap.wshift = bits_for((uint64_t)W) - 1;
    }
  }

  clk.mark("a3 tiles");
  // ---- a4: bucket entries by tile (stable)
  // One tile: the entries stay in CSR order, so the caller's values are read
  // in place and no per-entry row ids are needed (a5 works per row).
  const bool one_tile = ntiles <= 1;
  int32_t *b_icol = nullptr, *b_row = nullptr;
  const float* b_val = nullptr;
  std::vector<int64_t> tstart(ntiles + 1, 0);
  int64_t* d_ts = nullptr;  // tstart on the device
  // value map: entry indices stand in for the values through a4-a7
  const float* vsrc = A->val;
  if (o->value_map && nnz > 0) {
    int32_t* iota = tmp.get<int32_t>(nnz);
    hipLaunchKernelGGL(k_iota_i32, dim3(nblk(nnz, kB)), dim3(kB), 0, st, iota, nnz);
    HIPX(hipGetLastError());
    vsrc = (const float*)iota;
  }
  // With relabelled rows and several tiles (not TILE-COO, whose arrays keep
  // CSR order within a tile), the entries enter the tile passes in internal-
  // row order, so each tile's segments come out in increasing internal row
  // and the segment sort in a5 needs no passes over the row bits.
  const bool perm_rows = !one_tile && h->relabel && h->kernel != 1;
  const bool rows_in_order = one_tile || perm_rows || !h->relabel;
  if (nnz > 0) {
    int32_t* icol = tmp.get<int32_t>(nnz);
    int32_t* row_of = nullptr;
    float* pval = nullptr;
    int32_t* hist0 = nullptr;  // histogram of the first tile pass, when made by the permutation
    if (perm_rows) {
      int32_t* ilen = tmp.get<int32_t>(n_rows);
      int64_t* iptr = tmp.get<int64_t>(n_rows + 1);
      int64_t* istart = tmp.get<int64_t>(n_rows);
      hipLaunchKernelGGL(k_irow_len, dim3(nblk(n_rows, kB)), dim3(kB), 0, st, A->row_ptr, (const int32_t*)rowinv,
                         n_rows, ilen, istart);
      HIPX(hipGetLastError());
      const int64_t nsb = std::max<int64_t>(1, (n_rows + kScanTile - 1) / kScanTile);
      int64_t* bs = tmp.get<int64_t>(nsb + 1);
      excl_scan_async<int32_t, int64_t>(ilen, n_rows, iptr, bs, nsb, st);
      HIPX(hipMemcpyAsync(iptr + n_rows, bs + nsb, sizeof(int64_t), hipMemcpyDeviceToDevice, st));
      int32_t* irow = tmp.get<int32_t>(nnz);
      hipLaunchKernelGGL(k_expand_rows, dim3(nblk(n_rows, kB)), dim3(kB), 0, st, (const int64_t*)iptr, n_rows, irow);
      HIPX(hipGetLastError());
      row_of = tmp.get<int32_t>(nnz);
      pval = tmp.get<float>(nnz);
      // the first tile pass's histogram comes with the permutation when its
      // chunks are the permutation's blocks
      const int tb0 = std::min(8, bits_for((uint64_t)(ntiles - 1)));
      const CsPlan pl = cs_plan<TileItem>(nnz, tb0);
      const int64_t pblocks = (nnz + kPermBlock - 1) / kPermBlock;
      if (pl.chunk == kPermBlock) hist0 = tmp.get<int32_t>((int64_t)pl.nbuckets * pl.nchunks);
      hipLaunchKernelGGL((k_perm_entries<TileMap>), dim3((unsigned)pblocks), dim3(kPermBlock),
                         hist0 ? sizeof(int32_t) * (size_t)pl.nbuckets : 0, st, (const int32_t*)irow,
                         (const int64_t*)iptr, (const int64_t*)istart, A->col_idx, cpos, vsrc, nnz, icol, pval,
                         row_of, tmap, pl.nbuckets, pl.nchunks, hist0);
      HIPX(hipGetLastError());
      tmp.release(istart);
      tmp.release(irow);
      tmp.release(iptr);
      tmp.release(ilen);
      tmp.release(bs);
    } else {
      hipLaunchKernelGGL(k_icol, dim3(nblk(nnz, kB)), dim3(kB), 0, st, A->col_idx, cpos, nnz, icol);
      HIPX(hipGetLastError());
    }
    const int tb = bits_for((uint64_t)(ntiles > 1 ? ntiles - 1 : 0));
    if (one_tile) {
      b_icol = icol;
      b_val = vsrc;
    } else {
      if (!row_of) {
        row_of = tmp.get<int32_t>(nnz);
        hipLaunchKernelGGL(k_expand_rows, dim3(nblk(n_rows, kB)), dim3(kB), 0, st, A->row_ptr, n_rows, row_of);
        HIPX(hipGetLastError());
      }
      // LSD passes over 8-bit digits of the tile id; buffers alternate between
      // two sets (the caller's values are only read)
      int32_t* bi[2] = {tmp.get<int32_t>(nnz), icol};
      int32_t* br[2] = {tmp.get<int32_t>(nnz), row_of};
      float* bv[2] = {tmp.get<float>(nnz), pval};
      const int32_t* ci = icol;
      const int32_t* cr = row_of;
      const float* cv = pval ? pval : vsrc;
      int p = 0;
      for (int sh = 0; sh < tb; sh += 8, ++p) {
        const int s = p & 1;
        if (!bv[s]) bv[s] = tmp.get<float>(nnz);
        const int nb = std::min(8, tb - sh);
        cs_pass(TileOp{ci, cv, cr, bi[s], bv[s], br[s], tmap, sh}, nnz, nb, tmp, st, sh == 0 ? hist0 : nullptr);
        ci = bi[s];
        cr = br[s];
        cv = bv[s];
      }
      b_icol = (int32_t*)ci;
      b_row = (int32_t*)cr;
      b_val = cv;
    }
    clk.mark("a4 bucket passes");
    d_ts = tmp.get<int64_t>(ntiles + 1);
    hipLaunchKernelGGL(k_tile_bounds, dim3(nblk(ntiles + 1, kB)), dim3(kB), 0, st, b_icol, nnz, tmap, ntiles, d_ts);
    HIPX(hipGetLastError());
    HIPX(hipMemcpyAsync(tstart.data(), d_ts, sizeof(int64_t) * (ntiles + 1), hipMemcpyDeviceToHost, st));
    HIPX(hipStreamSynchronize(st));
  }
  h->tile_nnz.resize(ntiles);
  for (int t = 0; t < ntiles; ++t) h->tile_nnz[t] = tstart[t + 1] - tstart[t];
  h->tile_split.assign(ntiles, 0);
  for (int t = 0; t < ntiles; ++t) h->tile_split[t] = tile_split_len(h->split_len, h->tile_nnz[t], h->max_act_warp, h->S);
  int64_t* d_split_t = tmp.get<int64_t>(std::max(ntiles, 1));
  if (ntiles > 0)
    HIPX(hipMemcpyAsync(d_split_t, h->tile_split.data(), sizeof(int64_t) * ntiles, hipMemcpyHostToDevice, st));
  int32_t* first = tmp.get<int32_t>(n_rows);
  int32_t* touched = tmp.get<int32_t>(n_rows);
  if (n_rows > 0) {
    hipLaunchKernelGGL(k_fill_i32, dim3(nblk(n_rows, kB)), dim3(kB), 0, st, first, n_rows, (int32_t)0x7fffffff);
    hipLaunchKernelGGL(k_fill_i32, dim3(nblk(n_rows, kB)), dim3(kB), 0, st, touched, n_rows, (int32_t)0);
    HIPX(hipGetLastError());
  }

  clk.mark("a4 tile buckets");
  // ---- a5: segments (tile, row) and their sort by decreasing length
  int64_t nseg = 0;
  int32_t *rows_sorted = nullptr, *rows_len = nullptr, *srt_start = nullptr;
  std::vector<int64_t> trow(ntiles + 1, 0);
  // (length, rows) of every (tile, length) run, tile-major, and each tile's
  // first run (runs never span tiles: the tile is in the key's top bits)
  std::unique_ptr<Staged<LenRun>> run_list;
  std::vector<int64_t> tile_run;
  int64_t nruns = 0;
  if (nnz > 0) {
    int32_t *seg_start, *seg_row, *seg_tile, *seg_len;
    if (one_tile) {
      // one segment per non-empty row, emitted in increasing internal row
      int32_t* flags = tmp.get<int32_t>(n_rows);
      int32_t* pos = tmp.get<int32_t>(n_rows);
      hipLaunchKernelGGL(k_rowseg_flags, dim3(nblk(n_rows, kB)), dim3(kB), 0, st, A->row_ptr, rowinv, n_rows, flags);
      HIPX(hipGetLastError());
      nseg = excl_scan<int32_t, int32_t>(flags, n_rows, pos, tmp, st);
      seg_start = tmp.get<int32_t>(nseg);
      seg_row = tmp.get<int32_t>(nseg);
      seg_tile = tmp.get<int32_t>(nseg);
      seg_len = tmp.get<int32_t>(nseg);
      hipLaunchKernelGGL(k_rowseg_emit, dim3(nblk(n_rows, kB)), dim3(kB), 0, st, flags, pos, A->row_ptr, rowinv,
                         n_rows, seg_start, seg_row, seg_tile, seg_len);
      HIPX(hipGetLastError());
      tmp.release(flags);
      tmp.release(pos);
    } else {
      // heads counted per scan block, their block offsets scanned, then the
      // segments written at their positions (no per-entry flag array)
      const int64_t nb = (nnz + kScanTile - 1) / kScanTile;
      int64_t* bs = tmp.get<int64_t>(nb + 1);
      hipLaunchKernelGGL(k_seghead_count, dim3((unsigned)nb), dim3(kScanBlock), 0, st, b_row, nnz,
                         (const int64_t*)d_ts, ntiles, bs);
      HIPX(hipGetLastError());
      hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kScanBlock), 0, st, bs, nb, bs + nb);
      HIPX(hipGetLastError());
      HIPX(hipMemcpyAsync(&nseg, bs + nb, sizeof(int64_t), hipMemcpyDeviceToHost, st));
      HIPX(hipStreamSynchronize(st));
      seg_start = tmp.get<int32_t>(nseg);
      seg_row = tmp.get<int32_t>(nseg);
      seg_tile = tmp.get<int32_t>(nseg);
      seg_len = tmp.get<int32_t>(nseg);
      hipLaunchKernelGGL(k_seghead_emit, dim3((unsigned)nb), dim3(kScanBlock), 0, st, b_row, b_icol,
                         perm_rows ? (const int32_t*)nullptr : (const int32_t*)rowmap, nnz,
                         (const int64_t*)d_ts, ntiles, tmap, (const int64_t*)bs, seg_start, seg_row, seg_tile);
      HIPX(hipGetLastError());
      hipLaunchKernelGGL(k_seg_len, dim3(nblk(nseg, kB)), dim3(kB), 0, st, seg_start, nseg, nnz, seg_len);
      HIPX(hipGetLastError());
      tmp.release(bs);
    }
    clk.mark("a5 segment emission");
    if (h->n_panels > 0) {
      // row panels: every (panel, column tile) pair becomes a tile, panel-major
      const int32_t nct = ntiles;
      int32_t* d_pb = nullptr;
      h->panel_begin = make_panels(seg_tile, seg_row, seg_len, nseg, n_rows, d_split_t, h->n_panels,
                                   h->panel_rows, nct, tmp, st, &d_pb);
      h->n_panels = (int32_t)h->panel_begin.size() - 1;
      // segment tiles become (panel, column tile) tiles; first touches with them
      const int lds_pb = h->n_panels + 1 <= 8192 ? 1 : 0;
      hipLaunchKernelGGL(k_seg_panel_touch, dim3(nblk(nseg, kB)), dim3(kB),
                         lds_pb ? sizeof(int32_t) * (size_t)(h->n_panels + 1) : 0, st, seg_tile, seg_row, seg_len,
                         nseg, (const int32_t*)d_pb, h->n_panels, nct, lds_pb, (const int64_t*)d_split_t, first,
                         touched);
      HIPX(hipGetLastError());
      h->n_col_tiles = nct;
      ntiles = h->n_panels * nct;
      h->n_tiles = ntiles;
      std::vector<int64_t> cb = h->tile_col_begin, ce = h->tile_col_end, csp = h->tile_split;
      h->tile_col_begin.resize(ntiles);
      h->tile_col_end.resize(ntiles);
      h->tile_split.resize(ntiles);
      for (int g = 0; g < ntiles; ++g) {
        h->tile_col_begin[g] = cb[g % nct];
        h->tile_col_end[g] = ce[g % nct];
        h->tile_split[g] = csp[g % nct];
      }
      h->tile_nnz.assign(ntiles, 0);  // from the sorted segments below
      d_split_t = tmp.get<int64_t>(ntiles);
      HIPX(hipMemcpyAsync(d_split_t, h->tile_split.data(), sizeof(int64_t) * ntiles, hipMemcpyHostToDevice, st));
      HIPX(hipStreamSynchronize(st));
      trow.assign(ntiles + 1, 0);
    }
    clk.mark("a5 segments formed");
    if (h->n_panels == 0) {
      hipLaunchKernelGGL(k_first_touch, dim3(nblk(nseg, kB)), dim3(kB), 0, st, seg_tile, seg_len, seg_row, nseg,
                         (const int64_t*)d_split_t, first, touched);
      HIPX(hipGetLastError());
    }
    const int32_t maxlen = dev_max(seg_len, nseg, tmp, st);
    const int lb = bits_for((uint64_t)maxlen);
    const int rb = bits_for((uint64_t)(n_rows > 1 ? n_rows - 1 : 0));
    const int tb = bits_for((uint64_t)(ntiles > 1 ? ntiles - 1 : 0));
    if (lb + rb + tb > 64) throw Fail{TC_EUNSUPPORTED, "sort key of (tile, length, row) exceeds 64 bits"};
    uint64_t* k0 = tmp.get<uint64_t>(nseg);
    uint64_t* k1 = tmp.get<uint64_t>(nseg);
    int32_t* v0 = tmp.get<int32_t>(nseg);
    int32_t* v1 = tmp.get<int32_t>(nseg);
    hipLaunchKernelGGL(k_seg_keys, dim3(nblk(nseg, kB)), dim3(kB), 0, st, seg_tile, seg_len, seg_row, seg_start, nseg,
                       maxlen, lb, rb, k0, v0);
    HIPX(hipGetLastError());
    // segments already in increasing internal row within each tile (the
    // key's low rb bits): the stable passes over the length and tile bits
    // finish the order
    for (int sh = rows_in_order ? rb : 0; sh < lb + rb + tb; sh += 8) {
      cs_pass(RadixU64Op{k0, v0, k1, v1, sh}, nseg, 8, tmp, st);
      std::swap(k0, k1);
      std::swap(v0, v1);
    }
    clk.mark("a5 segments sorted");
    rows_sorted = hold<int32_t>(h, nseg);
    rows_len = hold<int32_t>(h, nseg);
    srt_start = tmp.get<int32_t>(nseg);
    hipLaunchKernelGGL(k_seg_decode, dim3(nblk(nseg, kB)), dim3(kB), 0, st, (const uint64_t*)k0, (const int32_t*)v0,
                       nseg, maxlen, lb, rb, rows_sorted, rows_len, srt_start);
    HIPX(hipGetLastError());
    int64_t* d_off = tmp.get<int64_t>(ntiles + 1);
    hipLaunchKernelGGL(k_key_bounds, dim3(nblk(ntiles + 1, kB)), dim3(kB), 0, st, k0, nseg, lb + rb, ntiles, d_off);
    HIPX(hipGetLastError());
    HIPX(hipMemcpyAsync(trow.data(), d_off, sizeof(int64_t) * (ntiles + 1), hipMemcpyDeviceToHost, st));
    if (h->n_panels > 0) {
      // entries of every (panel, column tile) tile: sums of its sorted rows' lengths
      int64_t* pre = tmp.get<int64_t>(nseg + 1);
      const int64_t tot = excl_scan<int32_t, int64_t>(rows_len, nseg, pre, tmp, st);
      HIPX(hipMemcpyAsync(pre + nseg, &tot, sizeof(int64_t), hipMemcpyHostToDevice, st));
      int64_t* d_tn = tmp.get<int64_t>(ntiles);
      hipLaunchKernelGGL(k_tile_entries, dim3(nblk(ntiles, kB)), dim3(kB), 0, st, (const int64_t*)pre,
                         (const int64_t*)d_off, ntiles, d_tn);
      HIPX(hipGetLastError());
      HIPX(hipMemcpyAsync(h->tile_nnz.data(), d_tn, sizeof(int64_t) * ntiles, hipMemcpyDeviceToHost, st));
    }
    // length runs
    int32_t* rflags = tmp.get<int32_t>(nseg);
    int32_t* rpos = tmp.get<int32_t>(nseg);
    hipLaunchKernelGGL(k_run_flags, dim3(nblk(nseg, kB)), dim3(kB), 0, st, k0, nseg, rb, rflags);
    HIPX(hipGetLastError());
    nruns = excl_scan<int32_t, int32_t>(rflags, nseg, rpos, tmp, st);
    int64_t* d_rp = tmp.get<int64_t>(nruns);
    int32_t* d_rl = tmp.get<int32_t>(nruns);
    hipLaunchKernelGGL(k_run_emit, dim3(nblk(nseg, kB)), dim3(kB), 0, st, rflags, rpos, rows_len, nseg, d_rp, d_rl);
    HIPX(hipGetLastError());
    LenRun* d_runs = tmp.get<LenRun>(nruns);
    hipLaunchKernelGGL(k_run_pairs, dim3(nblk(nruns, kB)), dim3(kB), 0, st, (const int64_t*)d_rp,
                       (const int32_t*)d_rl, nruns, nseg, d_runs);
    HIPX(hipGetLastError());
    int64_t* d_trun = tmp.get<int64_t>(ntiles + 1);
    hipLaunchKernelGGL(k_lower_bound_pre, dim3(nblk(ntiles + 1, kB)), dim3(kB), 0, st, (const int64_t*)d_rp, nruns,
                       (const int64_t*)d_off, (int)(ntiles + 1), d_trun);
    HIPX(hipGetLastError());
    run_list.reset(new Staged<LenRun>(nruns, st));
    tile_run.assign(ntiles + 1, 0);
    HIPX(hipMemcpyAsync(run_list->p, d_runs, sizeof(LenRun) * nruns, hipMemcpyDeviceToHost, st));
    HIPX(hipMemcpyAsync(tile_run.data(), d_trun, sizeof(int64_t) * (ntiles + 1), hipMemcpyDeviceToHost, st));
    HIPX(hipStreamSynchronize(st));
  }
  if (nnz == 0 && h->n_panels > 0) {
    h->n_panels = 0;
    h->n_col_tiles = 0;
  }
  h->d_rows_sorted = rows_sorted;
  h->d_rows_len = rows_len;
  h->n_rows_sorted = nseg;
  h->tile_row_off = trow;

  clk.mark("a5 segments");
  // ---- a6: workload sizes (Algorithm 2) and partition
  PerfTable table;
  if (o->perf_table) {
    std::string err;
    if (!load_perf_table(o->perf_table, &table, &err)) throw Fail{TC_EINVAL, err};
  } else {
    default_perf_table(&table);
  }
  PartitionParams pp{h->S, h->split_len, h->n_panels > 0 ? (int64_t)h->panel_waves : h->max_act_warp,
                     h->camping_pad};
  h->tile_wl.assign(ntiles, 0);
  h->tile_wl_begin.assign(ntiles + 1, 0);
  HostArray<HostWl>& wls = h->wls;
  wls.release();
  // Runs of each tile, then Algorithm 2 and the partition tile by tile; the
  // tiles are independent, so with many tiles (row panels) they are spread
  // over host threads, each writing its own tiles' workload lists.
  // (every run lies in one tile: the tile is in the key's top bits)
  std::vector<RunSpan> truns(ntiles);
  if (nruns > 0)
    for (int t = 0; t < ntiles; ++t)
      truns[t] = RunSpan{run_list->p + tile_run[t], (size_t)(tile_run[t + 1] - tile_run[t])};
  clk.mark("a6 runs");
  if (o->wl_policy == 1 && o->n_wl_per_tile < ntiles)
    throw Fail{TC_EINVAL, "wl_per_tile has fewer entries than tiles built"};
  std::vector<int64_t> tcount(ntiles, 0);  // workloads of each tile
  std::vector<int64_t> tchunk(ntiles, 0);  // of them, the leading chunk workloads (split rows come first)
  std::vector<int> tstray(ntiles, 0);
  std::vector<double> tmodel(ntiles, 0.0);
  std::vector<int> tbad(ntiles, 0);
  // per tile: padded elements and stored row ids of its workloads
  std::vector<int64_t> tdoff(ntiles + 1, 0), troff(ntiles + 1, 0);
  auto tile_job = [&](int64_t t) {
    const RunSpan& runs = truns[t];
    PartitionParams pt = pp;
    pt.split_len = (int32_t)h->tile_split[t];
    const bool sparse_t = (h->n_panels > 0 ? t % h->n_col_tiles : t) >= T;
    int64_t WLt;
    if (o->wl_policy == 1)
      WLt = o->wl_per_tile[t];
    else if (o->wl_policy == 2)
      WLt = o->wl_all;
    else if (o->panels < 0)
      WLt = kPanelWl;
    else
      WLt = choose_wl(runs, h->tile_nnz[t], table, sparse_t, pt);
    if (WLt < 1) {
      tbad[t] = 1;
      return;
    }
    h->tile_wl[t] = WLt;
    // the model's walk counts the workloads, so each tile's list is written
    // straight into its place below
    int64_t cnt = 0;
    if (!runs.empty()) tmodel[t] = model_time(runs, WLt, table, sparse_t, pt, &cnt);
    tcount[t] = cnt;
  };
  parallel_for(ntiles, 64, tile_job);
  clk.mark("a6 tile partitions");
  // workload offsets of every tile, then each tile's workloads written in
  // place in parallel with their padded elements and stored row ids
  for (int t = 0; t < ntiles; ++t) {
    if (tbad[t]) throw Fail{TC_EINVAL, "workload size must be >= 1"};
    h->model_us += tmodel[t];
    h->tile_wl_begin[t + 1] = h->tile_wl_begin[t] + tcount[t];
  }
  wls.reset(h->tile_wl_begin[ntiles]);
  parallel_for(ntiles, 64, [&](int64_t t) {
    if (tcount[t] == 0) return;
    PartitionParams pt = pp;
    pt.split_len = (int32_t)h->tile_split[t];
    HostWl* out = wls.data() + h->tile_wl_begin[t];
    partition_tile(truns[t], h->tile_wl[t], (int32_t)t, trow[t], pt, out);
    int64_t a = 0, r = 0, c = 0;
    while (c < tcount[t] && out[c].chunk >= 0) ++c;
    tchunk[t] = c;
    for (int64_t q = 0; q < tcount[t]; ++q) {
      const int64_t area = (int64_t)out[q].w_pad * out[q].h_pad;
      a += area + ((h->camping_pad && area % 512 == 0) ? 64 : 0);
      r += out[q].h_pad;
      if (q >= c && out[q].chunk >= 0) tstray[t] = 1;
    }
    tdoff[t + 1] = a;
    troff[t + 1] = r;
  });
  for (int t = 0; t < ntiles; ++t)
    if (tstray[t]) throw Fail{TC_EINVAL, "internal error: a chunk workload after a tile's first rows"};
  for (int t = 0; t < ntiles; ++t) {
    tdoff[t + 1] += tdoff[t];
    troff[t + 1] += troff[t];
  }
  clk.mark("a6 sizes and partition");
  h->d_tile_wl_begin = hold<int64_t>(h, ntiles + 1);
  HIPX(hipMemcpyAsync(h->d_tile_wl_begin, h->tile_wl_begin.data(), sizeof(int64_t) * (ntiles + 1),
                      hipMemcpyHostToDevice, st));
  const int64_t nwl = (int64_t)wls.size();
  h->n_wl = nwl;
  if (h->n_panels > 0) {
    // panel pass metadata: each tile's leading chunk workloads run on any
    // workgroup (their sums go to partial slots), listed per column tile
    const int32_t nct = h->n_col_tiles;
    std::vector<int64_t> ncb(ntiles), cbv(nct + 1, 0), chunks;
    for (int g = 0; g < ntiles; ++g) ncb[g] = h->tile_wl_begin[g] + tchunk[g];
    for (int t = 0; t < nct; ++t) {
      cbv[t] = (int64_t)chunks.size();
      for (int p = 0; p < h->n_panels; ++p)
        for (int64_t j = h->tile_wl_begin[p * nct + t]; j < ncb[p * nct + t]; ++j) chunks.push_back(j);
    }
    cbv[nct] = (int64_t)chunks.size();
    std::vector<int32_t> pb32(h->panel_begin.begin(), h->panel_begin.end());
    h->d_panel_ncb = hold<int64_t>(h, std::max<int64_t>(ntiles, 1));
    h->d_panel_cb = hold<int64_t>(h, nct + 1);
    h->d_panel_chunks = hold<int64_t>(h, std::max<int64_t>((int64_t)chunks.size(), 1));
    h->d_panel_begin = hold<int32_t>(h, h->n_panels + 1);
    HIPX(hipMemcpyAsync(h->d_panel_ncb, ncb.data(), sizeof(int64_t) * ntiles, hipMemcpyHostToDevice, st));
    HIPX(hipMemcpyAsync(h->d_panel_cb, cbv.data(), sizeof(int64_t) * (nct + 1), hipMemcpyHostToDevice, st));
    if (!chunks.empty())
      HIPX(hipMemcpyAsync(h->d_panel_chunks, chunks.data(), sizeof(int64_t) * chunks.size(), hipMemcpyHostToDevice,
                          st));
    HIPX(hipMemcpyAsync(h->d_panel_begin, pb32.data(), sizeof(int32_t) * pb32.size(), hipMemcpyHostToDevice, st));
    HIPX(hipStreamSynchronize(st));  // host vectors above go out of scope
  }

  clk.mark("a6 panel lists");
  // split rows: slots grouped by row, in (tile, chunk) order
  std::vector<int64_t> chunk_wl;
  for (int t = 0; t < ntiles; ++t)
    for (int64_t j = h->tile_wl_begin[t]; j < h->tile_wl_begin[t] + tchunk[t]; ++j) chunk_wl.push_back(j);
  std::vector<int32_t> chunk_row(chunk_wl.size()), chunk_first(chunk_wl.size());
  if (!chunk_wl.empty()) {
    // row ids of split rows (they sit at the start of their tile's sorted
    // rows) and the first tile that writes each
    const int64_t nc = (int64_t)chunk_wl.size();
    std::vector<int32_t> at(nc);
    for (int64_t q = 0; q < nc; ++q) at[q] = wls[chunk_wl[q]].row_begin;
    int32_t* d_at = tmp.get<int32_t>(nc);
    int32_t* d_r = tmp.get<int32_t>(nc);
    int32_t* d_f = tmp.get<int32_t>(nc);
    HIPX(hipMemcpyAsync(d_at, at.data(), sizeof(int32_t) * nc, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_chunk_rows, dim3(nblk(nc, kB)), dim3(kB), 0, st, (const int32_t*)rows_sorted,
                       (const int32_t*)first, (const int32_t*)d_at, nc, d_r, d_f);
    HIPX(hipGetLastError());
    HIPX(hipMemcpyAsync(chunk_row.data(), d_r, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, st));
    HIPX(hipMemcpyAsync(chunk_first.data(), d_f, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, st));
    HIPX(hipStreamSynchronize(st));
  }
  // chunks in increasing row, (tile, chunk) order kept within a row: a stable
  // LSD counting sort over 11-bit digits of the row (rows are int32 >= 0)
  std::vector<size_t> ord(chunk_wl.size()), ord2(chunk_wl.size());
  std::iota(ord.begin(), ord.end(), 0);
  {
    const int rbits = bits_for((uint64_t)std::max<int64_t>(n_rows - 1, 0));
    std::vector<size_t> cnt(2049);
    for (int sh = 0; sh < rbits; sh += 11) {
      std::fill(cnt.begin(), cnt.end(), 0);
      for (size_t q : ord) ++cnt[(((uint32_t)chunk_row[q] >> sh) & 2047u) + 1];
      for (size_t b = 1; b < cnt.size(); ++b) cnt[b] += cnt[b - 1];
      for (size_t q : ord) ord2[cnt[((uint32_t)chunk_row[q] >> sh) & 2047u]++] = q;
      ord.swap(ord2);
    }
  }
  std::vector<int32_t> slot_of(chunk_wl.size());
  std::vector<SplitRow> srows;
  for (size_t q = 0; q < ord.size(); ++q) {
    slot_of[ord[q]] = (int32_t)q;
    if (q == 0 || chunk_row[ord[q]] != chunk_row[ord[q - 1]])
      srows.push_back(SplitRow{chunk_row[ord[q]], (int32_t)q, 0, chunk_first[ord[q]] == 0x7fffffff ? 1 : 0});
    srows.back().n_slots++;
  }
  h->n_slots = (int64_t)chunk_wl.size();
  h->n_split_rows = (int64_t)srows.size();

  clk.mark("a6 split rows");
  // descriptors, per tile in parallel from the tile prefix sums, each
  // checked as it is made (a tile's leading chunk workloads take the partial
  // slots slot_of[cbase[t] ...])
  const int64_t doff = tdoff[ntiles], roff = troff[ntiles];
  if (doff >= ((int64_t)1 << 40)) throw Fail{TC_EUNSUPPORTED, "padded format too large"};
  h->nnz_pad = doff;
  h->n_rowid = roff;
  std::vector<int64_t> cbase(ntiles + 1, 0);
  for (int t = 0; t < ntiles; ++t) cbase[t + 1] = cbase[t] + tchunk[t];
  Staged<Wl> dwl(nwl, st);
  Staged<PackX> pxs(nwl, st);
  // ---- a7: pack, pipelined with the descriptors: the tiles go in a few
  // batches, and each batch's descriptors are copied and packed on the stream
  // while the host makes the next batch's
  h->d_idx = hold<int32_t>(h, doff);
  h->d_val = hold<float>(h, doff);
  h->d_rowid = hold<int32_t>(h, roff);
  h->d_wl = hold<Wl>(h, nwl);
  PackX* d_px = tmp.get<PackX>(nwl);
  Staged<int32_t> tfirst(ntiles, st);
  for (int t = 0; t < ntiles; ++t) tfirst[t] = (int32_t)h->tile_col_begin[t];
  int32_t* d_tfirst = tmp.get<int32_t>(ntiles);
  if (ntiles > 0) HIPX(hipMemcpyAsync(d_tfirst, tfirst.p, sizeof(int32_t) * ntiles, hipMemcpyHostToDevice, st));
  const int nbatch = ntiles >= 1024 ? 4 : 1;
  for (int bi = 0; bi < nbatch; ++bi) {
    const int64_t t0 = (int64_t)ntiles * bi / nbatch, t1 = (int64_t)ntiles * (bi + 1) / nbatch;
    std::atomic<int64_t> bad{INT64_MAX};
    parallel_for(t1 - t0, 16, [&](int64_t q) {
      const int64_t t = t0 + q;
      int64_t d = tdoff[t], r = troff[t];
      const int64_t jb = h->tile_wl_begin[t];
      const int64_t rb = h->tile_row_off[t], re = h->tile_row_off[t + 1];
      for (int64_t j = jb; j < h->tile_wl_begin[t + 1]; ++j) {
        HostWl& w = wls[j];
        const int64_t area = (int64_t)w.w_pad * w.h_pad;
        const int32_t extra = (h->camping_pad && area % 512 == 0) ? 64 : 0;
        w.data_off = d;
        w.rowid_off = r;
        const bool chunk = j - jb < tchunk[t];
        const Wl dd{d, r, w.w_pad, w.h_pad, w.n_rows,
                    chunk ? (int32_t)(kChunk | (slot_of[cbase[t] + (j - jb)] << 2)) : w.layout};
        dwl[j] = dd;
        pxs[j] = PackX{w.row_begin, chunk ? (int32_t)(w.chunk * h->tile_split[w.tile]) : -1, w.w, w.tile};
        if (!descriptor_ok(dd, w, t, rb, re, h->n_slots, doff, roff)) {
          int64_t cur = bad.load();
          while (j < cur && !bad.compare_exchange_weak(cur, j)) {
          }
        }
        d += area + extra;
        r += w.h_pad;
      }
    });
    if (bad.load() != INT64_MAX)
      throw Fail{TC_EINVAL, "internal error: workload " + std::to_string(bad.load()) + " (tile " +
                                std::to_string(wls[(size_t)bad.load()].tile) + ") addresses outside the packed arrays"};
    const int64_t j0 = h->tile_wl_begin[t0], nb = h->tile_wl_begin[t1] - j0;
    if (nb > 0) {
      HIPX(hipMemcpyAsync(h->d_wl + j0, dwl.p + j0, sizeof(Wl) * nb, hipMemcpyHostToDevice, st));
      HIPX(hipMemcpyAsync(d_px + j0, pxs.p + j0, sizeof(PackX) * nb, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_pack, dim3(nblk(nb * kPackSlices, kB / kWave)), dim3(kB), 0, st,
                         (const Wl*)(h->d_wl + j0), (const PackX*)(d_px + j0), nb, (const int32_t*)d_tfirst,
                         h->camping_pad ? 1 : 0, srt_start, rows_len, rows_sorted, b_icol, b_val,
                         (const int32_t*)first, h->d_idx, h->d_val, h->d_rowid, o->value_map ? pad_minus_one() : 0.0f);
      HIPX(hipGetLastError());
    }
  }
  clk.mark("a6 descriptors + a7 pack");
  if (o->value_map) {
    h->d_vmap = hold<int32_t>(h, doff);
    if (doff > 0) {
      hipLaunchKernelGGL(k_vmap_finish, dim3(nblk(doff, kB)), dim3(kB), 0, st, h->d_val, doff, A->val, h->d_vmap);
      HIPX(hipGetLastError());
    }
  }
  // TILE-COO: the bucketed entries themselves, with internal rows and the
  // first-touch flag of the coordinate kernel (a row's first tile stores)
  h->tile_coo_off = tstart;
  if (h->kernel == 1 && nnz > 0) {
    const int32_t* rows = b_row;
    if (!rows) {  // one tile: entries in CSR order
      int32_t* r = tmp.get<int32_t>(nnz);
      hipLaunchKernelGGL(k_expand_rows, dim3(nblk(n_rows, kB)), dim3(kB), 0, st, A->row_ptr, n_rows, r);
      HIPX(hipGetLastError());
      rows = r;
    }
    int64_t* d_ts = tmp.get<int64_t>(ntiles + 1);
    HIPX(hipMemcpyAsync(d_ts, tstart.data(), sizeof(int64_t) * (ntiles + 1), hipMemcpyHostToDevice, st));
    int32_t* cfirst = nullptr;
    if (ntiles > 1) {
      cfirst = tmp.get<int32_t>(n_rows);
      hipLaunchKernelGGL(k_fill_i32, dim3(nblk(n_rows, kB)), dim3(kB), 0, st, cfirst, n_rows, (int32_t)0x7fffffff);
      hipLaunchKernelGGL(k_coo_first, dim3(nblk(nnz, kB)), dim3(kB), 0, st, rows, (const int64_t*)d_ts, ntiles,
                         (const int32_t*)rowmap, nnz, cfirst);
      HIPX(hipGetLastError());
    }
    h->d_coo_row = hold<int32_t>(h, nnz);
    h->d_coo_col = hold<int32_t>(h, nnz);
    h->d_coo_val = hold<float>(h, nnz);
    hipLaunchKernelGGL(k_coo_pack, dim3(nblk(nnz, kB)), dim3(kB), 0, st, rows, (const int32_t*)b_icol, b_val,
                       (const int64_t*)d_ts, ntiles, (const int32_t*)rowmap, (const int32_t*)cfirst, nnz,
                       h->d_coo_row, h->d_coo_col, h->d_coo_val);
    HIPX(hipGetLastError());
  }
  // rows without any entry: every product writes their zero
  if (n_rows > 0) {
    int32_t* ef = tmp.get<int32_t>(n_rows);
    int32_t* ep = tmp.get<int32_t>(n_rows);
    hipLaunchKernelGGL(k_not, dim3(nblk(n_rows, kB)), dim3(kB), 0, st, (const int32_t*)touched, n_rows, ef);
    HIPX(hipGetLastError());
    h->n_empty = excl_scan<int32_t, int32_t>(ef, n_rows, ep, tmp, st);
    h->d_empty = hold<int32_t>(h, h->n_empty);
    hipLaunchKernelGGL(k_compact_idx, dim3(nblk(n_rows, kB)), dim3(kB), 0, st, (const int32_t*)ef,
                       (const int32_t*)ep, n_rows, h->d_empty);
    HIPX(hipGetLastError());
  }
  if (h->xcd_groups > 0 && n_rows > 0) {
    // rows tile 0 does not write: zeroed before the private copies are added
    int32_t* zf = tmp.get<int32_t>(n_rows);
    int32_t* zp = tmp.get<int32_t>(n_rows);
    hipLaunchKernelGGL(k_ne, dim3(nblk(n_rows, kB)), dim3(kB), 0, st, (const int32_t*)first, n_rows, 0, zf);
    HIPX(hipGetLastError());
    h->n_zero0 = excl_scan<int32_t, int32_t>(zf, n_rows, zp, tmp, st);
    h->d_zero0 = hold<int32_t>(h, h->n_zero0);
    hipLaunchKernelGGL(k_compact_idx, dim3(nblk(n_rows, kB)), dim3(kB), 0, st, (const int32_t*)zf,
                       (const int32_t*)zp, n_rows, h->d_zero0);
    HIPX(hipGetLastError());
    h->d_ypriv = hold<float>(h, (int64_t)h->xcd_groups * n_rows);
    HIPX(hipMemsetAsync(h->d_ypriv, 0, sizeof(float) * (size_t)h->xcd_groups * n_rows, st));
  }
  h->d_split = hold<SplitRow>(h, (int64_t)srows.size());
  h->d_partial = hold<double>(h, std::max<int64_t>(h->n_slots, 1) * 256);
  if (!srows.empty())
    HIPX(hipMemcpyAsync(h->d_split, srows.data(), sizeof(SplitRow) * srows.size(), hipMemcpyHostToDevice, st));
  std::vector<int64_t> psb;
  if (h->n_panels > 0) {
    // split rows of each panel (srows is in increasing row): [psb[p], psb[p+1])
    psb.assign(h->n_panels + 1, 0);
    size_t q = 0;
    for (int p = 0; p <= h->n_panels; ++p) {
      const int64_t lo = h->panel_begin[p];
      while (q < srows.size() && srows[q].row < lo) ++q;
      psb[p] = p == h->n_panels ? (int64_t)srows.size() : (int64_t)q;
    }
    h->d_panel_split_begin = hold<int64_t>(h, h->n_panels + 1);
    h->d_panel_yraw = hold<float>(h, std::max<int64_t>((int64_t)srows.size(), 1));
    HIPX(hipMemcpyAsync(h->d_panel_split_begin, psb.data(), sizeof(int64_t) * psb.size(), hipMemcpyHostToDevice, st));
  }
  h->d_xbuf = hold<float>(h, std::max(n_rows, n_cols));
  h->d_ybuf = hold<float>(h, std::max(n_rows, n_cols));
  h->d_red = hold<double>(h, 4096);
  h->d_counters = hold<unsigned long long>(h, std::max<int64_t>(ntiles, 1));
  HIPX(hipStreamSynchronize(st));
  clk.mark("a7 pack + metadata");
}

}  // namespace
}  // namespace tc

using namespace tc;

extern "C" tc_status tc_refresh_values(tc_handle* h, const float* d_val, tc_stream_t stream) {
  if (!h || (h->nnz > 0 && !d_val)) {
    set_error("tc_refresh_values: NULL argument");
    return TC_EINVAL;
  }
  if (!h->d_vmap) {
    set_error("tc_refresh_values: the handle was built without value_map");
    return TC_EINVAL;
  }
  if (h->nnz_pad > 0) {
    hipLaunchKernelGGL(k_refresh_vals, dim3(nblk(h->nnz_pad, kB)), dim3(kB), 0, (hipStream_t)stream,
                       (const int32_t*)h->d_vmap, h->nnz_pad, d_val, h->d_val);
    if (hipGetLastError() != hipSuccess) {
      set_error("tc_refresh_values: launch failed");
      return TC_EHIP;
    }
  }
  return TC_OK;
}

extern "C" void tc_build_opts_default(tc_build_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tile_width = 0;
  o->n_tiles = -1;
  o->wl_policy = 0;
  o->wave = 64;
  o->split_len = -1;
  o->relabel = -1;
}

extern "C" tc_status tc_build_tiled(const tc_csr* A, const tc_build_opts* opts, tc_stream_t stream, tc_handle** out) {
  auto t0 = std::chrono::steady_clock::now();
  if (!A || !out) {
    set_error("tc_build_tiled: NULL argument");
    return TC_EINVAL;
  }
  *out = nullptr;
  tc_build_opts def;
  tc_build_opts_default(&def);
  const tc_build_opts* o = opts ? opts : &def;
  if (A->n_rows < 0 || A->n_cols < 0 || A->nnz < 0) {
    set_error("tc_build_tiled: negative size");
    return TC_EINVAL;
  }
  if (A->nnz >= ((int64_t)1 << 31) || A->n_rows >= ((int64_t)1 << 30) || A->n_cols >= ((int64_t)1 << 31) - 1) {
    set_error("tc_build_tiled: sizes must fit 32-bit ids (nnz < 2^31, n_rows < 2^30)");
    return TC_EUNSUPPORTED;
  }
  if (!A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->val))) {
    set_error("tc_build_tiled: NULL CSR array");
    return TC_EINVAL;
  }
  if (o->tile_width < 0 || o->wave < 0 || o->split_len < -1 || o->xcd_groups < 0 || o->xcd_groups > 64 || o->kernel < 0 || o->kernel > 1 || (o->kernel == 1 && o->xcd_groups > 0) || o->value_map < 0 || o->value_map > 1 || (o->value_map && o->kernel == 1) || o->max_act_warp < 0 || o->wl_policy < 0 ||
      !(o->slices == 0 || o->slices == 1 || o->slices == 2 || o->slices == 4 || o->slices == 8) ||
      o->n_tile_bounds < 0 || o->lds_stage < -1 || o->lds_stage > 1 || o->panels < -1 || o->panel_rows < 0 ||
      !(o->panel_waves == 0 || o->panel_waves == 4 || o->panel_waves == 8 || o->panel_waves == 16) ||
      (o->panels != 0 && (o->xcd_groups > 0 || o->kernel == 1)) || (o->n_tile_bounds > 0 && (!o->tile_bounds || o->xcd_groups > 0)) ||
      o->wl_policy > 2 || (o->wl_policy == 1 && !o->wl_per_tile) || (o->relabel > 0 && A->n_rows != A->n_cols)) {
    set_error("tc_build_tiled: invalid option");
    return TC_EINVAL;
  }
  for (int i = 0; i < o->n_tile_bounds; ++i) {
    const int64_t b = o->tile_bounds[i];
    if (b <= (i ? (int64_t)o->tile_bounds[i - 1] : 0) || b > A->n_cols) {
      set_error("tc_build_tiled: tile_bounds must increase within (0, n_cols]");
      return TC_EINVAL;
    }
  }
  if ((o->alloc == nullptr) != (o->free == nullptr)) {
    set_error("tc_build_tiled: give both alloc and free or neither");
    return TC_EINVAL;
  }
  tc_handle* h = new tc_handle();
  h->n_rows = A->n_rows;
  h->n_cols = A->n_cols;
  h->nnz = A->nnz;
  // with automatic panels an unset width comes from the L2 in build()
  h->W = o->tile_width > 0 ? o->tile_width : (o->panels < 0 ? 0 : (1 << 23));
  h->S = o->wave > 0 ? o->wave : 64;
  h->split_len = o->split_len < 0 ? -1 : o->split_len;
  // automatic row panels with automatic sizes: workloads of kPanelWl entries
  // and rows split into chunks of twice that (measured best on MI355X; the
  // panel's wavefronts meet at a barrier after every tile, and Eq. 1-5 do not
  // charge the imbalance there)
  if (o->panels < 0 && o->split_len < 0) h->split_len = 2 * kPanelWl;
  h->camping_pad = o->camping_pad != 0;
  h->relabel = o->relabel < 0 ? (A->n_rows == A->n_cols) : (o->relabel != 0);
  h->max_act_warp = o->max_act_warp > 0 ? o->max_act_warp : 8192;
  h->xcd_groups = o->xcd_groups;
  h->kernel = o->kernel;
  h->slices = o->slices;
  h->lds_tiles = o->lds_stage + 1;  // 0 never, 1 automatic, 2 every tile that fits
  h->n_panels = o->panels;
  h->panel_rows = o->panels != 0 ? o->panel_rows : 0;
  h->panel_waves = o->panels != 0 ? (o->panel_waves > 0 ? o->panel_waves : 16) : 0;
  h->alloc = o->alloc;
  h->dfree = o->free;
  h->alloc_ctx = o->alloc_ctx;
  try {
    build(A, o, (hipStream_t)stream, h);
  } catch (const Fail& f) {
    (void)hipStreamSynchronize((hipStream_t)stream);
    set_error("tc_build_tiled: " + f.msg);
    tc_destroy(h);
    return f.st;
  } catch (const std::bad_alloc&) {
    (void)hipStreamSynchronize((hipStream_t)stream);
    set_error("tc_build_tiled: host allocation failed");
    tc_destroy(h);
    return TC_ENOMEM;
  }
  h->build_us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
  *out = h;
  return TC_OK;
}

extern "C" tc_status tc_csr_transpose(const tc_csr* A, int64_t* d_rpT, int32_t* d_colT, float* d_valT,
                                      int32_t* d_permT, tc_stream_t stream) {
  if (!A || !d_rpT || (A && A->nnz > 0 && (!A->row_ptr || !A->col_idx || (d_valT && !A->val)))) {
    set_error("tc_csr_transpose: NULL argument");
    return TC_EINVAL;
  }
  if (A->n_rows < 0 || A->n_cols < 0 || A->nnz < 0 || !A->row_ptr) {
    set_error("tc_csr_transpose: invalid sizes");
    return TC_EINVAL;
  }
  if (A->nnz >= ((int64_t)1 << 31) || A->n_rows >= ((int64_t)1 << 31) - 1 || A->n_cols >= ((int64_t)1 << 31) - 1) {
    set_error("tc_csr_transpose: sizes must fit 32-bit ids");
    return TC_EUNSUPPORTED;
  }
  try {
    transpose(A, d_rpT, d_colT, d_valT, d_permT, (hipStream_t)stream);
  } catch (const Fail& f) {
    set_error(std::string("tc_csr_transpose: ") + f.msg);
    return f.st;
  } catch (const std::bad_alloc&) {
    set_error("tc_csr_transpose: host allocation failed");
    return TC_ENOMEM;
  }
  return TC_OK;
}
