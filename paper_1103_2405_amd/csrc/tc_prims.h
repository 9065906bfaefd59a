// Device primitives of the format builder: a deterministic exclusive scan and
// one stable counting-sort pass.  Every sort of the builder (columns by
// length, entries by tile, rows by length) is a sequence of such passes, so
// the order of equal keys is always the input order and the result never
// depends on scheduling.
#pragma once

#include "tc_internal.h"

namespace tc {

constexpr int kScanBlock = 256;
constexpr int kScanPer = 16;
constexpr int64_t kScanTile = (int64_t)kScanBlock * kScanPer;

__device__ inline int lane_id() { return (int)__lane_id(); }

// v[i] = a[min(base + i, n - 1)] for the kScanPer items of one thread of the
// scan layout (n >= 1).  A run that lies inside [0, n) at a 16-byte aligned
// address is read with 16-byte loads: four lanes' runs then share each
// cache line request instead of sixteen.
template <typename T>
__device__ inline void load_run(const T* __restrict__ a, int64_t base, int64_t n, T (&v)[kScanPer]) {
  const T* p = a + min(base, n - 1);
  if ((sizeof(T) == 4 || sizeof(T) == 8) && base + kScanPer <= n && ((uintptr_t)p & 15) == 0) {
    constexpr int per = 16 / (int)sizeof(T);
#pragma unroll
    for (int q = 0; q < kScanPer / per; ++q) {
      const int4 w = reinterpret_cast<const int4*>(p)[q];
      __builtin_memcpy(&v[q * per], &w, 16);
    }
  } else {
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) v[i] = a[min(base + i, n - 1)];
  }
}

// a[base + i] = v[i] for base + i < n, with 16-byte stores for a whole
// aligned run
template <typename T>
__device__ inline void store_run(T* __restrict__ a, int64_t base, int64_t n, const T (&v)[kScanPer]) {
  T* p = a + base;
  if ((sizeof(T) == 4 || sizeof(T) == 8) && base + kScanPer <= n && ((uintptr_t)p & 15) == 0) {
    constexpr int per = 16 / (int)sizeof(T);
#pragma unroll
    for (int q = 0; q < kScanPer / per; ++q) {
      int4 w;
      __builtin_memcpy(&w, &v[q * per], 16);
      reinterpret_cast<int4*>(p)[q] = w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kScanPer; ++i)
      if (base + i < n) p[i] = v[i];
  }
}

// Inclusive scan across the 64 lanes of a wavefront.
template <typename T>
__device__ inline T wave_incl_scan(T v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T o = __shfl_up(v, d, kWave);
    if (lane >= d) v += o;
  }
  return v;
}

// Exclusive scan of one value per thread across a 256-thread block;
// *total receives the block sum.  Uses 4 + 1 LDS words.
template <typename T>
__device__ inline T block_excl_scan(T v, T* total) {
  __shared__ T wsum[kScanBlock / kWave];
  const int lane = lane_id(), wv = threadIdx.x / kWave;
  T inc = wave_incl_scan(v);
  if (lane == kWave - 1) wsum[wv] = inc;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kScanBlock / kWave; ++i) {
    if (i < wv) off += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

template <typename In>
__global__ void __launch_bounds__(kScanBlock) k_scan_reduce(const In* __restrict__ in, int64_t n,
                                                            int64_t* __restrict__ block_sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  In v[kScanPer];
  load_run(in, base, n, v);  // past n: in[n - 1], not added
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) s += base + i < n ? (int64_t)v[i] : 0;
  int64_t tot;
  block_excl_scan<int64_t>(s, &tot);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// Exclusive scan of nb block sums by one block (nb is at most a few 10^5).
__global__ void __launch_bounds__(kScanBlock) k_scan_blocks(int64_t* __restrict__ bs, int64_t nb,
                                                            int64_t* __restrict__ grand_total) {
  const int64_t per = (nb + kScanBlock - 1) / kScanBlock;
  const int64_t b0 = (int64_t)threadIdx.x * per;
  int64_t s = 0;
  for (int64_t i = 0; i < per; ++i)
    if (b0 + i < nb) s += bs[b0 + i];
  int64_t tot;
  int64_t off = block_excl_scan<int64_t>(s, &tot);
  for (int64_t i = 0; i < per; ++i)
    if (b0 + i < nb) {
      int64_t v = bs[b0 + i];
      bs[b0 + i] = off;
      off += v;
    }
  if (threadIdx.x == 0 && grand_total) *grand_total = tot;
}

template <typename In, typename Out>
__global__ void __launch_bounds__(kScanBlock) k_scan_down(const In* __restrict__ in, int64_t n,
                                                          const int64_t* __restrict__ bs,
                                                          Out* __restrict__ out) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  In v[kScanPer];
  load_run(in, base, n, v);
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    if (base + i >= n) v[i] = (In)0;
    s += (int64_t)v[i];
  }
  int64_t tot;
  int64_t off = block_excl_scan<int64_t>(s, &tot) + bs[blockIdx.x];
  Out o[kScanPer];
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    o[i] = (Out)off;
    off += (int64_t)v[i];
  }
  store_run(out, base, n, o);
}

// ---------------------------------------------------------------------------
// Stable counting-sort pass.  The input is cut into chunks of `chunk` items,
// one wavefront per chunk.  Pass 1 counts each chunk's buckets; an exclusive
// scan over the bucket-major count matrix gives every (bucket, chunk) its
// first output slot; pass 2 places the items (k_cs_scatter_staged).
//
// Op provides:  struct Item;                                   (one element)
//               __device__ Item load(int64_t k) const;
//               __device__ uint32_t bucket_of(const Item&) const;
//               __device__ void store(int64_t pos, const Item&) const;
// Every lane loads (a lane past the chunk's end reloads the chunk's first
// element) and only the stores are per lane: a load under a per-lane branch
// would wait for its data inside the branch, one element at a time.
constexpr int kCsBlock = 256;
constexpr int kCsWaves = kCsBlock / kWave;

template <class Op>
__global__ void __launch_bounds__(kCsBlock) k_cs_hist(Op op, int64_t n, int32_t nbuckets, int64_t chunk,
                                                      int64_t nchunks, int32_t* __restrict__ hist) {
  extern __shared__ int32_t cs_cnt[];
  const int lane = lane_id(), wv = threadIdx.x / kWave;
  const int64_t c = (int64_t)blockIdx.x * kCsWaves + wv;
  int32_t* cnt = cs_cnt + wv * nbuckets;
  for (int i = lane; i < nbuckets; i += kWave) cnt[i] = 0;
  __syncthreads();
  if (c < nchunks) {
    const int64_t first = c * chunk, end = min(n, (c + 1) * chunk);
    // four items per lane in flight, the next four loaded before these are
    // counted (lanes past the end reload the first item and count nothing)
    uint32_t nb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t k = first + u * kWave + lane;
      nb[u] = op.bucket_of(op.load(k < end ? k : first));
    }
    for (int64_t base0 = first; base0 < end; base0 += 4 * kWave) {
      uint32_t b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        b[u] = nb[u];
        const int64_t k = base0 + (4 + u) * kWave + lane;
        nb[u] = op.bucket_of(op.load(k < end ? k : first));
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (base0 + u * kWave + lane < end) atomicAdd(&cnt[b[u]], 1);
    }
  }
  __syncthreads();
  if (c < nchunks)
    for (int i = lane; i < nbuckets; i += kWave) hist[(int64_t)i * nchunks + c] = cnt[i];
}

// Pass 2: each wavefront walks its chunk in order, 64 items at a time, and
// ranks equal buckets inside the step by lane order (ballots over the
// bucket's bits), so equal keys keep their input order.  The items are placed
// in chunk-local bucket order in LDS; then every bucket's run of the chunk
// goes out with consecutive lanes, so the stores are coalesced and no global
// store sits between the loads of the walk.  hist holds the (bucket, chunk)
// counts; nbuckets must be a multiple of 64.
// Dynamic LDS per block: kCsWaves * (chunk * sizeof(Item) + 16 * nbuckets).
template <class Op>
__global__ void __launch_bounds__(kCsBlock) k_cs_scatter_staged(Op op, int64_t n, int32_t nbuckets, int32_t nbits,
                                                                int64_t chunk, int64_t nchunks,
                                                                const int64_t* __restrict__ offs,
                                                                const int32_t* __restrict__ hist) {
  using Item = typename Op::Item;
  extern __shared__ int64_t cs_stage[];
  const int lane = lane_id(), wv = threadIdx.x / kWave;
  const int64_t c = (int64_t)blockIdx.x * kCsWaves + wv;
  if (c >= nchunks) return;  // whole wavefront leaves; no block barrier below
  char* base = (char*)cs_stage + (size_t)wv * (chunk * sizeof(Item) + 16 * (size_t)nbuckets);
  Item* li = (Item*)base;
  int64_t* gst = (int64_t*)(base + chunk * sizeof(Item));  // bucket's first global slot for this chunk
  int32_t* lst = (int32_t*)(gst + nbuckets);                 // bucket's first local slot
  int32_t* lrun = lst + nbuckets;                            // next local slot
  // local starts: exclusive scan of this chunk's counts (lane l: buckets l*per ...)
  const int per = nbuckets / kWave;
  int32_t mine = 0;
  for (int q = 0; q < per; ++q) mine += hist[(int64_t)(lane * per + q) * nchunks + c];
  int32_t incl = mine;
  for (int o = 1; o < kWave; o <<= 1) {
    const int32_t t = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += t;
  }
  int32_t acc = incl - mine;
  for (int q = 0; q < per; ++q) {
    const int b = lane * per + q;
    lst[b] = acc;
    lrun[b] = acc;
    gst[b] = offs[(int64_t)b * nchunks + c];
    acc += hist[(int64_t)b * nchunks + c];
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const int64_t first = c * chunk, end = min(n, (c + 1) * chunk);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  Item nx[4];  // the next group's items, loaded while this group is placed
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t k = first + u * kWave + lane;
    nx[u] = op.load(k < end ? k : first);
  }
  for (int64_t base0 = first; base0 < end; base0 += 4 * kWave) {
    Item it[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      it[u] = nx[u];
      const int64_t k = base0 + (4 + u) * kWave + lane;
      nx[u] = op.load(k < end ? k : first);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t k = base0 + u * kWave + lane;
      const bool valid = k < end;
      const uint32_t b = op.bucket_of(it[u]);
      uint64_t peers = __ballot(valid);
      for (int bit = 0; bit < nbits; ++bit) {
        const bool set = (b >> bit) & 1u;
        const uint64_t bal = __ballot(set);
        peers &= set ? bal : ~bal;
      }
      const int32_t pos = valid ? lrun[b] + (int32_t)__popcll(peers & lt) : 0;
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      if (valid) li[pos] = it[u];
      if (valid && (peers >> lane) == 1ull) lrun[b] += (int32_t)__popcll(peers);
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
  }
  // out in local order: a bucket's run is consecutive lanes and slots
  const int32_t cl = (int32_t)(end - first);
  for (int32_t i = lane; i < cl; i += kWave) {
    const Item v = li[i];
    const uint32_t b = op.bucket_of(v);
    op.store(gst[b] + (i - lst[b]), v);
  }
}

}  // namespace tc
