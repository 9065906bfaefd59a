// RWR (Appendix F, Eq. 9) on many graphs per launch: tile t of every graph,
// the split rows of every graph and the update of every graph each run as one
// launch, so small graphs share the GPU.
#include <algorithm>
#include <cmath>
#include <vector>

#include "tc_host.h"

namespace tc {

namespace {

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
               GlobalX{(const float*)s.x}, (float*)s.y, (double*)s.partial);
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

}  // namespace
}  // namespace tc

using namespace tc;

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
