// Host side of the format builder: the throughput table, the performance
// model of one tile (Section 3.3, Algorithm 3, Eq. 1-5), the workload-size
// search (Algorithm 2) and the greedy partition of a tile into workloads
// (Solution 3).  A tile is described by its row-length histogram in
// decreasing length; the partition depends on nothing else, so the GPU only
// sends these histograms and receives the workload list.
//
// Readings where the paper is silent:
//  - rows longer than split_len are cut into chunks of split_len entries, each
//    a one-row row-major workload; they take no part in the size bounds (the
//    automatic split length is the tile's share per resident wavefront, so
//    that Algorithm 2's lower bound cannot exceed its upper bound by much);
//  - h = max(1, floor(WL / w)); a column-major workload pads h to a multiple
//    of S and then takes that many real rows when they remain;
//  - a row-major workload pads its rows to a multiple of S, except that with
//    S = 64 rows of at most 32 entries are padded to 32 (the paper pads to its
//    warp of 32 threads; a wavefront instruction then covers two such rows);
//  - the table is a grid over powers of two of the padded (w, h); a shape is
//    looked up at the nearest power of two of each side in log scale, ties
//    rounding up, clamped to the grid;
//  - the model runs in double precision in a fixed order: per round
//    mean = sum_perf / count, then time += area / mean.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <limits>
#include <map>
#include <sstream>

#include "tc_internal.h"

namespace tc {

namespace {
thread_local std::string g_err;

int64_t ceil_to(int64_t v, int64_t s) { return (v + s - 1) / s * s; }

// Padded length of a row-major workload's rows: a multiple of S, or half of
// S = 64 for rows of at most 32 entries (the paper's warp of 32; two such rows
// fill one 64-wide wavefront instruction).
int64_t rm_pad(int64_t w, int64_t S) { return S >= 64 && 2 * w <= S ? S / 2 : ceil_to(w, S); }

int nearest_log2(int64_t v) {
  if (v < 1) v = 1;
  int k = 63 - __builtin_clzll((unsigned long long)v);
  // compare v^2 with 2^(2k+1) without overflow for v < 2^31
  unsigned __int128 v2 = (unsigned __int128)v * (unsigned __int128)v;
  unsigned __int128 mid = (unsigned __int128)1 << (2 * k + 1);
  return v2 >= mid ? k + 1 : k;
}

// A run of identical consecutive workloads in emission order.
struct Batch {
  int32_t layout;
  int64_t w, w_pad, h_pad, n_rows;  // n_rows: real rows of each workload
  int64_t count;
  int64_t row_begin;                // first row (tile-local) of the first workload
  int64_t step;                     // rows consumed per workload
  int32_t chunk, n_chunks;          // >= 0 for one chunk of a split row
};

// Walk the greedy partition in emission order, calling f(batch) for every
// batch of identical workloads.
template <class F>
void walk(const RunSpan& runs, int64_t wl, const PartitionParams& p, F&& f) {
  int64_t R = 0;
  for (const auto& r : runs) R += r.count;
  const int64_t S = p.S;
  int64_t i = 0;
  size_t ri = 0;
  int64_t run_end = runs.empty() ? 0 : runs[0].count;
  while (i < R) {
    while (i >= run_end) run_end += runs[++ri].count;
    const int64_t w = runs[ri].len;
    if (p.split_len > 0 && w > p.split_len) {
      const int64_t nch = (w + p.split_len - 1) / p.split_len;
      for (; i < run_end; ++i)
        for (int64_t k = 0; k < nch; ++k) {
          const int64_t cw = std::min<int64_t>(p.split_len, w - k * p.split_len);
          f(Batch{kChunk, cw, ceil_to(cw, S), 1, 1, 1, i, 1, (int32_t)k, (int32_t)nch});
        }
      continue;
    }
    const int64_t hmax = std::max<int64_t>(1, wl / w);
    if (R - i <= hmax) {  // last workload of the tile
      const int64_t h = R - i;
      if (w >= h)
        f(Batch{kRM, w, rm_pad(w, S), h, h, 1, i, h, -1, 0});
      else
        f(Batch{kCM, w, w, ceil_to(h, S), h, 1, i, h, -1, 0});
      i = R;
      break;
    }
    if (w >= hmax) {
      const int64_t step = hmax;
      // workloads whose first row is in this run and that are not the tile's last
      const int64_t q = std::min((run_end - i + step - 1) / step, (R - i - hmax + step - 1) / step);
      f(Batch{kRM, w, rm_pad(w, S), hmax, hmax, q, i, step, -1, 0});
      i += q * step;
    } else {
      const int64_t hp = ceil_to(hmax, S);
      if (R - i < hp) {  // padded rows exceed what remains: take the rest
        f(Batch{kCM, w, w, hp, R - i, 1, i, R - i, -1, 0});
        i = R;
        break;
      }
      int64_t q = (run_end - i + hp - 1) / hp;
      q = std::min<int64_t>(q, (R - i) / hp);
      f(Batch{kCM, w, w, hp, hp, q, i, hp, -1, 0});
      i += q * hp;
    }
  }
}
}  // namespace

void set_error(const std::string& msg) { g_err = msg; }

int64_t tile_split_len(int32_t split_len, int64_t tile_nnz, int64_t max_act_warp, int32_t S) {
  if (split_len >= 0) return split_len;
  const int64_t share = (tile_nnz + max_act_warp - 1) / max_act_warp;
  return std::min<int64_t>(8192, std::max<int64_t>(S, ceil_to(share, S)));
}
const char* get_error() { return g_err.c_str(); }

int64_t PerfTable::perf(bool sparse_tile, int64_t w, int64_t h) const {
  int lw = std::min(nearest_log2(w), nw - 1);
  int lh = std::min(nearest_log2(h), nh - 1);
  return (sparse_tile ? sparse : dense)[(size_t)lw * nh + lh];
}

// Built-in table used until a measured one is given: modelled throughput of
// a wavefront on a w x h padded workload with a fixed per-workload cost and a
// per-row cost for row-major workloads (one cross-lane reduction per row).
void default_perf_table(PerfTable* t) {
  t->nw = 16;
  t->nh = 16;
  t->dense.assign(256, 0);
  t->sparse.assign(256, 0);
  for (int lw = 0; lw < 16; ++lw)
    for (int lh = 0; lh < 16; ++lh) {
      const double w = (double)(1 << lw), h = (double)(1 << lh);
      const double area = w * h;
      const bool rm = w >= h;
      const double over = 2048.0 + (rm ? 32.0 * h : 16.0 * (h / 64.0 + 1.0));
      const double v = 1.0e6 * area / (area + over);
      t->dense[lw * 16 + lh] = (int64_t)(v + 0.5);
      t->sparse[lw * 16 + lh] = (int64_t)(0.7 * v + 0.5);
    }
}

// Text table: lines "dense|sparse lw lh value", '#' comments.
bool load_perf_table(const char* path, PerfTable* t, std::string* err) {
  std::ifstream in(path);
  if (!in) {
    *err = std::string("cannot open performance table ") + path;
    return false;
  }
  std::map<std::pair<int, int>, int64_t> e[2];
  int nw = 0, nh = 0;
  std::string line;
  while (std::getline(in, line)) {
    auto hash = line.find('#');
    if (hash != std::string::npos) line.resize(hash);
    std::istringstream ss(line);
    std::string kind;
    int lw, lh;
    long long v;
    if (!(ss >> kind)) continue;
    if (!(ss >> lw >> lh >> v) || (kind != "dense" && kind != "sparse") || lw < 0 || lh < 0 || lw > 40 ||
        lh > 40 || v <= 0) {
      *err = "bad line in performance table: " + line;
      return false;
    }
    e[kind == "sparse"][{lw, lh}] = v;
    nw = std::max(nw, lw + 1);
    nh = std::max(nh, lh + 1);
  }
  if (nw == 0 || e[0].size() != (size_t)nw * nh || e[1].size() != (size_t)nw * nh) {
    *err = "performance table must give every (lw, lh) of its grid for dense and sparse";
    return false;
  }
  t->nw = nw;
  t->nh = nh;
  t->dense.assign((size_t)nw * nh, 0);
  t->sparse.assign((size_t)nw * nh, 0);
  for (auto& kv : e[0]) t->dense[(size_t)kv.first.first * nh + kv.first.second] = kv.second;
  for (auto& kv : e[1]) t->sparse[(size_t)kv.first.first * nh + kv.first.second] = kv.second;
  return true;
}

double model_time(const RunSpan& runs, int64_t wl, const PerfTable& table, bool sparse_tile,
                  const PartitionParams& p, int64_t* n_wl) {
  std::vector<double> P, Size;
  std::vector<int64_t> Cnt;
  int64_t j = 0;  // workload index
  walk(runs, wl, p, [&](const Batch& b) {
    const double perf = (double)table.perf(sparse_tile, b.w_pad, b.h_pad);
    const double area = (double)(b.w_pad * b.h_pad);
    int64_t left = b.count;
    while (left > 0) {
      const int64_t it = j / p.max_act_warp;
      const int64_t room = (it + 1) * p.max_act_warp - j;
      const int64_t c = std::min(left, room);
      if ((int64_t)P.size() <= it) {
        P.resize(it + 1, 0.0);
        Size.resize(it + 1, 0.0);
        Cnt.resize(it + 1, 0);
      }
      // integer-valued sums: exact in double, so the order of additions inside
      // a round cannot change the result
      P[it] += perf * (double)c;
      Size[it] += area * (double)c;
      Cnt[it] += c;
      j += c;
      left -= c;
    }
  });
  if (n_wl) *n_wl = j;
  double total = 0.0;
  for (size_t i = 0; i < P.size(); ++i) {
    const double mean = P[i] / (double)Cnt[i];
    total += Size[i] / mean;
  }
  return total;
}

int64_t choose_wl(const RunSpan& runs, int64_t tile_nnz, const PerfTable& table, bool sparse_tile,
                  const PartitionParams& p) {
  int64_t low = -1;
  for (const auto& r : runs)
    if (!(p.split_len > 0 && r.len > p.split_len)) {
      low = r.len;
      break;
    }
  if (low < 0) return p.split_len > 0 ? p.split_len : (runs.empty() ? 1 : runs[0].len);
  const int64_t up = tile_nnz / p.max_act_warp;
  if (up < low) return low;
  double best_t = std::numeric_limits<double>::infinity();
  int64_t best = 0;
  for (int64_t wl = low; wl <= up; wl += low) {
    const double t = model_time(runs, wl, table, sparse_tile, p);
    if (t < best_t) {
      best_t = t;
      best = wl;
    }
  }
  return best;
}

void partition_tile(const RunSpan& runs, int64_t wl, int32_t tile, int64_t row_base,
                    const PartitionParams& p, HostWl* out) {
  walk(runs, wl, p, [&](const Batch& b) {
    HostWl h;
    h.tile = tile;
    h.layout = b.layout == kCM ? kCM : kRM;
    h.w = (int32_t)b.w;
    h.w_pad = (int32_t)b.w_pad;
    h.h_pad = (int32_t)b.h_pad;
    h.n_rows = (int32_t)b.n_rows;
    h.chunk = b.layout == kChunk ? b.chunk : -1;
    h.n_chunks = b.layout == kChunk ? b.n_chunks : 0;
    h.data_off = 0;
    h.rowid_off = 0;
    for (int64_t q = 0; q < b.count; ++q) {
      h.row_begin = (int32_t)(row_base + b.row_begin + q * b.step);
      *out++ = h;
    }
  });
}

}  // namespace tc
