// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstdint>
#include <string>
#include <vector>

#include "tcspmv.h"

namespace tc {

constexpr int kWave = 64;

// Most floats of x a tile stages in LDS (160 KB, the LDS of one gfx950 CU).
constexpr int64_t kLdsMaxFloats = 40960;

// Row ids stored in `rowid` carry bit 30 when an earlier tile already wrote
// that row of y (the tile adds); without it the tile is the row's first
// writer and stores.  Rows are therefore limited to 2^30.
constexpr int32_t kAddFlag = 1 << 30;

// Workload layouts (Solution 3): row-major rectangles run one row at a time
// across the wavefront, column-major ones give each lane its own row; a chunk
// is one piece of a heavy row that was split across wavefronts.
enum : int32_t { kRM = 0, kCM = 1, kChunk = 2 };

// Device descriptor of one workload (32 bytes).
struct Wl {
  int64_t data_off;   // first element in idx/val
  int64_t rowid_off;  // first entry in rowid
  int32_t w_pad;      // elements per row as stored (RM, chunk) or columns (CM)
  int32_t h_pad;      // rows as stored (RM: real rows, CM: padded rows, chunk: 1)
  int32_t n_rows;     // real rows
  int32_t info;       // layout in bits 0-1; for chunks the partial slot in bits 2..31
};
static_assert(sizeof(Wl) == 32, "descriptor layout");

// One heavy row whose chunks (from any tile) are summed after the tile passes.
struct SplitRow {
  int32_t row;        // internal row id
  int32_t slot_begin; // first partial slot
  int32_t n_slots;    // chunks over all tiles, in (tile, chunk) order
  int32_t store;      // 1: no tile wrote the row, so the sum is stored, not added
};

// Host-side workload record (also what the format export returns).
struct HostWl {
  int32_t tile, layout, w, w_pad, h_pad, row_begin, n_rows, chunk, n_chunks;
  int64_t data_off, rowid_off;
};

// Throughput table over powers of two of (w, h) for the dense tiles and the
// sparse tile (Section 3.3: offline component of the performance model).
struct PerfTable {
  int nw = 0, nh = 0;
  std::vector<int64_t> dense, sparse;  // [lw * nh + lh]
  int64_t perf(bool sparse_tile, int64_t w, int64_t h) const;
};
bool load_perf_table(const char* path, PerfTable* t, std::string* err);
void default_perf_table(PerfTable* t);

// Length histogram of one tile's rows, in decreasing length.
struct LenRun {
  int64_t len;
  int64_t count;
};
// One tile's runs, a view into the build's run list.
struct RunSpan {
  const LenRun* p = nullptr;
  size_t n = 0;
  const LenRun* begin() const { return p; }
  const LenRun* end() const { return p + n; }
  size_t size() const { return n; }
  bool empty() const { return n == 0; }
  const LenRun& operator[](size_t i) const { return p[i]; }
};

struct PartitionParams {
  int32_t S;
  int32_t split_len;
  int64_t max_act_warp;
  bool camping_pad;
};

// Algorithm 2 / Algorithm 3 (performance model) for one tile.
int64_t choose_wl(const RunSpan& runs, int64_t tile_nnz, const PerfTable& table,
                  bool sparse_tile, const PartitionParams& p);
// n_wl (optional): the number of workloads of the partition
double model_time(const RunSpan& runs, int64_t wl, const PerfTable& table,
                  bool sparse_tile, const PartitionParams& p, int64_t* n_wl = nullptr);
// Split length of one tile: split_len >= 0 is used as given (0 = never
// split); -1 picks the tile's per-wavefront share of entries, rounded up to a
// multiple of S and kept within [S, 8192].
int64_t tile_split_len(int32_t split_len, int64_t tile_nnz, int64_t max_act_warp, int32_t S);
// Greedy packing of a tile into workloads (Solution 3), written to out[0, n)
// where n is the workload count model_time reports for the same arguments.
// row_base is the index of the tile's first row in the global sorted-row list.
void partition_tile(const RunSpan& runs, int64_t wl, int32_t tile, int64_t row_base,
                    const PartitionParams& p, HostWl* out);

// thread-local error message
void set_error(const std::string& msg);

// device memory pool (tc_mem.cpp): stream-ordered reuse of freed blocks
void* pool_alloc(size_t bytes, hipStream_t st);           // nullptr when out of memory
void pool_free(void* p, hipStream_t st, bool idle);       // idle: no queued work uses p
size_t pool_release_cached();
size_t pool_cached_bytes();

// host blocks kept for reuse (tc_mem.cpp): page-locked ones for the build's
// transfers, plain ones for a handle's host arrays.  A reused block is already
// mapped, so a build does not fault in fresh pages every time.
struct HostBlock {
  void* p = nullptr;
  size_t cap = 0;
  bool pinned = false;
};
HostBlock host_take(size_t bytes, bool pinned);  // throws std::bad_alloc when out of memory
void host_give(const HostBlock& b);
size_t host_release_cached();

// n items of a plain type in a reusable host block (contents uninitialised)
template <class T>
struct HostArray {
  HostBlock b;
  int64_t n = 0;
  HostArray() = default;
  HostArray(const HostArray&) = delete;
  HostArray& operator=(const HostArray&) = delete;
  ~HostArray() { release(); }
  void reset(int64_t count) {
    release();
    b = host_take(sizeof(T) * (size_t)(count > 0 ? count : 1), false);
    n = count;
  }
  void release() {
    if (b.p) host_give(b);
    b = HostBlock{};
    n = 0;
  }
  T* data() const { return (T*)b.p; }
  size_t size() const { return (size_t)n; }
  T& operator[](int64_t i) const { return data()[i]; }
};

}  // namespace tc

// The handle: every device buffer of one built matrix.
struct tc_handle {
  int64_t n_rows = 0, n_cols = 0, nnz = 0;
  int32_t W = 0, S = 64, split_len = 0, T = 0, n_tiles = 0;
  bool relabel = false, camping_pad = false;
  int64_t max_act_warp = 8192;
  int32_t slices = 0;               // row slices of the single-vector tile kernels (0 = automatic)
  int64_t nnz_pad = 0, n_rowid = 0, n_rows_sorted = 0, n_dangling = 0;
  int64_t n_wl = 0, n_slots = 0, n_split_rows = 0;
  double build_us = 0.0;
  double model_us = 0.0;            // Eq. 1-5 time of the built partition, all tiles

  // host copies of small metadata
  std::vector<int64_t> tile_col_begin, tile_col_end, tile_nnz, tile_wl, tile_split, tile_row_off;
  std::vector<int64_t> tile_wl_begin;  // workloads of tile t: [tile_wl_begin[t], tile_wl_begin[t+1])
  tc::HostArray<tc::HostWl> wls;   // every workload, in descriptor order

  // device buffers (owned)
  int32_t* d_cperm = nullptr;       // internal column -> original column
  int32_t* d_cpos = nullptr;        // original column -> internal column
  int32_t* d_rowmap = nullptr;      // original row -> internal row
  int32_t* d_rowinv = nullptr;      // internal row -> original row
  int32_t* d_clen = nullptr;        // column lengths (original ids)
  int32_t* d_rows_sorted = nullptr; // per-tile sorted internal rows
  int32_t* d_rows_len = nullptr;
  tc::Wl* d_wl = nullptr;
  int32_t* d_idx = nullptr;
  float* d_val = nullptr;
  int32_t* d_rowid = nullptr;
  tc::SplitRow* d_split = nullptr;
  double* d_partial = nullptr;
  float* d_xbuf = nullptr;          // internal-space x for spmv on user vectors
  float* d_ybuf = nullptr;
  double* d_red = nullptr;          // reduction scratch
  unsigned long long* d_counters = nullptr;  // per-tile work counters of the persistent pass
  int32_t* d_empty = nullptr;       // internal rows without any entry (zeroed by every product)
  int64_t n_empty = 0;
  // XCD schedule: tile 0 on every XCD, tiles 1..xcd_groups at once, tile g
  // pinned to the workgroups that land on XCD g-1, each writing its own y copy
  int32_t xcd_groups = 0;
  float* d_ypriv = nullptr;         // xcd_groups x n_rows, rows a tile never writes stay 0
  int32_t* d_zero0 = nullptr;       // rows tile 0 does not write (zeroed before the combine)
  int64_t* d_tile_wl_begin = nullptr;  // device copy of tile_wl_begin
  int64_t n_zero0 = 0;
  int n_cu = 256;                   // compute units of the device
  int32_t lds_tiles = 1;            // LDS staging of narrow tiles: 0 never, 1 automatic, 2 whenever it fits
  int64_t lds_floats = 0;           // floats of x one workgroup can stage (device limit)
  int64_t lds_cu_bytes = 0;         // LDS bytes per compute unit
  int64_t l2_bytes = 0;             // L2 bytes of one XCD (the L2 a workgroup's gathers see)
  int32_t* d_half = nullptr;        // HITS: 0/1 half of each internal index (lazily built)
  // row panels: tile g = panel g / n_col_tiles, column tile g % n_col_tiles
  int32_t n_panels = 0, n_col_tiles = 0, panel_rows = 0, panel_waves = 0;
  std::vector<int64_t> panel_begin;  // [n_panels + 1] internal rows
  int32_t* d_panel_begin = nullptr;  // device copy (int32)
  int64_t* d_panel_ncb = nullptr;    // [n_tiles] first workload of the tile that is not a split chunk
  int64_t* d_panel_chunks = nullptr; // chunk workloads of every column tile, panel order
  int64_t* d_panel_cb = nullptr;     // [n_col_tiles + 1] offsets into d_panel_chunks
  int64_t* d_panel_split_begin = nullptr;  // [n_panels + 1] first split row (d_split) of each panel
  float* d_panel_yraw = nullptr;     // [n_split_rows] a split row's sum over its unsplit segments (fused update)
  // value map (build option): the CSR entry of every padded slot, -1 for pads
  int32_t* d_vmap = nullptr;
  // TILE-COO (kernel == 1): every tile's entries in coordinate form
  int32_t kernel = 0;
  int32_t* d_coo_row = nullptr;     // internal row | kAddFlag when an earlier tile holds the row
  int32_t* d_coo_col = nullptr;     // internal column
  float* d_coo_val = nullptr;
  std::vector<int64_t> tile_coo_off;  // [n_tiles + 1]
  void* d_coo_carry = nullptr;      // per-wavefront partial sums of rows crossing intervals
  int64_t coo_carry_n = 0;
  // SpMM plan (lazily built): leading chunk workloads per tile, pieces per chunk
  bool mm_planned = false;
  std::vector<int64_t> mm_lead;
  int32_t mm_pieces = 1;
  double* d_mm_partial = nullptr;   // n_slots x pieces x k partial sums
  size_t mm_partial_bytes = 0;

  // allocator
  void* (*alloc)(size_t, void*) = nullptr;
  void (*dfree)(void*, void*) = nullptr;
  void* alloc_ctx = nullptr;
  std::vector<void*> owned;
  hipStream_t stream = nullptr;     // stream the handle was built on

  // growable workspace for SpMM and the drivers (device)
  void* d_ws = nullptr;
  size_t ws_bytes = 0;

  // timing of the tile kernels (optional)
  bool timing = false;
  double tile_kernel_ms = 0.0;
  int64_t tile_launches = 0;
  int64_t spmv_calls = 0;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
};
