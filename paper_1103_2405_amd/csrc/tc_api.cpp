// Handle queries, format export, kernel timing, destruction and errors.
#include <cstring>

#include "tc_internal.h"

namespace tc {
const char* get_error();
}

using namespace tc;

extern "C" const char* tc_last_error(void) { return get_error(); }

extern "C" tc_status tc_handle_info(const tc_handle* h, tc_info* info) {
  if (!h || !info) {
    set_error("tc_handle_info: NULL argument");
    return TC_EINVAL;
  }
  std::memset(info, 0, sizeof(*info));
  info->n_rows = h->n_rows;
  info->n_cols = h->n_cols;
  info->nnz = h->nnz;
  info->tile_width = h->W;
  info->wave = h->S;
  info->split_len = h->split_len;
  info->relabel = h->relabel ? 1 : 0;
  info->xcd_groups = h->xcd_groups;
  info->kernel = h->kernel;
  info->n_dense_tiles = h->T;
  info->n_tiles = h->n_tiles;
  info->n_workloads = h->n_wl;
  info->nnz_pad = h->nnz_pad;
  info->n_rowid = h->n_rowid;
  info->n_rows_sorted = h->n_rows_sorted;
  info->n_split_rows = h->n_split_rows;
  info->n_partials = h->n_slots;
  info->n_dangling = h->n_dangling;
  int64_t bytes = h->nnz_pad * 8 + h->n_rowid * 4 + h->n_wl * (int64_t)sizeof(Wl) + h->n_cols * 12 +
                  h->n_rows * 8 + h->n_rows_sorted * 8 + 2 * 4 * std::max(h->n_rows, h->n_cols) +
                  (int64_t)sizeof(double) * (std::max<int64_t>(h->n_slots, 1) * 256 + 4096) +
                  h->n_split_rows * (int64_t)sizeof(SplitRow) + (int64_t)h->ws_bytes;
  info->device_bytes = bytes;
  info->build_us = h->build_us;
  info->model_us = h->model_us;
  info->n_panels = h->n_panels;
  info->n_col_tiles = h->n_col_tiles;
  info->panel_rows = h->panel_rows;
  info->panel_waves = h->panel_waves;
  return TC_OK;
}

namespace {
template <class T>
hipError_t d2h(T* dst, const T* src, int64_t n) {
  if (!dst || n <= 0) return hipSuccess;
  return hipMemcpy(dst, src, sizeof(T) * (size_t)n, hipMemcpyDeviceToHost);
}
}  // namespace

extern "C" tc_status tc_export_format(const tc_handle* h, tc_format_view* v) {
  if (!h || !v) {
    set_error("tc_export_format: NULL argument");
    return TC_EINVAL;
  }
  if (hipDeviceSynchronize() != hipSuccess) {
    set_error("tc_export_format: device error before export");
    return TC_EHIP;
  }
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t r) {
    if (r != hipSuccess && e == hipSuccess) e = r;
  };
  chk(d2h(v->cperm, h->d_cperm, h->n_cols));
  chk(d2h(v->rowmap, h->d_rowmap, h->n_rows));
  chk(d2h(v->rows_sorted, h->d_rows_sorted, h->n_rows_sorted));
  chk(d2h(v->rows_len, h->d_rows_len, h->n_rows_sorted));
  chk(d2h(v->idx, h->d_idx, h->nnz_pad));
  chk(d2h(v->val, h->d_val, h->nnz_pad));
  chk(d2h(v->rowid, h->d_rowid, h->n_rowid));
  if (h->kernel == 1) {
    chk(d2h(v->coo_row, h->d_coo_row, h->nnz));
    chk(d2h(v->coo_col, h->d_coo_col, h->nnz));
    chk(d2h(v->coo_val, h->d_coo_val, h->nnz));
  }
  if (v->rowid)  // the first-writer flag is an implementation detail of the kernels
    for (int64_t k = 0; k < h->n_rowid; ++k)
      if (v->rowid[k] >= 0) v->rowid[k] &= ~kAddFlag;
  if (e != hipSuccess) {
    set_error(std::string("tc_export_format: ") + hipGetErrorString(e));
    return TC_EHIP;
  }
  for (int t = 0; t < h->n_tiles; ++t) {
    if (v->tile_col_begin) v->tile_col_begin[t] = h->tile_col_begin[t];
    if (v->tile_col_end) v->tile_col_end[t] = h->tile_col_end[t];
    if (v->tile_nnz) v->tile_nnz[t] = h->tile_nnz[t];
    if (v->tile_wl) v->tile_wl[t] = h->tile_wl[t];
    if (v->tile_split) v->tile_split[t] = h->tile_split[t];
  }
  if (v->panel_begin)
    for (size_t p = 0; p < h->panel_begin.size(); ++p) v->panel_begin[p] = h->panel_begin[p];
  if (v->tile_row_off)
    for (int t = 0; t <= h->n_tiles; ++t) v->tile_row_off[t] = h->tile_row_off.empty() ? 0 : h->tile_row_off[t];
  for (int64_t j = 0; j < h->n_wl; ++j) {
    const HostWl& w = h->wls[j];
    if (v->wl_tile) v->wl_tile[j] = w.tile;
    if (v->wl_layout) v->wl_layout[j] = w.layout;
    if (v->wl_w) v->wl_w[j] = w.w;
    if (v->wl_w_pad) v->wl_w_pad[j] = w.w_pad;
    if (v->wl_h_pad) v->wl_h_pad[j] = w.h_pad;
    if (v->wl_row_begin) v->wl_row_begin[j] = w.row_begin;
    if (v->wl_n_rows) v->wl_n_rows[j] = w.n_rows;
    if (v->wl_chunk) v->wl_chunk[j] = w.chunk;
    if (v->wl_n_chunks) v->wl_n_chunks[j] = w.n_chunks;
    if (v->wl_data_off) v->wl_data_off[j] = w.data_off;
    if (v->wl_rowid_off) v->wl_rowid_off[j] = w.rowid_off;
  }
  return TC_OK;
}

extern "C" tc_status tc_set_timing(tc_handle* h, int32_t enable) {
  if (!h) {
    set_error("tc_set_timing: NULL handle");
    return TC_EINVAL;
  }
  if (enable) {
    if (!h->ev_pool.empty()) (void)hipEventSynchronize(h->ev_pool[h->ev_used ? h->ev_used - 1 : 0]);
    h->tile_kernel_ms = 0.0;
    h->tile_launches = 0;
    h->spmv_calls = 0;
    h->ev_used = 0;
  }
  h->timing = enable != 0;
  return TC_OK;
}

extern "C" tc_status tc_get_timing(tc_handle* h, tc_timing* t) {
  if (!h || !t) {
    set_error("tc_get_timing: NULL argument");
    return TC_EINVAL;
  }
  if (h->ev_used > 0) {
    if (hipEventSynchronize(h->ev_pool[h->ev_used - 1]) != hipSuccess) {
      set_error("tc_get_timing: event synchronisation failed");
      return TC_EHIP;
    }
    for (size_t i = 0; i + 1 < h->ev_used; i += 2) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, h->ev_pool[i], h->ev_pool[i + 1]) == hipSuccess) h->tile_kernel_ms += ms;
    }
    h->ev_used = 0;
  }
  t->tile_kernel_ms = h->tile_kernel_ms;
  t->tile_launches = h->tile_launches;
  t->spmv_calls = h->spmv_calls;
  return TC_OK;
}

extern "C" void tc_destroy(tc_handle* h) {
  if (!h) return;
  (void)hipDeviceSynchronize();
  for (void* p : h->owned) {
    if (!p) continue;
    if (h->dfree)
      h->dfree(p, h->alloc_ctx);
    else
      tc::pool_free(p, nullptr, true);
  }
  if (h->d_ws) tc::pool_free(h->d_ws, nullptr, true);
  if (h->d_mm_partial) tc::pool_free(h->d_mm_partial, nullptr, true);
  if (h->d_coo_carry) tc::pool_free(h->d_coo_carry, nullptr, true);
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  delete h;
}

extern "C" size_t tc_release_cached_memory(void) { return tc::pool_release_cached() + tc::host_release_cached(); }
