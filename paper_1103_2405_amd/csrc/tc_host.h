// Host-side helpers shared by the library's entry points: errors, launches,
// the product passes and small transfers.
#pragma once

#include <string>

#include "tc_device.h"

namespace tc {

struct Err {
  tc_status st;
  std::string msg;
};

#define HIPC(call)                                                          \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) throw Err{TC_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

// the handle's growable device workspace (at least `bytes`)
void* workspace(tc_handle* h, size_t bytes, hipStream_t st);
// an event from the handle's pool (timing of tile launches)
hipEvent_t next_event(tc_handle* h);

// A tile-kernel launch; with timing on, bracketed by HIP events on its stream.
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

// LDS staging of tile t's x segment: the width to stage, or 0 (global gathers)
int64_t lds_tile_width(const tc_handle* h, int t);
int64_t lds_tile_blocks(const tc_handle* h, int64_t lw);

// Row slices of tile t's workloads (the build option, or the measured rule).
int32_t tile_slices(const tc_handle* h, int t, int64_t n_wl);
template <class K>
K pick_slices(int32_t s, K s1, K s2, K s4, K s8) {
  return s == 8 ? s8 : s == 4 ? s4 : s == 2 ? s2 : s1;
}

// y := A x in internal ids (x: n_cols, y: n_rows).
// fuse_combine: in the XCD schedule, leave y without the private copies (the
// caller adds them in its own pass); split rows are then added to y first.
// skip_zero: y's empty rows are still zero from an earlier product into the
// same y (nothing else writes them), so the zeroing launch can be left out.
// One launch of the row-panel pass y := A x (a handle with row panels); with
// pr, the pass writes the fused PageRank update of y instead (split rows are
// finished by the caller from pr->yraw and their chunks).
void panel_pass(tc_handle* h, const float* x, float* y, hipStream_t st, const PanelPr* pr);
// tilewise: one launch per tile even for a handle with row panels.
void spmv_internal(tc_handle* h, const float* x, float* y, hipStream_t st, bool fuse_combine = false,
                   bool skip_zero = false, bool tilewise = false);
// Y := A X for k right-hand sides in internal ids; epi: fused RWR restart.
// partial_ext: split-row partial sums go there (at least n_slots * pieces * k
// doubles) instead of the handle's pool buffer, and launches are not timed:
// the call then allocates nothing.
void spmm_internal(tc_handle* h, const float* X, float* Y, int32_t k, hipStream_t st, bool skip_empty = false,
                   const RwrEpi* epi = nullptr, double* partial_ext = nullptr);
// doubles of split-row partial sums spmm_internal needs for k right-hand sides
size_t spmm_partial_doubles(tc_handle* h, int32_t k);
// out row q = in row perm[q] (rows of w floats)
void gather_rows(const float* in, const int32_t* perm, int64_t n, int32_t w, float* out, hipStream_t st);
// one double from the device (synchronises the stream)
double read_f64(const double* d, hipStream_t st);
void need_square(const tc_handle* h, const char* who);

// Runs f, turning errors into a status and the thread's last-error message.
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

}  // namespace tc
