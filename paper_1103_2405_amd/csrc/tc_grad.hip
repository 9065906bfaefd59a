// Differentiable RWR with learned edge weights (Appendix F, Eq. 9 with
// w = softplus(theta . f)): the weights and their column normalisation, the
// checkpointed forward iterations, the adjoint pass and the chain to theta.
#include <algorithm>
#include <cmath>
#include <vector>

#include "tc_host.h"

namespace tc {

namespace {

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

}  // namespace
}  // namespace tc

using namespace tc;

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
