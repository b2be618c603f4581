// Sequential ALS (Algorithm 3, Section 4): topics are found k2 at a time.
// The factors keep their full width k; in block b the columns
// [k1, k1 + k2), k1 = b k2, are being solved, the columns before them are
// finished and the columns after them are zero.  With F the fixed factor
// (U in the V half) and X the one solved for (V), the deflated solve of
// Eqs. (seq-V)/(seq-U) for one row r of X is
//
//   x_r[blk] = max(0, (b_r[blk] - sum_{t < k1} x_r[t] G[t, blk]) W22)
//
// with b_r = (A_rows F)_r the raw product of the SpMM (all k columns, float
// in the working type), G = F^T F (float64) and W22 the inverse of G's
// [blk, blk] block (float64, k_gram.hip).  Finished columns are copied
// through and later columns stay zero, so the usual select and repack then
// rebuild the whole factor (a finished column already holds at most t
// entries and so is kept whole).
#include "nmf_device.h"

namespace nmfk {

namespace {

// One wave per row r; lanes = columns c (two per lane when k > 64).
template <typename T, int KPL>
__global__ __launch_bounds__(256) void k_seq_solve(const T* Bin, T* Xout, int64_t rows, int32_t k, int32_t k1,
                                                   int32_t k2, const int32_t* row_ptr, const uint8_t* topic,
                                                   const T* val, const double* G, const double* W22,
                                                   const int32_t* status) {
  if (*status != 0) return;
  const int64_t r = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (r >= rows) return;
  const int lane = lane_id();
  double y[KPL];
  T keep[KPL];
  bool in_blk[KPL];
#pragma unroll
  for (int q = 0; q < KPL; ++q) {
    const int c = lane + 64 * q;
    in_blk[q] = c >= k1 && c < k1 + k2;
    y[q] = in_blk[q] ? static_cast<double>(Bin[r * k + c]) : 0.0;
    keep[q] = T(0);
  }
  // the finished topics of this row: deflate, and keep their values (in the
  // first block there are none, and the solved factor may not exist yet:
  // its storage is not read)
  const int32_t e0 = k1 > 0 ? row_ptr[r] : 0;
  const int32_t e1 = k1 > 0 ? row_ptr[r + 1] : 0;
  for (int32_t e = e0; e < e1; ++e) {
    const int t = topic[e];
    if (t >= k1) continue;
    const T v = val[e];
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
      const int c = lane + 64 * q;
      if (in_blk[q]) y[q] = fma(-static_cast<double>(v), G[static_cast<int64_t>(t) * k + c], y[q]);
      if (c == t) keep[q] = v;
    }
  }
  // x[c] = sum_j y[k1 + j] W22[j][c - k1]
  double x[KPL];
#pragma unroll
  for (int q = 0; q < KPL; ++q) x[q] = 0.0;
  for (int j = 0; j < k2; ++j) {
    const int cj = k1 + j;
    const double yv = (KPL > 1 && cj >= 64) ? y[KPL - 1] : y[0];
    const double yj = __shfl(yv, cj & 63, 64);
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
      const int c = lane + 64 * q;
      if (in_blk[q]) x[q] = fma(yj, W22[static_cast<int64_t>(j) * k2 + (c - k1)], x[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < KPL; ++q) {
    const int c = lane + 64 * q;
    if (c < k) {
      T out = T(0);
      if (c < k1) out = keep[q];
      else if (in_blk[q]) out = static_cast<T>(x[q] > 0.0 ? x[q] : 0.0);
      Xout[r * k + c] = out;
    }
  }
}

// X (rows x k, dense): columns [k1, k1 + k2) <- U0b (rows x k2), later
// columns <- 0, earlier columns kept.
template <typename T>
__global__ __launch_bounds__(256) void k_seq_setup(T* X, const T* U0b, int64_t rows, int32_t k, int32_t k1,
                                                   int32_t k2) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= rows * k) return;
  const int64_t r = i / k;
  const int c = static_cast<int>(i - r * k);
  if (c < k1) return;
  X[i] = c < k1 + k2 ? U0b[r * k2 + (c - k1)] : T(0);
}

// U0b (rows x k2) <- the first k2 columns of X (rows x k).
template <typename T>
__global__ __launch_bounds__(256) void k_seq_save(const T* X, T* U0b, int64_t rows, int32_t k, int32_t k2) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= rows * k2) return;
  const int64_t r = i / k2;
  U0b[i] = X[r * k + (i - r * k2)];
}

// The storage high-water mark after a half-step: nnz(U) + nnz(V).
__global__ void k_seq_max(const int32_t* counts_a, const int32_t* counts_b, int64_t* max_nnz) {
  const int64_t cur = static_cast<int64_t>(*counts_a) + *counts_b;
  if (cur > *max_nnz) *max_nnz = cur;
}

unsigned grid_of(int64_t n, int per) { return static_cast<unsigned>((n + per - 1) / per); }

}  // namespace

template <typename T>
hipError_t seq_solve(nmf_handle* h, const T* B, T* X, int64_t rows, const Factor& F_old, const double* G,
                     const double* W22, int k1, int k2) {
  const unsigned blocks = grid_of(rows, 4);
  if (blocks == 0) return hipSuccess;
  if (h->k > 64)
    hipLaunchKernelGGL((k_seq_solve<T, 2>), dim3(blocks), dim3(256), 0, h->stream, B, X, rows, h->k, k1, k2,
                       F_old.row_ptr, F_old.topic, static_cast<const T*>(F_old.val), G, W22, h->status);
  else
    hipLaunchKernelGGL((k_seq_solve<T, 1>), dim3(blocks), dim3(256), 0, h->stream, B, X, rows, h->k, k1, k2,
                       F_old.row_ptr, F_old.topic, static_cast<const T*>(F_old.val), G, W22, h->status);
  return hipGetLastError();
}

template <typename T>
hipError_t seq_setup(nmf_handle* h, T* X, const T* U0b, int64_t rows, int k1, int k2) {
  const unsigned blocks = grid_of(rows * h->k, 256);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_seq_setup<T>, dim3(blocks), dim3(256), 0, h->stream, X, U0b, rows, h->k, k1, k2);
  return hipGetLastError();
}

template <typename T>
hipError_t seq_save(nmf_handle* h, const T* X, T* U0b, int64_t rows, int k2) {
  const unsigned blocks = grid_of(rows * k2, 256);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_seq_save<T>, dim3(blocks), dim3(256), 0, h->stream, X, U0b, rows, h->k, k2);
  return hipGetLastError();
}

hipError_t seq_max(nmf_handle* h, const Factor& a, const Factor& b) {
  hipLaunchKernelGGL(k_seq_max, dim3(1), dim3(1), 0, h->stream, a.counts, b.counts, h->met.max_nnz);
  return hipGetLastError();
}

template hipError_t seq_solve<float>(nmf_handle*, const float*, float*, int64_t, const Factor&, const double*,
                                     const double*, int, int);
template hipError_t seq_solve<double>(nmf_handle*, const double*, double*, int64_t, const Factor&, const double*,
                                      const double*, int, int);
template hipError_t seq_setup<float>(nmf_handle*, float*, const float*, int64_t, int, int);
template hipError_t seq_setup<double>(nmf_handle*, double*, const double*, int64_t, int, int);
template hipError_t seq_save<float>(nmf_handle*, const float*, float*, int64_t, int);
template hipError_t seq_save<double>(nmf_handle*, const double*, double*, int64_t, int);

}  // namespace nmfk
