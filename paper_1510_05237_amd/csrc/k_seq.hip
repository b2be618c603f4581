// Sequential ALS (Algorithm 3, Section 4): topics are found k2 at a time.
// The factors keep their full width k; in block b the columns
// [k1, k1 + k2), k1 = b k2, are being solved, the columns before them are
// finished and the columns after them are zero.  With F the fixed factor
// (U in the V half) and X the one solved for (V), the deflated solve of
// Eqs. (seq-V)/(seq-U) for one row r of X is
//
//   x_r[blk] = max(0, (b_r[blk] - sum_{t < k1} x_r[t] G[t, blk]) W22)
//
// with b_r = (A_rows F)_r the raw product of the SpMM (float in the working
// type; only the block's columns are read, and with k2 < k only they are
// gathered and stored), G = F^T F (float64) and W22 the inverse of G's
// [blk, blk] block (float64, k_gram.hip).  Finished columns are copied
// through and later columns stay zero, so the usual select and repack then
// rebuild the whole factor (a finished column already holds at most t
// entries and so is kept whole).
#include "nmf_device.h"

namespace nmfk {

namespace {

// Rows per wave in k_seq_solve: their loads are in flight together.
constexpr int kSeqRows = 4;

// kSeqRows consecutive rows per wave; lanes = columns c (two per lane when
// k > 64).  Bin and Xout may be the same array: a row is read whole before
// it is written.
template <typename T, int KPL>
__global__ __launch_bounds__(256) void k_seq_solve(const T* Bin, T* Xout, int64_t rows, int32_t k, int32_t k1,
                                                   int32_t k2, const int32_t* row_ptr, const uint8_t* topic,
                                                   const T* val, const double* G, const double* W22,
                                                   const int32_t* status) {
  if (*status != 0) return;
  const int64_t r0 = (static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6)) * kSeqRows;
  if (r0 >= rows) return;
  const int lane = lane_id();
  bool in_blk[KPL];
#pragma unroll
  for (int q = 0; q < KPL; ++q) in_blk[q] = lane + 64 * q >= k1 && lane + 64 * q < k1 + k2;
  double y[kSeqRows][KPL];
  T keep[kSeqRows][KPL];
  int32_t e0[kSeqRows], len[kSeqRows];
  int32_t most = 0;
#pragma unroll
  for (int u = 0; u < kSeqRows; ++u) {
    const int64_t r = r0 + u;
    const bool live = r < rows;
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
      y[u][q] = (live && in_blk[q]) ? static_cast<double>(Bin[r * k + lane + 64 * q]) : 0.0;
      keep[u][q] = T(0);
    }
    // the finished topics of the row (in the first block there are none, and
    // the solved factor may not exist yet: its storage is not read)
    e0[u] = (live && k1 > 0) ? row_ptr[r] : 0;
    len[u] = (live && k1 > 0) ? row_ptr[r + 1] - e0[u] : 0;
    most = max(most, len[u]);
  }
  // deflate with the finished topics and keep their values, entry i of every
  // row at once
  for (int32_t i = 0; i < most; ++i) {
    int t[kSeqRows];
    T v[kSeqRows];
#pragma unroll
    for (int u = 0; u < kSeqRows; ++u) {
      const bool act = i < len[u];
      t[u] = act ? static_cast<int>(topic[e0[u] + i]) : k;
      v[u] = act ? val[e0[u] + i] : T(0);
    }
#pragma unroll
    for (int u = 0; u < kSeqRows; ++u) {
      if (t[u] >= k1) continue;
#pragma unroll
      for (int q = 0; q < KPL; ++q) {
        const int c = lane + 64 * q;
        if (in_blk[q]) y[u][q] = fma(-static_cast<double>(v[u]), G[static_cast<int64_t>(t[u]) * k + c], y[u][q]);
        if (c == t[u]) keep[u][q] = v[u];
      }
    }
  }
  // x[c] = sum_j y[k1 + j] W22[j][c - k1]
  double x[kSeqRows][KPL];
#pragma unroll
  for (int u = 0; u < kSeqRows; ++u)
#pragma unroll
    for (int q = 0; q < KPL; ++q) x[u][q] = 0.0;
  for (int j = 0; j < k2; ++j) {
    const int cj = k1 + j;
    double w[KPL];
#pragma unroll
    for (int q = 0; q < KPL; ++q) w[q] = in_blk[q] ? W22[static_cast<int64_t>(j) * k2 + (lane + 64 * q - k1)] : 0.0;
#pragma unroll
    for (int u = 0; u < kSeqRows; ++u) {
      const double yv = (KPL > 1 && cj >= 64) ? y[u][KPL - 1] : y[u][0];
      const double yj = __shfl(yv, cj & 63, 64);
#pragma unroll
      for (int q = 0; q < KPL; ++q) x[u][q] = fma(yj, w[q], x[u][q]);
    }
  }
#pragma unroll
  for (int u = 0; u < kSeqRows; ++u) {
    const int64_t r = r0 + u;
    if (r >= rows) break;
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
      const int c = lane + 64 * q;
      if (c < k) {
        T out = T(0);
        if (c < k1) out = keep[u][q];
        else if (in_blk[q]) out = static_cast<T>(x[u][q] > 0.0 ? x[u][q] : 0.0);
        Xout[r * k + c] = out;
      }
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

// bits[w] bit i: row 32 w + i of the factor stores an entry in a topic of
// [c0, c0 + kw) (one lane per row; each wave writes two whole words).
__global__ __launch_bounds__(256) void k_window_bits(const int32_t* row_ptr, const uint8_t* topic, int64_t rows,
                                                     int32_t c0, int32_t kw, uint32_t* bits) {
  const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  bool in = false;
  if (r < rows)
    for (int32_t e = row_ptr[r]; e < row_ptr[r + 1] && !in; ++e) {
      const int t = topic[e];
      in = t >= c0 && t < c0 + kw;
    }
  const uint64_t b = __ballot(in);
  const int lane = threadIdx.x & 63;
  const int64_t w = r >> 5;
  if ((lane & 31) == 0 && w < (rows + 31) / 32) bits[w] = static_cast<uint32_t>(b >> lane);
}

// out[s][c] = F's compact dense row s, column c0 + c (c < kw), zero for
// kw <= c < ldn; rows past the factor's nonempty-row count are left alone.
__global__ __launch_bounds__(256) void k_narrow_rows(const float* dense, int32_t ld, const int32_t* counts,
                                                     int64_t rows, int32_t c0, int32_t kw, int32_t ldn, float* out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= rows * ldn) return;
  const int64_t s = i / ldn;
  if (s >= counts[1]) return;
  const int c = static_cast<int>(i - s * ldn);
  out[i] = c < kw ? dense[s * ld + c0 + c] : 0.f;
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
  const unsigned blocks = grid_of(rows, 4 * kSeqRows);
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

hipError_t window_bits(nmf_handle* h, const Factor& F, int c0, int kw, uint32_t* bits) {
  const unsigned blocks = grid_of(F.rows, 256);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_window_bits, dim3(blocks), dim3(256), 0, h->stream, F.row_ptr, F.topic, F.rows, c0, kw, bits);
  return hipGetLastError();
}

hipError_t narrow_rows(nmf_handle* h, const Factor& F, int c0, int kw, int ldn, float* out) {
  if (c0 < 0 || kw < 1 || c0 + kw > F.ld || ldn < kw) return hipErrorInvalidValue;
  const unsigned blocks = grid_of(F.rows * ldn, 256);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_narrow_rows, dim3(blocks), dim3(256), 0, h->stream, static_cast<const float*>(F.dense), F.ld,
                     F.counts, F.rows, c0, kw, ldn, out);
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
