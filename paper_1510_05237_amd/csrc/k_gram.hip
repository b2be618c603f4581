// Gram matrix of the fixed factor and its inverse: the (U^T U)^-1 and
// (V^T V)^-1 of Algorithms 1-2.
//
// G = F^T F is summed over the rows of F in the working type T: each of a
// fixed number of blocks owns a fixed slice of rows and keeps its partial
// k x k sums in registers (one thread per upper-triangle entry group), so
// the sums do not depend on scheduling.  The last block to finish (device
// ticket) adds the block partials in block order in float64, then, still in
// float64 and in LDS:
//  * dead topics (zero diagonal: an all-zero column of F) get an identity
//    row and column, which keeps that topic at exactly zero;
//  * Cholesky G = L L^T (a non-positive pivot elsewhere sets the sticky
//    status NMF_ERR_NOT_SPD);
//  * L^-1 by forward substitution (one thread per column, written into the
//    free upper triangle), then W = L^-T L^-1.
// G itself is stored without the dead-topic substitution (the error of
// Section 3.1 needs the true Gram matrices).
#include "nmf_device.h"

namespace nmfk {

namespace {

constexpr int kStageRows = 32;

struct GramArgs {
  const void* F;            // rows x k (compact rows of a factor, or a dense matrix)
  const int32_t* rows_dev;  // number of rows (device), or nullptr
  int64_t rows_host;
  int32_t k;
  void* partials;           // [kGramBlocks][ne] T
  int32_t* ticket;
  double* G;
  double* W;                // nullptr: no factorisation (plain Gram)
  int32_t* dead;
  int32_t* status;
  // storage high-water mark: max over calls of counts_a[0] + counts_b[0]
  const int32_t* counts_a;
  const int32_t* counts_b;
  int64_t* max_nnz;
};

__device__ __forceinline__ void tri_index(int e, int k, int* pa, int* pb) {
  // e enumerates (a, b), a <= b, row by row of the upper triangle
  int a = 0;
  int rowlen = k;
  while (e >= rowlen) {
    e -= rowlen;
    ++a;
    --rowlen;
  }
  *pa = a;
  *pb = a + e;
}

template <typename T, int JMAX>
__global__ __launch_bounds__(256) void k_gram(GramArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int last;
  __shared__ int bad;
  if (*g.status != 0) return;
  const int k = g.k;
  const int kpad = (k + 3) & ~3;
  const int ne = k * (k + 1) / 2;
  const int tid = threadIdx.x;
  const int64_t R = g.rows_dev ? static_cast<int64_t>(*g.rows_dev) : g.rows_host;
  const int P = gridDim.x;
  const int64_t lo = R * blockIdx.x / P;
  const int64_t hi = R * (blockIdx.x + 1) / P;
  T* stage = reinterpret_cast<T*>(smem);
  int ea[JMAX], eb[JMAX];
  T acc[JMAX];
#pragma unroll
  for (int j = 0; j < JMAX; ++j) {
    const int e = tid + 256 * j;
    int a = 0, b = 0;
    if (e < ne) tri_index(e, k, &a, &b);
    ea[j] = a;
    eb[j] = b;
    acc[j] = T(0);
  }
  const T* __restrict__ F = static_cast<const T*>(g.F);
  for (int64_t r0 = lo; r0 < hi; r0 += kStageRows) {
    const int nr = static_cast<int>(hi - r0 < kStageRows ? hi - r0 : kStageRows);
    __syncthreads();
    for (int i = tid; i < nr * k; i += 256) {
      const int rr = i / k, c = i - rr * k;
      stage[rr * kpad + c] = F[(r0 + rr) * k + c];
    }
    __syncthreads();
    for (int rr = 0; rr < nr; ++rr) {
      const T* row = stage + rr * kpad;
#pragma unroll
      for (int j = 0; j < JMAX; ++j) acc[j] = fma(row[ea[j]], row[eb[j]], acc[j]);
    }
  }
  T* part = static_cast<T*>(g.partials) + static_cast<int64_t>(blockIdx.x) * ne;
#pragma unroll
  for (int j = 0; j < JMAX; ++j) {
    const int e = tid + 256 * j;
    if (e < ne) part[e] = acc[j];
  }
  fence_release();
  __syncthreads();
  if (tid == 0) last = atomicAdd(g.ticket, 1) == P - 1;
  __syncthreads();
  if (!last) return;
  fence_acquire();

  double* A = reinterpret_cast<double*>(smem);  // [k][k]
  double* dinv = A + k * k;                     // [k]
  const T* allp = static_cast<const T*>(g.partials);
  for (int e = tid; e < ne; e += 256) {
    double s = 0.0;
    for (int b = 0; b < P; ++b) s += static_cast<double>(__builtin_nontemporal_load(&allp[static_cast<int64_t>(b) * ne + e]));
    int a, bb;
    tri_index(e, k, &a, &bb);
    A[a * k + bb] = s;
    A[bb * k + a] = s;
    g.G[a * k + bb] = s;
    g.G[bb * k + a] = s;
  }
  if (tid == 0) {
    *g.ticket = 0;
    bad = 0;
    if (g.max_nnz) {
      const int64_t cur = static_cast<int64_t>(*g.counts_a) + (g.counts_b ? *g.counts_b : 0);
      if (cur > *g.max_nnz) *g.max_nnz = cur;
    }
  }
  __syncthreads();
  if (g.W == nullptr) return;
  // dead topics
  if (tid == 0) {
    int nd = 0;
    for (int c = 0; c < k; ++c)
      if (A[c * k + c] == 0.0) ++nd;
    *g.dead = nd;
  }
  for (int c = 0; c < k; ++c) {
    if (A[c * k + c] == 0.0) {
      __syncthreads();
      for (int i = tid; i < k; i += 256) {
        A[c * k + i] = 0.0;
        A[i * k + c] = 0.0;
      }
      __syncthreads();
      if (tid == 0) A[c * k + c] = 1.0;
    }
  }
  __syncthreads();
  // right-looking Cholesky on the lower triangle
  for (int j = 0; j < k; ++j) {
    if (tid == 0) {
      const double d = A[j * k + j];
      if (!(d > 0.0)) {
        bad = 1;
        A[j * k + j] = 1.0;
      } else {
        A[j * k + j] = sqrt(d);
      }
    }
    __syncthreads();
    const double piv = A[j * k + j];
    for (int i = j + 1 + tid; i < k; i += 256) A[i * k + j] /= piv;
    __syncthreads();
    const int w = k - j - 1;
    for (int idx = tid; idx < w * w; idx += 256) {
      const int i = j + 1 + idx / w;
      const int l = j + 1 + idx % w;
      if (l <= i) A[i * k + l] -= A[i * k + j] * A[l * k + j];
    }
    __syncthreads();
  }
  if (bad) {
    if (tid == 0) atomicCAS(g.status, 0, static_cast<int32_t>(NMF_ERR_NOT_SPD));
    for (int i = tid; i < k * k; i += 256) g.W[i] = 0.0;
    return;
  }
  // column a of L^-1 by forward substitution; L^-1[r][a] (r > a) is kept at
  // A[a][r] (upper triangle), its diagonal in dinv
  for (int a = tid; a < k; a += 256) {
    const double da = 1.0 / A[a * k + a];
    dinv[a] = da;
    for (int r = a + 1; r < k; ++r) {
      double s = A[r * k + a] * da;
      for (int q = a + 1; q < r; ++q) s = fma(A[r * k + q], A[a * k + q], s);
      A[a * k + r] = -s / A[r * k + r];
    }
  }
  __syncthreads();
  // W = L^-T L^-1: W[a][b] = sum_{r >= max(a,b)} L^-1[r][a] L^-1[r][b]
  for (int e = tid; e < ne; e += 256) {
    int a, b;
    tri_index(e, k, &a, &b);  // a <= b
    double s = dinv[b] * (a == b ? dinv[a] : A[a * k + b]);
    for (int r = b + 1; r < k; ++r) s = fma(A[a * k + r], A[b * k + r], s);
    g.W[a * k + b] = s;
    g.W[b * k + a] = s;
  }
}

template <typename T>
hipError_t launch(nmf_handle* h, GramArgs& g) {
  const int k = h->k;
  const int kpad = (k + 3) & ~3;
  size_t lds = static_cast<size_t>(kStageRows) * kpad * sizeof(T);
  const size_t fac = (static_cast<size_t>(k) * k + k) * sizeof(double);
  if (fac > lds) lds = fac;
  if (k <= 64)
    hipLaunchKernelGGL((k_gram<T, 9>), dim3(kGramBlocks), dim3(256), lds, h->stream, g);
  else
    hipLaunchKernelGGL((k_gram<T, 33>), dim3(kGramBlocks), dim3(256), lds, h->stream, g);
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t gram(nmf_handle* h, const Factor& F, const Gram& out) {
  GramArgs g{};
  g.F = F.dense;
  g.rows_dev = F.counts + 1;
  g.k = h->k;
  g.partials = h->gram_partials;
  g.ticket = h->gram_ticket;
  g.G = out.G;
  g.W = out.W;
  g.dead = out.dead;
  g.status = h->status;
  // the other factor's count completes nnz(U) + nnz(V)
  const bool is_v = (&F == &h->V);
  g.counts_a = F.counts;
  g.counts_b = is_v ? h->U[h->cur_u].counts : h->V.counts;
  g.max_nnz = h->met.max_nnz;
  return launch<T>(h, g);
}

template <typename T>
hipError_t gram_dense(nmf_handle* h, const T* F, int64_t rows, double* G) {
  GramArgs g{};
  g.F = F;
  g.rows_dev = nullptr;
  g.rows_host = rows;
  g.k = h->k;
  g.partials = h->gram_partials;
  g.ticket = h->gram_ticket;
  g.G = G;
  g.W = nullptr;
  g.status = h->status;
  return launch<T>(h, g);
}

template hipError_t gram<float>(nmf_handle*, const Factor&, const Gram&);
template hipError_t gram<double>(nmf_handle*, const Factor&, const Gram&);
template hipError_t gram_dense<float>(nmf_handle*, const float*, int64_t, double*);
template hipError_t gram_dense<double>(nmf_handle*, const double*, int64_t, double*);

}  // namespace nmfk
