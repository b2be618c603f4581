// Gram matrix of the fixed factor and its inverse: the (U^T U)^-1 and
// (V^T V)^-1 of Algorithms 1-2.
//
//  1. k_gram_partial: G = F^T F is summed over the rows of F in the working
//     type T.  Each of kGramBlocks blocks owns a fixed slice of rows and keeps
//     its partial k x k sums (upper triangle) in registers.
//  2. k_gram_reduce: every block owns 64 upper-triangle entries; its four
//     waves add strided subsets of the block partials in float64 and the
//     four sums are combined in a fixed order, so G does not depend on
//     scheduling.
//  3. k_gram_factor (one block) factorizes in float64, in LDS:
//      * dead topics (zero diagonal: an all-zero column of F) get an identity
//        row and column, which keeps that topic at exactly zero;
//      * Cholesky G = L L^T, right-looking; a non-positive pivot elsewhere
//        sets the sticky status NMF_ERR_NOT_SPD;
//      * L^-1 overwrites L row by row (forward substitution on all columns
//        of the identity at once), then W = L^-T L^-1.
// G itself is stored without the dead-topic substitution (the error of
// Section 3.1 needs the true Gram matrices).
#include "nmf_device.h"

namespace nmfk {

namespace {

constexpr int kStageRows = 128;
constexpr int kReduceEntries = 64;  // upper-triangle entries per reduce block

struct GramArgs {
  const void* F;            // rows x k (compact rows of a factor, or a dense matrix)
  int32_t ld;               // row pitch of F (>= k)
  const int32_t* rows_dev;  // number of rows (device), or nullptr
  int64_t rows_host;
  int32_t k;
  void* partials;           // [kGramBlocks][ne] T
  double* G;
  double* W;                // nullptr: no factorisation (plain Gram)
  int32_t* dead;
  int32_t* status;
  // storage high-water mark: max over calls of counts_a[0] + counts_b[0]
  const int32_t* counts_a;
  const int32_t* counts_b;
  int64_t* max_nnz;
  int32_t two_mats;  // LDS holds a second k x k matrix for L^-1
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
__global__ __launch_bounds__(256) void k_gram_partial(GramArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
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
    // the batch is contiguous in F: eight independent loads per thread
    const int ld = g.ld;
    const int nel = nr * ld;
    for (int i0 = tid; i0 < nel; i0 += 256 * 8) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = i0 + 256 * u;
        v[u] = i < nel ? F[r0 * ld + i] : T(0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = i0 + 256 * u;
        const int rr = i / ld, c = i - rr * ld;
        if (i < nel && c < k) stage[rr * kpad + c] = v[u];
      }
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
}

// In-LDS float64 factorization of the k x k matrix A (full storage); writes
// W = A^-1.  X (k x k, may alias nothing) holds L^-1 when it is not null;
// otherwise L^-1 overwrites L row by row.  Returns false when a pivot is not
// positive.
__device__ bool factor_inverse(double* A, double* X, double* tmp, int* dead, int k, double* W,
                               int32_t* ndead) {
  const int tid = threadIdx.x;
  __shared__ int nd;
  if (tid == 0) nd = 0;
  __syncthreads();
  for (int c = tid; c < k; c += 256) {
    dead[c] = A[c * k + c] == 0.0;
    if (dead[c]) atomicAdd(&nd, 1);
  }
  __syncthreads();
  if (tid == 0) *ndead = nd;
  if (nd > 0) {
    for (int e = tid; e < k * k; e += 256) {
      const int i = e / k, j = e - (e / k) * k;
      if (dead[i] || dead[j]) A[e] = i == j ? 1.0 : 0.0;
    }
    __syncthreads();
  }
  // right-looking Cholesky on the lower triangle, two barriers per column.
  // The diagonal of L goes to tmp and replaces A's diagonal only at the end,
  // so every thread can read the pivot A[j][j] itself without a race.
  bool ok = true;
  for (int j = 0; j < k; ++j) {
    __syncthreads();  // the previous trailing update is complete
    const double d = A[j * k + j];
    if (!(d > 0.0)) ok = false;
    const double piv = d > 0.0 ? sqrt(d) : 1.0;
    if (tid == 0) tmp[j] = piv;
    for (int i = j + 1 + tid; i < k; i += 256) A[i * k + j] /= piv;
    __syncthreads();
    // trailing update: thread -> row i = j+1+tid/4, every 4th column
    for (int i = j + 1 + (tid >> 2); i < k; i += 64) {
      const double lij = A[i * k + j];
      for (int l = j + 1 + (tid & 3); l <= i; l += 4) A[i * k + l] = fma(-lij, A[l * k + j], A[i * k + l]);
    }
  }
  __syncthreads();
  for (int j = tid; j < k; j += 256) A[j * k + j] = tmp[j];
  __syncthreads();
  if (!ok) return false;
  if (X != nullptr) {
    // L^-1 by forward substitution on every column of the identity at once:
    // X = I; for j: X[j][:] /= L[j][j]; X[i][:] -= L[i][j] X[j][:] (i > j)
    for (int e = tid; e < k * k; e += 256) X[e] = (e / k) == (e % k) ? 1.0 : 0.0;
    __syncthreads();
    for (int j = 0; j < k; ++j) {
      const double ljj = A[j * k + j];
      for (int c = tid; c <= j; c += 256) X[j * k + c] /= ljj;
      __syncthreads();
      for (int i = j + 1 + (tid >> 2); i < k; i += 64) {
        const double lij = A[i * k + j];
        for (int c = (tid & 3); c <= j; c += 4) X[i * k + c] = fma(-lij, X[j * k + c], X[i * k + c]);
      }
      __syncthreads();
    }
  } else {
    // X = L^-1 overwrites L row by row:
    //   X[j][c] = (delta_jc - sum_{c <= i < j} L[j][i] X[i][c]) / L[j][j]
    X = A;
    for (int j = 0; j < k; ++j) {
      for (int i = tid; i <= j; i += 256) tmp[i] = A[j * k + i];
      __syncthreads();
      for (int c = tid; c <= j; c += 256) {
        double s = c == j ? 1.0 : 0.0;
        for (int i = c; i < j; ++i) s = fma(-tmp[i], A[i * k + c], s);
        A[j * k + c] = s / tmp[j];
      }
      __syncthreads();
    }
  }
  // W = X^T X: W[a][b] = sum_{r >= max(a,b)} X[r][a] X[r][b]
  const int ne = k * (k + 1) / 2;
  for (int e = tid; e < ne; e += 256) {
    int a, b;
    tri_index(e, k, &a, &b);  // a <= b
    double s0 = 0.0, s1 = 0.0;
    int r = b;
    for (; r + 1 < k; r += 2) {
      s0 = fma(X[r * k + a], X[r * k + b], s0);
      s1 = fma(X[(r + 1) * k + a], X[(r + 1) * k + b], s1);
    }
    if (r < k) s0 = fma(X[r * k + a], X[r * k + b], s0);
    const double sum = s0 + s1;
    W[a * k + b] = sum;
    W[b * k + a] = sum;
  }
  return true;
}

template <typename T>
__global__ __launch_bounds__(256) void k_gram_reduce(GramArgs g) {
  __shared__ double red[4][kReduceEntries];
  if (*g.status != 0) return;
  const int k = g.k;
  const int ne = k * (k + 1) / 2;
  const int lane = lane_id();
  const int wv = threadIdx.x >> 6;
  const int e = blockIdx.x * kReduceEntries + lane;
  const T* __restrict__ part = static_cast<const T*>(g.partials);
  double s = 0.0;
  if (e < ne) {
    // wave wv adds partials wv, wv + 4, ... in order, eight loads in flight
    int b = wv;
    for (; b + 28 < kGramBlocks; b += 32) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[static_cast<int64_t>(b + 4 * u) * ne + e];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += static_cast<double>(v[u]);
    }
    for (; b < kGramBlocks; b += 4) s += static_cast<double>(part[static_cast<int64_t>(b) * ne + e]);
  }
  red[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && e < ne) {
    const double t = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    int a, b;
    tri_index(e, k, &a, &b);
    g.G[a * k + b] = t;
    g.G[b * k + a] = t;
  }
}

// One block: the storage high-water mark, then W = G^-1 in float64.
__global__ __launch_bounds__(256) void k_gram_factor(GramArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (*g.status != 0) return;
  const int k = g.k;
  if (threadIdx.x == 0 && g.max_nnz) {
    const int64_t cur = static_cast<int64_t>(*g.counts_a) + (g.counts_b ? *g.counts_b : 0);
    if (cur > *g.max_nnz) *g.max_nnz = cur;
  }
  double* A = reinterpret_cast<double*>(smem);  // [k][k]
  double* tmp = A + k * k;                      // [k]
  int* dead = reinterpret_cast<int*>(tmp + k);  // [k]
  double* X = g.two_mats ? reinterpret_cast<double*>(dead + ((k + 1) & ~1)) : nullptr;  // [k][k]
  for (int i = threadIdx.x; i < k * k; i += 256) A[i] = g.G[i];
  __syncthreads();
  if (!factor_inverse(A, X, tmp, dead, k, g.W, g.dead)) {
    if (threadIdx.x == 0) atomicCAS(g.status, 0, static_cast<int32_t>(NMF_ERR_NOT_SPD));
    for (int i = threadIdx.x; i < k * k; i += 256) g.W[i] = 0.0;
  }
}

template <typename T>
hipError_t launch(nmf_handle* h, GramArgs& g) {
  const int k = h->k;
  const int kpad = (k + 3) & ~3;
  const size_t stage = static_cast<size_t>(kStageRows) * kpad * sizeof(T);
  size_t fac = (static_cast<size_t>(k) * k + k) * sizeof(double) + static_cast<size_t>((k + 1) & ~1) * sizeof(int);
  g.two_mats = fac + static_cast<size_t>(k) * k * sizeof(double) <= 150 * 1024 ? 1 : 0;
  if (g.two_mats) fac += static_cast<size_t>(k) * k * sizeof(double);
  if (k <= 64)
    hipLaunchKernelGGL((k_gram_partial<T, 9>), dim3(kGramBlocks), dim3(256), stage, h->stream, g);
  else
    hipLaunchKernelGGL((k_gram_partial<T, 33>), dim3(kGramBlocks), dim3(256), stage, h->stream, g);
  const int ne = k * (k + 1) / 2;
  const int rblocks = (ne + kReduceEntries - 1) / kReduceEntries;
  hipLaunchKernelGGL((k_gram_reduce<T>), dim3(rblocks), dim3(256), 0, h->stream, g);
  if (g.W) hipLaunchKernelGGL(k_gram_factor, dim3(1), dim3(256), fac, h->stream, g);
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t gram(nmf_handle* h, const Factor& F, const Gram& out) {
  GramArgs g{};
  g.F = F.dense;
  g.ld = F.ld;
  g.rows_dev = F.counts + 1;
  g.k = h->k;
  g.partials = h->gram_partials;
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
  g.ld = h->k;
  g.rows_dev = nullptr;
  g.rows_host = rows;
  g.k = h->k;
  g.partials = h->gram_partials;
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
