// Per-iteration metrics of Section 3.1 and the small helpers around them.
//
//   R = ||U_i - U_{i-1}||_F / ||U_i||_F, formed directly from the two
//       stored factors row by row (no cancellation, so R can fall to the
//       rounding floor);
//   E = ||A - U V^T||_F / ||A||_F with
//       ||A - U V^T||^2 = ||A||^2 - 2 <U, A V> + <U^T U, V^T V>,
//       where A V is the raw product kept by the U half-step and the two
//       Gram matrices come from the Gram kernels.
// Every sum is float64 over fixed blocks, added in block order by a
// one-block final kernel, so the history is reproducible bit for bit.
#include <cmath>

#include <algorithm>

#include "nmf_device.h"

namespace nmfk {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// sums three doubles over the block into out[0..2] (thread 0 holds them)
__device__ __forceinline__ void block_sum3(double a, double b, double c, double* sh, double* out) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int lane = __lane_id(), wv = threadIdx.x >> 6;
  if (lane == 0) {
    sh[wv * 3 + 0] = a;
    sh[wv * 3 + 1] = b;
    sh[wv * 3 + 2] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double x = 0, y = 0, z = 0;
    for (int w = 0; w < 4; ++w) {
      x += sh[w * 3 + 0];
      y += sh[w * 3 + 1];
      z += sh[w * 3 + 2];
    }
    out[0] = x;
    out[1] = y;
    out[2] = z;
  }
}

struct MetArgs {
  int64_t n;
  int32_t k;
  const int32_t* slot_new;
  const int32_t* slot_old;
  const void* dense_new;
  const void* dense_old;
  int32_t ld;     // row pitch of dense_new / dense_old
  const void* C;  // raw A V (n x k), or nullptr
  double* partials;
  const double* GU;
  const double* GV;
  const double* WU;   // inverses of G_U, G_V (conditioning indicator)
  const double* WV;
  unsigned long long* gathered;  // [2][kGathSlots], read into the record and cleared
  const double* nA2;
  double* ring;
  int64_t* it;
  const int32_t* nnz_u;
  const int32_t* nnz_v;
  const int32_t* dead_u;
  const int32_t* dead_v;
  int32_t record;  // 0: only nnz / dead counts (E, R = NaN)
  int32_t nparts;  // partial blocks of k_metrics
  int32_t* status;
};

template <typename T, int KPL>
__device__ __forceinline__ void k_metrics_body(const MetArgs& a, int blk, int nblk) {
  __shared__ double sh[12];
  __shared__ double tot[3];
  if (*a.status != 0) return;
  const int k = a.k;
  const int lane = lane_id();
  const int wv = threadIdx.x >> 6;
  double d2 = 0.0, n2 = 0.0, x = 0.0;
  if (a.record) {
    const int P = nblk;
    const int64_t lo = a.n * blk / P;
    const int64_t hi = a.n * (blk + 1) / P;
    const T* __restrict__ Dn = static_cast<const T*>(a.dense_new);
    const T* __restrict__ Do = static_cast<const T*>(a.dense_old);
    const T* __restrict__ C = static_cast<const T*>(a.C);
    for (int64_t base = lo + wv * 64; base < hi; base += 256) {
      const int64_t r = base + lane;
      int sn = -1, so = -1;
      if (r < hi) {
        sn = a.slot_new[r];
        so = a.slot_old[r];
      }
      uint64_t todo = __ballot(sn >= 0 || so >= 0);
      while (todo) {
        // four rows per step: their loads are in flight together
        int bb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          bb[u] = -1;
          if (todo) {
            bb[u] = __ffsll(static_cast<long long>(todo)) - 1;
            todo &= todo - 1;
          }
        }
        double un[4][KPL], uo[4][KPL], cv[4][KPL];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int b = bb[u] < 0 ? 0 : bb[u];
          const int s1 = bb[u] < 0 ? -1 : __shfl(sn, b, 64);
          const int s0 = bb[u] < 0 ? -1 : __shfl(so, b, 64);
#pragma unroll
          for (int q = 0; q < KPL; ++q) {
            const int c = lane + 64 * q;
            const bool in = c < k;
            un[u][q] = (in && s1 >= 0) ? static_cast<double>(Dn[static_cast<int64_t>(s1) * a.ld + c]) : 0.0;
            uo[u][q] = (in && s0 >= 0) ? static_cast<double>(Do[static_cast<int64_t>(s0) * a.ld + c]) : 0.0;
            cv[u][q] = (in && s1 >= 0 && C != nullptr) ? static_cast<double>(C[(base + b) * k + c]) : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int q = 0; q < KPL; ++q) {
            const double dd = un[u][q] - uo[u][q];
            d2 = fma(dd, dd, d2);
            n2 = fma(un[u][q], un[u][q], n2);
            x = fma(un[u][q], cv[u][q], x);
          }
      }
    }
  }
  block_sum3(d2, n2, x, sh, tot);
  if (threadIdx.x == 0) {
    double* p = a.partials + blk * 4;
    p[0] = tot[0];
    p[1] = tot[1];
    p[2] = tot[2];
  }
}
template <typename T, int KPL>
__global__ __launch_bounds__(256) void k_metrics(MetArgs a) { k_metrics_body<T, KPL>(a, blockIdx.x, gridDim.x); }
template <typename T, int KPL>
__global__ __launch_bounds__(256) void k_metrics_b(const MetArgs* as, const BlockMap* map) {
  const BlockMap m = map[blockIdx.x];
  const MetArgs a = as[m.prob];
  k_metrics_body<T, KPL>(a, m.blk, m.nblk);
}


// One block: add the block partials in block order, the quadratic term
// <G_U, G_V>, then E and R into the history ring.
__device__ __forceinline__ void k_metrics_final_body(const MetArgs& a, int blk, int nblk) {
  const int nparts = a.nparts;
  __shared__ double sh[12];
  __shared__ double tot[3];
  __shared__ double totq[3];
  if (*a.status != 0) return;
  const int k = a.k;
  // every load in flight at once: thread 0's scalars, the partials (thread t
  // adds blocks t, t + 256, ... in order, then a fixed tree) and G_U, G_V
  int64_t it = 0;
  double nA2 = 0.0;
  int32_t cnt[4] = {0, 0, 0, 0};
  if (threadIdx.x == 0) {
    it = *a.it;
    nA2 = *a.nA2;
    cnt[0] = *a.nnz_u;
    cnt[1] = *a.nnz_v;
    cnt[2] = *a.dead_u;
    cnt[3] = *a.dead_v;
  }
  constexpr int kPer = (kMetricBlocks + 255) / 256;
  double pd[kPer][3];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int b = threadIdx.x + 256 * j;
#pragma unroll
    for (int f = 0; f < 3; ++f) pd[j][f] = b < nparts ? a.partials[b * 4 + f] : 0.0;
  }
  // conditioning indicator and gathered-entry counts: each diagonal entry
  // and counter slot is loaded by its own thread (k <= 128 < 256)
  const bool have_w = a.GU != nullptr && a.WU != nullptr && a.GV != nullptr && a.WV != nullptr;
  double vl0 = 1.0, vl1 = 1.0;
  if (have_w && threadIdx.x < k) {
    const int c = threadIdx.x;
    const double gu = a.GU[c * k + c], wu = a.WU[c * k + c];
    const double gv = a.GV[c * k + c], wv = a.WV[c * k + c];
    if (gu > 0.0) vl0 = gu * wu;
    if (gv > 0.0) vl1 = gv * wv;
  }
  unsigned long long gl = 0ull;
  if (a.gathered != nullptr && threadIdx.x < 2 * kGathSlots) {
    gl = a.gathered[threadIdx.x];
    a.gathered[threadIdx.x] = 0ull;
  }
  double d = 0.0, n = 0.0, x = 0.0;
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    d += pd[j][0];
    n += pd[j][1];
    x += pd[j][2];
  }
  block_sum3(d, n, x, sh, tot);
  __syncthreads();
  double q = 0.0;
  if (a.record && a.GU != nullptr) {
    for (int i0 = threadIdx.x; i0 < k * k; i0 += 8 * 256) {
      double gu[8], gv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = i0 + 256 * u;
        gu[u] = i < k * k ? a.GU[i] : 0.0;
        gv[u] = i < k * k ? a.GV[i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) q = fma(gu[u], gv[u], q);
    }
  }
  block_sum3(q, 0.0, 0.0, sh, totq);
  // largest diagonal product per factor (fmax over waves, then blocks of
  // the wave's lanes); gathered counts: lanes 0-15 (V half), 16-31 (U half)
  __shared__ double shv[8];
  __shared__ unsigned long long shg[2];
  for (int o = 32; o > 0; o >>= 1) {
    vl0 = fmax(vl0, __shfl_xor(vl0, o, 64));
    vl1 = fmax(vl1, __shfl_xor(vl1, o, 64));
  }
  for (int o = 8; o > 0; o >>= 1) gl += __shfl_xor(gl, o, 64);
  if (__lane_id() == 0) {
    shv[(threadIdx.x >> 6) * 2] = vl0;
    shv[(threadIdx.x >> 6) * 2 + 1] = vl1;
  }
  if (threadIdx.x == 0) shg[0] = gl;
  if (threadIdx.x == kGathSlots) shg[1] = gl;
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double D = tot[0], N = tot[1], X = tot[2];
  double* rec = a.ring + (it % kHistRing) * H_FIELDS;
  double E = __builtin_nan(""), R = __builtin_nan("");
  if (a.record) {
    R = sqrt(D) / sqrt(N);
    const double e2 = nA2 - 2.0 * X + totq[0];
    E = sqrt(e2 > 0.0 ? e2 : 0.0) / sqrt(nA2);
    if (!isfinite(R) || !isfinite(E)) atomicCAS(a.status, 0, static_cast<int32_t>(NMF_ERR_NONFINITE));
  }
  rec[H_E] = E;
  rec[H_R] = R;
  rec[H_NNZU] = static_cast<double>(cnt[0]);
  rec[H_NNZV] = static_cast<double>(cnt[1]);
  rec[H_DEADU] = static_cast<double>(cnt[2]);
  rec[H_DEADV] = static_cast<double>(cnt[3]);
  // conditioning of each Gram matrix: the largest G_cc (G^-1)_cc over live
  // topics (>= 1; 1 for orthogonal columns; it bounds the condition number
  // from below and grows without bound as a column approaches the span of
  // the others)
  double vif[2] = {__builtin_nan(""), __builtin_nan("")};
  if (have_w)
    for (int f = 0; f < 2; ++f)
      vif[f] = fmax(fmax(shv[f], shv[2 + f]), fmax(shv[4 + f], shv[6 + f]));
  rec[H_VIFU] = vif[0];
  rec[H_VIFV] = vif[1];
  const unsigned long long gs[2] = {shg[0], shg[1]};
  rec[H_GATHV] = static_cast<double>(gs[0]);
  rec[H_GATHU] = static_cast<double>(gs[1]);
  *a.it = it + 1;
}
__global__ __launch_bounds__(256) void k_metrics_final(MetArgs a) { k_metrics_final_body(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(256) void k_metrics_final_b(const MetArgs* as, const BlockMap* map) {
  const BlockMap m = map[blockIdx.x];
  const MetArgs a = as[m.prob];
  k_metrics_final_body(a, m.blk, m.nblk);
}


// <U, C> for dense U, C (n x k): block partials ...
template <typename T>
__global__ __launch_bounds__(256) void k_loss(int64_t count, const T* U, const T* C, double* partials) {
  __shared__ double sh[12];
  __shared__ double tot[3];
  const int P = gridDim.x;
  const int64_t lo = count * blockIdx.x / P;
  const int64_t hi = count * (blockIdx.x + 1) / P;
  double x = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256)
    x = fma(static_cast<double>(U[i]), static_cast<double>(C[i]), x);
  block_sum3(x, 0.0, 0.0, sh, tot);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot[0];
}

// ... then L = ||A||^2 - 2 <U, C> + <G_U, G_V> (one block; GU may be null
// for a plain sum of the partials into *out).
__global__ __launch_bounds__(256) void k_loss_final(const double* partials, int nparts, const double* GU,
                                                    const double* GV, int k, const double* nA2,
                                                    double* out) {
  __shared__ double sh[12];
  __shared__ double tot[3];
  double x = 0.0;
  for (int b = threadIdx.x; b < nparts; b += 256) x += partials[b];
  double q = 0.0;
  if (GU != nullptr)
    for (int i = threadIdx.x; i < k * k; i += 256) q = fma(GU[i], GV[i], q);
  block_sum3(q, x, 0.0, sh, tot);
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double X = tot[1];
  *out = GU != nullptr ? *nA2 - 2.0 * X + tot[0] : X;
}

// out = g * (-2 B + 2 F G) for dense F, B (rows x k), G (k x k, float64)
template <typename T, int KPL>
__global__ __launch_bounds__(256) void k_grad(const T* F, const T* B, const double* G,
                                              const double* g_scale, int64_t rows, int k, T* out) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* sG = reinterpret_cast<double*>(smem);
  for (int i = threadIdx.x; i < k * k; i += 256) sG[i] = G[i];
  __syncthreads();
  const double gs = g_scale ? *g_scale : 1.0;
  const int lane = lane_id();
  const int64_t wg = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int64_t nw = static_cast<int64_t>(gridDim.x) * 4;
  for (int64_t r = wg; r < rows; r += nw) {
    double acc[KPL];
#pragma unroll
    for (int q = 0; q < KPL; ++q) acc[q] = 0.0;
    for (int a = 0; a < k; ++a) {
      const double f = static_cast<double>(F[r * k + a]);
#pragma unroll
      for (int q = 0; q < KPL; ++q) {
        const int c = lane + 64 * q;
        if (c < k) acc[q] = fma(f, sG[a * k + c], acc[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
      const int c = lane + 64 * q;
      if (c < k) {
        const double b = static_cast<double>(B[r * k + c]);
        out[r * k + c] = static_cast<T>(gs * (2.0 * acc[q] - 2.0 * b));
      }
    }
  }
}

template <typename T, int KPL>
__global__ __launch_bounds__(256) void k_densify(const int32_t* slot, const T* dense, int ld, int64_t rows,
                                                 int k, T* out) {
  const int lane = lane_id();
  const int64_t wg = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int64_t nw = static_cast<int64_t>(gridDim.x) * 4;
  for (int64_t r = wg; r < rows; r += nw) {
    const int s = slot[r];
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
      const int c = lane + 64 * q;
      if (c < k) out[r * k + c] = s >= 0 ? dense[static_cast<int64_t>(s) * ld + c] : T(0);
    }
  }
}

template <typename T>
__global__ void k_check(const T* x, int64_t count, int32_t* flag) {
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t st = static_cast<int64_t>(gridDim.x) * blockDim.x;
  bool bad = false;
  for (int64_t i = i0; i < count; i += st) {
    const T v = x[i];
    if (!(v >= T(0)) || !isfinite(v)) bad = true;
  }
  if (__ballot(bad) != 0 && __lane_id() == 0) atomicOr(flag, 1);
}

template <typename T>
__global__ __launch_bounds__(256) void k_sumsq(const T* x, int64_t count, double* partials) {
  __shared__ double sh[12];
  __shared__ double tot[3];
  const int P = gridDim.x;
  const int64_t lo = count * blockIdx.x / P;
  const int64_t hi = count * (blockIdx.x + 1) / P;
  double s = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
    const double v = static_cast<double>(x[i]);
    s = fma(v, v, s);
  }
  block_sum3(s, 0.0, 0.0, sh, tot);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot[0];
}

// Documents per (topic, label) for the clustering accuracy of Eq. (acc):
// a document belongs to every topic with a stored entry in its row of V.
// Thread = document; integer atomics, so the counts are exact.
__global__ void k_topic_counts(const int32_t* row_ptr, const uint8_t* topic, const int32_t* labels, int64_t rows,
                               int32_t n_labels, uint32_t* counts) {
  const int64_t d = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (d >= rows) return;
  const int32_t lab = labels[d];
  if (lab < 0 || lab >= n_labels) return;
  for (int32_t e = row_ptr[d]; e < row_ptr[d + 1]; ++e) atomicAdd(&counts[topic[e] * n_labels + lab], 1u);
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t count) {
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t st = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = i0; i < count; i += st) p[i] = v;
}

int grid_for(int64_t work, int per_block, int cap) {
  int64_t b = (work + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return static_cast<int>(b);
}

}  // namespace

template <typename T>
hipError_t metrics(nmf_handle* h, const Factor& Unew, const Factor& Uold, const T* C, bool record) {
  MetArgs a{};
  a.n = h->n;
  a.k = h->k;
  a.slot_new = Unew.slot;
  a.slot_old = Uold.slot;
  a.dense_new = Unew.dense;
  a.ld = Unew.ld;
  a.dense_old = Uold.dense;
  a.C = C;
  a.partials = h->met.partials;
  a.GU = h->gU.G;
  a.GV = h->gV.G;
  a.WU = h->w_stale ? nullptr : h->gU.W;
  a.WV = h->w_stale ? nullptr : h->gV.W;
  a.gathered = h->met.gathered;
  a.nA2 = h->met.nA2;
  a.ring = h->met.ring;
  a.it = h->met.it;
  a.nnz_u = Unew.counts;
  a.nnz_v = h->V.counts;
  a.dead_u = h->gU.dead;
  a.dead_v = h->gV.dead;
  a.record = record ? 1 : 0;
  a.status = h->status;
  // one partial block per 64 rows, at most kMetricBlocks
  a.nparts = static_cast<int32_t>(std::max<int64_t>(1, std::min<int64_t>(kMetricBlocks, (h->n + 63) / 64)));
  const unsigned P = static_cast<unsigned>(a.nparts);
  hipError_t e = h->k > 64 ? launch_rec(h, k_metrics<T, 2>, k_metrics_b<T, 2>, P, 256, 0, a)
                           : launch_rec(h, k_metrics<T, 1>, k_metrics_b<T, 1>, P, 256, 0, a);
  if (e != hipSuccess) return e;
  return launch_rec(h, k_metrics_final, k_metrics_final_b, 1, 256, 0, a);
}

template <typename T>
hipError_t loss_dot(nmf_handle* h, const T* U, const T* C, const double* GU, const double* GV,
                    double* loss_out) {
  hipLaunchKernelGGL((k_loss<T>), dim3(kMetricBlocks), dim3(256), 0, h->stream, h->n * h->k, U, C,
                     h->met.loss_parts);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, h->stream, h->met.loss_parts, kMetricBlocks, GU, GV,
                     h->k, h->met.nA2, loss_out);
  return hipGetLastError();
}

template <typename T>
hipError_t grad_combine(nmf_handle* h, const T* F, const T* B, const double* G,
                        const double* g_scale, int64_t rows, T* out) {
  const int blocks = grid_for(rows, 4, h->num_cus * 8);
  const size_t lds = static_cast<size_t>(h->k) * h->k * sizeof(double);
  if (h->k > 64)
    hipLaunchKernelGGL((k_grad<T, 2>), dim3(blocks), dim3(256), lds, h->stream, F, B, G, g_scale, rows,
                       h->k, out);
  else
    hipLaunchKernelGGL((k_grad<T, 1>), dim3(blocks), dim3(256), lds, h->stream, F, B, G, g_scale, rows,
                       h->k, out);
  return hipGetLastError();
}

template <typename T>
hipError_t densify(nmf_handle* h, const Factor& F, T* out) {
  const int blocks = grid_for(F.rows, 4, h->num_cus * 8);
  if (h->k > 64)
    hipLaunchKernelGGL((k_densify<T, 2>), dim3(blocks), dim3(256), 0, h->stream, F.slot,
                       static_cast<const T*>(F.dense), F.ld, F.rows, h->k, out);
  else
    hipLaunchKernelGGL((k_densify<T, 1>), dim3(blocks), dim3(256), 0, h->stream, F.slot,
                       static_cast<const T*>(F.dense), F.ld, F.rows, h->k, out);
  return hipGetLastError();
}

template <typename T>
hipError_t check_input(nmf_handle* h, const T* x, int64_t count, int32_t* flag) {
  if (count == 0) return hipSuccess;
  const int blocks = grid_for(count, 256 * 8, h->num_cus * 8);
  hipLaunchKernelGGL((k_check<T>), dim3(blocks), dim3(256), 0, h->stream, x, count, flag);
  return hipGetLastError();
}

template <typename T>
hipError_t sum_squares(nmf_handle* h, const T* x, int64_t count, double* out) {
  hipLaunchKernelGGL((k_sumsq<T>), dim3(kMetricBlocks), dim3(256), 0, h->stream, x, count, h->met.loss_parts);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, h->stream, h->met.loss_parts, kMetricBlocks, nullptr,
                     nullptr, 0, nullptr, out);
  return hipGetLastError();
}

hipError_t topic_counts(nmf_handle* h, const Factor& F, const int32_t* labels, int32_t n_labels, uint32_t* counts) {
  const unsigned blocks = static_cast<unsigned>((F.rows + 255) / 256);
  hipLaunchKernelGGL(k_topic_counts, dim3(blocks), dim3(256), 0, h->stream, F.row_ptr, F.topic, labels, F.rows,
                     n_labels, counts);
  return hipGetLastError();
}

hipError_t fill_i32(hipStream_t s, int32_t* p, int32_t v, int64_t count) {
  if (count == 0) return hipSuccess;
  const int blocks = grid_for(count, 256 * 4, 1024);
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks), dim3(256), 0, s, p, v, count);
  return hipGetLastError();
}

#define NMF_INST(T)                                                                            \
  template hipError_t metrics<T>(nmf_handle*, const Factor&, const Factor&, const T*, bool);  \
  template hipError_t loss_dot<T>(nmf_handle*, const T*, const T*, const double*,             \
                                  const double*, double*);                                    \
  template hipError_t grad_combine<T>(nmf_handle*, const T*, const T*, const double*,         \
                                      const double*, int64_t, T*);                            \
  template hipError_t densify<T>(nmf_handle*, const Factor&, T*);                             \
  template hipError_t check_input<T>(nmf_handle*, const T*, int64_t, int32_t*);               \
  template hipError_t sum_squares<T>(nmf_handle*, const T*, int64_t, double*);
NMF_INST(float)
NMF_INST(double)
#undef NMF_INST

}  // namespace nmfk
