// Fused sparse product + least-squares solve + projection of one ALS
// half-step (Algorithm 2, steps 1 and 3):
//
//   out_r = max(0, (sum_{p in row r} a_p F[col_p]) W)      W = (F^T F)^-1
//
// where the rows r are documents and F = U for the V half (A^T U), and the
// rows are terms and F = V for the U half (A V).  The sparse product
// accumulates in the working type T (float32 for the FP32 workloads); the
// k x k solve of the epilogue is float64.
//
// Mapping (wave64):
//  * each wave owns one work item: up to kRowGroup short rows, or one
//    kChunk-long piece of a long (Zipf-heavy) row;
//  * phase A, lanes = 64 consecutive nonzeros: coalesced loads of (col, a),
//    gather of the factor row's compact slot, ballot of the hits (rows of F
//    that are not empty), hits appended to a per-wave LDS queue;
//  * phase B, lanes = topics: for every queued hit one coalesced k-wide load
//    of the factor row and one FMA per lane;
//  * the epilogue multiplies the raw sums of a group of rows by W (held in
//    LDS as float64), clamps at zero, rounds to T and stores coalesced rows.
// Long rows: every chunk writes a partial sum; the last chunk to arrive
// (device-scope ticket) adds the partials in chunk order, so the result does
// not depend on scheduling.
#include "nmf_device.h"

namespace nmfk {

namespace {

template <typename T, int RG>
__host__ __device__ inline size_t spmm_per_wave(int k) {
  const int kpad = (k + 3) & ~3;
  return 64 * sizeof(int32_t) + 64 * sizeof(T) + static_cast<size_t>(RG) * kpad * sizeof(T);
}

template <typename T, int RG>
size_t spmm_lds_bytes(int k, bool raw) {
  const size_t w = raw ? 0 : static_cast<size_t>(k) * k * sizeof(double);
  return w + 4 * spmm_per_wave<T, RG>(k);
}

struct SpmmArgs {
  const int64_t* rowptr;
  const int32_t* col;
  const void* val;
  const WorkItem* items;
  int32_t n_items;
  int32_t* heavy_ticket;
  const int32_t* heavy_nchunks;
  const int32_t* heavy_part0;
  void* partials;
  const int32_t* slot;  // gather slot per factor row (nullptr: dense input)
  const void* F;        // compact dense factor rows (or the dense input)
  const double* W;
  void* X;
  void* C;
  int32_t k;
  const int32_t* status;
  int32_t* status_w;
};

template <typename T, int KPL>
__device__ __forceinline__ void accumulate(const SpmmArgs& a, int64_t p0, int64_t p1, T* acc,
                                           int32_t* q_off, T* q_a, bool dense_in) {
  const int lane = lane_id();
  const int32_t* __restrict__ col = a.col;
  const T* __restrict__ val = static_cast<const T*>(a.val);
  const T* __restrict__ F = static_cast<const T*>(a.F);
  const int k = a.k;
  for (int64_t base = p0; base < p1; base += 64) {
    const int64_t p = base + lane;
    const bool valid = p < p1;
    int32_t j = 0;
    T av = T(0);
    if (valid) {
      j = col[p];
      av = val[p];
    }
    int32_t s = -1;
    if (valid) s = dense_in ? j : a.slot[j];
    const bool hit = s >= 0;
    const uint64_t bal = __ballot(hit);
    if (hit) {
      const int pos = lane_rank(bal);
      q_off[pos] = s * k;
      q_a[pos] = av;
    }
    const int nh = __popcll(bal);
    int h = 0;
    // four hits per step keep four gathers in flight; the sums are still
    // formed in hit order
    for (; h + 4 <= nh; h += 4) {
      int32_t o0 = q_off[h], o1 = q_off[h + 1], o2 = q_off[h + 2], o3 = q_off[h + 3];
      T a0 = q_a[h], a1 = q_a[h + 1], a2 = q_a[h + 2], a3 = q_a[h + 3];
#pragma unroll
      for (int q = 0; q < KPL; ++q) {
        const int c = lane + 64 * q;
        if (c < k) {
          T f0 = F[o0 + c], f1 = F[o1 + c], f2 = F[o2 + c], f3 = F[o3 + c];
          acc[q] = fma(a0, f0, acc[q]);
          acc[q] = fma(a1, f1, acc[q]);
          acc[q] = fma(a2, f2, acc[q]);
          acc[q] = fma(a3, f3, acc[q]);
        }
      }
    }
    for (; h < nh; ++h) {
      const int32_t o = q_off[h];
      const T av2 = q_a[h];
#pragma unroll
      for (int q = 0; q < KPL; ++q) {
        const int c = lane + 64 * q;
        if (c < k) acc[q] = fma(av2, F[o + c], acc[q]);
      }
    }
  }
}

// tile layout: tile[rr * RG + r] = raw sum of row r, topic rr.
template <typename T, int KPL, int RG, bool RAW, bool STORE_C>
__device__ __forceinline__ void epilogue(const SpmmArgs& a, const T* tile, const double* sW,
                                         int nrows, int32_t r0) {
  const int lane = lane_id();
  const int k = a.k;
  T* __restrict__ X = static_cast<T*>(a.X);
  if (RAW) {
    for (int r = 0; r < nrows; ++r) {
#pragma unroll
      for (int q = 0; q < KPL; ++q) {
        const int c = lane + 64 * q;
        if (c < k) X[static_cast<int64_t>(r0 + r) * k + c] = tile[c * RG + r];
      }
    }
    return;
  }
  double out[RG][KPL];
#pragma unroll
  for (int r = 0; r < RG; ++r)
#pragma unroll
    for (int q = 0; q < KPL; ++q) out[r][q] = 0.0;
  for (int rr = 0; rr < k; ++rr) {
    double w[KPL];
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
      const int c = lane + 64 * q;
      w[q] = c < k ? sW[rr * k + c] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < RG; ++r) {
      const double b = static_cast<double>(tile[rr * RG + r]);
#pragma unroll
      for (int q = 0; q < KPL; ++q) out[r][q] = fma(b, w[q], out[r][q]);
    }
  }
  for (int r = 0; r < nrows; ++r) {
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
      const int c = lane + 64 * q;
      if (c < k) {
        const double x = out[r][q];
        const int64_t o = static_cast<int64_t>(r0 + r) * k + c;
        X[o] = static_cast<T>(x > 0.0 ? x : 0.0);
        if (STORE_C) static_cast<T*>(a.C)[o] = tile[c * RG + r];
      }
    }
  }
}

template <typename T, int KPL, int RG, bool RAW, bool STORE_C, bool DENSE_IN>
__global__ __launch_bounds__(256) void k_spmm(SpmmArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (*a.status != 0) return;
  const int k = a.k;
  const int lane = lane_id();
  const int wv = threadIdx.x >> 6;
  double* sW = reinterpret_cast<double*>(smem);
  unsigned char* wbase = smem + (RAW ? 0 : static_cast<size_t>(k) * k * sizeof(double));
  unsigned char* mine = wbase + wv * spmm_per_wave<T, RG>(k);
  int32_t* q_off = reinterpret_cast<int32_t*>(mine);
  T* q_a = reinterpret_cast<T*>(mine + 64 * sizeof(int32_t));
  T* tile = reinterpret_cast<T*>(mine + 64 * sizeof(int32_t) + 64 * sizeof(T));
  if (!RAW) {
    for (int i = threadIdx.x; i < k * k; i += blockDim.x) sW[i] = a.W[i];
  }
  __syncthreads();

  const int nw = gridDim.x * 4;
  for (int it = blockIdx.x * 4 + wv; it < a.n_items; it += nw) {
    const WorkItem wi = a.items[it];
    if (wi.heavy < 0) {
      const int nrows = wi.r1 - wi.r0;
      if (nrows > RG) {  // a plan built for another row group: refuse, never overrun the tile
        if (lane == 0) atomicCAS(a.status_w, 0, static_cast<int32_t>(NMF_ERR_DEVICE));
        continue;
      }
      for (int r = 0; r < nrows; ++r) {
        T acc[KPL];
#pragma unroll
        for (int q = 0; q < KPL; ++q) acc[q] = T(0);
        accumulate<T, KPL>(a, a.rowptr[wi.r0 + r], a.rowptr[wi.r0 + r + 1], acc, q_off, q_a,
                           DENSE_IN);
#pragma unroll
        for (int q = 0; q < KPL; ++q) {
          const int c = lane + 64 * q;
          if (c < k) tile[c * RG + r] = acc[q];
        }
      }
      epilogue<T, KPL, RG, RAW, STORE_C>(a, tile, sW, nrows, wi.r0);
    } else {
      T acc[KPL];
#pragma unroll
      for (int q = 0; q < KPL; ++q) acc[q] = T(0);
      accumulate<T, KPL>(a, wi.p0, wi.p1, acc, q_off, q_a, DENSE_IN);
      T* part = static_cast<T*>(a.partials);
#pragma unroll
      for (int q = 0; q < KPL; ++q) {
        const int c = lane + 64 * q;
        if (c < k) part[static_cast<int64_t>(wi.part) * k + c] = acc[q];
      }
      fence_release();
      int tk = 0;
      if (lane == 0) tk = atomicAdd(&a.heavy_ticket[wi.heavy], 1);
      tk = bcast_i32(tk, 0);
      const int nch = a.heavy_nchunks[wi.heavy];
      if (tk == nch - 1) {
        fence_acquire();
        const int32_t p0 = a.heavy_part0[wi.heavy];
#pragma unroll
        for (int q = 0; q < KPL; ++q) acc[q] = T(0);
        for (int j = 0; j < nch; ++j) {
#pragma unroll
          for (int q = 0; q < KPL; ++q) {
            const int c = lane + 64 * q;
            if (c < k) {
              const T v = __builtin_nontemporal_load(&part[static_cast<int64_t>(p0 + j) * k + c]);
              acc[q] += v;
            }
          }
        }
        if (lane == 0) a.heavy_ticket[wi.heavy] = 0;
#pragma unroll
        for (int q = 0; q < KPL; ++q) {
          const int c = lane + 64 * q;
          if (c < k) tile[c * RG + 0] = acc[q];
        }
        epilogue<T, KPL, RG, RAW, STORE_C>(a, tile, sW, 1, wi.r0);
      }
    }
  }
}

template <typename T, int KPL, int RG, bool RAW, bool STORE_C, bool DENSE_IN>
hipError_t launch(nmf_handle* h, const SpmmArgs& a) {
  const size_t lds = spmm_lds_bytes<T, RG>(a.k, RAW);
  auto kern = k_spmm<T, KPL, RG, RAW, STORE_C, DENSE_IN>;
  if (a.n_items == 0) return hipSuccess;
  // several resident blocks per CU; the LDS footprint decides how many fit
  int per_cu = static_cast<int>((160 * 1024) / (lds + 1024));
  if (per_cu < 1) per_cu = 1;
  if (per_cu > 8) per_cu = 8;
  int blocks = (a.n_items + 3) / 4;
  const int cap = h->num_cus * per_cu;
  if (blocks > cap) blocks = cap;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), lds, h->stream, a);
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t spmm(nmf_handle* h, const Plan& p, const Factor& F, const double* W, T* X, T* C,
                bool raw, const T* dense_in) {
  SpmmArgs a{};
  a.rowptr = p.rowptr;
  a.col = p.col;
  a.val = p.val;
  a.items = p.items;
  a.n_items = p.n_items;
  a.heavy_ticket = p.heavy_ticket;
  a.heavy_nchunks = p.heavy_nchunks;
  a.heavy_part0 = p.heavy_part0;
  a.partials = p.partials;
  a.slot = dense_in ? nullptr : F.slot;
  a.F = dense_in ? static_cast<const void*>(dense_in) : static_cast<const void*>(F.dense);
  a.W = W;
  a.X = X;
  a.C = C;
  a.k = h->k;
  a.status = h->status;
  a.status_w = h->status;
  const bool two = h->k > 64;
  const bool dense = dense_in != nullptr;
  if (raw) {
    if (dense)
      return two ? launch<T, 2, 4, true, false, true>(h, a) : launch<T, 1, 8, true, false, true>(h, a);
    return two ? launch<T, 2, 4, true, false, false>(h, a) : launch<T, 1, 8, true, false, false>(h, a);
  }
  if (C != nullptr)
    return two ? launch<T, 2, 4, false, true, false>(h, a) : launch<T, 1, 8, false, true, false>(h, a);
  return two ? launch<T, 2, 4, false, false, false>(h, a) : launch<T, 1, 8, false, false, false>(h, a);
}

template hipError_t spmm<float>(nmf_handle*, const Plan&, const Factor&, const double*, float*,
                                float*, bool, const float*);
template hipError_t spmm<double>(nmf_handle*, const Plan&, const Factor&, const double*, double*,
                                 double*, bool, const double*);

}  // namespace nmfk
