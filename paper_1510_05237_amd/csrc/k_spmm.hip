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
// Work items (built once per orientation of A): up to RG consecutive short
// rows with at most kChunk nonzeros in total, or one kChunk-long piece of a
// long (Zipf-heavy) row.  Per item, per 64 nonzeros (lanes span the item's
// rows):
//  * lanes = nonzeros: coalesced loads of (col, a) and one 8-byte gather of
//    the factor row's metadata {where, how many entries};
//  * factor rows with at most `sparse_row` entries are gathered entry by entry
//    (one {value, topic} load per entry, lanes still = nonzeros) and each
//    product is added into the wave's LDS accumulator at (row, topic).  One
//    wave owns the accumulator and LDS executes a wave's instructions in
//    order, so the sums are reproducible;
//  * denser factor rows are queued and then read as whole k-wide rows from
//    the compact dense copy of the factor, lanes = topics: one coalesced load
//    and one FMA per lane per row, eight rows in flight;
//  * the epilogue multiplies the item's raw row sums by W (float64, in LDS),
//    clamps at zero, rounds to T and stores whole rows.
// Pieces of long rows store their raw sums; k_spmm_heavy adds them in piece
// order and runs the same epilogue.
#include "nmf_device.h"

namespace nmfk {

namespace {

constexpr int kWaves = 8;  // waves per block

template <typename T, int RG>
__host__ __device__ inline size_t spmm_per_wave(int k) {
  const int kpad = (k + 3) & ~3;
  return 64 * (2 * sizeof(int32_t) + sizeof(T)) + static_cast<size_t>(RG) * kpad * sizeof(T);
}

template <typename T, int RG>
size_t spmm_lds_bytes(int k, bool raw) {
  const size_t w = raw ? 0 : static_cast<size_t>(k) * k * sizeof(double);
  return w + kWaves * spmm_per_wave<T, RG>(k);
}

struct SpmmArgs {
  const int64_t* rowptr;
  const int32_t* col;
  const void* val;
  const WorkItem* items;
  int32_t n_items;
  const int32_t* heavy_row;
  const int32_t* heavy_nchunks;
  const int32_t* heavy_part0;
  int32_t n_heavy;
  void* partials;
  const int2* meta;   // factor row metadata {dense row or first entry, entry count}
  int32_t sparse_row;  // rows with at most this many entries are gathered entry by entry
  const void* ents;   // stored factor entries {value, topic}
  const void* F;      // compact dense factor rows (or the dense input)
  const double* W;
  void* X;
  void* C;
  int32_t k;
  int32_t* status;
};

struct WaveLds {
  int32_t* q_off;
  int32_t* q_row;
  void* q_a;
  void* tile;
};

template <typename T, int RG>
__device__ __forceinline__ WaveLds wave_lds(unsigned char* smem, int k, bool raw, int wv) {
  unsigned char* base = smem + (raw ? 0 : static_cast<size_t>(k) * k * sizeof(double)) +
                        wv * spmm_per_wave<T, RG>(k);
  WaveLds w;
  w.q_off = reinterpret_cast<int32_t*>(base);
  w.q_row = reinterpret_cast<int32_t*>(base + 64 * sizeof(int32_t));
  w.q_a = base + 128 * sizeof(int32_t);
  w.tile = base + 128 * sizeof(int32_t) + 64 * sizeof(T);
  return w;
}

// Adds the nonzeros [p0, p1) of an item (rows bounded by rb[0..nrows]) times
// F into the LDS tile: tile[topic * RG + row].
template <typename T, int KPL, int RG, bool DENSE_IN>
__device__ __forceinline__ void accumulate(const SpmmArgs& a, int64_t p0, int64_t p1, const int64_t* rb,
                                           int nrows, const WaveLds& w) {
  const int lane = lane_id();
  const int k = a.k;
  const int32_t* __restrict__ col = a.col;
  const T* __restrict__ val = static_cast<const T*>(a.val);
  const T* __restrict__ F = static_cast<const T*>(a.F);
  const FactorEnt<T>* __restrict__ ents = static_cast<const FactorEnt<T>*>(a.ents);
  T* tile = static_cast<T*>(w.tile);
  T* q_a = static_cast<T*>(w.q_a);
  T acc[KPL];
#pragma unroll
  for (int q = 0; q < KPL; ++q) acc[q] = T(0);
  int cur_r = 0;
  for (int64_t base = p0; base < p1; base += 64) {
    const int64_t p = base + lane;
    const bool valid = p < p1;
    int32_t j = 0;
    T av = T(0);
    if (valid) {
      j = col[p];
      av = val[p];
    }
    int r = 0;
#pragma unroll
    for (int i = 1; i < RG; ++i) r += (i < nrows && p >= rb[i]) ? 1 : 0;
    int32_t x = 0, cnt = 0;
    if (valid) {
      if (DENSE_IN) {
        x = j;
        cnt = k;
      } else {
        const int2 m = a.meta[j];
        x = m.x;
        cnt = m.y;
      }
    }
    const bool sparse = !DENSE_IN && cnt > 0 && cnt <= a.sparse_row;
    // sparse factor rows: entry e of every lane's row per round; lanes start
    // at a rotated entry so that one round rarely adds twice to one topic
    const int rot = sparse ? lane % cnt : 0;
    for (int e = 0; __ballot(sparse && e < cnt) != 0; ++e) {
      if (sparse && e < cnt) {
        int idx = e + rot;
        if (idx >= cnt) idx -= cnt;
        const FactorEnt<T> en = ents[x + idx];
        atomicAdd(&tile[en.t * RG + r], av * en.v);
      }
    }
    // dense factor rows: queue, then one k-wide row per hit, lanes = topics
    const bool hit = DENSE_IN ? valid : cnt > a.sparse_row;
    const uint64_t bal = __ballot(hit);
    const int nh = __popcll(bal);
    if (nh == 0) continue;
    if (hit) {
      const int pos = lane_rank(bal);
      w.q_off[pos] = x * k;
      w.q_row[pos] = r;
      q_a[pos] = av;
    }
    // pad the queue to a multiple of 8 with zero-weight copies of row 0 of F
    // (same row index as the last hit), so the loop below needs no guards
    const int last_lane = 63 - __builtin_clzll(bal);
    const int r_last = __shfl(r, last_lane, 64);
    const int nh8 = (nh + 7) & ~7;
    if (lane < nh8 - nh) {
      w.q_off[nh + lane] = 0;
      w.q_row[nh + lane] = r_last;
      q_a[nh + lane] = T(0);
    }
    for (int h = 0; h < nh8; h += 8) {
      int32_t o[8], rr[8];
      T aa[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        o[u] = w.q_off[h + u];
        rr[u] = w.q_row[h + u];
        aa[u] = q_a[h + u];
      }
      T f[8][KPL];
#pragma unroll
      for (int q = 0; q < KPL; ++q) {
        const int c = lane + 64 * q;
        const int cc = c < k ? c : 0;
#pragma unroll
        for (int u = 0; u < 8; ++u) f[u][q] = F[o[u] + cc];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (rr[u] != cur_r) {  // rows are queued in order: flush on a change
#pragma unroll
          for (int q = 0; q < KPL; ++q) {
            const int c = lane + 64 * q;
            if (c < k) tile[c * RG + cur_r] += acc[q];
            acc[q] = T(0);
          }
          cur_r = rr[u];
        }
#pragma unroll
        for (int q = 0; q < KPL; ++q) acc[q] = fma(aa[u], f[u][q], acc[q]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < KPL; ++q) {
    const int c = lane + 64 * q;
    if (c < k) tile[c * RG + cur_r] += acc[q];
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
    double wv[KPL];
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
      const int c = lane + 64 * q;
      wv[q] = c < k ? sW[rr * k + c] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < RG; ++r) {
      const double b = static_cast<double>(tile[rr * RG + r]);
#pragma unroll
      for (int q = 0; q < KPL; ++q) out[r][q] = fma(b, wv[q], out[r][q]);
    }
  }
#pragma unroll
  for (int r = 0; r < RG; ++r) {
    if (r < nrows) {
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
}

template <typename T, int KPL, int RG>
__device__ __forceinline__ void clear_tile(T* tile, int k) {
  const int lane = lane_id();
#pragma unroll
  for (int q = 0; q < KPL; ++q) {
    const int c = lane + 64 * q;
    if (c < k) {
#pragma unroll
      for (int r = 0; r < RG; ++r) tile[c * RG + r] = T(0);
    }
  }
}

template <typename T, int KPL, int RG, bool RAW, bool STORE_C, bool DENSE_IN>
__global__ __launch_bounds__(512) void k_spmm(SpmmArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (*a.status != 0) return;
  const int k = a.k;
  const int lane = lane_id();
  const int wv = threadIdx.x >> 6;
  double* sW = reinterpret_cast<double*>(smem);
  const WaveLds w = wave_lds<T, RG>(smem, k, RAW, wv);
  T* tile = static_cast<T*>(w.tile);
  if (!RAW) {
    for (int i = threadIdx.x; i < k * k; i += blockDim.x) sW[i] = a.W[i];
  }
  __syncthreads();

  const int nw = gridDim.x * kWaves;
  for (int it = blockIdx.x * kWaves + wv; it < a.n_items; it += nw) {
    const WorkItem wi = a.items[it];
    clear_tile<T, KPL, RG>(tile, k);
    if (wi.heavy < 0) {
      const int nrows = wi.r1 - wi.r0;
      if (nrows > RG) {  // a plan built for another row group: refuse, never overrun the tile
        if (lane == 0) atomicCAS(a.status, 0, static_cast<int32_t>(NMF_ERR_DEVICE));
        continue;
      }
      int64_t rb[RG + 1];
#pragma unroll
      for (int i = 0; i <= RG; ++i) rb[i] = a.rowptr[wi.r0 + (i < nrows ? i : nrows)];
      accumulate<T, KPL, RG, DENSE_IN>(a, rb[0], rb[nrows], rb, nrows, w);
      epilogue<T, KPL, RG, RAW, STORE_C>(a, tile, sW, nrows, wi.r0);
    } else {
      int64_t rb[RG + 1];
#pragma unroll
      for (int i = 0; i <= RG; ++i) rb[i] = i == 0 ? wi.p0 : wi.p1;
      accumulate<T, KPL, RG, DENSE_IN>(a, wi.p0, wi.p1, rb, 1, w);
      T* part = static_cast<T*>(a.partials);
#pragma unroll
      for (int q = 0; q < KPL; ++q) {
        const int c = lane + 64 * q;
        if (c < k) part[static_cast<int64_t>(wi.part) * k + c] = tile[c * RG];
      }
    }
  }
}

// Long rows: add the pieces' raw sums in piece order, then the epilogue.
template <typename T, int KPL, int RG, bool RAW, bool STORE_C>
__global__ __launch_bounds__(512) void k_spmm_heavy(SpmmArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (*a.status != 0) return;
  const int k = a.k;
  const int lane = lane_id();
  const int wv = threadIdx.x >> 6;
  double* sW = reinterpret_cast<double*>(smem);
  const WaveLds w = wave_lds<T, RG>(smem, k, RAW, wv);
  T* tile = static_cast<T*>(w.tile);
  if (!RAW) {
    for (int i = threadIdx.x; i < k * k; i += blockDim.x) sW[i] = a.W[i];
  }
  __syncthreads();
  const T* part = static_cast<const T*>(a.partials);
  const int nw = gridDim.x * kWaves;
  for (int hh = blockIdx.x * kWaves + wv; hh < a.n_heavy; hh += nw) {
    const int nch = a.heavy_nchunks[hh];
    const int p0 = a.heavy_part0[hh];
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
      const int c = lane + 64 * q;
      if (c < k) {
        T s = T(0);
        int j = 0;
        for (; j + 8 <= nch; j += 8) {  // eight loads in flight, added in order
          T v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) v[u] = part[static_cast<int64_t>(p0 + j + u) * k + c];
#pragma unroll
          for (int u = 0; u < 8; ++u) s += v[u];
        }
        for (; j < nch; ++j) s += part[static_cast<int64_t>(p0 + j) * k + c];
        tile[c * RG] = s;
      }
    }
    epilogue<T, KPL, RG, RAW, STORE_C>(a, tile, sW, 1, a.heavy_row[hh]);
  }
}

template <typename T, int KPL, int RG, bool RAW, bool STORE_C, bool DENSE_IN>
hipError_t launch(nmf_handle* h, const SpmmArgs& a) {
  const size_t lds = spmm_lds_bytes<T, RG>(a.k, RAW);
  int per_cu = static_cast<int>((160 * 1024) / (lds + 512));
  if (per_cu < 1) per_cu = 1;
  if (per_cu > 4) per_cu = 4;
  if (a.n_items > 0) {
    int blocks = (a.n_items + kWaves - 1) / kWaves;
    const int cap = h->num_cus * per_cu;
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL((k_spmm<T, KPL, RG, RAW, STORE_C, DENSE_IN>), dim3(blocks), dim3(64 * kWaves), lds,
                       h->stream, a);
  }
  if (a.n_heavy > 0) {
    int blocks = (a.n_heavy + kWaves - 1) / kWaves;
    const int cap = h->num_cus * per_cu;
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL((k_spmm_heavy<T, KPL, RG, RAW, STORE_C>), dim3(blocks), dim3(64 * kWaves), lds,
                       h->stream, a);
  }
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t spmm(nmf_handle* h, const Plan& p, const Factor& F, const double* W, T* X, T* C,
                bool raw, const T* dense_in, int sparse_row) {
  SpmmArgs a{};
  a.rowptr = p.rowptr;
  a.col = p.col;
  a.val = p.val;
  a.items = p.items;
  a.n_items = p.n_items;
  a.heavy_row = p.heavy_row;
  a.heavy_nchunks = p.heavy_nchunks;
  a.heavy_part0 = p.heavy_part0;
  a.n_heavy = p.n_heavy;
  a.partials = p.partials;
  a.meta = dense_in ? nullptr : F.meta;
  a.sparse_row = sparse_row;
  a.ents = F.packed;
  a.F = dense_in ? static_cast<const void*>(dense_in) : static_cast<const void*>(F.dense);
  a.W = W;
  a.X = X;
  a.C = C;
  a.k = h->k;
  a.status = h->status;
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
                                float*, bool, const float*, int);
template hipError_t spmm<double>(nmf_handle*, const Plan&, const Factor&, const double*, double*,
                                 double*, bool, const double*, int);

}  // namespace nmfk
