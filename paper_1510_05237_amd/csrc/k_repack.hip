// Sparse repack of a factor after selection (Algorithm 2, steps 2 and 4:
// the kept entries are stored as a sparse matrix, Section 3's sparse
// storage of U and V).
//
// Input: per-row keep masks (bit c of row r set when entry (r, c) survives)
// and the dense pre-selection matrix X holding the values.  Output, all in
// row order (so the result is deterministic whatever order the masks were
// set in):
//  * row-compressed sparse factor: row_ptr[rows+1], topic[], val[] with
//    topics ascending within a row;
//  * the SpMM gather cache: slot[r] (compact index of a nonempty row or -1),
//    rowid[slot], and every nonempty row expanded to k dense values;
//  * counts[0] = nnz, counts[1] = number of nonempty rows.
// Two kernels: per-block counts + (last block) scan of the block totals;
// then per-block local scan and write-out.  The masks are cleared as they
// are consumed.
#include "nmf_device.h"

namespace nmfk {

namespace {

constexpr int kScanRows = 256;  // rows per block, one per thread

struct RepackArgs {
  const void* X;
  int64_t rows;
  int32_t k;
  int32_t mw;
  uint32_t* mask;
  int32_t* part_cnt;  // [blocks]
  int32_t* part_ne;   // [blocks]
  int32_t* ticket;
  Factor F;
  const int32_t* status;
};

__device__ __forceinline__ int row_count(const uint32_t* mask, int64_t r, int mw) {
  int c = 0;
  for (int w = 0; w < mw; ++w) c += __popc(mask[r * mw + w]);
  return c;
}

__global__ __launch_bounds__(256) void k_scan_count(RepackArgs a) {
  __shared__ int tmp[8];
  __shared__ int last;
  __shared__ int seg_tmp[8];
  if (*a.status != 0) return;
  const int64_t r = static_cast<int64_t>(blockIdx.x) * kScanRows + threadIdx.x;
  int cnt = 0;
  if (r < a.rows) cnt = row_count(a.mask, r, a.mw);
  const int ne = cnt > 0;
  int tot_c, tot_n;
  block_excl_scan_256(cnt, tmp, &tot_c);
  block_excl_scan_256(ne, tmp, &tot_n);
  if (threadIdx.x == 0) {
    a.part_cnt[blockIdx.x] = tot_c;
    a.part_ne[blockIdx.x] = tot_n;
  }
  fence_release();
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(a.ticket, 1) == static_cast<int>(gridDim.x) - 1;
  __syncthreads();
  if (!last) return;
  fence_acquire();
  // exclusive scan of the block totals: each thread scans one contiguous
  // segment, the segment sums are scanned across the block
  const int P = gridDim.x;
  const int seg = (P + 255) / 256;
  const int s0 = threadIdx.x * seg;
  int sc = 0, sn = 0;
  for (int i = s0; i < s0 + seg && i < P; ++i) {
    sc += __hip_atomic_load(&a.part_cnt[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    sn += __hip_atomic_load(&a.part_ne[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  int all_c, all_n;
  int oc = block_excl_scan_256(sc, seg_tmp, &all_c);
  int on = block_excl_scan_256(sn, seg_tmp, &all_n);
  for (int i = s0; i < s0 + seg && i < P; ++i) {
    const int vc = __hip_atomic_load(&a.part_cnt[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int vn = __hip_atomic_load(&a.part_ne[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    a.part_cnt[i] = oc;
    a.part_ne[i] = on;
    oc += vc;
    on += vn;
  }
  if (threadIdx.x == 0) {
    a.F.counts[0] = all_c;
    a.F.counts[1] = all_n;
    a.F.row_ptr[a.rows] = all_c;
    *a.ticket = 0;
  }
}

template <typename T, int KPL>
__global__ __launch_bounds__(256) void k_build(RepackArgs a) {
  __shared__ int tmp[8];
  __shared__ uint32_t smask[kScanRows * 4];
  __shared__ int s_rp[kScanRows];
  __shared__ int s_slot[kScanRows];
  if (*a.status != 0) return;
  const int mw = a.mw;
  const int k = a.k;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kScanRows;
  const int64_t r = r0 + threadIdx.x;
  int cnt = 0;
  if (r < a.rows) {
    for (int w = 0; w < mw; ++w) {
      const uint32_t m = a.mask[r * mw + w];
      smask[threadIdx.x * 4 + w] = m;
      cnt += __popc(m);
    }
  }
  const int ne = cnt > 0;
  int tc, tn;
  const int lc = block_excl_scan_256(cnt, tmp, &tc);
  const int ln = block_excl_scan_256(ne, tmp, &tn);
  const int rp = a.part_cnt[blockIdx.x] + lc;
  const int sl = ne ? a.part_ne[blockIdx.x] + ln : -1;
  if (r < a.rows) {
    a.F.row_ptr[r] = rp;
    a.F.slot[r] = sl;
    if (ne) a.F.rowid[sl] = static_cast<int32_t>(r);
    for (int w = 0; w < mw; ++w) a.mask[r * mw + w] = 0u;
  }
  s_rp[threadIdx.x] = rp;
  s_slot[threadIdx.x] = sl;
  __syncthreads();
  // write-out: each wave takes 64 rows; lanes = topics for every nonempty row
  const int lane = lane_id();
  const int wv = threadIdx.x >> 6;
  const T* __restrict__ X = static_cast<const T*>(a.X);
  T* __restrict__ dense = static_cast<T*>(a.F.dense);
  T* __restrict__ fval = static_cast<T*>(a.F.val);
  const int lr = wv * 64 + lane;
  uint64_t todo = __ballot(s_slot[lr] >= 0);
  while (todo) {
    const int b = __ffsll(static_cast<long long>(todo)) - 1;
    todo &= todo - 1;
    const int i = wv * 64 + b;
    const int64_t row = r0 + i;
    const int s = s_slot[i];
    const int base = s_rp[i];
    uint32_t mwords[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) mwords[w] = w < mw ? smask[i * 4 + w] : 0u;
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
      const int c = lane + 64 * q;
      if (c < k) {
        uint32_t word = 0;
        int below = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          if (w == (c >> 5))
            word = mwords[w];
          else if (w < (c >> 5))
            below += __popc(mwords[w]);
        }
        const bool bit = (word >> (c & 31)) & 1u;
        const T v = bit ? X[row * k + c] : T(0);
        dense[static_cast<int64_t>(s) * k + c] = v;
        if (bit) {
          below += __popc(word & ((1u << (c & 31)) - 1u));
          fval[base + below] = v;
          a.F.topic[base + below] = static_cast<uint8_t>(c);
        }
      }
    }
  }
}

}  // namespace

template <typename T>
hipError_t repack(nmf_handle* h, const T* X, int64_t rows, const Factor& out_f) {
  RepackArgs a{};
  a.X = X;
  a.rows = rows;
  a.k = h->k;
  a.mw = h->mask_words;
  a.mask = h->sel.mask;
  const int blocks = static_cast<int>((rows + kScanRows - 1) / kScanRows);
  a.part_cnt = h->sel.scan_part;
  a.part_ne = h->sel.scan_part + blocks + 1;
  a.ticket = h->sel.ticket + 1;
  a.F = out_f;
  a.status = h->status;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan_count, dim3(blocks), dim3(256), 0, h->stream, a);
  if (h->k > 64)
    hipLaunchKernelGGL((k_build<T, 2>), dim3(blocks), dim3(256), 0, h->stream, a);
  else
    hipLaunchKernelGGL((k_build<T, 1>), dim3(blocks), dim3(256), 0, h->stream, a);
  return hipGetLastError();
}

template hipError_t repack<float>(nmf_handle*, const float*, int64_t, const Factor&);
template hipError_t repack<double>(nmf_handle*, const double*, int64_t, const Factor&);

}  // namespace nmfk
