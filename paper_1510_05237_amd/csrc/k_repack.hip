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
//  * what the SpMM gathers: per row {compact dense row when the row has more
//    than `sparse_row` entries, else its first entry; entry count}, per entry
//    {value, topic}, and every nonempty row expanded to k dense values
//    (slot[r] = its compact index or -1, rowid[slot] = r);
//  * counts[0] = nnz, counts[1] = number of nonempty rows.
// Two kernels: per-block totals, then per-block offsets (sum of the earlier
// block totals), a local scan and the write-out.  The masks are cleared as
// they are consumed.
#include "nmf_device.h"

namespace nmfk {

namespace {

constexpr int kRowsPerThread = 1;
constexpr int kScanRows = 256 * kRowsPerThread;  // rows per block
constexpr int kBuildInFlight = 8;  // nonempty rows whose value loads are in flight together

struct RepackArgs {
  const void* X;
  int64_t rows;
  int32_t k;
  int32_t mw;
  uint32_t* mask;
  int32_t* part_cnt;  // [blocks]
  int32_t* part_ne;   // [blocks]
  Factor F;
  int32_t sparse_row;
  const int32_t* status;
};

__device__ __forceinline__ int row_count(const uint32_t* mask, int64_t r, int mw) {
  int c = 0;
  for (int w = 0; w < mw; ++w) c += __popc(mask[r * mw + w]);
  return c;
}

__device__ __forceinline__ int block_sum_256(int v, int* tmp) {
  int t;
  block_excl_scan_256(v, tmp, &t);
  return t;
}

__device__ __forceinline__ void k_scan_count_body(const RepackArgs& a, int blk, int nblk) {
  __shared__ int tmp[8];
  if (*a.status != 0) return;
  const int64_t r0 = static_cast<int64_t>(blk) * kScanRows + threadIdx.x * kRowsPerThread;
  int cnt = 0, ne = 0;
#pragma unroll
  for (int i = 0; i < kRowsPerThread; ++i) {
    const int64_t r = r0 + i;
    if (r < a.rows) {
      const int c = row_count(a.mask, r, a.mw);
      cnt += c;
      ne += c > 0;
    }
  }
  const int tc = block_sum_256(cnt, tmp);
  const int tn = block_sum_256(ne, tmp);
  if (threadIdx.x == 0) {
    a.part_cnt[blk] = tc;
    a.part_ne[blk] = tn;
  }
}
__global__ __launch_bounds__(256) void k_scan_count(RepackArgs a) { k_scan_count_body(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(256) void k_scan_count_b(const RepackArgs* as, const BlockMap* map) {
  const BlockMap m = map[blockIdx.x];
  const RepackArgs a = as[m.prob];
  k_scan_count_body(a, m.blk, m.nblk);
}


template <typename T, int KPL>
__device__ __forceinline__ void k_build_body(const RepackArgs& a, int blk, int nblk) {
  __shared__ int tmp[8];
  __shared__ uint32_t smask[kScanRows * 4];
  __shared__ int s_rp[kScanRows];
  __shared__ int s_slot[kScanRows];
  if (*a.status != 0) return;
  const int mw = a.mw;
  const int k = a.k;
  const int tid = threadIdx.x;
  // offsets of this block: the totals of all earlier blocks
  int oc = 0, on = 0;
  for (int b = tid; b < static_cast<int>(blk); b += 256) {
    oc += a.part_cnt[b];
    on += a.part_ne[b];
  }
  const int off_c = block_sum_256(oc, tmp);
  const int off_n = block_sum_256(on, tmp);
  const int64_t rb0 = static_cast<int64_t>(blk) * kScanRows;
  const int64_t r0 = rb0 + tid * kRowsPerThread;
  int cnt[kRowsPerThread];
  int tc = 0, tn = 0;
#pragma unroll
  for (int i = 0; i < kRowsPerThread; ++i) {
    const int64_t r = r0 + i;
    const int li = tid * kRowsPerThread + i;
    int c = 0;
    if (r < a.rows) {
      for (int w = 0; w < mw; ++w) {
        const uint32_t m = a.mask[r * mw + w];
        smask[li * 4 + w] = m;
        c += __popc(m);
      }
    }
    cnt[i] = c;
    tc += c;
    tn += c > 0;
  }
  int bc, bn;
  int lc = block_excl_scan_256(tc, tmp, &bc);
  int ln = block_excl_scan_256(tn, tmp, &bn);
  lc += off_c;
  ln += off_n;
#pragma unroll
  for (int i = 0; i < kRowsPerThread; ++i) {
    const int64_t r = r0 + i;
    const int li = tid * kRowsPerThread + i;
    const bool ne = cnt[i] > 0;
    const int sl = ne ? ln : -1;
    // row table word of rows [32 w, 32 w + 32) (kScanRows is a multiple of
    // 64, so a word is one half of a wave): its nonempty bits, and the
    // nonempty rows before it
    const uint64_t bw = __ballot(ne);
    if ((r & 31) == 0 && r < a.rows)
      a.F.rowtab[r >> 5] = make_int2(static_cast<int>(static_cast<uint32_t>(bw >> (lane_id() & 32))), ln);
    s_rp[li] = lc;
    s_slot[li] = sl;
    if (r < a.rows) {
      a.F.row_ptr[r] = lc;
      a.F.slot[r] = sl;
      a.F.meta[r] = make_int2(cnt[i] > a.sparse_row ? sl : lc, cnt[i]);
      if (ne) a.F.rowid[sl] = static_cast<int32_t>(r);
      for (int w = 0; w < mw; ++w) a.mask[r * mw + w] = 0u;
    }
    lc += cnt[i];
    ln += ne ? 1 : 0;
  }
  if (blk == nblk - 1 && tid == 255) {
    // lc / ln now hold the totals over every block
    a.F.counts[0] = lc;
    a.F.counts[1] = ln;
    a.F.row_ptr[a.rows] = lc;
  }
  __syncthreads();
  // write-out: each wave takes 64 rows at a time; lanes = topics for every
  // nonempty row
  const int lane = lane_id();
  const int wv = tid >> 6;
  const int ld = a.F.ld;
  const T* __restrict__ X = static_cast<const T*>(a.X);
  T* __restrict__ dense = static_cast<T*>(a.F.dense);
  T* __restrict__ fval = static_cast<T*>(a.F.val);
  FactorEnt<T>* __restrict__ ents = static_cast<FactorEnt<T>*>(a.F.packed);
  for (int g = wv * 64; g < kScanRows; g += 256) {
    uint64_t todo = __ballot(s_slot[g + lane] >= 0);
    while (todo) {
      int ib[kBuildInFlight];
      int nb = 0;
#pragma unroll
      for (int u = 0; u < kBuildInFlight; ++u) {
        ib[u] = -1;
        if (todo) {
          ib[u] = g + __ffsll(static_cast<long long>(todo)) - 1;
          todo &= todo - 1;
          ++nb;
        }
      }
      T xv[kBuildInFlight][KPL];
#pragma unroll
      for (int u = 0; u < kBuildInFlight; ++u)
#pragma unroll
        for (int q = 0; q < KPL; ++q) {
          const int c = lane + 64 * q;
          xv[u][q] = (ib[u] >= 0 && c < k) ? X[(rb0 + ib[u]) * k + c] : T(0);
        }
#pragma unroll
      for (int u = 0; u < kBuildInFlight; ++u) {
        if (ib[u] < 0) continue;
        const int i = ib[u];
        const int s = s_slot[i];
        const int base = s_rp[i];
        uint32_t mwords[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) mwords[w] = w < mw ? smask[i * 4 + w] : 0u;
#pragma unroll
        for (int q = 0; q < KPL; ++q) {
          const int c = lane + 64 * q;
          if (c < ld) {  // columns k..ld-1 of the dense copy are padding: no bit is set there
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
            const T v = bit ? xv[u][q] : T(0);
            dense[static_cast<int64_t>(s) * ld + c] = v;
            if (bit) {
              below += __popc(word & ((1u << (c & 31)) - 1u));
              fval[base + below] = v;
              a.F.topic[base + below] = static_cast<uint8_t>(c);
              FactorEnt<T> en;
              en.v = v;
              en.t = static_cast<uint32_t>(c);
              ents[base + below] = en;
            }
          }
        }
      }
      (void)nb;
    }
  }
}
template <typename T, int KPL>
__global__ __launch_bounds__(256) void k_build(RepackArgs a) { k_build_body<T, KPL>(a, blockIdx.x, gridDim.x); }
template <typename T, int KPL>
__global__ __launch_bounds__(256) void k_build_b(const RepackArgs* as, const BlockMap* map) {
  const BlockMap m = map[blockIdx.x];
  const RepackArgs a = as[m.prob];
  k_build_body<T, KPL>(a, m.blk, m.nblk);
}


}  // namespace

template <typename T>
hipError_t repack(nmf_handle* h, const T* X, int64_t rows, const Factor& out_f, int sparse_row) {
  RepackArgs a{};
  a.sparse_row = sparse_row;
  a.X = X;
  a.rows = rows;
  a.k = h->k;
  a.mw = h->mask_words;
  a.mask = h->sel.mask;
  const int blocks = static_cast<int>((rows + kScanRows - 1) / kScanRows);
  a.part_cnt = h->sel.scan_part;
  a.part_ne = h->sel.scan_part + blocks + 1;
  a.F = out_f;
  a.status = h->status;
  hipError_t e = launch_rec(h, k_scan_count, k_scan_count_b, blocks, 256, 0, a);
  if (e != hipSuccess) return e;
  if (h->k > 64) return launch_rec(h, k_build<T, 2>, k_build_b<T, 2>, blocks, 256, 0, a);
  return launch_rec(h, k_build<T, 1>, k_build_b<T, 1>, blocks, 256, 0, a);
}

template hipError_t repack<float>(nmf_handle*, const float*, int64_t, const Factor&, int);
template hipError_t repack<double>(nmf_handle*, const double*, int64_t, const Factor&, int);

}  // namespace nmfk
