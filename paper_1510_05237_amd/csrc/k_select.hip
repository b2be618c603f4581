// Per-column top-t selection of a clamped pre-selection matrix X (rows x k,
// row-major): Section 2's rule (keep the t largest entries) applied to every
// column separately as in Section 4.  Exactly min(t, #positive) entries
// survive per column; among entries equal to the t-th largest value the
// lowest rows win, i.e. the kept set is the t largest under the order
// (value descending, row ascending).  Only strictly positive entries are
// candidates (zeros are never stored).
//
// Radix select on the IEEE bits of the positive values (they order like
// unsigned integers):
//  1. hist:    per-column histogram of the first digit (the 8 bits under
//              the sign bit: the exponent for float32), block-private in LDS,
//              flushed with integer atomics; then one block picks, per
//              column, the digit b1 holding the t-th largest entry.
//  2. collect: one pass over X: entries whose digit is above b1 are kept
//              (bit set in the per-row keep mask); entries with digit b1 are
//              appended to the column's candidate list.
//  3. refine:  one block per column narrows the candidates digit by digit
//              (remaining value bits, then the row bits for the tie-break),
//              keeping whole digits above the threshold, until at most 64
//              remain; one wave then ranks those by comparing all pairs.
// Only integer atomics are used, so the kept set does not depend on
// scheduling; the row-compressed factor is then built in row order from the
// keep masks (k_repack.hip).
//
// Whole-matrix form (Algorithm 2 as printed, Section 2): the same passes with
// one histogram, one threshold and one candidate list for all entries; a
// candidate's "row" is its row-major flat index r * k + c, so ties at the
// t-th largest value go to the lowest (row, column) in row-major order.
#include <algorithm>

#include "nmf_device.h"

namespace nmfk {

namespace {

constexpr int kRowsPerBlock = kSelBlockRows;  // rows of X per hist/collect block
constexpr int kPadBins = kBins + 1;
constexpr int kFinish = 64;  // candidates ranked directly by one wave
constexpr int kHistRows = 8;                       // rows in flight per wave in k_hist
constexpr int kHistThreads = 1024;                 // k_hist block: 16 waves, one block per CU
constexpr int kCollectRows = kRowsPerBlock / 4;    // k_collect: every row of a wave's share at once
static_assert(kRowsPerBlock == 4 * kCollectRows, "k_collect: each of the 4 waves reads kCollectRows rows");

struct SelArgs {
  const void* X;
  int64_t rows;
  int32_t k;
  int32_t mw;  // mask words per row
  int64_t t;
  int32_t mode;
  int32_t hist_rows;  // rows of X per hist block
  uint32_t* hist;
  ColSel* sel;
  int32_t* cand_cnt;  // column c, sub-list s at cand_cnt[(c * kSelSub + s) * kCntStride]
  int64_t sub;        // entries per sub-list
  void* candA;
  void* candB;
  int64_t stride;
  uint32_t* mask;
  int32_t* ticket;
  int32_t* status;
  int32_t flat_k;  // whole-matrix form: k (candidates carry r * k + c); 0 per column
};

template <typename T, int KPL, bool WHOLE>
__device__ __forceinline__ void k_hist_body(const SelArgs& a, int blk, int nblk) {
  using KO = KeyOf<T>;
  extern __shared__ __align__(16) unsigned char smem[];
  uint32_t* h = reinterpret_cast<uint32_t*>(smem);  // [k][kPadBins] (whole matrix: [1][kPadBins])
  if (*a.status != 0) return;
  const int k = a.k;
  const int nh = WHOLE ? 1 : k;
  for (int i = threadIdx.x; i < nh * kPadBins; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const int lane = lane_id();
  const int wv = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const T* __restrict__ X = static_cast<const T*>(a.X);
  const int64_t r_begin = static_cast<int64_t>(blk) * a.hist_rows;
  int64_t r_end = r_begin + a.hist_rows;
  if (r_end > a.rows) r_end = a.rows;
  // kHistRows rows per wave per step keep that many loads in flight
  for (int64_t r = r_begin + wv; r < r_end; r += nw * kHistRows) {
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
      const int c = lane + 64 * q;
      if (c < k) {
        typename KO::K key[kHistRows];
#pragma unroll
        for (int u = 0; u < kHistRows; ++u) key[u] = r + nw * u < r_end ? KO::key(X[(r + nw * u) * k + c]) : 0;
#pragma unroll
        for (int u = 0; u < kHistRows; ++u)
          if (key[u] != 0) atomicAdd(&h[(WHOLE ? 0 : c * kPadBins) + top_digit<T>(key[u])], 1u);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nh * kBins; i += blockDim.x) {
    const int c = i / kBins, d = i - c * kBins;
    const uint32_t v = h[c * kPadBins + d];
    if (v) atomicAdd(&a.hist[i], v);
  }
}
template <typename T, int KPL, bool WHOLE>
__global__ __launch_bounds__(kHistThreads) void k_hist(SelArgs a) { k_hist_body<T, KPL, WHOLE>(a, blockIdx.x, gridDim.x); }
template <typename T, int KPL, bool WHOLE>
__global__ __launch_bounds__(kHistThreads) void k_hist_b(const SelArgs* as, const BlockMap* map) {
  const BlockMap m = map[blockIdx.x];
  const SelArgs a = as[m.prob];
  k_hist_body<T, KPL, WHOLE>(a, m.blk, m.nblk);
}


// The threshold digit of every column from the full histogram, one wave per
// column; the histogram is cleared for the next use.
__device__ __forceinline__ void k_pick_body(const SelArgs& a, int blk, int nblk) {
  if (*a.status != 0) return;
  const int k = a.k;
  const int lane = lane_id();
  const int nw = nblk * (blockDim.x >> 6);
  for (int c = blk * (blockDim.x >> 6) + (threadIdx.x >> 6); c < k; c += nw) {
    uint4* hc = reinterpret_cast<uint4*>(a.hist + static_cast<size_t>(c) * kBins);
    const uint4 q = hc[lane];
    hc[lane] = make_uint4(0u, 0u, 0u, 0u);
    const uint32_t v[4] = {q.x, q.y, q.z, q.w};
    int64_t npos = static_cast<int64_t>(q.x) + q.y + q.z + q.w;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) npos += __shfl_xor(npos, d, 64);
    ColSel s;
    s.npos = static_cast<int32_t>(npos);
    s.all = (a.mode == NMF_MODE_NONE || npos <= a.t) ? 1 : 0;
    s.b1 = -1;
    s.need = 0;
    if (!s.all) {
      int64_t above = 0;
      s.b1 = wave_pick_bin(v, a.t, &above);
      s.need = static_cast<int32_t>(a.t - above);
    }
    if (lane == 0) a.sel[c] = s;
  }
}
__global__ __launch_bounds__(256) void k_pick(SelArgs a) { k_pick_body(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(256) void k_pick_b(const SelArgs* as, const BlockMap* map) {
  const BlockMap m = map[blockIdx.x];
  const SelArgs a = as[m.prob];
  k_pick_body(a, m.blk, m.nblk);
}


// Candidates are staged per (wave, column): a lane owns its column's slots
// in its wave's region (at most kCollectRows, one per row the wave reads), so
// staging needs no atomics.  Block b then appends its regions, in wave order,
// to sub-list b % kSelSub of each column (of the one list in the
// whole-matrix form) with one atomic per column; spreading the blocks over
// kSelSub counters keeps them from queueing on one address.  k_refine
// concatenates the sub-lists.
template <typename T, int KPL, bool WHOLE>
__device__ __forceinline__ void k_collect_body(const SelArgs& a, int blk, int nblk) {
  using KO = KeyOf<T>;
  using C = Cand<T>;
  __shared__ int32_t lcnt[4][kMaxK];  // staged entries per (wave, column)
  __shared__ int32_t lbase[kMaxK];
  __shared__ int32_t loff[4 * kMaxK];  // whole-matrix form: offset of each (wave, column) region
  __shared__ int tmp[8];
  extern __shared__ __align__(16) unsigned char smem[];
  C* stage = reinterpret_cast<C*>(smem);  // [wave][slot < kCollectRows][k]
  if (*a.status != 0) return;
  const int k = a.k;
  const int lane = lane_id();
  const int wv = threadIdx.x >> 6;
  ColSel s[KPL];
  int cnt[KPL];
#pragma unroll
  for (int q = 0; q < KPL; ++q) {
    const int c = lane + 64 * q;
    s[q] = c < k ? a.sel[WHOLE ? 0 : c] : ColSel{0, 0, 1, 0};
    cnt[q] = 0;
  }
  const T* __restrict__ X = static_cast<const T*>(a.X);
  const int64_t r_begin = static_cast<int64_t>(blk) * kRowsPerBlock;
  int64_t r_end = r_begin + kRowsPerBlock;
  if (r_end > a.rows) r_end = a.rows;
  C* wstage = stage + static_cast<size_t>(wv) * kCollectRows * k;
  // the wave reads every fourth row of the block (kCollectRows of them), all
  // loads in flight at once
  const int64_t r4 = r_begin + wv;
  typename KO::K keys[kCollectRows][KPL];
#pragma unroll
  for (int u = 0; u < kCollectRows; ++u)
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
      const int c = lane + 64 * q;
      keys[u][q] = (c < k && r4 + 4 * u < r_end) ? KO::key(X[(r4 + 4 * u) * k + c]) : 0;
    }
#pragma unroll
  for (int u = 0; u < kCollectRows; ++u) {
    const int64_t r = r4 + 4 * u;
    if (r >= r_end) break;
    uint64_t keep_bits[KPL];
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
      const int c = lane + 64 * q;
      bool keep = false;
      const auto key = keys[u][q];
      if (key != 0) {  // zero for lanes past k
        const int d = top_digit<T>(key);
        keep = s[q].all || d > s[q].b1;
        if (!s[q].all && d == s[q].b1) {
          C cd;
          cd.key = key;
          cd.row = WHOLE ? static_cast<uint32_t>(r * k + c) : static_cast<uint32_t>(r);
          wstage[cnt[q] * k + c] = cd;
          ++cnt[q];
        }
      }
      keep_bits[q] = __ballot(keep);
    }
    // the wave owns row r: its keep-mask words (zero until now: the repack
    // clears them after use) are plain stores; the threshold bin's picks are
    // added by k_refine after this kernel
    if (lane < a.mw) {
      const int q = lane >> 1;
      const uint64_t b = keep_bits[q < KPL ? q : 0];
      const uint32_t word = (lane & 1) ? static_cast<uint32_t>(b >> 32) : static_cast<uint32_t>(b);
      if (word) a.mask[r * a.mw + lane] = word;
    }
  }
#pragma unroll
  for (int q = 0; q < KPL; ++q) {
    const int c = lane + 64 * q;
    if (c < k) lcnt[wv][c] = cnt[q];
  }
  __syncthreads();
  C* __restrict__ out = static_cast<C*>(a.candA);
  if (WHOLE) {
    // one list: regions in (wave, column) order after one offset for the block
    int v = 0;
    for (int f = 2 * threadIdx.x; f < 2 * threadIdx.x + 2; ++f)
      if (f < 4 * k) v += lcnt[f / k][f % k];
    int tot;
    int o = block_excl_scan_256(v, tmp, &tot);
    for (int f = 2 * threadIdx.x; f < 2 * threadIdx.x + 2; ++f)
      if (f < 4 * k) {
        loff[f] = o;
        o += lcnt[f / k][f % k];
      }
    if (threadIdx.x == 0) lbase[0] = tot ? atomicAdd(&a.cand_cnt[(blk % kSelSub) * kCntStride], tot) : 0;
    __syncthreads();
    C* mine = out + (blk % kSelSub) * a.sub * k + lbase[0];
    for (int f = wv; f < 4 * k; f += 4) {
      const int w = f / k, c = f % k;
      const int n = lcnt[w][c];
      for (int i = lane; i < n; i += 64) mine[loff[f] + i] = stage[(static_cast<size_t>(w) * kCollectRows + i) * k + c];
    }
    return;
  }
  for (int c = threadIdx.x; c < k; c += 256) {
    const int n = lcnt[0][c] + lcnt[1][c] + lcnt[2][c] + lcnt[3][c];
    lbase[c] = n ? atomicAdd(&a.cand_cnt[(c * kSelSub + blk % kSelSub) * kCntStride], n) : 0;
  }
  __syncthreads();
  // per column, lanes span every (wave, slot) pair
  for (int c = wv; c < k; c += 4) {
    const int n0 = lcnt[0][c], n1 = lcnt[1][c], n2 = lcnt[2][c];
    for (int j = lane; j < 4 * kCollectRows; j += 64) {
      const int w = j / kCollectRows, i = j - w * kCollectRows;
      const int before = (w > 0 ? n0 : 0) + (w > 1 ? n1 : 0) + (w > 2 ? n2 : 0);
      if (i < lcnt[w][c])
        out[static_cast<int64_t>(c) * a.stride + (blk % kSelSub) * a.sub + lbase[c] + before + i] =
            stage[(static_cast<size_t>(w) * kCollectRows + i) * k + c];
    }
  }
}
template <typename T, int KPL, bool WHOLE>
__global__ __launch_bounds__(256) void k_collect(SelArgs a) { k_collect_body<T, KPL, WHOLE>(a, blockIdx.x, gridDim.x); }
template <typename T, int KPL, bool WHOLE>
__global__ __launch_bounds__(256) void k_collect_b(const SelArgs* as, const BlockMap* map) {
  const BlockMap m = map[blockIdx.x];
  const SelArgs a = as[m.prob];
  k_collect_body<T, KPL, WHOLE>(a, m.blk, m.nblk);
}


// digit of a candidate under the compound order; `kb` value bits and `rb`
// row bits remain below the digits already fixed
template <typename T>
__device__ __forceinline__ int cand_digit(const Cand<T>& cd, int kb, int rb, int* width) {
  if (kb > 0) {
    const int w = kb < 8 ? kb : 8;
    *width = w;
    return static_cast<int>((cd.key >> (kb - w)) & ((1u << w) - 1));
  }
  const int w = rb < 8 ? rb : 8;
  *width = w;
  const uint32_t nr = ~cd.row;
  return static_cast<int>((nr >> (rb - w)) & ((1u << w) - 1));
}

__device__ __forceinline__ void mark(uint32_t* mask, int mw, uint32_t row, int c) {
  atomicOr(&mask[static_cast<int64_t>(row) * mw + (c >> 5)], 1u << (c & 31));
}

// Keep a refined candidate of list c (whole-matrix form: decode its flat index).
__device__ __forceinline__ void mark_cand(const SelArgs& a, uint32_t row, int c) {
  if (a.flat_k > 0)
    mark(a.mask, a.mw, row / static_cast<uint32_t>(a.flat_k), static_cast<int>(row % static_cast<uint32_t>(a.flat_k)));
  else
    mark(a.mask, a.mw, row, c);
}

template <typename T>
__device__ __forceinline__ void k_refine_body(const SelArgs& a, int blk, int nblk) {
  using C = Cand<T>;
  __shared__ uint32_t h[kBins];
  __shared__ int s_bin, s_need, s_n, s_cnt;
  __shared__ int s_off[kSelSub + 1];
  const int c = blk;
  const int tid = threadIdx.x;
  // the sub-list counters: read, then cleared for the next selection (also
  // after an error, so that no later selection appends past a sub-list)
  int32_t* cnt = a.cand_cnt + static_cast<int64_t>(c) * kSelSub * kCntStride;
  if (tid == 0) {
    int o = 0;
    for (int q = 0; q < kSelSub; ++q) {
      s_off[q] = o;
      o += cnt[q * kCntStride];
    }
    s_off[kSelSub] = o;
  }
  __syncthreads();
  if (tid < kSelSub) cnt[tid * kCntStride] = 0;
  if (*a.status != 0) return;
  const ColSel s = a.sel[c];
  if (s.all || s.need <= 0) return;
  int need = s.need;
  int n = s_off[kSelSub];
  // concatenate the sub-lists (sub-list q holds entries [s_off[q], s_off[q+1])
  // of the whole list), four entries in flight per thread
  C* lists = static_cast<C*>(a.candA) + static_cast<int64_t>(c) * a.stride;
  C* src = static_cast<C*>(a.candB) + static_cast<int64_t>(c) * a.stride;
  C* dst = lists;
  {
    const int64_t sub = a.flat_k > 0 ? a.sub * a.flat_k : a.sub;
    const int NT = blockDim.x;
    for (int i0 = tid; i0 < n; i0 += 4 * NT) {
      C v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + u * NT;
        if (i < n) {
          int q = 0;
#pragma unroll
          for (int x = 1; x < kSelSub; ++x) q += i >= s_off[x] ? 1 : 0;
          v[u] = lists[q * sub + (i - s_off[q])];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (i0 + u * NT < n) src[i0 + u * NT] = v[u];
    }
    __syncthreads();
  }
  int kb = KeyOf<T>::bits - 9;
  int rb = 32;
  while (n > kFinish && (kb > 0 || rb > 0)) {
    const int NT = blockDim.x;
    for (int i = tid; i < kBins; i += NT) h[i] = 0;
    __syncthreads();
    int width;
    for (int i = tid; i < n; i += 4 * NT) {
      C v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (i + NT * u < n) v[u] = src[i + NT * u];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (i + NT * u < n) atomicAdd(&h[cand_digit<T>(v[u], kb, rb, &width)], 1u);
    }
    __syncthreads();
    if (tid < 64) {
      const uint32_t v[4] = {h[4 * tid], h[4 * tid + 1], h[4 * tid + 2], h[4 * tid + 3]};
      int64_t above = 0;
      const int bin = wave_pick_bin(v, need, &above);
      if (tid == 0) {
        s_bin = bin;
        s_need = need - static_cast<int>(above);
        s_n = static_cast<int>(h[bin]);
        s_cnt = 0;
      }
    }
    __syncthreads();
    const int bin = s_bin;
    // each wave takes 256 consecutive entries per step (four per lane)
    for (int i0 = (tid >> 6) * 256; i0 < n; i0 += 4 * NT) {
      C cd[4];
      int d[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + 64 * u + __lane_id();
        d[u] = -1;
        if (i < n) {
          cd[u] = src[i];
          d[u] = cand_digit<T>(cd[u], kb, rb, &width);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (d[u] > bin) mark_cand(a, cd[u].row, c);
        // one LDS atomic per wave for the equal-digit entries
        const uint64_t eq = __ballot(d[u] == bin);
        int base = 0;
        if (__lane_id() == 0 && eq) base = atomicAdd(&s_cnt, __popcll(eq));
        base = __shfl(base, 0, 64);
        if (d[u] == bin) dst[base + lane_rank(eq)] = cd[u];
      }
    }
    if (kb > 0)
      kb -= kb < 8 ? kb : 8;
    else
      rb -= rb < 8 ? rb : 8;
    need = s_need;
    n = s_n;
    C* tmp = src;
    src = dst;
    dst = tmp;
    __syncthreads();
  }
  // finish: rank the remaining candidates under the compound order (value
  // descending, row ascending) on one wave, lane = candidate, and keep the
  // first `need`.  Distinct rows make every compound key distinct, so the
  // ranks are distinct; once every digit is fixed at most one candidate is
  // left, so more than kFinish means a corrupted list, which is reported
  // instead of read past.
  if (n > kFinish) {
    if (tid == 0) atomicCAS(a.status, 0, static_cast<int32_t>(NMF_ERR_DEVICE));
    return;
  }
  if (tid < 64) {
    C me;
    me.key = 0;
    me.row = 0xFFFFFFFFu;
    if (tid < n) me = src[tid];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      C o;
      o.key = __shfl(me.key, j, 64);
      o.row = __shfl(me.row, j, 64);
      rank += cand_before<T>(o, me) ? 1 : 0;
    }
    if (tid < n && rank < need) mark_cand(a, me.row, c);
  }
}
template <typename T>
__global__ __launch_bounds__(1024) void k_refine(SelArgs a) { k_refine_body<T>(a, blockIdx.x, gridDim.x); }
template <typename T>
__global__ __launch_bounds__(1024) void k_refine_b(const SelArgs* as, const BlockMap* map) {
  const BlockMap m = map[blockIdx.x];
  const SelArgs a = as[m.prob];
  k_refine_body<T>(a, m.blk, m.nblk);
}


template <typename T, int KPL, bool WHOLE>
hipError_t run(nmf_handle* h, SelArgs& a) {
  const unsigned blocks = static_cast<unsigned>((a.rows + kRowsPerBlock - 1) / kRowsPerBlock);
  // one 16-wave histogram block per compute unit the problem has: enough
  // rows each that the flush of the block histograms stays small
  const int64_t want = static_cast<int64_t>(h->hist_cus);
  a.hist_rows = static_cast<int32_t>(std::max<int64_t>(kRowsPerBlock, (a.rows + want - 1) / want));
  const unsigned hblocks = static_cast<unsigned>((a.rows + a.hist_rows - 1) / a.hist_rows);
  const size_t hbytes = static_cast<size_t>(WHOLE ? 1 : a.k) * kPadBins * sizeof(uint32_t);
  const size_t stage = static_cast<size_t>(a.k) * kRowsPerBlock * sizeof(Cand<T>);
  hipError_t e;
  // the whole-matrix form picks and refines one list: k = 1 for those passes
  SelArgs one = a;
  if (WHOLE) {
    one.k = 1;
    one.flat_k = a.k;
  }
  if ((e = launch_rec(h, k_hist<T, KPL, WHOLE>, k_hist_b<T, KPL, WHOLE>, hblocks, kHistThreads, hbytes, a)) !=
      hipSuccess)
    return e;
  if ((e = launch_rec(h, k_pick, k_pick_b, (one.k + 3) / 4, 256, 0, one)) != hipSuccess) return e;
  if ((e = launch_rec(h, k_collect<T, KPL, WHOLE>, k_collect_b<T, KPL, WHOLE>, blocks, 256, stage, a)) != hipSuccess)
    return e;
  return launch_rec(h, k_refine<T>, k_refine_b<T>, one.k, 1024, 0, one);
}

}  // namespace

template <typename T>
hipError_t select_topt(nmf_handle* h, const T* X, int64_t rows, int64_t t, int mode,
                       const Factor& out_f) {
  (void)out_f;
  SelArgs a{};
  a.X = X;
  a.rows = rows;
  a.k = h->k;
  a.mw = h->mask_words;
  a.t = t;
  a.mode = mode;
  a.hist = h->sel.hist;
  a.sel = h->sel.sel;
  a.cand_cnt = h->sel.cand_cnt;
  a.sub = h->sel.cand_sub;
  a.candA = h->sel.candA;
  a.candB = h->sel.candB;
  a.stride = h->sel.cand_stride;
  a.mask = h->sel.mask;
  a.ticket = h->sel.ticket;
  a.status = h->status;
  a.flat_k = 0;
  if (mode == NMF_MODE_WHOLE) {
    a.stride = h->sel.cand_stride * h->k;  // the one list may use every list's room
    return h->k > 64 ? run<T, 2, true>(h, a) : run<T, 1, true>(h, a);
  }
  return h->k > 64 ? run<T, 2, false>(h, a) : run<T, 1, false>(h, a);
}

// Keep every nonzero entry (used to load given factors).
template <typename T, int KPL>
__global__ __launch_bounds__(256) void k_mark_nonzero(const T* X, int64_t rows, int k, int mw,
                                                      uint32_t* mask) {
  const int lane = lane_id();
  const int64_t r = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (r >= rows) return;
  uint64_t bits[KPL];
#pragma unroll
  for (int q = 0; q < KPL; ++q) {
    const int c = lane + 64 * q;
    bits[q] = __ballot(c < k && X[r * k + c] != T(0));
  }
  if (lane < mw) {
    const int q = lane >> 1;
    const uint64_t b = bits[q < KPL ? q : 0];
    mask[r * mw + lane] = (lane & 1) ? static_cast<uint32_t>(b >> 32) : static_cast<uint32_t>(b);
  }
}

template <typename T>
hipError_t mark_nonzero(nmf_handle* h, const T* X, int64_t rows) {
  const int blocks = static_cast<int>((rows + 3) / 4);
  if (blocks == 0) return hipSuccess;
  if (h->k > 64)
    hipLaunchKernelGGL((k_mark_nonzero<T, 2>), dim3(blocks), dim3(256), 0, h->stream, X, rows, h->k,
                       h->mask_words, h->sel.mask);
  else
    hipLaunchKernelGGL((k_mark_nonzero<T, 1>), dim3(blocks), dim3(256), 0, h->stream, X, rows, h->k,
                       h->mask_words, h->sel.mask);
  return hipGetLastError();
}

template hipError_t select_topt<float>(nmf_handle*, const float*, int64_t, int64_t, int, const Factor&);
template hipError_t select_topt<double>(nmf_handle*, const double*, int64_t, int64_t, int, const Factor&);
template hipError_t mark_nonzero<float>(nmf_handle*, const float*, int64_t);
template hipError_t mark_nonzero<double>(nmf_handle*, const double*, int64_t);

}  // namespace nmfk
