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
// long (Zipf-heavy) row.  One wave owns an item and its accumulator (in LDS).
// Per step of 64 nonzeros (lanes span the item's rows; the wide form takes
// two per lane):
//  * lanes = nonzeros: coalesced loads of (col, a) and one 8-byte gather of
//    the factor row's metadata {where, how many entries};
//  * factor rows with at most `sparse_row` entries are gathered entry by entry
//    (one {value, topic} load per entry, lanes still = nonzeros); no
//    floating-point atomics add their products: an item of one row appends
//    them to a list in a fixed order that is summed with lanes = topics (see
//    scan_list), an item of several rows adds each at (row, topic) of the
//    accumulator in claim sub-rounds where the lowest lane goes first (see
//    ordered_add);
//  * a raw product may cover a window of the factor's columns (sequential
//    ALS), with a bitmap in LDS of the factor rows that store anything in it:
//    the other nonzeros are skipped before their metadata gather;
//  * denser factor rows are queued in row order and then read whole from the
//    compact dense copy of the factor, lanes = topics, eight rows in flight;
//    the running sums for the current row stay in registers and go to the
//    accumulator when the row changes;
//  * the epilogue multiplies the item's raw row sums by W (float64, in LDS),
//    clamps at zero, rounds to T and stores whole rows.
// Pieces of long rows store their raw sums; k_spmm_heavy adds them in piece
// order and runs the same epilogue.  One wave owns each accumulator and LDS
// executes a wave's instructions in order, so the sums are reproducible.
#include <algorithm>

#include "nmf_device.h"

namespace nmfk {

namespace {

constexpr int kWaves = 16;  // most waves per block (fewer when W and the wave buffers exceed the LDS)
constexpr size_t kLdsBytes = 160 * 1024;
// Dense-row queue: one step's hits (64, or 128 in the wide form) padded to
// whole batches of 8.
template <bool WIDE>
constexpr int queue_len() {
  return WIDE ? 136 : 64;
}

// Each wave's accumulator has a row slot for all 64 * KPL lanes of every
// topic slice (RG * 64 * KPL = 512 entries), so lanes past k can add their
// zero-weight sums without a guard and the row-change test stays uniform.
constexpr int kTileEntries = 512;

// Dense factor rows in flight per wave in the queue loop (per topic slice:
// halved when each lane holds two topics).
constexpr int kQueueBatch = 8;

// Claim table of the ordered entry-by-entry adds (one per wave): slot
// (row, topic) of the accumulator hashes to entry (topic + 16 row) % 128.
constexpr int kClaims = 128;
// Piece sums of a long row in flight at once in k_spmm_heavy.
constexpr int kHeavyLoads = 32;
// Sub-rounds before the claim table is cleared and the tag restarts (tags
// stay far from overflowing the 32-bit entries).
constexpr int32_t kTagMax = 1 << 22;

// Restarts the tag and clears the wave's claim table once the tag has grown
// large (wave-uniform).
__device__ __forceinline__ void claim_restart(int32_t* claim, int32_t& tag) {
  if (tag >= kTagMax) {
    for (int i = lane_id(); i < kClaims; i += 64) claim[i] = 0;
    tag = 0;
  }
}

// Per wave: the queue's values, byte offsets and item rows, then the
// accumulator, then the claim table.
template <typename T, int RG, bool WIDE>
__host__ __device__ inline size_t spmm_per_wave(int) {
  constexpr size_t Q = queue_len<WIDE>();
  return Q * (sizeof(T) + sizeof(uint32_t)) + (Q + 15) / 16 * 16 + kTileEntries * sizeof(T) +
         kClaims * sizeof(int32_t);
}

// LDS of one block: W (or, for a raw product, the row filter), then each
// wave's buffers.
__host__ __device__ inline size_t spmm_head_bytes(int k, bool raw, int filter_words) {
  return raw ? (static_cast<size_t>(filter_words) * sizeof(uint32_t) + 15) / 16 * 16
             : static_cast<size_t>(k) * k * sizeof(double);
}
template <typename T, int RG, bool WIDE>
size_t spmm_lds_bytes(int k, bool raw, int waves, int filter_words = 0) {
  return spmm_head_bytes(k, raw, filter_words) + waves * spmm_per_wave<T, RG, WIDE>(k);
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
  const int2* meta;    // factor row metadata {dense row or first entry, entry count}
  int32_t sparse_row;  // rows with at most this many entries are gathered entry by entry
  const void* ents;    // stored factor entries {value, topic}
  const void* F;       // compact dense factor rows (or the dense input)
  int32_t ld;          // row pitch of F
  uint32_t F_bytes;    // bytes of F (its loads are range-checked against this)
  const double* W;
  void* X;
  void* C;
  int32_t k;           // topics of the product (the column window's width)
  int32_t c0;          // first factor column of the window (stored entries are shifted by it)
  int32_t x_ld;        // raw output: row pitch of X and first column written
  int32_t x_c0;
  const uint32_t* filter;  // raw products only: bit j set when factor row j can contribute
  int32_t filter_words;    // (null: every row); staged in LDS, other nonzeros are skipped
  int32_t* status;
  unsigned long long* gathered;  // [kGathSlots] entries gathered (null: not counted)
};

// A stored entry's topic within the column window [c0, c0 + k); an entry
// outside it adds zero (to topic 0).
template <typename T>
__device__ __forceinline__ FactorEnt<T> in_window(FactorEnt<T> en, int c0, int k) {
  const int t = static_cast<int>(en.t) - c0;
  const bool in = static_cast<unsigned>(t) < static_cast<unsigned>(k);
  return FactorEnt<T>{in ? en.v : T(0), in ? static_cast<uint32_t>(t) : 0u};
}

struct WaveLds {
  uint32_t* q_off;  // dense-row queue: byte offset of the factor row in F
  uint8_t* q_r;     //                  row within the item
  void* q_a;        //                  the nonzero's value
  void* tile;       // accumulator: tile[topic * RG + row]
  int32_t* claim;   // claim table of the ordered adds (tags of earlier sub-rounds; zero at start)
  const uint32_t* filt;  // row filter in LDS (null: none)
};

template <typename T, int RG, bool WIDE>
__device__ __forceinline__ WaveLds wave_lds(unsigned char* smem, size_t wave0, int k, int wv) {
  constexpr int Q = queue_len<WIDE>();
  unsigned char* base = smem + wave0 + wv * spmm_per_wave<T, RG, WIDE>(k);
  WaveLds w;
  w.q_a = base;  // T first: 8-byte aligned for double
  w.q_off = reinterpret_cast<uint32_t*>(base + Q * sizeof(T));
  w.q_r = base + Q * (sizeof(T) + sizeof(uint32_t));
  w.tile = base + Q * (sizeof(T) + sizeof(uint32_t)) + (Q + 15) / 16 * 16;
  w.claim = reinterpret_cast<int32_t*>(static_cast<unsigned char*>(w.tile) + kTileEntries * sizeof(T));
  w.filt = nullptr;
  return w;
}

// Block prologue: W into LDS (unless raw); returns the LDS offset of the
// waves' buffers.
template <bool RAW>
__device__ __forceinline__ size_t load_block(const SpmmArgs& a, unsigned char* smem) {
  const int k = a.k;
  if (!RAW) {
    double* sW = reinterpret_cast<double*>(smem);
    for (int i = threadIdx.x; i < k * k; i += blockDim.x) sW[i] = a.W[i];
  } else if (a.filter != nullptr) {
    uint32_t* f = reinterpret_cast<uint32_t*>(smem);
    for (int i = threadIdx.x; i < a.filter_words; i += blockDim.x) f[i] = a.filter[i];
  }
  __syncthreads();
  return spmm_head_bytes(k, RAW, a.filter != nullptr ? a.filter_words : 0);
}

// Wave-uniform copy of a value every lane holds (an SGPR operand).
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uniform(double v) {
  const long long b = __double_as_longlong(v);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(b));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(b >> 32));
  return __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(hi) << 32) | lo));
}

// A load of F at a byte offset through a buffer resource: the hardware
// returns zero for offsets at or past the resource's size.
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, static_cast<int>(off), 0, 0));
}
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, static_cast<int>(off), 0, 0));
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  // raw buffer (stride 0): 32-bit elements, range-checked by byte offset
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), static_cast<short>(0), static_cast<int>(bytes),
                                           0x00020000);
}

// Adds queued entries [h, h + B) into the accumulator: B factor rows in
// flight, lanes = topics, sums for the current row kept in acc.  A row's
// address is its queued byte offset plus the lane's topic offset (one
// vector add; the queued words are LDS broadcasts).  Rows are queued in
// order, so a batch whose first and last entries share an item row lies in
// that row: it needs one row test instead of one per entry.
template <typename T, int KPL, int RG, int B>
__device__ __forceinline__ void queue_batch(const WaveLds& w, __amdgpu_buffer_rsrc_t F, int h,
                                            const uint32_t* lo, const bool* live, T* acc, int& cur_r) {
  const int lane = lane_id();
  T* tile = static_cast<T*>(w.tile);
  const T* q_a = static_cast<const T*>(w.q_a);
  const int ra = static_cast<int>(uniform(static_cast<uint32_t>(w.q_r[h])));
  const int rb = static_cast<int>(uniform(static_cast<uint32_t>(w.q_r[h + B - 1])));
  uint32_t off[B];
  T aa[B];
#pragma unroll
  for (int u = 0; u < B; ++u) {
    off[u] = w.q_off[h + u];
    aa[u] = q_a[h + u];
  }
  // lanes past k load nothing (their quarter-waves then touch no line)
  T f[B][KPL];
#pragma unroll
  for (int q = 0; q < KPL; ++q) {
    if (live[q]) {
#pragma unroll
      for (int u = 0; u < B; ++u) f[u][q] = buf_load<T>(F, off[u] + lo[q]);
    } else {
#pragma unroll
      for (int u = 0; u < B; ++u) f[u][q] = T(0);
    }
  }
  auto flush = [&](int rr) {
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
      tile[(lane + 64 * q) * RG + cur_r] += acc[q];
      acc[q] = T(0);
    }
    cur_r = rr;
  };
  if (ra == rb) {
    if (ra != cur_r) flush(ra);
#pragma unroll
    for (int u = 0; u < B; ++u)
#pragma unroll
      for (int q = 0; q < KPL; ++q) acc[q] = fma(aa[u], f[u][q], acc[q]);
  } else {
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int rr = static_cast<int>(uniform(static_cast<uint32_t>(w.q_r[h + u])));
      if (rr != cur_r) flush(rr);
#pragma unroll
      for (int q = 0; q < KPL; ++q) acc[q] = fma(aa[u], f[u][q], acc[q]);
    }
  }
}

// Adds the queued entries [0, n8) (n8 a multiple of 8, in row order): whole
// batches of kQueueBatch rows, then the tail in batches of halving size.
// Lanes past k add zeros into unused accumulator slots.
template <typename T, int KPL, int RG>
__device__ __forceinline__ void run_queue(const WaveLds& w, __amdgpu_buffer_rsrc_t F, int n8, int k, T* acc,
                                          int& cur_r) {
  const int lane = lane_id();
  uint32_t lo[KPL];
  bool live[KPL];
#pragma unroll
  for (int q = 0; q < KPL; ++q) {
    const int c = lane + 64 * q;
    live[q] = c < k;
    lo[q] = static_cast<uint32_t>(c) * static_cast<uint32_t>(sizeof(T));
  }
  constexpr int QB = kQueueBatch / KPL < 8 ? 8 : kQueueBatch / KPL;
  int h = 0;
  for (; h + QB <= n8; h += QB) queue_batch<T, KPL, RG, QB>(w, F, h, lo, live, acc, cur_r);
  if constexpr (QB > 32) {
    if (h + 32 <= n8) {
      queue_batch<T, KPL, RG, 32>(w, F, h, lo, live, acc, cur_r);
      h += 32;
    }
  }
  if constexpr (QB > 16) {
    if (h + 16 <= n8) {
      queue_batch<T, KPL, RG, 16>(w, F, h, lo, live, acc, cur_r);
      h += 16;
    }
  }
  if constexpr (QB > 8) {
    if (h + 8 <= n8) queue_batch<T, KPL, RG, 8>(w, F, h, lo, live, acc, cur_r);
  }
}

// Queues a step's dense hits (one per lane, or two in the wide form: lane
// positions base + 64 * s) in step order = row order, padded to whole
// batches of 8 with zero-weight reads of the first factor row at the last
// hit's row; returns the padded length.  `ldb` is F's row pitch in bytes.
template <typename T, int NS>
__device__ __forceinline__ int queue_hits(const WaveLds& w, const bool* hit, const int32_t* x, const int* r,
                                          const T* av, uint32_t ldb) {
  const int lane = lane_id();
  T* q_a = static_cast<T*>(w.q_a);
  uint64_t bal[NS];
  int before[NS];
  int nh = 0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    bal[s] = __ballot(hit[s]);
    before[s] = nh;
    nh += __popcll(bal[s]);
  }
  if (nh == 0) return 0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (hit[s]) {
      const int pos = before[s] + lane_rank(bal[s]);
      w.q_off[pos] = static_cast<uint32_t>(x[s]) * ldb;
      w.q_r[pos] = static_cast<uint8_t>(r[s]);
      q_a[pos] = av[s];
    }
  }
  int last_s = 0;
#pragma unroll
  for (int s = 1; s < NS; ++s)
    if (bal[s]) last_s = s;
  int r_src = r[0];
#pragma unroll
  for (int s = 1; s < NS; ++s)
    if (s == last_s) r_src = r[s];
  const int r_last = __shfl(r_src, 63 - __builtin_clzll(bal[last_s]), 64);
  const int nh8 = (nh + 7) & ~7;
  if (lane < nh8 - nh) {
    w.q_off[nh + lane] = 0u;
    w.q_r[nh + lane] = static_cast<uint8_t>(r_last);
    q_a[nh + lane] = T(0);
  }
  return nh8;
}

// Adds v into tile[slot] on every lane where `pend` holds.  Lanes of one
// call that add to the same slot do so in ascending lane order: in each
// sub-round every pending lane writes the tag (sub-round << 6 | 63 - lane)
// into its slot's claim entry with an integer atomicMax (the result does not
// depend on the order in which the hardware applies the lanes, and tags of
// earlier sub-rounds are smaller), and the lane that finds its own tag there
// adds; the winners of a sub-round hold distinct slots, so their adds never
// collide.  The rest try again.  Different slots that share a claim entry
// only wait one more sub-round.  The sums are therefore the same on every
// run.  `tag` counts the wave's sub-rounds (wave-uniform; the claim table
// starts at zero).
template <typename T, int RG>
__device__ __forceinline__ void ordered_add(T* tile, int32_t* claim, int32_t& tag, int t, int r, T v, bool pend) {
  const int lane = lane_id();
  const int slot = t * RG + r;
  int32_t* cl = &claim[(t + 16 * r) & (kClaims - 1)];
  while (__ballot(pend) != 0) {
    claim_restart(claim, tag);
    ++tag;
    const int32_t mine = (tag << 6) | (63 - lane);
    if (pend) __hip_atomic_fetch_max(cl, mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    const bool win = pend && __hip_atomic_load(cl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == mine;
    if (win) {
      __hip_atomic_fetch_add(&tile[slot], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      pend = false;
    }
  }
}

// A single-row item's entry-by-entry products are not added into the
// accumulator one by one: each step appends them, in a fixed order (round,
// then nonzero), to a list kept in the wave's accumulator space (unused
// until the item ends: the row's sums stay in registers), and the list is
// then summed with lanes = topics, each lane adding the entries of its topic
// in list order.  No two lanes ever add to one place.
constexpr int kListCap = 256;

template <typename T, int KPL>
__device__ __forceinline__ void scan_list(const int32_t* lt, const T* lw, int n, T* acc) {
  const int lane = lane_id();
  int j = 0;
  for (; j + 4 <= n; j += 4) {
    int tv[4];
    T wv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      tv[u] = lt[j + u];
      wv[u] = lw[j + u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < KPL; ++q) acc[q] += tv[u] == lane + 64 * q ? wv[u] : T(0);
  }
  for (; j < n; ++j) {
    const int tv = lt[j];
    const T wv = lw[j];
#pragma unroll
    for (int q = 0; q < KPL; ++q) acc[q] += tv == lane + 64 * q ? wv : T(0);
  }
}

// Adds the nonzeros [p0, p1) of an item (rows bounded by rb[0..nrows]) times
// F into the accumulator.
//  * Narrow form (64 nonzeros per step): loads are predicated on the lanes
//    that need them, so a gather costs only its active lanes.  Suits factors
//    whose rows are mostly dense (few lanes take the entry-by-entry path).
//  * Wide form (128 nonzeros per step, two per lane): every global load of a
//    step is issued unconditionally at an in-bounds address (lanes past the
//    end re-read the last nonzero, inactive gathers read entry 0) and masked
//    afterwards, so twice as many loads are in flight per step and none waits
//    at the end of a divergent branch.  Suits very sparse factors, where the
//    wave mostly waits on the metadata and entry gathers.
template <typename T, int KPL, int RG, bool DENSE_IN, bool WIDE>
__device__ __forceinline__ void accumulate(const SpmmArgs& a, int64_t p0, int64_t p1, const int64_t* rb,
                                           int nrows, const WaveLds& w, uint32_t& gath, int32_t& tag) {
  constexpr int NS = WIDE ? 2 : 1;
  const int lane = lane_id();
  const int k = a.k;
  const int32_t* __restrict__ col = a.col;
  const T* __restrict__ val = static_cast<const T*>(a.val);
  const __amdgpu_buffer_rsrc_t Fr = make_rsrc(a.F, a.F_bytes);
  const uint32_t ldb = static_cast<uint32_t>(a.ld) * static_cast<uint32_t>(sizeof(T));
  const FactorEnt<T>* __restrict__ ents = static_cast<const FactorEnt<T>*>(a.ents);
  T* tile = static_cast<T*>(w.tile);
  T acc[KPL];
#pragma unroll
  for (int q = 0; q < KPL; ++q) acc[q] = T(0);
  int cur_r = 0;
  for (int64_t base = p0; base < p1; base += 64 * NS) {
    int64_t p[NS];
    bool valid[NS];
    int32_t j[NS], x[NS], cnt[NS];
    T av[NS];
    int r[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      p[s] = base + 64 * s + lane;
      valid[s] = p[s] < p1;
      if (WIDE) {
        const int64_t pc = valid[s] ? p[s] : p1 - 1;
        j[s] = __builtin_nontemporal_load(&col[pc]);
        av[s] = __builtin_nontemporal_load(&val[pc]);
      } else {
        j[s] = 0;
        av[s] = T(0);
        if (valid[s]) {
          j[s] = col[p[s]];
          av[s] = val[p[s]];
        }
      }
      r[s] = 0;
#pragma unroll
      for (int i = 1; i < RG; ++i) r[s] += (i < nrows && p[s] >= rb[i]) ? 1 : 0;
    }
    if (!DENSE_IN && w.filt != nullptr) {
      // nonzeros whose factor row has nothing in the column window add nothing
#pragma unroll
      for (int s = 0; s < NS; ++s) valid[s] = valid[s] && ((w.filt[j[s] >> 5] >> (j[s] & 31)) & 1u) != 0u;
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (DENSE_IN) {
        x[s] = j[s];
        cnt[s] = valid[s] ? k : 0;
      } else if (WIDE) {
        const int2 m = a.meta[valid[s] ? j[s] : 0];
        x[s] = m.x;
        cnt[s] = valid[s] ? m.y : 0;
        av[s] = valid[s] ? av[s] : T(0);
      } else {
        x[s] = 0;
        cnt[s] = 0;
        if (valid[s]) {
          const int2 m = a.meta[j[s]];
          x[s] = m.x;
          cnt[s] = m.y;
        }
      }
    }
    if (!DENSE_IN) {
#pragma unroll
      for (int s = 0; s < NS; ++s) gath += static_cast<uint32_t>(cnt[s]);
      // sparse factor rows, entry by entry; lanes start at a rotated entry so
      // that one round rarely adds twice to one topic
      bool sparse[NS];
      int rot[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        sparse[s] = cnt[s] > 0 && cnt[s] <= a.sparse_row;
        rot[s] = sparse[s] ? lane % cnt[s] : 0;
      }
      if (nrows == 1) {
        // one row: the products go to the list (see scan_list), which is
        // summed into the row's registers whenever it could overflow and at
        // the end of the step
        int32_t* lt = reinterpret_cast<int32_t*>(tile);
        T* lw = reinterpret_cast<T*>(lt + kListCap);
        int nl = 0;
        for (int e = 0; __ballot((sparse[0] && e < cnt[0]) || (sparse[NS - 1] && e < cnt[NS - 1])) != 0; ++e) {
          bool act[NS];
          uint64_t bal[NS];
          int tot = 0;
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            act[s] = sparse[s] && e < cnt[s];
            bal[s] = __ballot(act[s]);
            tot += __popcll(bal[s]);
          }
          if (nl + tot > kListCap) {
            __builtin_amdgcn_wave_barrier();
            scan_list<T, KPL>(lt, lw, nl, acc);
            __builtin_amdgcn_wave_barrier();
            nl = 0;
          }
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            if (act[s]) {
              int idx = e + rot[s];
              if (idx >= cnt[s]) idx -= cnt[s];
              const FactorEnt<T> en = in_window(ents[x[s] + idx], a.c0, k);
              const int pos = nl + lane_rank(bal[s]);
              lt[pos] = static_cast<int32_t>(en.t);
              lw[pos] = av[s] * en.v;
            }
            nl += __popcll(bal[s]);
          }
        }
        __builtin_amdgcn_wave_barrier();
        scan_list<T, KPL>(lt, lw, nl, acc);
        __builtin_amdgcn_wave_barrier();
      } else if (WIDE) {
        // entries e and e + 1 of every row per round; a round only runs when
        // some lane has an entry left, so entry 0 exists and serves as the
        // inactive lanes' address
        for (int e = 0; __ballot((sparse[0] && e < cnt[0]) || (sparse[NS - 1] && e < cnt[NS - 1])) != 0;
             e += 2) {
          FactorEnt<T> en[NS][2];
          bool act[NS][2];
#pragma unroll
          for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int d = 0; d < 2; ++d) {
              act[s][d] = sparse[s] && e + d < cnt[s];
              int idx = e + d + rot[s];
              if (idx >= cnt[s]) idx -= cnt[s];
              en[s][d] = in_window(ents[act[s][d] ? x[s] + idx : 0], a.c0, k);
            }
#pragma unroll
          for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int d = 0; d < 2; ++d)
              ordered_add<T, RG>(tile, w.claim, tag, static_cast<int>(en[s][d].t), r[s], av[s] * en[s][d].v, act[s][d]);
        }
      } else {
        for (int e = 0; __ballot(sparse[0] && e < cnt[0]) != 0; ++e) {
          const bool act = sparse[0] && e < cnt[0];
          FactorEnt<T> en{T(0), 0u};
          if (act) {
            int idx = e + rot[0];
            if (idx >= cnt[0]) idx -= cnt[0];
            en = in_window(ents[x[0] + idx], a.c0, k);
          }
          ordered_add<T, RG>(tile, w.claim, tag, static_cast<int>(en.t), r[0], av[0] * en.v, act);
        }
      }
    }
    // dense factor rows: queued, then one k-wide row per hit, lanes = topics
    bool hit[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) hit[s] = DENSE_IN ? valid[s] : cnt[s] > a.sparse_row;
    const int nq = queue_hits<T, NS>(w, hit, x, r, av, ldb);
    run_queue<T, KPL, RG>(w, Fr, nq, k, acc, cur_r);
  }
  if (!DENSE_IN && nrows == 1) {
    // the accumulator space held the list: the row's sums replace it
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int i = 0; i < kTileEntries / 64; ++i) tile[lane + 64 * i] = T(0);
    __builtin_amdgcn_wave_barrier();
  }
#pragma unroll
  for (int q = 0; q < KPL; ++q) tile[(lane + 64 * q) * RG + cur_r] += acc[q];
}

// tile layout: tile[rr * RG + r] = raw sum of row r, topic rr.
template <typename T, int KPL, int RG, bool RAW, bool STORE_C>
__device__ __forceinline__ void epilogue(const SpmmArgs& a, const T* tile, const double* sW,
                                         int nrows, int32_t r0) {
  const int lane = lane_id();
  const int k = a.k;
  T* __restrict__ X = static_cast<T*>(a.X);
  // a non-finite sum or solution (float32 overflow) raises the sticky
  // NONFINITE status instead of being clamped to zero
  bool bad = false;
  if (RAW) {
    for (int r = 0; r < nrows; ++r) {
#pragma unroll
      for (int q = 0; q < KPL; ++q) {
        const int c = lane + 64 * q;
        if (c < k) {
          const T x = tile[c * RG + r];
          bad |= !isfinite(x);
          X[static_cast<int64_t>(r0 + r) * a.x_ld + a.x_c0 + c] = x;
        }
      }
    }
    if (__ballot(bad) != 0 && lane == 0) atomicCAS(a.status, 0, static_cast<int32_t>(NMF_ERR_NONFINITE));
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
          const T y = static_cast<T>(x > 0.0 ? x : 0.0);
          bad |= !isfinite(x) || !isfinite(y);
          X[o] = y;
          if (STORE_C) static_cast<T*>(a.C)[o] = tile[c * RG + r];
        }
      }
    }
  }
  if (__ballot(bad) != 0 && lane == 0) atomicCAS(a.status, 0, static_cast<int32_t>(NMF_ERR_NONFINITE));
}

template <typename T, int KPL, int RG>
__device__ __forceinline__ void clear_tile(T* tile, int) {
  const int lane = lane_id();
#pragma unroll
  for (int i = 0; i < kTileEntries / 64; ++i) tile[lane + 64 * i] = T(0);
}

// Block `blk` of a grid of `nblk` blocks over the items of one problem.
template <typename T, int KPL, int RG, bool RAW, bool STORE_C, bool DENSE_IN, bool WIDE>
__device__ __forceinline__ void spmm_body(const SpmmArgs& a, int blk, int nblk) {
  static_assert(RG * 64 * KPL <= kTileEntries, "accumulator too small for the row group");
  extern __shared__ __align__(16) unsigned char smem[];
  if (*a.status != 0) return;
  const int k = a.k;
  const int lane = lane_id();
  const int wv = threadIdx.x >> 6;
  const size_t wave0 = load_block<RAW>(a, smem);
  const double* sW = reinterpret_cast<const double*>(smem);
  WaveLds w = wave_lds<T, RG, WIDE>(smem, wave0, k, wv);
  if (RAW && a.filter != nullptr) w.filt = reinterpret_cast<const uint32_t*>(smem);
  T* tile = static_cast<T*>(w.tile);
#pragma unroll
  for (int i = 0; i < kClaims / 64; ++i) w.claim[lane + 64 * i] = 0;

  const int bw = blockDim.x >> 6;
  const int nw = nblk * bw;
  uint32_t gath = 0;  // this lane's gathered entries (fits: at most k per nonzero it loads)
  int32_t tag = 0;    // sub-rounds of the ordered adds so far (wave-uniform)
  for (int it = blk * bw + wv; it < a.n_items; it += nw) {
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
      accumulate<T, KPL, RG, DENSE_IN, WIDE>(a, rb[0], rb[nrows], rb, nrows, w, gath, tag);
      epilogue<T, KPL, RG, RAW, STORE_C>(a, tile, sW, nrows, wi.r0);
    } else {
      int64_t rb[RG + 1];
#pragma unroll
      for (int i = 0; i <= RG; ++i) rb[i] = i == 0 ? wi.p0 : wi.p1;
      accumulate<T, KPL, RG, DENSE_IN, WIDE>(a, wi.p0, wi.p1, rb, 1, w, gath, tag);
      T* part = static_cast<T*>(a.partials);
#pragma unroll
      for (int q = 0; q < KPL; ++q) {
        const int c = lane + 64 * q;
        if (c < k) part[static_cast<int64_t>(wi.part) * k + c] = tile[c * RG];
      }
    }
  }
  if (a.gathered != nullptr) {
    unsigned long long g = gath;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) g += __shfl_xor(g, d, 64);
    if (lane == 0 && g != 0) atomicAdd(&a.gathered[(blk * bw + wv) % kGathSlots], g);
  }
}

template <typename T, int KPL, int RG, bool RAW, bool STORE_C, bool DENSE_IN, bool WIDE>
__global__ __launch_bounds__(64 * kWaves) void k_spmm(SpmmArgs a) {
  spmm_body<T, KPL, RG, RAW, STORE_C, DENSE_IN, WIDE>(a, blockIdx.x, gridDim.x);
}
template <typename T, int KPL, int RG, bool RAW, bool STORE_C, bool DENSE_IN, bool WIDE>
__global__ __launch_bounds__(64 * kWaves) void k_spmm_b(const SpmmArgs* as, const BlockMap* map) {
  const BlockMap m = map[blockIdx.x];
  const SpmmArgs a = as[m.prob];
  spmm_body<T, KPL, RG, RAW, STORE_C, DENSE_IN, WIDE>(a, m.blk, m.nblk);
}

// Long rows: add the pieces' raw sums in piece order, then the epilogue.
template <typename T, int KPL, int RG, bool RAW, bool STORE_C>
__device__ __forceinline__ void spmm_heavy_body(const SpmmArgs& a, int blk, int nblk) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (*a.status != 0) return;
  const int k = a.k;
  const int lane = lane_id();
  const int wv = threadIdx.x >> 6;
  double* sW = reinterpret_cast<double*>(smem);
  if (!RAW) {
    for (int i = threadIdx.x; i < k * k; i += blockDim.x) sW[i] = a.W[i];
  }
  __syncthreads();
  const size_t wave0 = RAW ? 0 : static_cast<size_t>(k) * k * sizeof(double);
  T* tile = reinterpret_cast<T*>(smem + wave0) + static_cast<size_t>(wv) * kTileEntries;
  const T* part = static_cast<const T*>(a.partials);
  const int bw = blockDim.x >> 6;
  const int nw = nblk * bw;
  for (int hh = blk * bw + wv; hh < a.n_heavy; hh += nw) {
    const int nch = a.heavy_nchunks[hh];
    const int p0 = a.heavy_part0[hh];
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
      const int c = lane + 64 * q;
      if (c < k) {
        // kHeavyLoads loads in flight (the longest rows of a billion-nonzero
        // corpus have thousands of pieces), added in piece order
        T s = T(0);
        int j = 0;
        for (; j + kHeavyLoads <= nch; j += kHeavyLoads) {
          T v[kHeavyLoads];
#pragma unroll
          for (int u = 0; u < kHeavyLoads; ++u) v[u] = part[static_cast<int64_t>(p0 + j + u) * k + c];
#pragma unroll
          for (int u = 0; u < kHeavyLoads; ++u) s += v[u];
        }
        for (; j < nch; ++j) s += part[static_cast<int64_t>(p0 + j) * k + c];
        tile[c * RG] = s;
      }
    }
    epilogue<T, KPL, RG, RAW, STORE_C>(a, tile, sW, 1, a.heavy_row[hh]);
  }
}

template <typename T, int KPL, int RG, bool RAW, bool STORE_C>
__global__ __launch_bounds__(64 * kWaves) void k_spmm_heavy(SpmmArgs a) {
  spmm_heavy_body<T, KPL, RG, RAW, STORE_C>(a, blockIdx.x, gridDim.x);
}
template <typename T, int KPL, int RG, bool RAW, bool STORE_C>
__global__ __launch_bounds__(64 * kWaves) void k_spmm_heavy_b(const SpmmArgs* as, const BlockMap* map) {
  const BlockMap m = map[blockIdx.x];
  const SpmmArgs a = as[m.prob];
  spmm_heavy_body<T, KPL, RG, RAW, STORE_C>(a, m.blk, m.nblk);
}

template <typename T, int KPL, int RG, bool RAW, bool STORE_C, bool DENSE_IN, bool WIDE>
hipError_t launch(nmf_handle* h, const SpmmArgs& a, int waves_max) {
  // W (float64, k x k) is shared by the block; with large k fewer waves fit
  int waves = std::min(waves_max, kWaves);
  const int fw = a.filter != nullptr ? a.filter_words : 0;
  while (waves > 1 && spmm_lds_bytes<T, RG, WIDE>(a.k, RAW, waves, fw) > kLdsBytes) waves /= 2;
  const size_t lds = spmm_lds_bytes<T, RG, WIDE>(a.k, RAW, waves, fw);
  if (lds > kLdsBytes) return hipErrorInvalidValue;
  // one wave of blocks: as many as are resident at once (registers and LDS),
  // so no block starts late and the strided item loop stays balanced
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_spmm<T, KPL, RG, RAW, STORE_C, DENSE_IN, WIDE>,
                                                   64 * waves, lds) != hipSuccess)
    return hipErrorInvalidValue;
  if (per_cu < 1) per_cu = 1;
  const int cap = h->num_cus * per_cu;
  const int items = std::min((a.n_items + waves - 1) / waves, cap);
  hipError_t e = launch_rec(h, k_spmm<T, KPL, RG, RAW, STORE_C, DENSE_IN, WIDE>,
                            k_spmm_b<T, KPL, RG, RAW, STORE_C, DENSE_IN, WIDE>, static_cast<unsigned>(items),
                            64u * waves, lds, a);
  if (e != hipSuccess) return e;
  const int heavy = std::min((a.n_heavy + waves - 1) / waves, cap);
  return launch_rec(h, k_spmm_heavy<T, KPL, RG, RAW, STORE_C>, k_spmm_heavy_b<T, KPL, RG, RAW, STORE_C>,
                    static_cast<unsigned>(heavy), 64u * waves, lds, a);
}

template <typename T>
hipError_t spmm_stream(nmf_handle* h, const Plan& p, const Factor& F, const double* W, T* X, T* C,
                       bool raw, const T* dense_in, int sparse_row, bool wide, int waves,
                       const ColWindow* win = nullptr, const uint32_t* filter = nullptr, int32_t filter_words = 0) {
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
  a.ld = dense_in ? h->k : F.ld;
  a.F_bytes = static_cast<uint32_t>(F.rows * a.ld * static_cast<int64_t>(sizeof(T)));
  a.W = W;
  a.X = X;
  a.C = C;
  a.k = h->k;
  a.c0 = 0;
  a.x_ld = h->k;
  a.x_c0 = 0;
  if (win != nullptr) {
    // raw product of factor columns [c0, c0 + kw): dense rows are read from
    // column c0 on, stored entries are shifted into the window
    if (!raw || dense_in != nullptr || win->kw < 1 || win->c0 < 0 || win->c0 + win->kw > h->k ||
        win->x_c0 < 0 || win->x_c0 + win->kw > win->x_ld)
      return hipErrorInvalidValue;
    a.k = win->kw;
    a.c0 = win->c0;
    a.x_ld = win->x_ld;
    a.x_c0 = win->x_c0;
    a.F = static_cast<const T*>(F.dense) + win->c0;
    a.F_bytes -= static_cast<uint32_t>(win->c0 * sizeof(T));
    a.filter = filter;
    a.filter_words = filter_words;
  }
  a.status = h->status;
  a.gathered = dense_in ? nullptr : h->met.gathered + (&p == &h->planA ? kGathSlots : 0);
  const bool two = a.k > 64;
  const bool dense = dense_in != nullptr;
  if (p.n_hot > 0) return hipErrorInvalidValue;  // a hot block belongs to the fused V-half kernel
  if (raw) {
    if (dense)
      return two ? launch<T, 2, 4, true, false, true, false>(h, a, waves) : launch<T, 1, 8, true, false, true, false>(h, a, waves);
    return two ? launch<T, 2, 4, true, false, false, false>(h, a, waves) : launch<T, 1, 8, true, false, false, false>(h, a, waves);
  }
  if (C != nullptr) {
    if (wide)
      return two ? launch<T, 2, 4, false, true, false, true>(h, a, waves) : launch<T, 1, 8, false, true, false, true>(h, a, waves);
    return two ? launch<T, 2, 4, false, true, false, false>(h, a, waves) : launch<T, 1, 8, false, true, false, false>(h, a, waves);
  }
  if (wide)
    return two ? launch<T, 2, 4, false, false, false, true>(h, a, waves) : launch<T, 1, 8, false, false, false, true>(h, a, waves);
  return two ? launch<T, 2, 4, false, false, false, false>(h, a, waves) : launch<T, 1, 8, false, false, false, false>(h, a, waves);
}

}  // namespace

// Every product records the same number of launches (the stream, its long
// rows and an empty one; or the fused V-half kernel and two empty ones), so
// that the launch sequences of a batch's problems line up.
template <typename T>
hipError_t spmm(nmf_handle* h, const Plan& p, const Factor& F, const double* W, T* X, T* C,
                bool raw, const T* dense_in, int sparse_row, bool wide, int waves) {
  if constexpr (sizeof(T) == 4) {
    if (h->use_vhalf && &p == &h->planAt) {
      if (C != nullptr) return hipErrorInvalidValue;
      hipError_t e = vhalf(h, p, F, dense_in, X, raw ? nullptr : W, waves);
      if (e != hipSuccess) return e;
      if ((e = vhalf_placeholder(h)) != hipSuccess) return e;
      return vhalf_placeholder(h);
    }
  }
  hipError_t e = spmm_stream<T>(h, p, F, W, X, C, raw, dense_in, sparse_row, wide, waves);
  if (e != hipSuccess) return e;
  return vhalf_placeholder(h);
}

// Raw product over a column window of the factor (see ColWindow).
template <typename T>
hipError_t spmm_window(nmf_handle* h, const Plan& p, const Factor& F, T* X, const ColWindow& win, int sparse_row,
                       const Factor& S) {
  if constexpr (sizeof(T) == 4) {
    if (h->use_vhalf && &p == &h->planAt) {
      // the fused kernel reads 16-byte groups of 16-byte aligned rows: the
      // window's columns at a pitch of kw rounded up to 4, which never
      // exceeds the pitch of S's own dense copy (k rounded up to 4 or more)
      const int32_t ldn = (win.kw + 3) / 4 * 4;
      if (F.rows * ldn > S.rows * S.ld) return hipErrorInvalidValue;
      hipError_t e = narrow_rows(h, F, win.c0, win.kw, ldn, static_cast<float*>(S.dense));
      if (e != hipSuccess) return e;
      Factor Fn = F;
      Fn.dense = S.dense;
      Fn.ld = ldn;
      return vhalf_window(h, p, Fn, X, win);
    }
  }
  // the filter bitmap goes through S's values; it is used while it fits in
  // there and in a quarter of the LDS
  const int64_t fw = (F.rows + 31) / 32;
  const bool filt = fw * 4 <= static_cast<int64_t>(kLdsBytes / 4) &&
                    fw * 4 <= S.rows * static_cast<int64_t>(h->k) * static_cast<int64_t>(sizeof(T));
  if (filt) {
    hipError_t e = window_bits(h, F, win.c0, win.kw, static_cast<uint32_t*>(S.val));
    if (e != hipSuccess) return e;
  }
  return spmm_stream<T>(h, p, F, nullptr, X, nullptr, true, nullptr, sparse_row, false, 8, &win,
                        filt ? static_cast<const uint32_t*>(S.val) : nullptr, static_cast<int32_t>(fw));
}

template hipError_t spmm<float>(nmf_handle*, const Plan&, const Factor&, const double*, float*,
                                float*, bool, const float*, int, bool, int);
template hipError_t spmm_window<float>(nmf_handle*, const Plan&, const Factor&, float*, const ColWindow&, int,
                                       const Factor&);
template hipError_t spmm_window<double>(nmf_handle*, const Plan&, const Factor&, double*, const ColWindow&, int,
                                        const Factor&);
template hipError_t spmm<double>(nmf_handle*, const Plan&, const Factor&, const double*, double*,
                                 double*, bool, const double*, int, bool, int);

}  // namespace nmfk
