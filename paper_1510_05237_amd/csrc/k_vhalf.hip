// V half-step of Algorithm 2 (step 1) for float32 factors with k <= 64, as
// one fused kernel:
//
//   V_pre[r] = max(0, (sum_{p in doc r} a_p U[term_p]) W),   W = (U^T U)^-1
//
// (W null: the raw sums are stored instead, for the loss products).
//
// Work unit: a tile of 16 consecutive documents owned by one wave, from
// their nonzeros to their stored rows of V_pre.
//
//  * Hot terms.  The terms that occur in the most documents (their rows of A
//    were split off into a dense documents x hot block when the handle was
//    created) are a dense product: after the rest of the tile has streamed,
//    the wave loads its 16 documents' hot columns as float4 per lane
//    (holding them during the stream would spill registers at 16 waves per
//    block) and multiplies them by U's
//    hot rows, staged once per block in LDS, on the fp32 matrix cores
//    (v_mfma_f32_16x16x4f32), computing the transposed product
//    (U_H^T)(A_H^T): element i of tile tt then holds document r0 + m,
//    topic 16 tt + 4 q + i for lane (m = lane % 16, q = lane / 16).
//  * Every other nonzero is streamed straight into the registers that the
//    hot product accumulates into: lane (m, q) owns document r0 + m and the
//    topics 16 tt + 4 q + i (the fp32 MFMA result layout).  Per step each
//    document's next 16 nonzeros are read, four per lane, as one 16-byte
//    load of terms and one of values; U's row table, staged once per block
//    in LDS (one word per 32 terms: which of them have a nonempty row of U,
//    and how many nonempty rows precede them), gives each term's row in the
//    compact dense copy of U without a global load.  The document's four
//    lanes then take its 16 nonzeros in order (each broadcast from the lane
//    that read it): a nonempty row is read as one 16-byte load per topic
//    group and multiply-added into the lane's sums; empty rows are skipped.
//    Every sum is formed in nonzero order in one lane: no atomics, no
//    cross-lane reduction, and two runs are bitwise identical.
//  * Epilogue: the float64 solve runs
//    on the matrix cores (v_mfma_f64_16x16x4f64) with the raw sums as the A
//    operand straight from registers and W from LDS (the contraction order
//    of raw W is free); the result holds document r0 + q + 4 i, topic
//    16 tt + m in element i; it is clamped at zero, rounded to float32 and
//    stored.  A non-finite sum or solution raises the sticky NONFINITE
//    status instead of being clamped.
#include <algorithm>

#include "nmf_device.h"

namespace nmfk {

namespace {

typedef float vh_f4 __attribute__((ext_vector_type(4)));
typedef double vh_d4 __attribute__((ext_vector_type(4)));
typedef int vh_i4 __attribute__((ext_vector_type(4)));

constexpr int kVhTile = 16;                       // documents per wave tile
constexpr int kVhTopics = 64;                     // topic slots (k <= 64)
constexpr int kVhWavesMax = 16;
// Streamed rows a lane reads at once: 8 / NT, so that the rows in flight
// take the same registers whatever k (two 52-topic rows, or eight of 16).
template <int NT>
constexpr int vh_group() {
  return NT == 1 ? 8 : NT == 2 ? 4 : 2;
}
constexpr int kVhHotChunk = 8;                    // 16-column groups of the hot block read at once
constexpr size_t kVhLds = 160 * 1024;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t vh_rsrc(const void* p, uint32_t bytes) {
  // raw buffer: range-checked by byte offset (zero is returned past the end)
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), static_cast<short>(0), static_cast<int>(bytes),
                                           0x00020000);
}
__device__ __forceinline__ vh_f4 vh_load4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(vh_f4, __builtin_amdgcn_raw_buffer_load_b128(r, static_cast<int>(off), 0, 0));
}
__device__ __forceinline__ vh_i4 vh_load4i(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(vh_i4, __builtin_amdgcn_raw_buffer_load_b128(r, static_cast<int>(off), 0, 0));
}
__device__ __forceinline__ float vh_load1(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, static_cast<int>(off), 0, 0));
}
__device__ __forceinline__ int vh_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Four consecutive topics of a factor row at a byte offset: one 16-byte load
// from the compact dense copy (rows 16-byte aligned); four 4-byte loads from
// a caller's dense input, whose rows are only 4-byte aligned.
template <bool DENSE_IN>
__device__ __forceinline__ vh_f4 vh_row4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  if (DENSE_IN) return vh_f4{vh_load1(r, off), vh_load1(r, off + 4u), vh_load1(r, off + 8u), vh_load1(r, off + 12u)};
  return vh_load4(r, off);
}

struct VhArgs {
  const int64_t* rowptr;   // [rows + 1]: documents' nonzeros of the non-hot terms
  const int32_t* col;      // term of each nonzero
  const float* val;
  uint32_t stream_bytes;   // bytes of col (and of val), padding and spare entries included
  const int2* rowtab;      // U row table (see Factor::rowtab); null for a dense input
  int32_t tab_words;       // words of the row table
  const int32_t* sdf;      // per U row: streamed nonzeros of its term (gathered-entry count)
  const int32_t* urp;      // U's row pointers [n_u + 1] (entries per row)
  int64_t n_u;             // rows of U
  const float* F;          // compact dense U rows (pitch ld), or the dense input (pitch k)
  int32_t ld;
  uint32_t F_bytes;        // bytes of F (every load of it is range-checked)
  const float* hot;        // [rows][hot_ld]: hot block (null when n_hot == 0)
  const int32_t* hot_col;  // [n_hot]: U row of hot column h
  const int32_t* warm_col; // [n_warm]: U row of warm term w (stream term -2 - w)
  int32_t n_warm;
  int32_t hot_ld;          // multiple of 16, <= kMaxHot
  int32_t n_hot;
  const int32_t* slot;     // U row -> compact dense row (-1: empty), null for a dense input
  int64_t rows;            // documents
  int32_t k;
  const double* W;         // k x k, or null: X receives the raw sums
  float* X;                // [rows][k]; raw sums: pitch x_ld from column x_c0
  int32_t x_ld;
  int32_t x_c0;
  int32_t* status;
  unsigned long long* gathered;  // [kGathSlots]: U entries of the streamed rows (null: not counted)
};

// LDS of a block: U's hot rows (MFMA operand layout), W, U's row table,
// then U's warm rows (64 floats each).
__host__ __device__ inline size_t vh_block_lds(int hot_ld, int k, bool solve, int tab_words, int n_warm) {
  size_t b = static_cast<size_t>(hot_ld) * kVhTopics * sizeof(float);
  if (solve) b += static_cast<size_t>(k) * k * sizeof(double);
  b += static_cast<size_t>(tab_words) * sizeof(int2);
  b = (b + 15) / 16 * 16;
  return b + static_cast<size_t>(n_warm) * kVhTopics * sizeof(float);
}
__host__ __device__ inline size_t vh_warm_offset(int hot_ld, int k, bool solve, int tab_words) {
  return vh_block_lds(hot_ld, k, solve, tab_words, 0);
}

// The tile's streamed nonzeros into acc: lane (m, q) adds, for every nonzero
// (term j, value a) of document r0 + m, a times topics 16 tt + 4 q .. + 3 of
// U's row j to acc[tt], in nonzero order.  [rb, re): the document's
// nonzeros (empty past the tile's last document).
template <int NT, bool DENSE_IN>
__device__ __forceinline__ void vh_stream(const VhArgs& a, int64_t rb, int64_t re, const int2* stab,
                                          const float* warm, vh_f4* acc) {
  const int lane = lane_id();
  const int m = lane & 15, q = lane >> 4;
  const __amdgpu_buffer_rsrc_t Fr = vh_rsrc(a.F, a.F_bytes);
  // every document's run starts at a multiple of four entries (padded with
  // term -1) and the arrays carry four spare entries past their end, so the
  // 16-byte reads are aligned and a read at a document's end stays inside
  const __amdgpu_buffer_rsrc_t cr = vh_rsrc(a.col, a.stream_bytes);
  const __amdgpu_buffer_rsrc_t vr = vh_rsrc(a.val, a.stream_bytes);
  const uint32_t ldb = static_cast<uint32_t>(a.ld) * 4u;
  const uint32_t lo = 16u * static_cast<uint32_t>(q);
  bool live[NT];
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) live[tt] = 16 * tt + 4 * q < a.k;
  // steps of 16 nonzeros per document, as many as the tile's longest needs
  int ns = static_cast<int>((re - rb + 15) >> 4);
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) ns = max(ns, __shfl_xor(ns, o, 64));
  ns = vh_uniform(ns);
  // the next step's terms and values are read while this step's rows are
  // gathered
  int64_t p = rb + 4 * q;
  vh_i4 cv = vh_load4i(cr, static_cast<uint32_t>(p) * 4u);
  vh_f4 av = vh_load4(vr, static_cast<uint32_t>(p) * 4u);
  for (int s = 0; s < ns; ++s, p += 16) {
    const vh_i4 cur = cv;
    const vh_f4 cav = av;
    if (s + 1 < ns) {
      cv = vh_load4i(cr, static_cast<uint32_t>(p + 16) * 4u);
      av = vh_load4(vr, static_cast<uint32_t>(p + 16) * 4u);
    }
    // sl: compact row of U (>= 0), warm row w (-2 - w) or nothing (-1)
    int sl[4];
    if (DENSE_IN) {
#pragma unroll
      for (int e = 0; e < 4; ++e) sl[e] = (p + e < re) ? cur[e] : -1;
    } else {
      // each term's word of the row table (all four read at once): is its U
      // row nonempty, and which compact row is it
      int2 w[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) w[e] = stab[cur[e] >= 0 ? (cur[e] >> 5) : 0];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t bit = 1u << (cur[e] & 31);
        const bool hit = p + e < re && cur[e] >= 0 && (static_cast<uint32_t>(w[e].x) & bit) != 0u;
        sl[e] = hit ? w[e].y + __popc(static_cast<uint32_t>(w[e].x) & (bit - 1u)) : (p + e < re && cur[e] < -1 ? cur[e] : -1);
      }
    }
    // the document's 16 nonzeros in order, G rows in flight per lane
    constexpr int G = vh_group<NT>();
#pragma unroll 1
    for (int jj = 0; jj < 16; jj += G) {
      int sj[G];
      float aj[G];
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const int e = (jj + u) & 3;  // element e of the lane that read nonzero jj + u
        const int src = 16 * ((jj + u) >> 2) + m;
        const int se = e == 0 ? sl[0] : e == 1 ? sl[1] : e == 2 ? sl[2] : sl[3];
        const float ae = e == 0 ? cav[0] : e == 1 ? cav[1] : e == 2 ? cav[2] : cav[3];
        sj[u] = __shfl(se, src, 64);
        aj[u] = __shfl(ae, src, 64);
      }
      vh_f4 f[G][NT];
#pragma unroll
      for (int u = 0; u < G; ++u) {
        if (sj[u] >= 0) {
#pragma unroll
          for (int tt = 0; tt < NT; ++tt)
            f[u][tt] = live[tt] ? vh_row4<DENSE_IN>(Fr, static_cast<uint32_t>(sj[u]) * ldb + lo + 64u * tt)
                                : vh_f4{0.f, 0.f, 0.f, 0.f};
        } else if (sj[u] < -1) {
          const float* wr = warm + (-2 - sj[u]) * kVhTopics + 4 * q;
#pragma unroll
          for (int tt = 0; tt < NT; ++tt) f[u][tt] = *reinterpret_cast<const vh_f4*>(wr + 16 * tt);
        } else {
#pragma unroll
          for (int tt = 0; tt < NT; ++tt) f[u][tt] = vh_f4{0.f, 0.f, 0.f, 0.f};
        }
      }
#pragma unroll
      for (int u = 0; u < G; ++u)
#pragma unroll
        for (int tt = 0; tt < NT; ++tt)
          if (sj[u] != -1) acc[tt] += aj[u] * f[u][tt];
    }
  }
}

template <int NT, bool DENSE_IN>
__device__ __forceinline__ void vh_body(const VhArgs& a, int blk, int nblk) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int bw = blockDim.x >> 6;
  if (*a.status != 0) return;
  const int k = a.k;
  const int H = a.n_hot > 0 ? a.hot_ld : 0;
  const bool solve = a.W != nullptr;
  const int tw = DENSE_IN ? 0 : a.tab_words;
  float* ub = reinterpret_cast<float*>(smem);  // [H / 16][4][64][4]
  double* sW = reinterpret_cast<double*>(smem + static_cast<size_t>(H) * kVhTopics * sizeof(float));
  int2* stab = reinterpret_cast<int2*>(reinterpret_cast<unsigned char*>(sW) +
                                       (solve ? static_cast<size_t>(k) * k * sizeof(double) : 0));
  float* warm = reinterpret_cast<float*>(smem + vh_warm_offset(H, k, solve, tw));
  // stage U's hot rows (zeros for empty rows and topics past k) and W
  if (H > 0) {
    const __amdgpu_buffer_rsrc_t fr = vh_rsrc(a.F, a.F_bytes);
    for (int i = threadIdx.x; i < H * kVhTopics; i += blockDim.x) {
      const int hc = i / kVhTopics, c = i - hc * kVhTopics;
      int64_t off = -1;
      if (hc < a.n_hot) {
        const int r = a.hot_col[hc];
        const int s = a.slot != nullptr ? a.slot[r] : r;
        if (s >= 0) off = static_cast<int64_t>(s) * a.ld * 4;
      }
      const float v = vh_load1(fr, static_cast<uint32_t>(off < 0 ? 0 : off) + 4u * static_cast<uint32_t>(c));
      ub[(((hc >> 4) * 4 + ((hc >> 2) & 3)) * kVhTopics + c) * 4 + (hc & 3)] = (off >= 0 && c < k) ? v : 0.f;
    }
  }
  if (solve)
    for (int i = threadIdx.x; i < k * k; i += blockDim.x) sW[i] = a.W[i];
  for (int i = threadIdx.x; i < tw; i += blockDim.x) stab[i] = a.rowtab[i];
  // stage U's warm rows (zeros for empty rows and topics past k)
  if (a.n_warm > 0) {
    const __amdgpu_buffer_rsrc_t fr = vh_rsrc(a.F, a.F_bytes);
    for (int i = threadIdx.x; i < a.n_warm * kVhTopics; i += blockDim.x) {
      const int w = i / kVhTopics, c = i - w * kVhTopics;
      const int r = a.warm_col[w];
      const int s = a.slot != nullptr ? a.slot[r] : r;
      const int64_t off = s >= 0 ? static_cast<int64_t>(s) * a.ld * 4 : 0;
      const float v = vh_load1(fr, static_cast<uint32_t>(off) + 4u * static_cast<uint32_t>(c));
      warm[i] = (s >= 0 && c < k) ? v : 0.f;
    }
  }
  // gathered-entry count (the streamed nonzeros times the entries of their
  // terms' rows of U), this block's share of the terms
  uint32_t gath = 0;
  if (!DENSE_IN && a.gathered != nullptr)
    for (int64_t r = static_cast<int64_t>(blk) * blockDim.x + threadIdx.x; r < a.n_u;
         r += static_cast<int64_t>(nblk) * blockDim.x)
      gath += static_cast<uint32_t>(a.sdf[r]) * static_cast<uint32_t>(a.urp[r + 1] - a.urp[r]);
  __syncthreads();

  const int lane = lane_id();
  const int wv = threadIdx.x >> 6;
  const int m = lane & 15, q = lane >> 4;
  const int64_t tiles = (a.rows + kVhTile - 1) / kVhTile;
  const __amdgpu_buffer_rsrc_t hr = vh_rsrc(a.hot, static_cast<uint32_t>(H > 0 ? a.rows * H * 4 : 0));
  // wave w of the launch takes tiles w, w + W, w + 2 W, ...: the waves
  // running at once work on neighbouring documents
  const int64_t nw = static_cast<int64_t>(nblk) * bw;
  for (int64_t t = static_cast<int64_t>(blk) * bw + wv; t < tiles; t += nw) {
    const int64_t r0 = kVhTile * t;
    const int nrows = static_cast<int>(a.rows - r0 < kVhTile ? a.rows - r0 : kVhTile);
    // the hot columns of the 16 documents (rows past the end read as zero)
    const uint32_t abase = static_cast<uint32_t>((r0 + m) * H + 4 * q) * 4u;
    const int64_t rb = a.rowptr[r0 + (m < nrows ? m : nrows)];
    const int64_t re = a.rowptr[r0 + (m + 1 < nrows ? m + 1 : nrows)];
    // streamed part first, then the hot product adds on the same sums
    vh_f4 acc[4];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) acc[tt] = vh_f4{0.f, 0.f, 0.f, 0.f};
    vh_stream<NT, DENSE_IN>(a, rb, re, stab, warm, acc);
    // hot product: tile tt = (U_H^T)(topics 16 tt ..) x (A_H^T)(.., docs),
    // the hot columns read eight 16-column groups at a time
    for (int g0 = 0; g0 < H / 16; g0 += kVhHotChunk) {
      vh_f4 arow4[kVhHotChunk];
#pragma unroll
      for (int g = 0; g < kVhHotChunk; ++g)
        arow4[g] = 16 * (g0 + g) < H ? vh_load4(hr, abase + 64u * (g0 + g)) : vh_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int gg = 0; gg < kVhHotChunk; ++gg) {
        const int g = g0 + gg;
        if (16 * g >= H) break;
        const vh_f4 av = arow4[gg];
        vh_f4 bv[4];
#pragma unroll
        for (int tt = 0; tt < NT; ++tt)
          bv[tt] = *reinterpret_cast<const vh_f4*>(&ub[((g * 4 + q) * kVhTopics + 16 * tt + m) * 4]);
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) acc[tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[tt].x, av.x, acc[tt], 0, 0, 0);
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) acc[tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[tt].y, av.y, acc[tt], 0, 0, 0);
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) acc[tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[tt].z, av.z, acc[tt], 0, 0, 0);
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) acc[tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[tt].w, av.w, acc[tt], 0, 0, 0);
      }
    }
    // raw sums of document r0 + m, topic 16 tt + 4 q + i (topics past k,
    // which a dense input's next row may have filled, are zeroed)
    float raw[4][4];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
      for (int i = 0; i < 4; ++i) raw[tt][i] = 16 * tt + 4 * q + i < k ? acc[tt][i] : 0.f;
    bool bad = false;
    const int64_t ra = r0 + m;
    if (!solve) {
#pragma unroll
      for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = 16 * tt + 4 * q + i;
          if (ra < a.rows && c < k) {
            bad |= !isfinite(raw[tt][i]);
            a.X[ra * a.x_ld + a.x_c0 + c] = raw[tt][i];
          }
        }
      if (__ballot(bad) != 0 && lane == 0) atomicCAS(a.status, 0, static_cast<int32_t>(NMF_ERR_NONFINITE));
      continue;
    }
    // float64 solve on the matrix cores: out (16 docs x 64 topics) =
    // raw (16 x k) W (k x 64); step (tt, i) takes in lane (m, q) the raw sum
    // of topic rr = 16 tt + 4 q + i as the A operand's column q and
    // W[rr][16 t2 + m] as the B operand's row q
    vh_d4 o[4];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) o[tt] = vh_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (16 * tt + i >= k) break;
        const int rr = 16 * tt + 4 * q + i;
        const double av = static_cast<double>(raw[tt][i]);
#pragma unroll
        for (int t2 = 0; t2 < NT; ++t2) {
          const int c = 16 * t2 + m;
          const double bv = (rr < k && c < k) ? sW[rr * k + c] : 0.0;
          o[t2] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, o[t2], 0, 0, 0);
        }
      }
    // o[tt][i]: document r0 + q + 4 i, topic 16 tt + m
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t r = r0 + q + 4 * i;
        const int c = 16 * tt + m;
        if (r < a.rows && c < k) {
          const float y = static_cast<float>(o[tt][i] > 0.0 ? o[tt][i] : 0.0);
          bad |= !isfinite(o[tt][i]) || !isfinite(y);
          a.X[r * k + c] = y;
        }
      }
    if (__ballot(bad) != 0 && lane == 0) atomicCAS(a.status, 0, static_cast<int32_t>(NMF_ERR_NONFINITE));
  }
  if (a.gathered != nullptr) {
    unsigned long long g = gath;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) g += __shfl_xor(g, d, 64);
    if (lane == 0 && g != 0) atomicAdd(&a.gathered[(blk * bw + wv) % kGathSlots], g);
  }
}

template <int NT, bool DENSE_IN>
__global__ __launch_bounds__(64 * kVhWavesMax) void k_vhalf(VhArgs a) {
  vh_body<NT, DENSE_IN>(a, blockIdx.x, gridDim.x);
}
template <int NT, bool DENSE_IN>
__global__ __launch_bounds__(64 * kVhWavesMax) void k_vhalf_b(const VhArgs* as, const BlockMap* map) {
  const BlockMap mp = map[blockIdx.x];
  const VhArgs a = as[mp.prob];
  vh_body<NT, DENSE_IN>(a, mp.blk, mp.nblk);
}

// The batched form for every topic-tile count: one launch serves all the
// problems of a batch, each block running its problem's instantiation
// (the LDS of the launch is the largest any problem needs).
__global__ __launch_bounds__(64 * kVhWavesMax) void k_vhalf_any_b(const VhArgs* as, const BlockMap* map) {
  const BlockMap mp = map[blockIdx.x];
  const VhArgs a = as[mp.prob];
  switch ((a.k + 15) / 16) {
    case 1: vh_body<1, false>(a, mp.blk, mp.nblk); break;
    case 2: vh_body<2, false>(a, mp.blk, mp.nblk); break;
    case 3: vh_body<3, false>(a, mp.blk, mp.nblk); break;
    default: vh_body<4, false>(a, mp.blk, mp.nblk); break;
  }
}

template <int NT, bool DENSE_IN>
hipError_t vh_launch(nmf_handle* h, const VhArgs& a, int waves_max) {
  const size_t blk_lds = vh_block_lds(a.n_hot > 0 ? a.hot_ld : 0, a.k, a.W != nullptr,
                                      a.rowtab != nullptr ? a.tab_words : 0, a.n_warm);
  int waves = std::min(std::max(waves_max, 1), kVhWavesMax);
  const size_t lds = blk_lds;
  if (lds > kVhLds) return hipErrorInvalidValue;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_vhalf<NT, DENSE_IN>, 64 * waves, lds) != hipSuccess)
    return hipErrorInvalidValue;
  if (per_cu < 1) per_cu = 1;
  const int64_t tiles = (a.rows + kVhTile - 1) / kVhTile;
  const unsigned blocks =
      static_cast<unsigned>(std::min<int64_t>((tiles + waves - 1) / waves, static_cast<int64_t>(h->num_cus) * per_cu));
  return launch_rec(h, k_vhalf<NT, DENSE_IN>, DENSE_IN ? k_vhalf_b<NT, DENSE_IN> : k_vhalf_any_b, blocks, 64u * waves,
                    lds, a);
}

template <bool DENSE_IN>
hipError_t vh_dispatch(nmf_handle* h, const VhArgs& a, int waves) {
  switch ((a.k + 15) / 16) {
    case 1: return vh_launch<1, DENSE_IN>(h, a, waves);
    case 2: return vh_launch<2, DENSE_IN>(h, a, waves);
    case 3: return vh_launch<3, DENSE_IN>(h, a, waves);
    default: return vh_launch<4, DENSE_IN>(h, a, waves);
  }
}

}  // namespace

hipError_t vhalf(nmf_handle* h, const Plan& p, const Factor& F, const float* dense_in, float* X, const double* W,
                 int waves) {
  // byte offsets into the hot block, the stream, F and X are 32-bit
  if (h->k > kVhTopics || p.hot_ld > kMaxHot || (p.rows + kVhTile) * p.hot_ld * 4 >= (int64_t{1} << 32) ||
      (p.rows + kVhTile) * h->k * 4 >= (int64_t{1} << 32) || (p.nnz + 4) * 4 >= (int64_t{1} << 32))
    return hipErrorInvalidValue;
  VhArgs a{};
  a.rowptr = p.rowptr;
  a.col = p.col;
  a.val = static_cast<const float*>(p.val);
  a.stream_bytes = static_cast<uint32_t>((p.nnz + 4) * 4);  // the padded stream and its spare entries
  a.rowtab = dense_in ? nullptr : F.rowtab;
  a.tab_words = dense_in ? 0 : static_cast<int32_t>((F.rows + 31) / 32);
  a.sdf = p.sdf;
  a.urp = F.row_ptr;
  a.n_u = F.rows;
  a.F = dense_in ? dense_in : static_cast<const float*>(F.dense);
  a.ld = dense_in ? h->k : F.ld;
  a.F_bytes = static_cast<uint32_t>(dense_in ? h->n * h->k * 4 : F.rows * F.ld * 4);
  a.hot = static_cast<const float*>(p.hot);
  a.hot_col = p.hot_col;
  a.warm_col = p.warm_col;
  a.n_warm = p.n_warm;
  a.hot_ld = p.hot_ld;
  a.n_hot = p.n_hot;
  a.slot = dense_in ? nullptr : F.slot;
  a.rows = p.rows;
  a.k = h->k;
  a.W = W;
  a.X = X;
  a.x_ld = h->k;
  a.x_c0 = 0;
  a.status = h->status;
  a.gathered = dense_in ? nullptr : h->met.gathered;
  return dense_in ? vh_dispatch<true>(h, a, waves) : vh_dispatch<false>(h, a, waves);
}

hipError_t vhalf_window(nmf_handle* h, const Plan& p, const Factor& F, float* X, const ColWindow& win) {
  if (win.kw < 1 || win.kw > kVhTopics || win.x_c0 < 0 || win.x_c0 + win.kw > win.x_ld || F.ld < win.kw ||
      F.ld % 4 != 0 || p.hot_ld > kMaxHot || (p.rows + kVhTile) * p.hot_ld * 4 >= (int64_t{1} << 32) ||
      (p.rows + kVhTile) * win.x_ld * 4 >= (int64_t{1} << 32) || (p.nnz + 4) * 4 >= (int64_t{1} << 32) ||
      F.rows * F.ld * 4 >= (int64_t{1} << 32))
    return hipErrorInvalidValue;
  VhArgs a{};
  a.rowptr = p.rowptr;
  a.col = p.col;
  a.val = static_cast<const float*>(p.val);
  a.stream_bytes = static_cast<uint32_t>((p.nnz + 4) * 4);
  a.rowtab = F.rowtab;
  a.tab_words = static_cast<int32_t>((F.rows + 31) / 32);
  a.sdf = p.sdf;
  a.urp = F.row_ptr;
  a.n_u = F.rows;
  a.F = static_cast<const float*>(F.dense);
  a.ld = F.ld;
  a.F_bytes = static_cast<uint32_t>(F.rows * F.ld * 4);
  a.hot = static_cast<const float*>(p.hot);
  a.hot_col = p.hot_col;
  a.warm_col = p.warm_col;
  a.n_warm = p.n_warm;
  a.hot_ld = p.hot_ld;
  a.n_hot = p.n_hot;
  a.slot = F.slot;
  a.rows = p.rows;
  a.k = win.kw;
  a.W = nullptr;
  a.X = X;
  a.x_ld = win.x_ld;
  a.x_c0 = win.x_c0;
  a.status = h->status;
  a.gathered = h->met.gathered;
  return vh_dispatch<false>(h, a, h->waves[0]);
}

// Empty launches in the places of a product's second and third kernels, so
// that problems of a batch with and without this kernel record equally long
// launch sequences.
hipError_t vhalf_placeholder(nmf_handle* h) {
  VhArgs a{};
  return launch_rec(h, k_vhalf<4, false>, k_vhalf_b<4, false>, 0, 64, 0, a);
}

}  // namespace nmfk
