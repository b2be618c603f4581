// Hot block of the V half (float32, k <= 64).
//
// The terms that occur in the most documents (rows of A with at least
// kHotDensity * m nonzeros, at most kMaxHot of them) are kept out of the
// V-half sparse stream: their entries are stored as a dense docs x hot
// block.  For those columns A^T U is close to a dense product (with Zipf
// term frequencies the 128 densest terms fill about a third of their block),
// so it runs on the matrix cores instead of as per-nonzero gathers of U rows.  k_spmm first leaves the raw sums of the rest of each
// document's stream in X; this kernel adds the hot block's product and, in
// the solving form, applies the epilogue of Algorithm 2 step 1:
//   X_r = max(0, (cold_r + hot_r) W),  W = (U^T U)^-1 (float64).
//
// Layout: a wave owns 16 documents and all 64 topic slots.  The hot product
// is computed transposed, (U_H^T)(A_H^T), as four 16-topic x 16-document
// tiles, one 16x16x4 MFMA per tile and four hot columns: lane l (m = l % 16,
// q = l / 16) loads hot columns 16 g + 4 q .. + 3 of document r0 + m as one
// float4 (the B operand's column m, rows q, one per MFMA) and reads U's rows
// of the same hot columns from LDS, staged as ub[g][q][topic][s] so that one
// 16-byte load gives its four A operands.  Element i of tile tt then holds
// document r0 + m, topic 16 tt + 4 q + i.  The float64 solve (raw W) is a
// second product on the matrix cores whose contraction order is free: step
// (tt, i) takes, in lane (m, q), the raw sum the lane holds for topic
// rr = 16 tt + 4 q + i as its A operand and W[rr][16 t2 + m] as its B
// operand, so the raw sums never leave registers; the float64 result holds
// document r0 + q + 4 i, topic 16 t2 + m in element i.
#include <algorithm>

#include "nmf_device.h"

namespace nmfk {

namespace {

typedef float hot_f4 __attribute__((ext_vector_type(4)));
typedef double hot_d4 __attribute__((ext_vector_type(4)));

// Range-checked buffer loads (the hardware returns zero past the resource's
// size), so that the tile's loads carry no branches and the MFMAs can start as
// soon as their own operands have arrived.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t hot_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), static_cast<short>(0), static_cast<int>(bytes),
                                           0x00020000);
}
__device__ __forceinline__ hot_f4 hot_load4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(hot_f4, __builtin_amdgcn_raw_buffer_load_b128(r, static_cast<int>(off), 0, 0));
}
__device__ __forceinline__ float hot_load1(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, static_cast<int>(off), 0, 0));
}

constexpr int kHotWaves = 8;
constexpr int kHotTopics = 64;  // topic slots per wave (k <= 64)

struct HotArgs {
  const float* hot;        // [rows][hot_ld]
  const int32_t* hot_col;  // [n_hot]: U row of hot column h
  int32_t hot_ld;          // a multiple of 16
  int32_t n_hot;
  const int32_t* slot;  // compact index of each U row (-1: empty), or null for a dense input
  const float* F;       // compact dense U rows, or the dense input
  int32_t ld;           // row pitch of F
  uint32_t F_bytes;     // bytes of F (staging loads are range-checked against it)
  int64_t rows;         // documents
  int32_t k;
  const double* W;  // k x k, or null: X receives the raw sums
  float* X;         // in: raw sums of the rest of the stream; out: as above
  int32_t* status;
};

size_t hot_lds_bytes(int hot_ld, int k, bool solve) {
  size_t b = static_cast<size_t>(hot_ld) * kHotTopics * sizeof(float);
  if (solve) b += static_cast<size_t>(k) * k * sizeof(double);
  return b;
}

// NT: 16-topic tiles in use (ceil(k / 16)); the product and the solve skip the rest.
template <int NT>
__device__ __forceinline__ void k_hot_body(const HotArgs& a, int blk, int nblk) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (*a.status != 0) return;
  const int k = a.k;
  const int H = a.hot_ld;
  float* ub = reinterpret_cast<float*>(smem);  // [H / 16][4][64][4]
  double* sW = reinterpret_cast<double*>(smem + static_cast<size_t>(H) * kHotTopics * sizeof(float));
  // where each hot column's U row starts in F (-1: an empty row, staged as
  // zeros), then every staged value with independent range-checked loads,
  // several in flight per thread
  __shared__ int64_t s_off[kMaxHot];
  for (int hc = threadIdx.x; hc < H; hc += blockDim.x) {
    int64_t off = -1;
    if (hc < a.n_hot) {
      const int r = a.hot_col[hc];
      const int s = a.slot != nullptr ? a.slot[r] : r;
      if (s >= 0) off = static_cast<int64_t>(s) * a.ld * 4;
    }
    s_off[hc] = off;
  }
  __syncthreads();
  const __amdgpu_buffer_rsrc_t fr = hot_rsrc(a.F, a.F_bytes);
  constexpr int kStage = kMaxHot * kHotTopics / (64 * kHotWaves);  // values per thread at most
  float sv[kStage];
#pragma unroll
  for (int u = 0; u < kStage; ++u) {
    const int i = threadIdx.x + u * 64 * kHotWaves;
    const int hc = (i / kHotTopics) < H ? i / kHotTopics : 0, c = i % kHotTopics;
    const int64_t off = s_off[hc];
    const float v = hot_load1(fr, static_cast<uint32_t>(off < 0 ? 0 : off) + 4u * static_cast<uint32_t>(c));
    sv[u] = (off >= 0 && c < k) ? v : 0.f;
  }
#pragma unroll
  for (int u = 0; u < kStage; ++u) {
    const int i = threadIdx.x + u * 64 * kHotWaves;
    const int hc = i / kHotTopics, c = i - hc * kHotTopics;
    if (hc < H) ub[(((hc >> 4) * 4 + ((hc >> 2) & 3)) * kHotTopics + c) * 4 + (hc & 3)] = sv[u];
  }
  if (a.W != nullptr) {
    constexpr int kWStage = kHotTopics * kHotTopics / (64 * kHotWaves);
    const __amdgpu_buffer_rsrc_t wr = hot_rsrc(a.W, static_cast<uint32_t>(k * k * 8));
    double wv[kWStage];
#pragma unroll
    for (int u = 0; u < kWStage; ++u) {
      const int i = threadIdx.x + u * 64 * kHotWaves;
      wv[u] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(wr, 8 * i, 0, 0));
    }
#pragma unroll
    for (int u = 0; u < kWStage; ++u) {
      const int i = threadIdx.x + u * 64 * kHotWaves;
      if (i < k * k) sW[i] = wv[u];
    }
  }
  __syncthreads();
  const int lane = lane_id();
  const int m = lane & 15, q = lane >> 4;
  const int bw = blockDim.x >> 6;
  const int64_t nw = static_cast<int64_t>(nblk) * bw;
  const int64_t tiles = (a.rows + 15) / 16;
  constexpr int HG = kMaxHot / 16;
  const __amdgpu_buffer_rsrc_t hr = hot_rsrc(a.hot, static_cast<uint32_t>(a.rows * H * 4));
  const __amdgpu_buffer_rsrc_t xr = hot_rsrc(a.X, static_cast<uint32_t>(a.rows * k * 4));
  for (int64_t t = static_cast<int64_t>(blk) * bw + (threadIdx.x >> 6); t < tiles; t += nw) {
    const int64_t r0 = 16 * t;
    const int64_t ra = r0 + m;
    // every load of the tile in flight at once: the documents' hot columns
    // (rows past the end read as zero) and the raw sums the stream left in X
    // (topics past k are zeroed after the load)
    const uint32_t abase = static_cast<uint32_t>(ra * H + 4 * q) * 4u;
    hot_f4 arow4[HG];
#pragma unroll
    for (int g = 0; g < HG; ++g)
      arow4[g] = 16 * g < H ? hot_load4(hr, abase + 64u * g) : hot_f4{0.f, 0.f, 0.f, 0.f};
    // cold[tt][i]: raw sum of document r0 + m, topic 16 tt + 4 q + i (the
    // layout of the transposed product below)
    const uint32_t xbase = static_cast<uint32_t>(ra * k + 4 * q) * 4u;
    float cold[4][4];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float v = hot_load1(xr, xbase + static_cast<uint32_t>(16 * tt + i) * 4u);
        cold[tt][i] = 16 * tt + 4 * q + i < k ? v : 0.f;
      }
    // transposed product: tile tt = (U_H^T)(topics 16 tt ..) x (A_H^T)(.., docs),
    // element i of lane (m, q) = document r0 + m, topic 16 tt + 4 q + i
    hot_f4 acc[4];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) acc[tt] = hot_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int g = 0; g < HG; ++g) {
      if (16 * g >= H) break;
      const hot_f4 av = arow4[g];
      hot_f4 bv[4];
#pragma unroll
      for (int tt = 0; tt < NT; ++tt)
        bv[tt] = *reinterpret_cast<const hot_f4*>(&ub[((g * 4 + q) * kHotTopics + 16 * tt + m) * 4]);
      // consecutive MFMAs go to different tiles, so none waits on the one before
#pragma unroll
      for (int tt = 0; tt < NT; ++tt) acc[tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[tt].x, av.x, acc[tt], 0, 0, 0);
#pragma unroll
      for (int tt = 0; tt < NT; ++tt) acc[tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[tt].y, av.y, acc[tt], 0, 0, 0);
#pragma unroll
      for (int tt = 0; tt < NT; ++tt) acc[tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[tt].z, av.z, acc[tt], 0, 0, 0);
#pragma unroll
      for (int tt = 0; tt < NT; ++tt) acc[tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[tt].w, av.w, acc[tt], 0, 0, 0);
    }
    float raw[4][4];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
      for (int i = 0; i < 4; ++i) raw[tt][i] = cold[tt][i] + acc[tt][i];
    // a non-finite sum or solution (float32 overflow) raises the sticky
    // NONFINITE status instead of being clamped to zero
    bool bad = false;
    if (a.W == nullptr) {
#pragma unroll
      for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = 16 * tt + 4 * q + i;
          if (ra < a.rows && c < k) {
            bad |= !isfinite(raw[tt][i]);
            a.X[ra * k + c] = raw[tt][i];
          }
        }
      if (__ballot(bad) != 0 && lane == 0) atomicCAS(a.status, 0, static_cast<int32_t>(NMF_ERR_NONFINITE));
      continue;
    }
    // the float64 solve on the matrix cores: out (16 docs x 64 topics) =
    // raw (16 x k) W (k x 64).  The step (tt, i) takes, in lane (m, q), the
    // raw sum the lane already holds, raw[doc m][rr = 16 tt + 4 q + i], as
    // the A operand's column q and W[rr][16 tt' + m] as the B operand's row
    // q; steps whose four rr are all past k are skipped.
    hot_d4 o[4];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) o[tt] = hot_d4{0.0, 0.0, 0.0, 0.0};
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
    // o[tt][i]: document r0 + q + 4 i, topic 16 tt + m (the float64 form
    // interleaves the rows)
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
}
template <int NT>
__global__ __launch_bounds__(64 * kHotWaves) void k_hot(HotArgs a) { k_hot_body<NT>(a, blockIdx.x, gridDim.x); }
template <int NT>
__global__ __launch_bounds__(64 * kHotWaves) void k_hot_b(const HotArgs* as, const BlockMap* map) {
  const BlockMap mp = map[blockIdx.x];
  const HotArgs a = as[mp.prob];
  k_hot_body<NT>(a, mp.blk, mp.nblk);
}

}  // namespace

hipError_t hot_placeholder(nmf_handle* h) {
  HotArgs a{};
  return launch_rec(h, k_hot<4>, k_hot_b<4>, 0, 64 * kHotWaves, 0, a);
}

hipError_t hot_finish(nmf_handle* h, const Plan& p, const Factor& F, const float* dense_in, float* X,
                      const double* W) {
  // the tile loads address the block and X with 32-bit byte offsets
  if (p.n_hot <= 0 || h->k > kHotTopics || p.hot_ld > kMaxHot ||
      (p.rows + 16) * p.hot_ld * 4 >= (int64_t{1} << 32) || (p.rows + 16) * h->k * 4 >= (int64_t{1} << 32))
    return hipErrorInvalidValue;
  HotArgs a{};
  a.hot = static_cast<const float*>(p.hot);
  a.hot_col = p.hot_col;
  a.hot_ld = p.hot_ld;
  a.n_hot = p.n_hot;
  a.slot = dense_in ? nullptr : F.slot;
  a.F = dense_in ? dense_in : static_cast<const float*>(F.dense);
  a.ld = dense_in ? h->k : F.ld;
  a.F_bytes = static_cast<uint32_t>(dense_in ? h->n * h->k * 4 : F.rows * F.ld * 4);
  a.rows = p.rows;
  a.k = h->k;
  a.W = W;
  a.X = X;
  a.status = h->status;
  const int64_t tiles = (p.rows + 15) / 16;
  const unsigned blocks =
      static_cast<unsigned>(std::min<int64_t>((tiles + kHotWaves - 1) / kHotWaves, 2 * h->num_cus));
  const size_t lds = hot_lds_bytes(p.hot_ld, h->k, W != nullptr);
  switch ((h->k + 15) / 16) {
    case 1: return launch_rec(h, k_hot<1>, k_hot_b<1>, blocks, 64 * kHotWaves, lds, a);
    case 2: return launch_rec(h, k_hot<2>, k_hot_b<2>, blocks, 64 * kHotWaves, lds, a);
    case 3: return launch_rec(h, k_hot<3>, k_hot_b<3>, blocks, 64 * kHotWaves, lds, a);
    default: return launch_rec(h, k_hot<4>, k_hot_b<4>, blocks, 64 * kHotWaves, lds, a);
  }
}

}  // namespace nmfk
