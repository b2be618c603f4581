// Hot block of the V half (float32, k <= 64).
//
// The terms that occur in the most documents (rows of A with at least
// kHotDensity * m nonzeros, at most kMaxHot of them) are kept out of the
// V-half sparse stream: their entries are stored as a dense docs x hot
// block.  For those columns A^T U is a dense product (the block is 12 % to
// 85 % full), so it runs on the matrix cores instead of as per-nonzero
// gathers of U rows.  k_spmm first leaves the raw sums of the rest of each
// document's stream in X; this kernel adds the hot block's product and, in
// the solving form, applies the epilogue of Algorithm 2 step 1:
//   X_r = max(0, (cold_r + hot_r) W),  W = (U^T U)^-1 (float64).
//
// Layout of the product: a wave owns 16 documents and all 64 topic slots
// (four 16-topic tiles), one 16x16x4 MFMA per tile and four hot columns.
// Lane l (m = l % 16, q = l / 16) loads hot columns 16 g + 4 q .. + 3 of
// document r0 + m as one float4 and feeds them to four MFMAs as the A
// operand's column q; the B operand of the same MFMA, row q, is U's row of
// the same hot column, staged in LDS as ub[g][q][topic][s] so that a lane
// reads its four values with one 16-byte load.  Tile tt then holds the sums
// for document r0 + 4 q + i, topic 16 tt + m in element i.  The solve is a
// second product on the matrix cores, in float64: the 16 documents' raw sums
// (through a per-wave LDS tile) times W, 16x16x4 float64 MFMAs with the same
// operand layout; their result holds document r0 + q + 4 i in element i.
#include <algorithm>

#include "nmf_device.h"

namespace nmfk {

namespace {

typedef float hot_f4 __attribute__((ext_vector_type(4)));
typedef double hot_d4 __attribute__((ext_vector_type(4)));

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
  int64_t rows;         // documents
  int32_t k;
  const double* W;  // k x k, or null: X receives the raw sums
  float* X;         // in: raw sums of the rest of the stream; out: as above
  int32_t* status;
};

size_t hot_lds_bytes(int hot_ld, int k, bool solve) {
  size_t b = static_cast<size_t>(hot_ld) * kHotTopics * sizeof(float);
  if (solve) b += static_cast<size_t>((k * k + 1) & ~1) * sizeof(double) + kHotWaves * kHotTopics * 16 * sizeof(float);
  return b;
}

__device__ __forceinline__ void k_hot_body(const HotArgs& a, int blk, int nblk) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (*a.status != 0) return;
  const int k = a.k;
  const int H = a.hot_ld;
  float* ub = reinterpret_cast<float*>(smem);  // [H / 16][4][64][4]
  double* sW = reinterpret_cast<double*>(smem + static_cast<size_t>(H) * kHotTopics * sizeof(float));
  // per-wave raw tile [topic][16 docs], 16-byte aligned
  float* rt = reinterpret_cast<float*>(sW + ((k * k + 1) & ~1)) + (threadIdx.x >> 6) * kHotTopics * 16;
  for (int i = threadIdx.x; i < H * kHotTopics; i += blockDim.x) {
    const int hc = i / kHotTopics, c = i - hc * kHotTopics;
    float v = 0.f;
    if (hc < a.n_hot && c < k) {
      const int r = a.hot_col[hc];
      if (a.slot != nullptr) {
        const int s = a.slot[r];
        if (s >= 0) v = a.F[static_cast<int64_t>(s) * a.ld + c];
      } else {
        v = a.F[static_cast<int64_t>(r) * a.ld + c];
      }
    }
    ub[(((hc >> 4) * 4 + ((hc >> 2) & 3)) * kHotTopics + c) * 4 + (hc & 3)] = v;
  }
  if (a.W != nullptr)
    for (int i = threadIdx.x; i < k * k; i += blockDim.x) sW[i] = a.W[i];
  __syncthreads();
  const int lane = lane_id();
  const int m = lane & 15, q = lane >> 4;
  const int bw = blockDim.x >> 6;
  const int64_t nw = static_cast<int64_t>(nblk) * bw;
  const int64_t tiles = (a.rows + 15) / 16;
  constexpr int HG = kMaxHot / 16;
  for (int64_t t = static_cast<int64_t>(blk) * bw + (threadIdx.x >> 6); t < tiles; t += nw) {
    const int64_t r0 = 16 * t;
    const int64_t ra = r0 + m;
    // every load of the tile in flight at once: the documents' hot columns
    // and the raw sums the stream left in X
    const float* __restrict__ arow = a.hot + ra * H + 4 * q;
    hot_f4 arow4[HG];
#pragma unroll
    for (int g = 0; g < HG; ++g)
      arow4[g] = (16 * g < H && ra < a.rows) ? *reinterpret_cast<const hot_f4*>(arow + 16 * g)
                                             : hot_f4{0.f, 0.f, 0.f, 0.f};
    float cold[4][4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t r = r0 + 4 * q + i;
        const int c = 16 * tt + m;
        cold[tt][i] = (r < a.rows && c < k) ? a.X[r * k + c] : 0.f;
      }
    hot_f4 acc[4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) acc[tt] = hot_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int g = 0; g < HG; ++g) {
      if (16 * g >= H) break;
      const hot_f4 av = arow4[g];
#pragma unroll
      for (int tt = 0; tt < 4; ++tt) {
        const hot_f4 bv = *reinterpret_cast<const hot_f4*>(&ub[((g * 4 + q) * kHotTopics + 16 * tt + m) * 4]);
        acc[tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv.x, acc[tt], 0, 0, 0);
        acc[tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv.y, acc[tt], 0, 0, 0);
        acc[tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, bv.z, acc[tt], 0, 0, 0);
        acc[tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, bv.w, acc[tt], 0, 0, 0);
      }
    }
    if (a.W == nullptr) {
#pragma unroll
      for (int tt = 0; tt < 4; ++tt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t r = r0 + 4 * q + i;
          const int c = 16 * tt + m;
          if (r < a.rows && c < k) a.X[r * k + c] = cold[tt][i] + acc[tt][i];
        }
      continue;
    }
    // raw sums of the 16 documents, topic-major, then the float64 solve on
    // the matrix cores: out (16 docs x 64 topics) = raw (16 x k) W (k x 64),
    // one 16x16x4 MFMA per topic tile and four rows of W; lane l feeds
    // raw[doc m][rr = 4 s + q] and W[4 s + q][16 tt + m]
#pragma unroll
    for (int tt = 0; tt < 4; ++tt)
#pragma unroll
      for (int i = 0; i < 4; ++i) rt[(16 * tt + m) * 16 + 4 * q + i] = cold[tt][i] + acc[tt][i];
    hot_d4 o[4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) o[tt] = hot_d4{0.0, 0.0, 0.0, 0.0};
    for (int s4 = 0; s4 < k; s4 += 4) {
      const int rr = s4 + q;
      const double av = rr < k ? static_cast<double>(rt[rr * 16 + m]) : 0.0;
#pragma unroll
      for (int tt = 0; tt < 4; ++tt) {
        const int c = 16 * tt + m;
        const double bv = (rr < k && c < k) ? sW[rr * k + c] : 0.0;
        o[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, o[tt], 0, 0, 0);
      }
    }
    // o[tt][i]: document r0 + q + 4 i, topic 16 tt + m (the float64 form
    // interleaves the rows)
#pragma unroll
    for (int tt = 0; tt < 4; ++tt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t r = r0 + q + 4 * i;
        const int c = 16 * tt + m;
        if (r < a.rows && c < k) a.X[r * k + c] = static_cast<float>(o[tt][i] > 0.0 ? o[tt][i] : 0.0);
      }
  }
}
__global__ __launch_bounds__(64 * kHotWaves) void k_hot(HotArgs a) { k_hot_body(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(64 * kHotWaves) void k_hot_b(const HotArgs* as, const BlockMap* map) {
  const BlockMap mp = map[blockIdx.x];
  const HotArgs a = as[mp.prob];
  k_hot_body(a, mp.blk, mp.nblk);
}

}  // namespace

hipError_t hot_placeholder(nmf_handle* h) {
  HotArgs a{};
  return launch_rec(h, k_hot, k_hot_b, 0, 64 * kHotWaves, 0, a);
}

hipError_t hot_finish(nmf_handle* h, const Plan& p, const Factor& F, const float* dense_in, float* X,
                      const double* W) {
  if (p.n_hot <= 0 || h->k > kHotTopics || p.hot_ld > kMaxHot) return hipErrorInvalidValue;
  HotArgs a{};
  a.hot = static_cast<const float*>(p.hot);
  a.hot_col = p.hot_col;
  a.hot_ld = p.hot_ld;
  a.n_hot = p.n_hot;
  a.slot = dense_in ? nullptr : F.slot;
  a.F = dense_in ? dense_in : static_cast<const float*>(F.dense);
  a.ld = dense_in ? h->k : F.ld;
  a.rows = p.rows;
  a.k = h->k;
  a.W = W;
  a.X = X;
  a.status = h->status;
  const int64_t tiles = (p.rows + 15) / 16;
  const unsigned blocks =
      static_cast<unsigned>(std::min<int64_t>((tiles + kHotWaves - 1) / kHotWaves, 2 * h->num_cus));
  return launch_rec(h, k_hot, k_hot_b, blocks, 64 * kHotWaves, hot_lds_bytes(p.hot_ld, h->k, W != nullptr), a);
}

}  // namespace nmfk
