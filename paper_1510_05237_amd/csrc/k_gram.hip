// Gram matrix of the fixed factor and its inverse: the (U^T U)^-1 and
// (V^T V)^-1 of Algorithms 1-2.
//
//  1. G = F^T F is summed over the rows of F in the working type T.  Each of
//     kGramBlocks blocks owns a fixed slice of rows.  float32: k_gram_mfma,
//     a dense contraction on the matrix cores (v_mfma_f32_16x16x4f32, four
//     rows per instruction, the upper-triangle 16 x 16 tiles of G in
//     accumulator registers); float64: k_gram_partial, the upper-triangle
//     sums in registers, one FMA per entry and row.
//  2. k_gram_reduce: every block owns 64 upper-triangle entries; its four
//     waves add strided subsets of the block partials in float64 and the
//     four sums are combined in a fixed order, so G does not depend on
//     scheduling.
//  3. k_gram_block (one block) inverts in float64 (see there):
//      * dead topics (zero diagonal: an all-zero column of F) get an identity
//        row and column, which keeps that topic at exactly zero;
//      * a pivot that is not positive elsewhere (G not positive definite)
//        sets the sticky status NMF_ERR_NOT_SPD.
// G itself is stored without the dead-topic substitution (the error of
// Section 3.1 needs the true Gram matrices).
#include <algorithm>

#include "nmf_device.h"

namespace nmfk {

namespace {

constexpr int kStageRows = 128;
constexpr int kReduceEntries = 64;  // upper-triangle entries per reduce block

struct GramArgs {
  const void* F;            // rows x k (compact rows of a factor, or a dense matrix)
  int32_t ld;               // row pitch of F (>= k)
  const int32_t* rows_dev;  // number of rows (device), or nullptr
  int64_t rows_host;
  int32_t k;
  void* partials;           // [kGramBlocks][ne] T
  double* G;
  double* W;                // nullptr: no factorisation (plain Gram)
  int32_t* dead;
  int32_t* status;
  // storage high-water mark: max over calls of counts_a[0] + counts_b[0]
  const int32_t* counts_a;
  const int32_t* counts_b;
  int64_t* max_nnz;
  int32_t nparts;  // partial blocks (grid of the partial kernel)
};

__device__ __forceinline__ void tri_index(int e, int k, int* pa, int* pb) {
  // e enumerates (a, b), a <= b, row by row of the upper triangle
  int a = 0;
  int rowlen = k;
  while (e >= rowlen) {
    e -= rowlen;
    ++a;
    --rowlen;
  }
  *pa = a;
  *pb = a + e;
}

template <typename T, int JMAX>
__device__ __forceinline__ void k_gram_partial_body(const GramArgs& g, int blk, int nblk) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (*g.status != 0) return;
  const int k = g.k;
  const int kpad = (k + 3) & ~3;
  const int ne = k * (k + 1) / 2;
  const int tid = threadIdx.x;
  const int64_t R = g.rows_dev ? static_cast<int64_t>(*g.rows_dev) : g.rows_host;
  const int P = nblk;
  const int64_t lo = R * blk / P;
  const int64_t hi = R * (blk + 1) / P;
  T* stage = reinterpret_cast<T*>(smem);
  int ea[JMAX], eb[JMAX];
  T acc[JMAX];
#pragma unroll
  for (int j = 0; j < JMAX; ++j) {
    const int e = tid + 256 * j;
    int a = 0, b = 0;
    if (e < ne) tri_index(e, k, &a, &b);
    ea[j] = a;
    eb[j] = b;
    acc[j] = T(0);
  }
  const T* __restrict__ F = static_cast<const T*>(g.F);
  for (int64_t r0 = lo; r0 < hi; r0 += kStageRows) {
    const int nr = static_cast<int>(hi - r0 < kStageRows ? hi - r0 : kStageRows);
    __syncthreads();
    // the batch is contiguous in F: eight independent loads per thread
    const int ld = g.ld;
    const int nel = nr * ld;
    for (int i0 = tid; i0 < nel; i0 += 256 * 8) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = i0 + 256 * u;
        v[u] = i < nel ? F[r0 * ld + i] : T(0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = i0 + 256 * u;
        const int rr = i / ld, c = i - rr * ld;
        if (i < nel && c < k) stage[rr * kpad + c] = v[u];
      }
    }
    __syncthreads();
    for (int rr = 0; rr < nr; ++rr) {
      const T* row = stage + rr * kpad;
#pragma unroll
      for (int j = 0; j < JMAX; ++j) acc[j] = fma(row[ea[j]], row[eb[j]], acc[j]);
    }
  }
  T* part = static_cast<T*>(g.partials) + static_cast<int64_t>(blk) * ne;
#pragma unroll
  for (int j = 0; j < JMAX; ++j) {
    const int e = tid + 256 * j;
    if (e < ne) part[e] = acc[j];
  }
}
template <typename T, int JMAX>
__global__ __launch_bounds__(256) void k_gram_partial(GramArgs g) { k_gram_partial_body<T, JMAX>(g, blockIdx.x, gridDim.x); }
template <typename T, int JMAX>
__global__ __launch_bounds__(256) void k_gram_partial_b(const GramArgs* as, const BlockMap* map) {
  const BlockMap m = map[blockIdx.x];
  const GramArgs g = as[m.prob];
  k_gram_partial_body<T, JMAX>(g, m.blk, m.nblk);
}


template <typename T>
__device__ __forceinline__ void k_gram_reduce_body(const GramArgs& g, int blk, int nblk) {
  __shared__ double red[4][kReduceEntries];
  if (*g.status != 0) return;
  const int k = g.k;
  const int ne = k * (k + 1) / 2;
  const int lane = lane_id();
  const int wv = threadIdx.x >> 6;
  const int e = blk * kReduceEntries + lane;
  const T* __restrict__ part = static_cast<const T*>(g.partials);
  double s = 0.0;
  if (e < ne) {
    // wave wv adds partials wv, wv + 4, ... in order, eight loads in flight
    int b = wv;
    for (; b + 28 < g.nparts; b += 32) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[static_cast<int64_t>(b + 4 * u) * ne + e];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += static_cast<double>(v[u]);
    }
    for (; b < g.nparts; b += 4) s += static_cast<double>(part[static_cast<int64_t>(b) * ne + e]);
  }
  red[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && e < ne) {
    const double t = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    int a, b;
    tri_index(e, k, &a, &b);
    g.G[a * k + b] = t;
    g.G[b * k + a] = t;
  }
}
template <typename T>
__global__ __launch_bounds__(256) void k_gram_reduce(GramArgs g) { k_gram_reduce_body<T>(g, blockIdx.x, gridDim.x); }
template <typename T>
__global__ __launch_bounds__(256) void k_gram_reduce_b(const GramArgs* as, const BlockMap* map) {
  const BlockMap m = map[blockIdx.x];
  const GramArgs g = as[m.prob];
  k_gram_reduce_body<T>(g, m.blk, m.nblk);
}


typedef float mfma_f4 __attribute__((ext_vector_type(4)));

// G partials on the matrix cores (float32, k <= 16 * NB).  A 16 x 4 by
// 4 x 16 product with the four rows r0..r0+3 of F as the inner dimension:
// lane l supplies F[r0 + l / 16][16 t + l % 16] for topic block t, which is
// both the A operand (F^T, topics x rows) of block t and the B operand (F,
// rows x topics) of block t; the accumulator of tile (ta, tb) then holds
// G[16 ta + 4 (l / 16) + i][16 tb + l % 16] in its element i.  Each wave sums
// a contiguous slice of the block's rows; the block adds its waves' tiles in
// wave order and stores the upper triangle like k_gram_partial.
template <int NB>
__device__ __forceinline__ void k_gram_mfma_body(const GramArgs& g, int blk, int nblk) {
  constexpr int NP = NB * (NB + 1) / 2;  // tiles (ta <= tb)
  __shared__ float red[4][NP][64][4];
  if (*g.status != 0) return;
  const int k = g.k;
  const int ld = g.ld;
  const int lane = lane_id();
  const int wv = threadIdx.x >> 6;
  const int64_t R = g.rows_dev ? static_cast<int64_t>(*g.rows_dev) : g.rows_host;
  const int P = nblk;
  const int64_t blo = R * blk / P, bhi = R * (blk + 1) / P;
  const int64_t lo = blo + (bhi - blo) * wv / 4, hi = blo + (bhi - blo) * (wv + 1) / 4;
  const float* __restrict__ F = static_cast<const float*>(g.F);
  mfma_f4 acc[NP];
#pragma unroll
  for (int t = 0; t < NP; ++t) acc[t] = mfma_f4{0.f, 0.f, 0.f, 0.f};
  const int kr = lane >> 4;  // row within a group of four
  const int cl = lane & 15;  // topic within a block of 16
  for (int64_t r0 = lo; r0 < hi; r0 += 8) {
    // two groups of four rows, all loads in flight together
    float f[2][NB];
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      const int64_t r = r0 + 4 * s2 + kr;
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        const int c = 16 * t + cl;
        f[s2][t] = (r < hi && c < k) ? F[r * ld + c] : 0.f;
      }
    }
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      int pi = 0;
#pragma unroll
      for (int ta = 0; ta < NB; ++ta)
#pragma unroll
        for (int tb = ta; tb < NB; ++tb) {
          acc[pi] = __builtin_amdgcn_mfma_f32_16x16x4f32(f[s2][ta], f[s2][tb], acc[pi], 0, 0, 0);
          ++pi;
        }
    }
  }
#pragma unroll
  for (int t = 0; t < NP; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) red[wv][t][lane][i] = acc[t][i];
  __syncthreads();
  const int ne = k * (k + 1) / 2;
  float* part = static_cast<float*>(g.partials) + static_cast<int64_t>(blk) * ne;
  for (int x = threadIdx.x; x < NP * 256; x += 256) {
    const int t = x >> 8, l = (x >> 2) & 63, i = x & 3;
    const float v = ((red[0][t][l][i] + red[1][t][l][i]) + red[2][t][l][i]) + red[3][t][l][i];
    // tile t -> (ta, tb)
    int ta = 0, rem = t;
    while (rem >= NB - ta) {
      rem -= NB - ta;
      ++ta;
    }
    const int tb = ta + rem;
    const int a = 16 * ta + 4 * (l >> 4) + i, b = 16 * tb + (l & 15);
    if (a <= b && b < k) part[a * k - a * (a - 1) / 2 + (b - a)] = v;
  }
}
template <int NB>
__global__ __launch_bounds__(256) void k_gram_mfma(GramArgs g) { k_gram_mfma_body<NB>(g, blockIdx.x, gridDim.x); }
template <int NB>
__global__ __launch_bounds__(256) void k_gram_mfma_b(const GramArgs* as, const BlockMap* map) {
  const BlockMap m = map[blockIdx.x];
  const GramArgs g = as[m.prob];
  k_gram_mfma_body<NB>(g, m.blk, m.nblk);
}


// One block: the storage high-water mark, then W = G^-1 in float64 by the
// symmetric sweep operator on the positive definite G.  Sweeping pivot p
// maps a to b with
//   b_pp = -1 / a_pp,  b_ip = a_ip / a_pp,  b_pj = a_pj / a_pp,
//   b_ij = a_ij - a_ip a_pj / a_pp          (i, j != p),
// which keeps the matrix symmetric; sweeping every pivot in order leaves
// -G^-1.  Its p-th pivot is the p-th Schur complement diagonal, i.e. the
// square of the Cholesky diagonal L_pp, so a pivot that is not positive
// (NOT_SPD) occurs exactly where the Cholesky factorization of G fails.
// Dead topics (G_cc = 0) get identity rows and columns first, which the
// sweep leaves as -1 on the diagonal (W_cc = 1).
//
// The pivots are swept four at a time.  Sweeping a pivot set P at once
// (B = a_PP, positive definite as a Schur complement of G) maps a to b with
//   b_PP = -B^-1,  b_Pj = B^-1 a_Pj,  b_iP = a_iP B^-1,
//   b_ij = a_ij - a_iP B^-1 a_Pj            (i, j not in P),
// the same matrix as sweeping P's pivots one at a time, and its pivots are
// the same Schur complement diagonals (checked the same way).  The KM x KM
// register matrix (KM = 64 H, k <= KM) is split into blocks of four rows;
// wave w of the 16 owns blocks w and, when H = 2, w + 16, and lane c holds
// columns c and c + 64.  The wave that owns the next block reads its 4 x 4
// diagonal block (through LDS), sweeps it in registers (b = -B^-1), forms
// T = B^-1 a_P. for every column and publishes a_P. and T; by symmetry
// (a_iP = a_Pi) every other row's update needs only these, so a block of
// four pivots takes one barrier.
constexpr int kFactorThreads = 1024;
constexpr int kPiv = 4;

// 1 / d for a pivot d > 0: the hardware reciprocal estimate refined by two
// Newton-Raphson steps r <- r + r (1 - d r), each of which squares the
// relative error; a pivot below 2^-1000 (where the estimate may flush) takes
// the IEEE division.  d is the same in every lane, so the branch is uniform.
__device__ __forceinline__ double pivot_recip(double d) {
  if (!(d >= 0x1p-1000)) return 1.0 / d;
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// The owner wave of the block of pivots p0..p0+bs-1 (its rows e): sweep the
// diagonal block into b = -B^-1, then t[q][h] = (B^-1 a_P.)[q][c + 64 h];
// publishes a_P. (its rows as they stand) and T.  The diagonal block reaches
// every lane through `dg` (written by its own lanes, read back by the same
// wave, whose LDS accesses complete in order).  Returns false on a pivot
// that is not positive.
template <int H>
__device__ __forceinline__ bool block_pivot(const double (&e)[kPiv][H], int p0, int bs, double (&b)[kPiv][kPiv],
                                            double (&t)[kPiv][H], double (*rs)[kPiv], double (*ts)[kPiv],
                                            double (*dg)[kPiv], int c) {
  // the block's four columns lie in one half (p0 is a multiple of 4)
  const int h0 = p0 >> 6, cl = p0 & 63;
  if (c >= cl && c < cl + kPiv)
#pragma unroll
    for (int q = 0; q < kPiv; ++q) {
      double v = e[q][0];
#pragma unroll
      for (int h = 1; h < H; ++h)
        if (h == h0) v = e[q][h];
      dg[q][c - cl] = v;
    }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int q = 0; q < kPiv; ++q)
#pragma unroll
    for (int l = 0; l < kPiv; ++l) b[q][l] = dg[q][l];
  bool ok = true;
#pragma unroll
  for (int p = 0; p < kPiv; ++p) {
    if (p >= bs) break;
    const double d = b[p][p];
    ok = ok && d > 0.0;
    const double ip = pivot_recip(d);
    double rp[kPiv];
#pragma unroll
    for (int l = 0; l < kPiv; ++l) rp[l] = b[p][l] * ip;
#pragma unroll
    for (int i = 0; i < kPiv; ++i) {
      if (i == p) continue;
      const double aip = b[i][p];
#pragma unroll
      for (int l = 0; l < kPiv; ++l)
        if (l != p) b[i][l] = fma(-aip, rp[l], b[i][l]);
      b[i][p] = aip * ip;
    }
#pragma unroll
    for (int l = 0; l < kPiv; ++l)
      if (l != p) b[p][l] = rp[l];
    b[p][p] = -ip;
  }
  // rows/columns of the block past bs are zero padding and stay zero
#pragma unroll
  for (int q = 0; q < kPiv; ++q)
#pragma unroll
    for (int h = 0; h < H; ++h) {
      double v = 0.0;
#pragma unroll
      for (int l = 0; l < kPiv; ++l) v = fma(-b[q][l], e[l][h], v);
      t[q][h] = v;
    }
#pragma unroll
  for (int q = 0; q < kPiv; ++q)
#pragma unroll
    for (int h = 0; h < H; ++h) {
      rs[c + 64 * h][q] = e[q][h];
      ts[c + 64 * h][q] = t[q][h];
    }
  return ok;
}

template <int H>
__device__ __forceinline__ void k_gram_block_body(const GramArgs& g, int blk, int nblk) {
  constexpr int KM = 64 * H;
  constexpr int NW = kFactorThreads / 64;
  static_assert(NW * kPiv * H == KM, "16 waves of H blocks of four rows");
  __shared__ double rs[2][KM][kPiv];  // rs[.][c][l] = a_{p0+l, c}
  __shared__ double ts[2][KM][kPiv];  // ts[.][c][q] = (B^-1 a_P.)[q][c]
  __shared__ double dg[kPiv][kPiv];   // the owner's diagonal block
  __shared__ int s_dead[KM];
  __shared__ int s_nd, s_bad;
  if (*g.status != 0) return;
  const int k = g.k;
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_nd = 0;
    s_bad = 0;
    if (g.max_nnz) {
      const int64_t cur = static_cast<int64_t>(*g.counts_a) + (g.counts_b ? *g.counts_b : 0);
      if (cur > *g.max_nnz) *g.max_nnz = cur;
    }
  }
  __syncthreads();
  for (int c = tid; c < KM; c += kFactorThreads) {
    const int d = c < k && g.G[c * k + c] == 0.0;
    s_dead[c] = d;
    if (d) atomicAdd(&s_nd, 1);
  }
  __syncthreads();
  if (tid == 0) *g.dead = s_nd;
  const int c = lane_id();
  const int wv = tid >> 6;  // owns row blocks wv (and wv + 16)
  double e[H][kPiv][H];     // e[lb][q][h]: row kPiv (wv + 16 lb) + q, column c + 64 h
#pragma unroll
  for (int lb = 0; lb < H; ++lb)
#pragma unroll
    for (int q = 0; q < kPiv; ++q)
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int i = kPiv * (wv + NW * lb) + q, col = c + 64 * h;
        double v = 0.0;
        if (i < k && col < k) v = (s_dead[i] || s_dead[col]) ? (i == col ? 1.0 : 0.0) : g.G[i * k + col];
        e[lb][q][h] = v;
      }
  const int nbk = (k + kPiv - 1) / kPiv;
  double b[kPiv][kPiv], t[kPiv][H];
  if (wv == 0 && !block_pivot<H>(e[0], 0, k < kPiv ? k : kPiv, b, t, rs[0], ts[0], dg, c) && c == 0) s_bad = 1;
  __syncthreads();
  for (int j = 0; j < nbk; ++j) {
    const int buf = j & 1;
    const int p0 = kPiv * j;
    const int bs = k - p0 < kPiv ? k - p0 : kPiv;
#pragma unroll
    for (int lb = 0; lb < H; ++lb) {
      const int jb = wv + NW * lb;
      if (jb >= nbk) continue;
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int col = c + 64 * h;
        const bool cp = col >= p0 && col < p0 + bs;
        const int m = (col - p0) & (kPiv - 1);
        if (jb == j) {
          // the block's own rows: -B^-1 inside the block, T elsewhere
#pragma unroll
          for (int q = 0; q < kPiv; ++q) {
            if (q >= bs) break;
            double w = b[q][0];
#pragma unroll
            for (int l = 1; l < kPiv; ++l)
              if (m == l) w = b[q][l];
            e[lb][q][h] = cp ? w : t[q][h];
          }
        } else {
          const double t0 = ts[buf][col][0], t1 = ts[buf][col][1], t2 = ts[buf][col][2], t3 = ts[buf][col][3];
#pragma unroll
          for (int q = 0; q < kPiv; ++q) {
            const int i = kPiv * jb + q;
            if (cp) {
              e[lb][q][h] = ts[buf][i][m];  // a_iP B^-1 = (B^-1 a_Pi)^T by symmetry
            } else {
              double v = e[lb][q][h];
              v = fma(-rs[buf][i][0], t0, v);
              v = fma(-rs[buf][i][1], t1, v);
              v = fma(-rs[buf][i][2], t2, v);
              v = fma(-rs[buf][i][3], t3, v);
              e[lb][q][h] = v;
            }
          }
        }
      }
    }
    // the owner of the next block sweeps its diagonal block (a different
    // wave from this block's: blocks go round the 16 waves)
    if (j + 1 < nbk && wv == ((j + 1) % NW)) {
      const int n0 = p0 + kPiv;
      const int nbs = k - n0 < kPiv ? k - n0 : kPiv;
      bool ok = true;
#pragma unroll
      for (int lb = 0; lb < H; ++lb)
        if ((j + 1) / NW == lb) ok = block_pivot<H>(e[lb], n0, nbs, b, t, rs[buf ^ 1], ts[buf ^ 1], dg, c);
      if (!ok && c == 0) s_bad = 1;
    }
    __syncthreads();
  }
  if (s_bad) {
    if (tid == 0) atomicCAS(g.status, 0, static_cast<int32_t>(NMF_ERR_NOT_SPD));
    for (int x = tid; x < k * k; x += kFactorThreads) g.W[x] = 0.0;
    return;
  }
#pragma unroll
  for (int lb = 0; lb < H; ++lb)
#pragma unroll
    for (int q = 0; q < kPiv; ++q)
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const int i = kPiv * (wv + NW * lb) + q, col = c + 64 * h;
        if (i < k && col < k) g.W[i * k + col] = -e[lb][q][h];
      }
}
template <int H>
__global__ __launch_bounds__(kFactorThreads) void k_gram_block(GramArgs g) {
  k_gram_block_body<H>(g, blockIdx.x, gridDim.x);
}
template <int H>
__global__ __launch_bounds__(kFactorThreads) void k_gram_block_b(const GramArgs* as, const BlockMap* map) {
  const BlockMap m = map[blockIdx.x];
  const GramArgs g = as[m.prob];
  k_gram_block_body<H>(g, m.blk, m.nblk);
}


template <typename T>
hipError_t launch(nmf_handle* h, GramArgs& g, int64_t rows_bound) {
  const int k = h->k;
  const int kpad = (k + 3) & ~3;
  const size_t stage = static_cast<size_t>(kStageRows) * kpad * sizeof(T);
  // one partial block per 64 possible rows, at most kGramBlocks
  g.nparts = static_cast<int32_t>(std::max<int64_t>(1, std::min<int64_t>(kGramBlocks, (rows_bound + 63) / 64)));
  const unsigned P = static_cast<unsigned>(g.nparts);
  hipError_t e;
  if (sizeof(T) == 4) {
    if (k <= 32)
      e = launch_rec(h, k_gram_mfma<2>, k_gram_mfma_b<2>, P, 256, 0, g);
    else if (k <= 64)
      e = launch_rec(h, k_gram_mfma<4>, k_gram_mfma_b<4>, P, 256, 0, g);
    else
      e = launch_rec(h, k_gram_mfma<8>, k_gram_mfma_b<8>, P, 256, 0, g);
  } else if (k <= 64) {
    e = launch_rec(h, k_gram_partial<T, 9>, k_gram_partial_b<T, 9>, P, 256, stage, g);
  } else {
    e = launch_rec(h, k_gram_partial<T, 33>, k_gram_partial_b<T, 33>, P, 256, stage, g);
  }
  if (e != hipSuccess) return e;
  const int ne = k * (k + 1) / 2;
  const unsigned rblocks = static_cast<unsigned>((ne + kReduceEntries - 1) / kReduceEntries);
  if ((e = launch_rec(h, k_gram_reduce<T>, k_gram_reduce_b<T>, rblocks, 256, 0, g)) != hipSuccess) return e;
  if (!g.W) return hipSuccess;
  if (k <= 64) return launch_rec(h, k_gram_block<1>, k_gram_block_b<1>, 1, kFactorThreads, 0, g);
  return launch_rec(h, k_gram_block<2>, k_gram_block_b<2>, 1, kFactorThreads, 0, g);
}

}  // namespace

template <typename T>
hipError_t gram(nmf_handle* h, const Factor& F, const Gram& out) {
  GramArgs g{};
  g.F = F.dense;
  g.ld = F.ld;
  g.rows_dev = F.counts + 1;
  g.k = h->k;
  g.partials = h->gram_partials;
  g.G = out.G;
  g.W = out.W;
  g.dead = out.dead;
  g.status = h->status;
  // the other factor's count completes nnz(U) + nnz(V)
  const bool is_v = (&F == &h->V);
  g.counts_a = F.counts;
  g.counts_b = is_v ? h->U[h->cur_u].counts : h->V.counts;
  g.max_nnz = h->met.max_nnz;
  return launch<T>(h, g, F.rows);
}

template <typename T>
hipError_t gram_dense(nmf_handle* h, const T* F, int64_t rows, double* G) {
  GramArgs g{};
  g.F = F;
  g.ld = h->k;
  g.rows_dev = nullptr;
  g.rows_host = rows;
  g.k = h->k;
  g.partials = h->gram_partials;
  g.G = G;
  g.W = nullptr;
  g.status = h->status;
  return launch<T>(h, g, rows);
}

// G = F^T F only (no inverse, no storage mark).
template <typename T>
hipError_t gram_plain(nmf_handle* h, const Factor& F, double* G) {
  GramArgs g{};
  g.F = F.dense;
  g.ld = F.ld;
  g.rows_dev = F.counts + 1;
  g.k = h->k;
  g.partials = h->gram_partials;
  g.G = G;
  g.W = nullptr;
  g.status = h->status;
  return launch<T>(h, g, F.rows);
}

namespace {
__global__ void k_copy_block(const double* G, int32_t k, int32_t k1, int32_t k2, double* Gb) {
  for (int i = threadIdx.x; i < k2 * k2; i += blockDim.x) {
    const int a = i / k2, b = i - a * k2;
    Gb[i] = G[static_cast<int64_t>(k1 + a) * k + (k1 + b)];
  }
}
}  // namespace

// W22 = inverse of the [k1, k1 + k2) diagonal block of the k x k matrix G,
// by the same float64 sweep kernel as the full inverse (dead topics
// of the block get identity rows; a non-positive pivot is NMF_ERR_NOT_SPD).
// Gb: k2 x k2 scratch; dead: one int of scratch.
hipError_t block_inverse(nmf_handle* h, const double* G, int k1, int k2, double* Gb, double* W22, int32_t* dead) {
  hipLaunchKernelGGL(k_copy_block, dim3(1), dim3(256), 0, h->stream, G, h->k, k1, k2, Gb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  GramArgs g{};
  g.G = Gb;
  g.W = W22;
  g.k = k2;
  g.dead = dead;
  g.status = h->status;
  if (k2 <= 64)
    hipLaunchKernelGGL(k_gram_block<1>, dim3(1), dim3(kFactorThreads), 0, h->stream, g);
  else
    hipLaunchKernelGGL(k_gram_block<2>, dim3(1), dim3(kFactorThreads), 0, h->stream, g);
  return hipGetLastError();
}

template hipError_t gram_plain<float>(nmf_handle*, const Factor&, double*);
template hipError_t gram_plain<double>(nmf_handle*, const Factor&, double*);
template hipError_t gram<float>(nmf_handle*, const Factor&, const Gram&);
template hipError_t gram<double>(nmf_handle*, const Factor&, const Gram&);
template hipError_t gram_dense<float>(nmf_handle*, const float*, int64_t, double*);
template hipError_t gram_dense<double>(nmf_handle*, const double*, int64_t, double*);

}  // namespace nmfk
