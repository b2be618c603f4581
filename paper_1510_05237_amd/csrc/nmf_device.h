// Device-side helpers shared by the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "nmf_internal.h"

namespace nmfk {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Number of set bits of `mask` below this lane (rank among the set lanes).
__device__ __forceinline__ int lane_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

__device__ __forceinline__ int bcast_i32(int v, int src) { return __shfl(v, src, 64); }

// Order-preserving unsigned key of a non-negative value (its IEEE bits).
// Only strictly positive values are candidates of the select, so key 0 means
// "not a candidate"; -0.0 never reaches here because the clamp writes +0.0.
template <typename T> struct KeyOf;
template <> struct KeyOf<float> {
  using K = uint32_t;
  static constexpr int bits = 32;
  __device__ static K key(float x) { return __float_as_uint(x); }
  __device__ static float val(K k) { return __uint_as_float(k); }
};
template <> struct KeyOf<double> {
  using K = uint64_t;
  static constexpr int bits = 64;
  __device__ static K key(double x) { return static_cast<uint64_t>(__double_as_longlong(x)); }
  __device__ static double val(K k) { return __longlong_as_double(static_cast<long long>(k)); }
};

// First select digit: the 8 bits below the (always zero) sign bit.
template <typename T>
__device__ __forceinline__ int top_digit(typename KeyOf<T>::K key) {
  return static_cast<int>((key >> (KeyOf<T>::bits - 9)) & 0xFF);
}

// A select candidate: the value's key and its row.  The compound order is
// (key descending, row ascending), i.e. larger value first and, among equal
// values, the lowest row first.
template <typename T>
struct Cand {
  typename KeyOf<T>::K key;
  uint32_t row;
};

template <typename T>
__device__ __forceinline__ bool cand_before(const Cand<T>& a, const Cand<T>& b) {
  return a.key > b.key || (a.key == b.key && a.row < b.row);
}

// Block-wide exclusive scan of one int per thread over NW waves (blockDim.x
// == 64 * NW).  `tmp` must hold NW ints of shared memory.  Returns the
// exclusive prefix; *total receives the block total.
template <int NW>
__device__ __forceinline__ int block_excl_scan(int v, int* tmp, int* total) {
  const int lane = __lane_id();
  const int wv = threadIdx.x >> 6;
  // inclusive scan inside the wave
  int x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) tmp[wv] = x;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    int s = tmp[w];
    if (w < wv) off += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}
__device__ __forceinline__ int block_excl_scan_256(int v, int* tmp, int* total) {
  return block_excl_scan<4>(v, tmp, total);
}
__device__ __forceinline__ int block_excl_scan_1024(int v, int* tmp, int* total) {
  return block_excl_scan<16>(v, tmp, total);
}

// Radix-select step on one wave: given the 256-bin histogram of the
// remaining candidates (lane l holds bins 4l .. 4l + 3 in v[0..3]) and need
// >= 1, find the bin holding the need-th largest candidate: returns it and
// sets *above to the count in higher bins.  Requires need <= the total.
__device__ __forceinline__ int wave_pick_bin(const uint32_t* v, int64_t need, int64_t* above) {
  const int lane = __lane_id();
  const int64_t mine = static_cast<int64_t>(v[0]) + v[1] + v[2] + v[3];
  // inclusive suffix sums over lanes (lane l: bins 4l and higher)
  int64_t suf = mine;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t y = __shfl_down(suf, d, 64);
    if (lane + d < 64) suf += y;
  }
  const int64_t higher = suf - mine;  // bins above this lane's four
  const bool here = higher < need && suf >= need;
  const uint64_t hb = __ballot(here);
  const int src = __builtin_ctzll(hb);  // exactly one lane qualifies
  int bin = 0;
  int64_t acc = higher;
  if (here) {
    bin = 4 * lane;
    for (int i = 3; i >= 0; --i) {
      if (acc + v[i] >= need) {
        bin = 4 * lane + i;
        break;
      }
      acc += v[i];
    }
  }
  *above = __shfl(acc, src, 64);
  return __shfl(bin, src, 64);
}

// Issues a kernel on the handle's stream, or, while the handle records,
// appends the launch (with the kernel's batched form) to the record.  A grid
// of zero blocks is recorded too, so that every problem of a batch records
// the same sequence of launches.
template <typename Args>
hipError_t launch_rec(nmf_handle* h, void (*single)(Args), void (*batched)(const Args*, const BlockMap*),
                      unsigned grid, unsigned block, size_t lds, const Args& a) {
  if (h->rec) {
    LaunchRecord r;
    r.batched = reinterpret_cast<const void*>(batched);
    r.args.resize(sizeof(Args));
    __builtin_memcpy(r.args.data(), &a, sizeof(Args));
    r.grid = grid;
    r.block = block;
    r.lds = lds;
    h->rec->push_back(std::move(r));
    return hipSuccess;
  }
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(single, dim3(grid), dim3(block), lds, h->stream, a);
  return hipGetLastError();
}

// Release/acquire fences at device (agent) scope around inter-block tickets.
__device__ __forceinline__ void fence_release() { __threadfence(); }
__device__ __forceinline__ void fence_acquire() { __threadfence(); }

}  // namespace nmfk
