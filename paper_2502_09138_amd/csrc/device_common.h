// Device helpers shared by the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tpc_internal.h"

namespace tpc {

constexpr int kWave = 64;

// isqrt of a non-negative 64-bit integer (exact).
__device__ __forceinline__ int64_t isqrt64(int64_t q) {
  int64_t s = (int64_t)sqrt((double)q);
  while (s * s > q) --s;
  while ((s + 1) * (s + 1) <= q) ++s;
  return s;
}

// C1 grid dimensions of a row with n hits.
__device__ __forceinline__ void grid_dims(uint32_t n, int k, int ly, int lz, int& ny, int& nz) {
  const int64_t B = max((int64_t)1, (int64_t)(n / (uint32_t)k));
  const int64_t q = (B * (int64_t)ly) / (int64_t)lz;
  int64_t s = isqrt64(q);
  s = s < 1 ? 1 : (s > B ? B : s);
  ny = (int)s;
  nz = (int)max((int64_t)1, B / s);
}

// C1 bin of one coordinate: float32, one rounding per operation, no contraction.
__device__ __forceinline__ int bin1(float v, float lo, float inv_w, int n) {
#pragma clang fp contract(off)
  const float a = v - lo;
  const float b = (float)n * inv_w;
  float u = a * b;
  if (!(u >= 0.0f)) u = 0.0f;
  const float top = (float)(n - 1);
  if (u > top) u = top;
  return (int)u;
}

__device__ __forceinline__ uint32_t bin_base(const DevPtrs& d, uint32_t sr) { return d.row_off[sr] + 2u * sr; }

// Wave-level inclusive scan (64 lanes) of 32/64-bit unsigned values.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    T y = __shfl_up(x, off, kWave);
    if (lane >= off) x += y;
  }
  return x;
}

// Block exclusive scan of one value per thread.  `wsum` is LDS scratch of
// blockDim/64 entries.  Returns the exclusive prefix; *total receives the sum.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* wsum, T* total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  T inc = wave_inclusive_scan(v);
  if (lane == kWave - 1) wsum[w] = inc;
  __syncthreads();
  T before = 0, all = 0;
  for (int i = 0; i < nw; ++i) {
    T s = wsum[i];
    if (i < w) before += s;
    all += s;
  }
  __syncthreads();
  *total = all;
  return before + inc - v;
}

// Exclusive scan of arr[0..n) in LDS by one block, in place; arr[n] = total.
__device__ __forceinline__ void block_scan_array(uint32_t* arr, uint32_t n, uint32_t* wsum) {
  const uint32_t nt = blockDim.x;
  const uint32_t chunk = (n + nt - 1) / nt;
  const uint32_t b0 = min(n, threadIdx.x * chunk), b1 = min(n, b0 + chunk);
  uint32_t s = 0;
  for (uint32_t i = b0; i < b1; ++i) s += arr[i];
  uint32_t total;
  uint32_t run = block_exclusive_scan<uint32_t>(s, wsum, &total);
  for (uint32_t i = b0; i < b1; ++i) {
    const uint32_t v = arr[i];
    arr[i] = run;
    run += v;
  }
  if (threadIdx.x == 0) arr[n] = total;
  __syncthreads();
}

// XCD-aware grid-stride schedule over n items.  Workgroups are dispatched
// round-robin over the 8 XCDs (block b -> XCD b % 8), each with its own L2; this
// gives XCD x the contiguous virtual blocks [x*per, (x+1)*per), so items that
// share data (tracklets of one sector) are served from one L2.  The grid must be
// a multiple of kXcds.  Usage: for (uint32_t vb = s.first; vb < s.end; vb += s.stride)
constexpr uint32_t kXcds = 8;
struct XcdSched {
  uint32_t first, end, stride;
};
__device__ __forceinline__ XcdSched xcd_sched(uint32_t n_items) {
  const uint32_t need = (n_items + blockDim.x - 1) / blockDim.x;
  const uint32_t per = (need + kXcds - 1) / kXcds;
  const uint32_t xcd = blockIdx.x % kXcds;
  return XcdSched{xcd * per + blockIdx.x / kXcds, min(need, (xcd + 1) * per), gridDim.x / kXcds};
}
inline uint32_t xcd_grid(uint32_t blocks) { return (blocks + kXcds - 1) / kXcds * kXcds; }

}  // namespace tpc
