// Device-wide exclusive scans (reduce, scan of block sums, down-sweep).
// out[i] = sum(in[0..i)) for i in [0, n]; out[n] is the total.
#include "device_common.h"

namespace tpc {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = kScanBlock / kThreads;   // 4 per thread

template <typename T>
__device__ __forceinline__ uint32_t scan_count(uint32_t n, const uint32_t* n_dev, uint32_t n_max) {
  return n_dev ? min(*n_dev, n_max) : n;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_scan_reduce(const T* in, uint32_t n, const uint32_t* n_dev,
                                                          uint32_t n_max, unsigned long long* blocks) {
  __shared__ T wsum[kThreads / kWave];
  const uint32_t cnt = scan_count<T>(n, n_dev, n_max);
  const uint32_t base = blockIdx.x * kScanBlock;
  if (base >= cnt && blockIdx.x != 0) return;
  T s = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const uint32_t i = base + threadIdx.x * kItems + k;
    if (i < cnt) s += in[i];
  }
  T total;
  block_exclusive_scan<T>(s, wsum, &total);
  if (threadIdx.x == 0) blocks[blockIdx.x] = (unsigned long long)total;
}

template <typename T>
__global__ void __launch_bounds__(1024) k_scan_blocks(unsigned long long* blocks, uint32_t n, const uint32_t* n_dev,
                                                      uint32_t n_max) {
  __shared__ unsigned long long wsum[1024 / kWave];
  const uint32_t cnt = scan_count<T>(n, n_dev, n_max);
  const uint32_t nb = (cnt + kScanBlock - 1) / kScanBlock;
  const uint32_t per = (nb + blockDim.x - 1) / blockDim.x;
  const uint32_t b0 = min(nb, threadIdx.x * per), b1 = min(nb, b0 + per);
  unsigned long long s = 0;
  for (uint32_t i = b0; i < b1; ++i) s += blocks[i];
  unsigned long long total;
  unsigned long long run = block_exclusive_scan<unsigned long long>(s, wsum, &total);
  for (uint32_t i = b0; i < b1; ++i) {
    const unsigned long long v = blocks[i];
    blocks[i] = run;
    run += v;
  }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_scan_down(const T* in, T* out, uint32_t n, const uint32_t* n_dev,
                                                        uint32_t n_max, const unsigned long long* blocks) {
  __shared__ T wsum[kThreads / kWave];
  const uint32_t cnt = scan_count<T>(n, n_dev, n_max);
  const uint32_t base = blockIdx.x * kScanBlock;
  if (cnt == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0;
    return;
  }
  if (base >= cnt) return;
  T v[kItems];
  T s = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const uint32_t i = base + threadIdx.x * kItems + k;
    v[k] = i < cnt ? in[i] : (T)0;
    s += v[k];
  }
  T total;
  T run = block_exclusive_scan<T>(s, wsum, &total) + (T)blocks[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const uint32_t i = base + threadIdx.x * kItems + k;
    if (i < cnt) out[i] = run;
    run += v[k];
    if (i + 1 == cnt) out[cnt] = run;
  }
}

template <typename T>
void scan_impl(const T* in, T* out, uint32_t n, const uint32_t* n_dev, uint32_t n_max, unsigned long long* blocks,
               hipStream_t s) {
  const uint32_t span = n_dev ? n_max : n;
  const uint32_t nb = span == 0 ? 1 : (span + kScanBlock - 1) / kScanBlock;
  hipLaunchKernelGGL(k_scan_reduce<T>, dim3(nb), dim3(kThreads), 0, s, in, n, n_dev, n_max, blocks);
  hipLaunchKernelGGL(k_scan_blocks<T>, dim3(1), dim3(1024), 0, s, blocks, n, n_dev, n_max);
  hipLaunchKernelGGL(k_scan_down<T>, dim3(nb), dim3(kThreads), 0, s, in, out, n, n_dev, n_max, blocks);
}

}  // namespace

void launch_scan_u32(const uint32_t* in, uint32_t* out, uint32_t n, unsigned long long* blocks, hipStream_t s) {
  scan_impl<uint32_t>(in, out, n, nullptr, 0, blocks, s);
}

void launch_scan_u64(const unsigned long long* in, unsigned long long* out, const uint32_t* n_dev, uint32_t n_max,
                     unsigned long long* blocks, hipStream_t s) {
  scan_impl<unsigned long long>(in, out, 0, n_dev, n_max, blocks, s);
}

}  // namespace tpc
