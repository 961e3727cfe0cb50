// K3 + K4: neighbour cleaner and start-hit finder -- steps C3 and C4.
//
// k_clean (one workgroup per row) keeps only mutual links, flags chain starts
// (computed from the C2 snapshot, so it needs no other workgroup's output) and
// counts them per row.  After a scan of the per-row counts, k_starts writes
// the start list in canonical order with a wavefront ballot + prefix count
// inside each row.
#include "device_common.h"

namespace tpc {
namespace {

constexpr int kThreads = 256;

__global__ void __launch_bounds__(kThreads) k_clean(DevPtrs d) {
  __shared__ uint32_t wsum[kThreads / kWave];
  const uint32_t sr = blockIdx.x;
  const uint32_t a = d.row_off[sr], n = d.row_off[sr + 1] - a;
  uint32_t cnt = 0;
  for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
    const int32_t h = (int32_t)(a + j);
    const int32_t u = d.up0[h], dn = d.down0[h];
    const int32_t u1 = (u >= 0 && d.down0[u] == h) ? u : -1;
    const int32_t d1 = (dn >= 0 && d.up0[dn] == h) ? dn : -1;
    d.up1[h] = u1;
    d.down1[h] = d1;
    bool start = false;
    if (d1 == -1 && u1 >= 0) {
      const int32_t uu = d.up0[u1];
      start = uu >= 0 && d.down0[uu] == u1;   // up1[u1] >= 0
    }
    d.sflag[h] = start ? 1 : 0;
    cnt += start;
  }
  uint32_t total;
  block_exclusive_scan<uint32_t>(cnt, wsum, &total);
  if (threadIdx.x == 0) d.row_nstart[sr] = total;
}

__global__ void __launch_bounds__(kThreads) k_starts(DevPtrs d) {
  __shared__ uint32_t wsum[kThreads / kWave];
  const uint32_t sr = blockIdx.x;
  const uint32_t a = d.row_off[sr], n = d.row_off[sr + 1] - a;
  if (sr == 0 && threadIdx.x == 0) {
    const uint32_t ns = d.row_start_off[d.SR];
    d.hdr->n_starts = ns;
    if (ns > d.tcap) atomicOr(&d.hdr->error_flags, 2u);
  }
  uint32_t run = d.row_start_off[sr];
  for (uint32_t j0 = 0; j0 < n; j0 += blockDim.x) {
    const uint32_t j = j0 + threadIdx.x;
    const uint32_t f = (j < n) ? d.sflag[a + j] : 0u;
    uint32_t total;
    const uint32_t pre = block_exclusive_scan<uint32_t>(f, wsum, &total);
    if (f) {
      const uint32_t idx = run + pre;
      if (idx < d.tcap) {
        d.start_pos[idx] = a + j;
        d.start_sr[idx] = sr;
      }
    }
    run += total;
  }
}

}  // namespace

void launch_clean_starts(const DevPtrs& d, uint32_t, hipStream_t s) {
  if (d.SR == 0) return;
  hipLaunchKernelGGL(k_clean, dim3(d.SR), dim3(kThreads), 0, s, d);
  launch_scan_u32(d.row_nstart, d.row_start_off, d.SR, d.scan_blocks, s);
  hipLaunchKernelGGL(k_starts, dim3(d.SR), dim3(kThreads), 0, s, d);
}

}  // namespace tpc
