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

// kBatch hits per thread at a time: each level of the dependent gathers
// (own links, the linked hits' links, the next hit's links) is issued for the
// whole batch before the next level needs it.
constexpr int kBatch = 4;

// Rows go to the XCDs (block b runs on XCD b % kXcds) in groups of kRowGroup
// consecutive rows, group g on XCD g % kXcds, so that the links of rows r - 1
// and r + 1 that a row reads are mostly in its own XCD's L2.
constexpr uint32_t kRowGroup = 16;

__global__ void __launch_bounds__(kThreads) k_clean(DevPtrs d) {
  __shared__ uint32_t wsum[kThreads / kWave];
  const uint32_t l = blockIdx.x / kXcds;
  const uint32_t sr = ((l / kRowGroup) * kXcds + blockIdx.x % kXcds) * kRowGroup + l % kRowGroup;
  if (sr >= d.SR) return;
  const uint32_t a = d.row_off[sr], n = d.row_off[sr + 1] - a;
  uint32_t cnt = 0;
  for (uint32_t j0 = threadIdx.x; j0 < n; j0 += kBatch * kThreads) {
    int32_t u[kBatch], dn[kBatch], uback[kBatch], dback[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      const uint32_t j = j0 + q * kThreads;
      u[q] = j < n ? d.up0[a + j] : -1;
      dn[q] = j < n ? d.down0[a + j] : -1;
    }
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      uback[q] = u[q] >= 0 ? d.down0[u[q]] : -1;
      dback[q] = dn[q] >= 0 ? d.up0[dn[q]] : -1;
    }
    int32_t u1[kBatch], d1[kBatch], uu[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      const int32_t h = (int32_t)(a + j0 + q * kThreads);
      u1[q] = (u[q] >= 0 && uback[q] == h) ? u[q] : -1;
      d1[q] = (dn[q] >= 0 && dback[q] == h) ? dn[q] : -1;
      uu[q] = (d1[q] == -1 && u1[q] >= 0) ? d.up0[u1[q]] : -1;
    }
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      const uint32_t j = j0 + q * kThreads;
      const bool start = uu[q] >= 0 && d.down0[uu[q]] == u1[q];   // up1[u1] >= 0
      if (j < n) {
        const int32_t h = (int32_t)(a + j);
        d.up1[h] = u1[q];
        d.down1[h] = d1[q];
        d.sflag[h] = start ? 1 : 0;
        cnt += start;
      }
    }
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
  const uint32_t groups = (d.SR + kRowGroup - 1) / kRowGroup;
  hipLaunchKernelGGL(k_clean, dim3((groups + kXcds - 1) / kXcds * kXcds * kRowGroup), dim3(kThreads), 0, s, d);
  launch_scan_u32(d.row_nstart, d.row_start_off, d.SR, d.scan_blocks, s);
  hipLaunchKernelGGL(k_starts, dim3(d.SR), dim3(kThreads), 0, s, d);
}

}  // namespace tpc
