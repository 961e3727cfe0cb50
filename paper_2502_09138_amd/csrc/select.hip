// K6: tracklet selector and canonical output -- steps C6 and C7.
//
// k_claim: every valid tracklet raises W[hit] to its key with a 64-bit
//   atomicMax (commutative, so the result does not depend on scheduling).
// k_own:   counts the hits each tracklet still owns and decides acceptance;
//   packs (owned << 32) | accepted for one 64-bit scan that yields both the
//   track index and the cluster offset.
// k_emit:  writes accepted tracks at their scanned slots (tracklet order =
//   ascending start position = canonical order).
// k_finish: track and cluster totals, capacity flags, final offset.
#include "device_common.h"

namespace tpc {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ unsigned long long key_of(uint32_t nhits, uint32_t start_pos) {
  return ((unsigned long long)nhits << 32) | (unsigned long long)(0xFFFFFFFFu - start_pos);
}

__device__ __forceinline__ uint32_t n_tracklets(const DevPtrs& d) { return min(d.hdr->n_starts, d.tcap); }

// Row loops are unrolled by kUnroll with all loads issued before use, so a
// lane keeps kUnroll independent gathers in flight instead of one.
constexpr int kUnroll = 8;

template <class Fn>
__device__ __forceinline__ void for_rows(const DevPtrs& d, uint32_t i, int32_t rin, int32_t rout, Fn fn) {
  const uint32_t T = d.tcap;
  for (int32_t r = rin; r <= rout; r += kUnroll) {
    int32_t h[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) h[u] = (r + u <= rout) ? d.tk_rowhit[(size_t)(r + u) * T + i] : -1;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) fn(h[u]);
  }
}

__global__ void __launch_bounds__(kThreads) k_claim(DevPtrs d, KfConst k) {
  const uint32_t nt = n_tracklets(d), T = d.tcap;
  const XcdSched sch = xcd_sched(nt);
  for (uint32_t vb = sch.first; vb < sch.end; vb += sch.stride) {
    const uint32_t i = vb * blockDim.x + threadIdx.x;
    if (i >= nt) continue;
    const int32_t nh = d.tk_info[i];
    if (nh < k.min_tracklet_hits) continue;
    const unsigned long long key = key_of((uint32_t)nh, d.start_pos[i]);
    const int32_t rin = d.tk_info[T + i], rout = d.tk_info[2 * T + i];
    for (int32_t r = rin; r <= rout; r += kUnroll) {
      int32_t h[kUnroll];
      unsigned long long w[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) h[u] = (r + u <= rout) ? d.tk_rowhit[(size_t)(r + u) * T + i] : -1;
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) w[u] = h[u] >= 0 ? d.W[h[u]] : ~0ull;
      // max is monotone: skip the atomic where the word already holds a larger key
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
        if (w[u] < key) atomicMax(&d.W[h[u]], key);
    }
  }
}

__global__ void __launch_bounds__(kThreads) k_own(DevPtrs d, KfConst k) {
  const uint32_t nt = n_tracklets(d), T = d.tcap;
  const XcdSched sch = xcd_sched(nt);
  for (uint32_t vb = sch.first; vb < sch.end; vb += sch.stride) {
    const uint32_t i = vb * blockDim.x + threadIdx.x;
    if (i >= nt) continue;
    const int32_t nh = d.tk_info[i];
    unsigned long long packed = 0;
    if (nh >= k.min_tracklet_hits) {
      const unsigned long long key = key_of((uint32_t)nh, d.start_pos[i]);
      const int32_t rin = d.tk_info[T + i], rout = d.tk_info[2 * T + i];
      uint32_t owned = 0;
      for_rows(d, i, rin, rout, [&](int32_t h) { owned += (h >= 0 && d.W[h] == key) ? 1u : 0u; });
      const float need = k.min_owned_frac * (float)nh;
      if ((int32_t)owned >= k.min_track_hits && (float)owned >= need)
        packed = ((unsigned long long)owned << 32) | 1ull;
    }
    d.tk_pack[i] = packed;
  }
}

__global__ void __launch_bounds__(kThreads) k_emit(DevPtrs d, KfConst k) {
  const uint32_t nt = n_tracklets(d), T = d.tcap;
  const XcdSched sch = xcd_sched(nt);
  for (uint32_t vb = sch.first; vb < sch.end; vb += sch.stride) {
    const uint32_t i = vb * blockDim.x + threadIdx.x;
    if (i >= nt) continue;
    const unsigned long long pk = d.tk_pack[i];
    if (!(pk & 1ull)) continue;
    const unsigned long long pre = d.tk_scan[i];
    const uint32_t ti = (uint32_t)(pre & 0xFFFFFFFFull);
    const unsigned long long co = pre >> 32;
    const uint32_t owned = (uint32_t)(pk >> 32);
    if (ti >= d.max_tracks || co + owned > d.max_track_clusters) continue;   // flagged in k_finish
    const int32_t nh = d.tk_info[i];
    const unsigned long long key = key_of((uint32_t)nh, d.start_pos[i]);
    const int32_t rin = d.tk_info[T + i], rout = d.tk_info[2 * T + i];
    uint32_t o = (uint32_t)co;
    for_rows(d, i, rin, rout, [&](int32_t h) {
      if (h >= 0 && d.W[h] == key) d.out_clusters[o++] = d.sid[h];
    });
    d.out_sector[ti] = d.start_sr[i] / d.R;
    d.out_start[ti] = d.start_pos[i];
    d.out_first[ti] = (uint32_t)co;
    d.out_xref[ti] = d.rows[rin].x;
#pragma unroll
    for (int q = 0; q < 5; ++q) d.out_param[(size_t)ti * 5 + q] = d.tk_param[(size_t)q * T + i];
#pragma unroll
    for (int q = 0; q < 15; ++q) d.out_cov[(size_t)ti * 15 + q] = d.tk_cov[(size_t)q * T + i];
    d.out_chi2[ti] = d.tk_chi2[i];
    d.out_ndf[ti] = 2 * nh - 5;
  }
}

__global__ void k_finish(DevPtrs d) {
  const uint32_t nt = n_tracklets(d);
  const unsigned long long tot = d.tk_scan[nt];
  uint32_t ntr = (uint32_t)(tot & 0xFFFFFFFFull);
  unsigned long long ncl = tot >> 32;
  uint32_t flags = 0;
  if (ntr > d.max_tracks) flags |= 4u;
  if (ncl > d.max_track_clusters) flags |= 8u;
  if (flags) atomicOr(&d.hdr->error_flags, flags);
  d.hdr->n_tracks = ntr;
  d.hdr->n_track_clusters = ncl;
  if (!flags) d.out_first[ntr] = (uint32_t)ncl;
}

}  // namespace

void launch_select(const DevPtrs& d, const KfConst& k, hipStream_t s) {
  uint32_t blocks = (d.tcap + kThreads - 1) / kThreads;
  if (blocks > 8192) blocks = 8192;
  blocks = xcd_grid(blocks == 0 ? 1 : blocks);
  hipLaunchKernelGGL(k_claim, dim3(blocks), dim3(kThreads), 0, s, d, k);
  hipLaunchKernelGGL(k_own, dim3(blocks), dim3(kThreads), 0, s, d, k);
  launch_scan_u64(d.tk_pack, d.tk_scan, &d.hdr->n_starts, d.tcap, d.scan_blocks, s);
  hipLaunchKernelGGL(k_emit, dim3(blocks), dim3(kThreads), 0, s, d, k);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(1), 0, s, d);
}

}  // namespace tpc
