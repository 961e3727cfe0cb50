// C10/C11: track-model compression of the clusters of a completed request,
// and its decoding.
//
// Encoding writes, per track, the model (x_ref and six coefficients of the
// second-order expansion of the fitted helix around x_ref) and, per track
// cluster, its row and the quantised residuals (k_y, k_z) to that model; the
// clusters on no track are listed raw, in input order.  Decoding rebuilds the
// clusters from the stream.  Every float32 step is written out in the order the
// definition gives, with contraction off, so the codes are the same bits as
// any other evaluation of the definition; the coefficients are computed in
// double (IEEE division and square root) and rounded once.
//
// All work is one lane per track or per cluster, bound by HBM traffic: about
// 40 B per track (6 coefficients, x_ref, offset) and 13 B per track cluster
// (id, row, codes, raw pair) for the encoding, the same order for the
// decoding; the clusters on no track cost a flag and 9 B each.  The decoder
// does not search per cluster: a wave takes kChunk * 64 consecutive track
// clusters, and each lane finds its track once and then walks forward with
// its clusters.  (The encoder searches its track and row per cluster: both
// searches run over small arrays that stay in cache, which measured faster
// than chunks of clusters per lane or a per-cluster row word.)
#include <algorithm>

#include "device_common.h"

namespace tpc {
namespace {

constexpr int kThreads = 256;
constexpr int16_t kEscape = -32768;
constexpr uint32_t kChunk = 16;   // track clusters per decoding lane between two track searches

__device__ __forceinline__ uint32_t grid_stride() { return gridDim.x * blockDim.x; }
__device__ __forceinline__ uint32_t gtid() { return blockIdx.x * blockDim.x + threadIdx.x; }

// Last index k with a[k] <= v in the ascending array a[0..n] (a[0] <= v).
__device__ __forceinline__ uint32_t last_le(const uint32_t* a, uint32_t n, uint32_t v) {
  uint32_t lo = 0, hi = n;   // a[lo] <= v < a[hi] (a[n] treated as +inf)
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (a[mid] <= v) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Track of cluster position j, from a track t0 at or before it (first[t0] <= j),
// never past the last track.
__device__ __forceinline__ uint32_t walk_track(const uint32_t* first, uint32_t n_tracks, uint32_t t0, uint64_t j) {
  uint32_t t = t0;
  while (t + 1 < n_tracks && first[t + 1] <= j) ++t;
  return t;
}

// c0 + u * (c1 + u * c2), u = xr - x_ref, float32, no fused multiply-add.
__device__ __forceinline__ float predict(float xr, float x_ref, float c0, float c1, float c2) {
#pragma clang fp contract(off)
  const float u = xr - x_ref;
  const float inner = c1 + u * c2;
  const float outer = u * inner;
  return c0 + outer;
}

__global__ void __launch_bounds__(kThreads) k_codec_tracks(CodecArgs a) {
  if (gtid() == 0) {
    *a.n_escaped = 0;
    if (a.n_tracks == 0) a.first[0] = 0;
  }
  for (uint32_t t = gtid(); t < a.n_tracks; t += grid_stride()) {
    const float* p = a.param + 5 * (size_t)t;
    float* c = a.coef + 6 * (size_t)t;
    const double s = p[2], T = p[3], qpt = p[4];
    if (fabs(s) < 1.0) {
      const double kappa = a.bk * qpt;
      const double cc = sqrt(1.0 - s * s);
      const double ic = 1.0 / cc;
      const double ic3 = ic * ic * ic;
      c[0] = p[0];
      c[1] = (float)(s * ic);
      c[2] = (float)(0.5 * kappa * ic3);
      c[3] = p[1];
      c[4] = (float)(T * ic);
      c[5] = (float)(((0.5 * T) * s) * kappa * ic3);
    } else {
      for (int q = 0; q < 6; ++q) c[q] = 0.0f;   // no model: every cluster of the track is escaped
    }
    a.x_ref[t] = a.xref_in[t];
    a.first[t] = a.first_in[t];
    if (t + 1 == a.n_tracks) a.first[t + 1] = a.first_in[t + 1];
  }
}

// Every cluster starts unassigned (1), before k_codec_clusters clears the track clusters.
__global__ void __launch_bounds__(kThreads) k_codec_unmark(CodecArgs a) {
  for (uint32_t i = gtid(); i < a.N; i += grid_stride()) a.unf[i] = 1u;
}

__global__ void __launch_bounds__(kThreads) k_codec_clusters(CodecArgs a) {
#pragma clang fp contract(off)
  uint32_t esc = 0;
  for (uint64_t j = gtid(); j < a.n_cl; j += grid_stride()) {
    const uint32_t t = last_le(a.first_in, a.n_tracks, (uint32_t)j);
    const uint32_t id = a.clusters[j];
    a.unf[id] = 0u;
    const uint32_t r = last_le(a.row_off, a.SR, id) % a.R;
    a.row[j] = (uint8_t)r;
    const float* c = a.coef + 6 * (size_t)t;
    const float xr = a.rows[r].x, xref = a.xref_in[t];
    const float py = predict(xr, xref, c[0], c[1], c[2]);
    const float pz = predict(xr, xref, c[3], c[4], c[5]);
    const float ym = a.y[id], zm = a.z[id];
    const float vy = (ym - py) * a.inv_qy;
    const float vz = (zm - pz) * a.inv_qz;
    const bool model = fabsf(a.param[5 * (size_t)t + 2]) < 1.0f;
    short2 k;
    float2 raw = make_float2(0.0f, 0.0f);
    if (model && fabsf(vy) <= 32767.0f && fabsf(vz) <= 32767.0f) {
      k = make_short2((short)(int)rintf(vy), (short)(int)rintf(vz));
    } else {
      k = make_short2(kEscape, 0);
      raw = make_float2(ym, zm);
      ++esc;
    }
    reinterpret_cast<short2*>(a.code)[j] = k;
    reinterpret_cast<float2*>(a.raw)[j] = raw;
  }
  // escaped clusters: one atomic per wave
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) esc += (uint32_t)__shfl_xor((int)esc, off, kWave);
  if (threadIdx.x % kWave == 0 && esc) atomicAdd(a.n_escaped, esc);
}

// The clusters on no track, raw, in input order: counted per (sector, row)
// slot (one block each), the counts scanned, then each slot's block lists its
// own in order.
__global__ void __launch_bounds__(kThreads) k_codec_row_count(CodecArgs a) {
  __shared__ uint32_t wsum[kThreads / kWave];
  const uint32_t sr = blockIdx.x;
  const uint32_t b = a.row_off[sr], e = a.row_off[sr + 1];
  uint32_t c = 0;
  for (uint32_t i = b + threadIdx.x; i < e; i += kThreads) c += a.unf[i];
  uint32_t total;
  (void)block_exclusive_scan<uint32_t>(c, wsum, &total);
  if (threadIdx.x == 0) a.row_cnt[sr] = total;
}

__global__ void __launch_bounds__(kThreads) k_codec_row_emit(CodecArgs a) {
  __shared__ uint32_t wsum[kThreads / kWave];
  const uint32_t sr = blockIdx.x;
  const uint32_t b = a.row_off[sr], e = a.row_off[sr + 1];
  uint32_t base = a.row_pos[sr];
  for (uint32_t i0 = b; i0 < e; i0 += kThreads) {   // block-uniform chunks
    const uint32_t i = i0 + threadIdx.x;
    const uint32_t f = i < e ? a.unf[i] : 0u;
    uint32_t total;
    const uint32_t k = base + block_exclusive_scan<uint32_t>(f, wsum, &total);
    if (f) {
      a.un_row[k] = (uint8_t)(sr % a.R);
      reinterpret_cast<float2*>(a.un_yz)[k] = make_float2(a.y[i], a.z[i]);
    }
    base += total;
  }
}

__global__ void __launch_bounds__(kThreads) k_codec_decode(DecodeArgs a) {
#pragma clang fp contract(off)
  const uint64_t span = (uint64_t)kWave * kChunk;
  const uint32_t lane = threadIdx.x % kWave;
  const uint64_t wave = gtid() / kWave, waves = grid_stride() / kWave;
  for (uint64_t base = wave * span; base < a.n_cl; base += waves * span) {   // wave-uniform bounds
    uint32_t t = 0;
    bool found = false;
    for (uint32_t k = 0; k < kChunk; ++k) {
      const uint64_t j = base + lane + (uint64_t)k * kWave;
      if (j >= a.n_cl) break;
      const short2 c2 = reinterpret_cast<const short2*>(a.code)[j];
      const uint8_t r = a.row[j];
      float y, z;
      if (c2.x == kEscape) {
        const float2 raw = reinterpret_cast<const float2*>(a.raw)[j];
        y = raw.x;
        z = raw.y;
      } else {
        t = found ? walk_track(a.first, a.n_tracks, t, j) : last_le(a.first, a.n_tracks, (uint32_t)j);
        found = true;
        const float* c = a.coef + 6 * (size_t)t;
        const float xr = a.rows[r].x, xref = a.x_ref[t];
        const float py = predict(xr, xref, c[0], c[1], c[2]);
        const float pz = predict(xr, xref, c[3], c[4], c[5]);
        const float dy = (float)c2.x * a.q_y;
        const float dz = (float)c2.y * a.q_z;
        y = py + dy;
        z = pz + dz;
      }
      a.y_out[j] = y;
      a.z_out[j] = z;
      a.row_out[j] = r;
    }
  }
  for (uint64_t k = gtid(); k < a.n_un; k += grid_stride()) {
    const float2 v = reinterpret_cast<const float2*>(a.un_yz)[k];
    a.y_out[a.n_cl + k] = v.x;
    a.z_out[a.n_cl + k] = v.y;
    a.row_out[a.n_cl + k] = a.un_row[k];
  }
}

uint32_t blocks_for(uint64_t n) {
  const uint64_t b = (n + kThreads - 1) / kThreads;
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(b, 8192));
}

}  // namespace

void launch_codec_encode(const CodecArgs& a, unsigned long long* scan_blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_codec_tracks, dim3(blocks_for(a.n_tracks)), dim3(kThreads), 0, s, a);
  hipLaunchKernelGGL(k_codec_unmark, dim3(blocks_for(a.N)), dim3(kThreads), 0, s, a);
  hipLaunchKernelGGL(k_codec_clusters, dim3(blocks_for(a.n_cl)), dim3(kThreads), 0, s, a);
  if (a.SR == 0) return;
  hipLaunchKernelGGL(k_codec_row_count, dim3(a.SR), dim3(kThreads), 0, s, a);
  launch_scan_u32(a.row_cnt, a.row_pos, a.SR, scan_blocks, s);
  hipLaunchKernelGGL(k_codec_row_emit, dim3(a.SR), dim3(kThreads), 0, s, a);
}

void launch_codec_decode(const DecodeArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_codec_decode, dim3(blocks_for(std::max<uint64_t>((a.n_cl + kChunk - 1) / kChunk, a.n_un))),
                     dim3(kThreads), 0, s, a);
}

}  // namespace tpc
