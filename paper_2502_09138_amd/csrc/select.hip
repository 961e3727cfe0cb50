// K6: tracklet selector and canonical output -- steps C6 and C7.
//
// Ownership key.  The definition orders tracklets by (nHits, then smaller
// startPos).  Tracklet index i in the start list is ascending in startPos, so
// key32 = (nHits << 23) | (2^23 - 1 - i) orders them identically (nHits <= 255,
// i < 2^23 = the tracklet capacity limit) in 4 bytes instead of 8.
//
// Tiled selection (the default).  Every tracklet's hits lie in one sector, and
// the row -> hit columns are stored row-major over tracklets, so the tracklets
// of a sector read one row as a contiguous segment.  A workgroup owns a tile =
// (sector, block of consecutive rows) and keeps the tile's ownership words in
// LDS:
//   k_claim_tiles  every valid tracklet of the sector raises W_tile[hit] with an
//                  LDS atomicMax; the tile is then written to W (coalesced) --
//                  every position is written, so W needs no clearing -- and,
//                  from the same LDS copy, each tracklet's owned hits in the
//                  tile are counted -> own_part;
//   k_accept       sums the tiles, applies the acceptance rule, turns own_part
//                  into per-tile prefixes and packs (owned << 32) | accepted for
//                  one 64-bit scan giving track index and cluster offset;
//   k_records      writes the per-track records (canonical order = tracklet
//                  order = ascending start position) and the track -> tracklet
//                  list;
//   k_emit_tiles   walks the sector's tracks (not all its tracklets) and writes
//                  the owned cluster ids of each at offset + prefix, row by row
//                  (ascending row order);
//   (k_records also writes the totals and capacity flags.)
// Rows too large for an LDS tile use the same steps with W in global memory,
// one thread per tracklet (k_claim_g / k_own_g / k_emit_g).
#include "device_common.h"

namespace tpc {
namespace {

constexpr int kThreads = 256;
constexpr int kUnroll = 8;

__device__ __forceinline__ uint32_t key32(uint32_t nh, uint32_t i) { return (nh << 23) | (0x7FFFFFu - i); }
__device__ __forceinline__ uint32_t n_tracklets(const DevPtrs& d) { return min(d.hdr->n_starts, d.tcap); }

struct Tile {
  uint32_t s, ra, rb, first, n, ts, te;
};

// Tiles go to the XCDs (block b runs on XCD b % kXcds) in groups of half a
// sector's tiles, group g on XCD g % kXcds: a sector's tracklet arrays, which
// every tile of the sector scans, are then read through two L2s instead of
// all eight.  Returns the tile (sector-major), or at least S * n_tiles for a
// block without one.
__device__ __forceinline__ uint32_t tile_index(const DevPtrs& d, uint32_t n_tiles) {
  const uint32_t G = (n_tiles + 1) / 2, l = blockIdx.x / kXcds;
  return ((l / G) * kXcds + blockIdx.x % kXcds) * G + l % G;
}

__device__ __forceinline__ Tile tile_of(const DevPtrs& d, uint32_t v, uint32_t tile_rows, uint32_t n_tiles) {
  Tile t;
  t.s = v / n_tiles;
  const uint32_t tt = v % n_tiles;
  t.ra = tt * tile_rows;
  t.rb = min(d.R, t.ra + tile_rows);
  const uint32_t srb = t.s * d.R;
  t.first = d.row_off[srb + t.ra];
  t.n = d.row_off[srb + t.rb] - t.first;
  const uint32_t T = n_tracklets(d);
  t.ts = min(d.row_start_off[srb], T);
  t.te = min(d.row_start_off[srb + d.R], T);
  return t;
}

// A thread takes kBatch of the sector's tracklets at a time and issues all
// their loads (tracklet info, then the tile's rows of each) before using any,
// so a tile's loop over the tracklets is not one dependent load chain per
// tracklet.  Tiles have at most kTileRowsMax rows.
constexpr int kBatch = 4;
constexpr int kTileRowsMax = 4;

struct TileHits {
  int32_t h[kBatch][kTileRowsMax];   // hit in tile row ra + rr, -1 if none or outside [rin, rout]
  uint32_t key[kBatch];
};

template <int kT>
__device__ __forceinline__ void tile_hits(const DevPtrs& d, const KfConst& k, const Tile& tl, uint32_t i0,
                                          TileHits& th) {
  const uint32_t T = d.tcap;
  int32_t nh[kBatch], rin[kBatch], rout[kBatch];
#pragma unroll
  for (int u = 0; u < kBatch; ++u) {
    const uint32_t i = i0 + u * kT;
    const bool in = i < tl.te;
    nh[u] = in ? d.tk_info[i] : 0;
    rin[u] = in ? d.tk_info[T + i] : 0;
    rout[u] = in ? d.tk_info[2 * T + i] : -1;
  }
#pragma unroll
  for (int u = 0; u < kBatch; ++u) {
    const uint32_t i = i0 + u * kT;
    const bool ok = i < tl.te && nh[u] >= k.min_tracklet_hits;
    const int32_t lo = max((int32_t)tl.ra, rin[u]), hi = min((int32_t)tl.rb - 1, rout[u]);
    th.key[u] = key32((uint32_t)nh[u], i);
#pragma unroll
    for (int rr = 0; rr < kTileRowsMax; ++rr) {
      const int32_t r = (int32_t)tl.ra + rr;
      th.h[u][rr] = (ok && r >= lo && r <= hi) ? d.tk_rowhit[(size_t)r * T + i] : -1;
    }
  }
}

template <int kT>
__global__ void __launch_bounds__(kT) k_claim_tiles(DevPtrs d, KfConst k, uint32_t tile_rows, uint32_t n_tiles) {
  extern __shared__ uint32_t wt[];
  const uint32_t v = tile_index(d, n_tiles);
  if (v >= d.S * n_tiles) return;
  const Tile tl = tile_of(d, v, tile_rows, n_tiles);
  const uint32_t T = d.tcap;
  for (uint32_t j = threadIdx.x; j < tl.n; j += blockDim.x) wt[j] = 0u;
  __syncthreads();
  for (uint32_t i0 = tl.ts + threadIdx.x; i0 < tl.te; i0 += kBatch * kT) {
    TileHits th;
    tile_hits<kT>(d, k, tl, i0, th);
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
#pragma unroll
      for (int rr = 0; rr < kTileRowsMax; ++rr)
        if (th.h[u][rr] >= 0) atomicMax(&wt[(uint32_t)th.h[u][rr] - tl.first], th.key[u]);
  }
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < tl.n; j += blockDim.x) d.W[tl.first + j] = wt[j];
  // every claim on the tile's rows is in: count each tracklet's owned hits here
  const uint32_t tt = v % n_tiles;
  for (uint32_t i0 = tl.ts + threadIdx.x; i0 < tl.te; i0 += kBatch * kT) {
    TileHits th;
    tile_hits<kT>(d, k, tl, i0, th);
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const uint32_t i = i0 + u * kT;
      uint32_t cnt = 0;
#pragma unroll
      for (int rr = 0; rr < kTileRowsMax; ++rr)
        cnt += (th.h[u][rr] >= 0 && wt[(uint32_t)th.h[u][rr] - tl.first] == th.key[u]) ? 1u : 0u;
      if (i < tl.te) d.own_part[(size_t)tt * T + i] = (uint8_t)cnt;
    }
  }
}

constexpr int kAcceptBatch = 8;

__global__ void __launch_bounds__(kThreads) k_accept(DevPtrs d, KfConst k, uint32_t tile_rows) {
  const uint32_t nt = n_tracklets(d), T = d.tcap;
  const XcdSched sch = xcd_sched(nt);
  for (uint32_t vb = sch.first; vb < sch.end; vb += sch.stride) {
    const uint32_t i = vb * blockDim.x + threadIdx.x;
    if (i >= nt) continue;
    const int32_t nh = d.tk_info[i];
    unsigned long long packed = 0;
    if (nh >= k.min_tracklet_hits) {
      // owned hits lie only in the tiles that overlap [rin, rout]
      const uint32_t t0 = (uint32_t)d.tk_info[T + i] / tile_rows, t1 = (uint32_t)d.tk_info[2 * T + i] / tile_rows;
      uint32_t owned = 0;
      for (uint32_t tb = t0; tb <= t1; tb += kAcceptBatch) {   // the batch's loads go out before its stores
        uint32_t c[kAcceptBatch];
#pragma unroll
        for (int j = 0; j < kAcceptBatch; ++j) c[j] = tb + j <= t1 ? d.own_part[(size_t)(tb + j) * T + i] : 0u;
#pragma unroll
        for (int j = 0; j < kAcceptBatch; ++j)
          if (tb + j <= t1) {
            d.own_part[(size_t)(tb + j) * T + i] = (uint8_t)owned;   // prefix before this tile
            owned += c[j];
          }
      }
      const float need = k.min_owned_frac * (float)nh;
      if ((int32_t)owned >= k.min_track_hits && (float)owned >= need)
        packed = ((unsigned long long)owned << 32) | 1ull;
    }
    d.tk_pack[i] = packed;
  }
}

template <int kT>
__global__ void __launch_bounds__(kT) k_emit_tiles(DevPtrs d, KfConst k, uint32_t tile_rows, uint32_t n_tiles) {
  extern __shared__ uint32_t wt[];
  const uint32_t v = tile_index(d, n_tiles);
  if (v >= d.S * n_tiles) return;
  const Tile tl = tile_of(d, v, tile_rows, n_tiles);
  const uint32_t T = d.tcap, tt = v % n_tiles;
  for (uint32_t j = threadIdx.x; j < tl.n; j += blockDim.x) wt[j] = d.W[tl.first + j];
  // the sector's tracks: [track index of its first tracklet, ... of the next sector's), in track order
  const uint32_t v0 = (uint32_t)(d.tk_scan[tl.ts] & 0xFFFFFFFFull);
  const uint32_t v1 = min((uint32_t)(d.tk_scan[tl.te] & 0xFFFFFFFFull), d.max_tracks);
  __syncthreads();
  // kBatch tracks per thread at a time, each stage's loads issued together
  for (uint32_t vb = v0 + threadIdx.x; vb < v1; vb += kBatch * kT) {
    uint32_t i[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) i[u] = vb + u * kT < v1 ? d.acc_list[vb + u * kT] : 0u;
    bool go[kBatch];
    uint32_t o[kBatch], key[kBatch];
    int32_t lo[kBatch], hi[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const bool in = vb + u * kT < v1;
      const unsigned long long pk = in ? d.tk_pack[i[u]] : 0ull;
      const unsigned long long co = in ? d.tk_scan[i[u]] >> 32 : 0ull;
      const int32_t nh = in ? d.tk_info[i[u]] : 0;
      lo[u] = max((int32_t)tl.ra, in ? d.tk_info[T + i[u]] : 0);
      hi[u] = min((int32_t)tl.rb - 1, in ? d.tk_info[2 * T + i[u]] : -1);
      const uint32_t pre = in ? d.own_part[(size_t)tt * T + i[u]] : 0u;
      go[u] = in && co + (pk >> 32) <= d.max_track_clusters && lo[u] <= hi[u];   // capacity: flagged by finish()
      key[u] = key32((uint32_t)nh, i[u]);
      o[u] = (uint32_t)co + pre;
    }
    int32_t h[kBatch][kTileRowsMax];
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
#pragma unroll
      for (int rr = 0; rr < kTileRowsMax; ++rr) {
        const int32_t r = (int32_t)tl.ra + rr;
        h[u][rr] = (go[u] && r >= lo[u] && r <= hi[u]) ? d.tk_rowhit[(size_t)r * T + i[u]] : -1;
      }
    uint32_t id[kBatch][kTileRowsMax];
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
#pragma unroll
      for (int rr = 0; rr < kTileRowsMax; ++rr) {
        const bool own = h[u][rr] >= 0 && wt[(uint32_t)h[u][rr] - tl.first] == key[u];
        if (!own) h[u][rr] = -1;
        id[u][rr] = own ? d.sid[h[u][rr]] : 0u;
      }
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
#pragma unroll
      for (int rr = 0; rr < kTileRowsMax; ++rr)
        if (h[u][rr] >= 0) d.out_clusters[o[u]++] = id[u][rr];
  }
}

// Totals and capacity flags (one thread).
__device__ __forceinline__ void finish(const DevPtrs& d) {
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

__global__ void __launch_bounds__(kThreads) k_records(DevPtrs d, KfConst k) {
  const uint32_t nt = n_tracklets(d), T = d.tcap;
  if (blockIdx.x == 0 && threadIdx.x == 0) finish(d);
  const XcdSched sch = xcd_sched(nt);
  for (uint32_t vb = sch.first; vb < sch.end; vb += sch.stride) {
    const uint32_t i = vb * blockDim.x + threadIdx.x;
    if (i >= nt) continue;
    const unsigned long long pk = d.tk_pack[i];
    if (!(pk & 1ull)) continue;
    const unsigned long long pre = d.tk_scan[i];
    const uint32_t ti = (uint32_t)(pre & 0xFFFFFFFFull);
    const unsigned long long co = pre >> 32;
    if (ti >= d.max_tracks) continue;                          // flagged by finish()
    d.acc_list[ti] = i;                                        // track -> tracklet, for the tiled emit
    if (co + (pk >> 32) > d.max_track_clusters) continue;
    const int32_t nh = d.tk_info[i];
    d.out_sector[ti] = d.start_sr[i] / d.R;
    d.out_start[ti] = d.start_pos[i];
    d.out_first[ti] = (uint32_t)co;
    d.out_xref[ti] = d.rows[d.tk_info[T + i]].x;
#pragma unroll
    for (int q = 0; q < 5; ++q) d.out_param[(size_t)ti * 5 + q] = d.tk_param[(size_t)q * T + i];
#pragma unroll
    for (int q = 0; q < 15; ++q) d.out_cov[(size_t)ti * 15 + q] = d.tk_cov[(size_t)q * T + i];
    d.out_chi2[ti] = d.tk_chi2[i];
    d.out_ndf[ti] = 2 * nh - 5;
  }
}

// ---- global-memory variant for rows too large for an LDS tile ----
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

__global__ void __launch_bounds__(kThreads) k_clear_w(DevPtrs d) {
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < d.N; j += gridDim.x * blockDim.x) d.W[j] = 0u;
}

__global__ void __launch_bounds__(kThreads) k_claim_g(DevPtrs d, KfConst k) {
  const uint32_t nt = n_tracklets(d), T = d.tcap;
  const XcdSched sch = xcd_sched(nt);
  for (uint32_t vb = sch.first; vb < sch.end; vb += sch.stride) {
    const uint32_t i = vb * blockDim.x + threadIdx.x;
    if (i >= nt) continue;
    const int32_t nh = d.tk_info[i];
    if (nh < k.min_tracklet_hits) continue;
    const uint32_t key = key32((uint32_t)nh, i);
    for_rows(d, i, d.tk_info[T + i], d.tk_info[2 * T + i], [&](int32_t h) {
      if (h >= 0 && d.W[h] < key) atomicMax(&d.W[h], key);   // max is monotone: skip when already larger
    });
  }
}

__global__ void __launch_bounds__(kThreads) k_own_g(DevPtrs d, KfConst k) {
  const uint32_t nt = n_tracklets(d), T = d.tcap;
  const XcdSched sch = xcd_sched(nt);
  for (uint32_t vb = sch.first; vb < sch.end; vb += sch.stride) {
    const uint32_t i = vb * blockDim.x + threadIdx.x;
    if (i >= nt) continue;
    const int32_t nh = d.tk_info[i];
    unsigned long long packed = 0;
    if (nh >= k.min_tracklet_hits) {
      const uint32_t key = key32((uint32_t)nh, i);
      uint32_t owned = 0;
      for_rows(d, i, d.tk_info[T + i], d.tk_info[2 * T + i],
               [&](int32_t h) { owned += (h >= 0 && d.W[h] == key) ? 1u : 0u; });
      const float need = k.min_owned_frac * (float)nh;
      if ((int32_t)owned >= k.min_track_hits && (float)owned >= need)
        packed = ((unsigned long long)owned << 32) | 1ull;
    }
    d.tk_pack[i] = packed;
  }
}

__global__ void __launch_bounds__(kThreads) k_emit_g(DevPtrs d, KfConst k) {
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
    if (ti >= d.max_tracks || co + (pk >> 32) > d.max_track_clusters) continue;
    const uint32_t key = key32((uint32_t)d.tk_info[i], i);
    uint32_t o = (uint32_t)co;
    for_rows(d, i, d.tk_info[T + i], d.tk_info[2 * T + i], [&](int32_t h) {
      if (h >= 0 && d.W[h] == key) d.out_clusters[o++] = d.sid[h];
    });
  }
}


}  // namespace

void launch_select(const DevPtrs& d, const KfConst& k, uint32_t tile_rows, hipStream_t s) {
  const uint32_t blocks = xcd_grid(std::min<uint32_t>(8192, std::max<uint32_t>(1, (d.tcap + kThreads - 1) / kThreads)));
  if (tile_rows > 0 && tile_rows <= (uint32_t)kTileRowsMax && d.S > 0) {
    const uint32_t n_tiles = (d.R + tile_rows - 1) / tile_rows;
    const size_t lds = (size_t)d.tile_cap * sizeof(uint32_t);
    const uint32_t G = (n_tiles + 1) / 2, groups = (d.S * n_tiles + G - 1) / G;
    const dim3 tiles((groups + kXcds - 1) / kXcds * kXcds * G);   // every group slot of every XCD
    // workgroup size of the tile kernels: their LDS holds the tile's ownership words (up to 48 KB),
    // which bounds the workgroups per CU, so larger workgroups put more waves on each tile
    const uint32_t nt = d.k6_threads == 1024 ? 1024u : d.k6_threads == 256 ? 256u : 512u;
    if (nt == 1024) hipLaunchKernelGGL(k_claim_tiles<1024>, tiles, dim3(nt), lds, s, d, k, tile_rows, n_tiles);
    else if (nt == 256) hipLaunchKernelGGL(k_claim_tiles<256>, tiles, dim3(nt), lds, s, d, k, tile_rows, n_tiles);
    else hipLaunchKernelGGL(k_claim_tiles<512>, tiles, dim3(nt), lds, s, d, k, tile_rows, n_tiles);
    hipLaunchKernelGGL(k_accept, dim3(blocks), dim3(kThreads), 0, s, d, k, tile_rows);
    launch_scan_u64(d.tk_pack, d.tk_scan, &d.hdr->n_starts, d.tcap, d.scan_blocks, s);
    hipLaunchKernelGGL(k_records, dim3(blocks), dim3(kThreads), 0, s, d, k);
    if (nt == 1024) hipLaunchKernelGGL(k_emit_tiles<1024>, tiles, dim3(nt), lds, s, d, k, tile_rows, n_tiles);
    else if (nt == 256) hipLaunchKernelGGL(k_emit_tiles<256>, tiles, dim3(nt), lds, s, d, k, tile_rows, n_tiles);
    else hipLaunchKernelGGL(k_emit_tiles<512>, tiles, dim3(nt), lds, s, d, k, tile_rows, n_tiles);
  } else {
    hipLaunchKernelGGL(k_clear_w, dim3(xcd_grid(std::min<uint32_t>(8192, std::max<uint32_t>(1, (d.N + kThreads - 1) / kThreads)))),
                       dim3(kThreads), 0, s, d);
    hipLaunchKernelGGL(k_claim_g, dim3(blocks), dim3(kThreads), 0, s, d, k);
    hipLaunchKernelGGL(k_own_g, dim3(blocks), dim3(kThreads), 0, s, d, k);
    launch_scan_u64(d.tk_pack, d.tk_scan, &d.hdr->n_starts, d.tcap, d.scan_blocks, s);
    hipLaunchKernelGGL(k_emit_g, dim3(blocks), dim3(kThreads), 0, s, d, k);
    hipLaunchKernelGGL(k_records, dim3(blocks), dim3(kThreads), 0, s, d, k);
  }
}

}  // namespace tpc
