// K2: neighbour finder -- step C2 of the tracker definition.
//
// One wave per tile of up to 64 consecutive hits of one row (so every lane
// owns one hit, whatever the row size).  Rows are sorted z-line-major, so the
// candidates any hit of the tile can reach in an adjacent row lie in one
// contiguous run of that row's z-lines: the z-lines covering the tile's
// [z_min - w_z, z_max + w_z] (the same padded window and float32 bin rule the
// per-hit search uses, so every per-hit range is inside the staged run).  The
// run's hits and bin starts are staged into LDS with coalesced loads and all
// candidate tests read LDS; a run larger than the stage reads global memory.
//
// All window tests and the pair deviation use float32 with contraction off, in
// the order the definition writes them, so the argmin is bit-identical to any
// other evaluation of the definition.
#include <algorithm>

#include "device_common.h"

namespace tpc {
namespace {

constexpr int kThreads = 64;             // one wave; one hit per lane
constexpr uint32_t kSliceHits = 256;     // staged hits per adjacent row
// Staged bin starts per adjacent row, and waves per SIMD.  The 4-slot kernel
// stages 128 (5 KB of LDS per wave) and is held to 72 VGPRs, which lets seven
// waves share a SIMD instead of six (-7% on the 32-orbit frame).  The 8-slot
// kernel keeps 256 and its 89 VGPRs (five waves): held to 80 for six waves it
// spills, 4% faster on the uneven chunks but its spill stores triple its HBM
// traffic; at seven waves it runs twice as long.
template <int kUpSlots>
constexpr uint32_t slice_bins() { return kUpSlots == 4 ? 128u : 256u; }
template <int kUpSlots>
constexpr int link_waves() { return kUpSlots == 4 ? 7 : 5; }

struct RowView {
  const float2* yz;        // indexed by position - off
  const uint32_t* bs;      // bin starts (global positions), indexed by bin - bofs
  uint32_t off;            // global sorted position of yz[0]
  int bofs;                // first bin held in bs
  int ny, nz;
  float y_lo, inv_wy, z_lo, inv_wz;
};

// Candidates of the bins covering a window around (y, z): fn(q, (y, z)) for
// every hit q (relative to v.off) of those bins.  A lane walks its z-lines as
// one flat sequence of groups of kGroup hits whose reads are issued together
// (indices clamped to the z-line), so a wave runs for the largest per-lane
// candidate count rather than the sum of per-line maxima.  The order in which
// candidates are visited does not matter: every decision below breaks ties
// explicitly.
constexpr int kGroup = 4;

template <class Fn>
__device__ __forceinline__ void for_window(const RowView& v, float y, float z, float wy, float wz, Fn fn) {
#pragma clang fp contract(off)
  const float py = wy + kWinPad, pz = wz + kWinPad;
  const int iy0 = bin1(y - py, v.y_lo, v.inv_wy, v.ny), iy1 = bin1(y + py, v.y_lo, v.inv_wy, v.ny);
  const int iz0 = bin1(z - pz, v.z_lo, v.inv_wz, v.nz), iz1 = bin1(z + pz, v.z_lo, v.inv_wz, v.nz);
  int iz = iz0;
  uint32_t q = v.bs[iz * v.ny + iy0 - v.bofs] - v.off, hi = v.bs[iz * v.ny + iy1 + 1 - v.bofs] - v.off;
  for (;;) {
    while (q >= hi && iz < iz1) {
      ++iz;
      q = v.bs[iz * v.ny + iy0 - v.bofs] - v.off;
      hi = v.bs[iz * v.ny + iy1 + 1 - v.bofs] - v.off;
    }
    if (q >= hi) break;
    float2 c[kGroup];
#pragma unroll
    for (int j = 0; j < kGroup; ++j) c[j] = v.yz[min(q + j, hi - 1)];
#pragma unroll
    for (int j = 0; j < kGroup; ++j)
      if (q + j < hi) fn(q + j, c[j]);
    q += kGroup;
  }
}

// Candidate slots per lane for the passing hits of row r+1 (mean 1.6, max 7
// on a central event), held in registers; a hit with more falls back to
// rescanning the window.  Two instances: 8 slots (dense frames, where more
// slots avoid rescans) and 4 (sparse frames: leaner code and six waves per
// SIMD instead of five); the tuning knob TPC_KNOB_LINK_SLOTS chooses.
// Links of one hit (sorted position p, coordinates h) of row rc between rows dn and up.
template <int kUpSlots>
__device__ __forceinline__ void link_hit(const DevPtrs& d, uint32_t p, float2 h, const RowView& dn, const RowView& up,
                                         const RowConst& rc, float rho) {
#pragma clang fp contract(off)
  const float t = rc.t;
  int32_t bu = -1, bd = -1;
  float best = 0.0f;
  // passing candidates of row r+1, collected once (registers: unrolled, predicated slot writes)
  int nu = 0;
  uint32_t sq[kUpSlots];
  float2 sc[kUpSlots];
  for_window(up, h.x, h.y, rc.wy_up, rc.wz_up, [&](uint32_t qu, float2 pu) {
    if (!(fabsf(pu.x - h.x) <= rc.wy_up && fabsf(pu.y - h.y) <= rc.wz_up)) return;
#pragma unroll
    for (int j = 0; j < kUpSlots; ++j)
      if (j == nu) {
        sq[j] = qu;
        sc[j] = pu;
      }
    ++nu;
  });
  if (nu == 0) {
    d.up0[p] = -1;
    d.down0[p] = -1;
    return;
  }
  auto pair = [&](const float2 pd, int32_t gd, uint32_t qu, const float2 pu) {
    const float yp = pd.x + t * (pu.x - pd.x);
    const float zp = pd.y + t * (pu.y - pd.y);
    const float ey = h.x - yp, ez = h.y - zp;
    const float dev = ey * ey + rho * (ez * ez);
    if (!(dev <= rc.dmax)) return;
    const int32_t gu = (int32_t)(up.off + qu);
    if (bu < 0 || dev < best || (dev == best && (gu < bu || (gu == bu && gd < bd)))) {
      best = dev;
      bu = gu;
      bd = gd;
    }
  };
  for_window(dn, h.x, h.y, rc.wy_dn, rc.wz_dn, [&](uint32_t qd, float2 pd) {
    if (!(fabsf(pd.x - h.x) <= rc.wy_dn && fabsf(pd.y - h.y) <= rc.wz_dn)) return;
    const int32_t gd = (int32_t)(dn.off + qd);
    if (nu <= kUpSlots) {
#pragma unroll
      for (int k = 0; k < kUpSlots; ++k)
        if (k < nu) pair(pd, gd, sq[k], sc[k]);
    } else {
      for_window(up, h.x, h.y, rc.wy_up, rc.wz_up, [&](uint32_t qu, float2 pu) {
        if (fabsf(pu.x - h.x) <= rc.wy_up && fabsf(pu.y - h.y) <= rc.wz_up) pair(pd, gd, qu, pu);
      });
    }
  });
  d.up0[p] = bu;
  d.down0[p] = bd;
}

__device__ __forceinline__ float wave_minf(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fminf(v, __shfl_xor(v, off, kWave));
  return v;
}
__device__ __forceinline__ float wave_maxf(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, kWave));
  return v;
}

// View of adjacent row sr restricted to the z-lines reachable from z in
// [zmin, zmax] with window half-width wz; staged into (lyz, lbs) when it fits.
template <uint32_t kBins>
__device__ __forceinline__ RowView adjacent_view(const DevPtrs& d, uint32_t sr, float zmin, float zmax, float wz,
                                                 bool stage, float2* lyz, uint32_t* lbs) {
#pragma clang fp contract(off)
  const uint32_t R = d.R;
  const RowConst rc = d.rows[sr % R];
  const SectorConst sc = d.secs[sr / R];
  const uint2 meta = d.row_meta[sr];
  RowView v;
  v.ny = (int)(meta.y & 0xFFFFu);
  v.nz = (int)(meta.y >> 16);
  v.y_lo = rc.y_lo;
  v.inv_wy = rc.inv_wy;
  v.z_lo = sc.z_lo;
  v.inv_wz = sc.inv_wz;
  const uint32_t* bs = d.bin_start + meta.x;
  const float pz = wz + kWinPad;
  const int iz0 = bin1(zmin - pz, v.z_lo, v.inv_wz, v.nz), iz1 = bin1(zmax + pz, v.z_lo, v.inv_wz, v.nz);
  const uint32_t b0 = (uint32_t)(iz0 * v.ny), b1 = (uint32_t)((iz1 + 1) * v.ny);   // bins [b0, b1), starts [b0, b1]
  const uint32_t s0 = bs[b0], s1 = bs[b1];
  if (stage && s1 - s0 <= kSliceHits && b1 - b0 + 1 <= kBins) {
    for (uint32_t j = threadIdx.x; j < s1 - s0; j += kThreads) lyz[j] = d.syz[s0 + j];
    for (uint32_t j = threadIdx.x; j <= b1 - b0; j += kThreads) lbs[j] = bs[b0 + j];
    v.yz = lyz;
    v.bs = lbs;
    v.off = s0;
    v.bofs = (int)b0;
  } else {
    v.off = d.row_off[sr];
    v.yz = d.syz + v.off;
    v.bs = bs;
    v.bofs = 0;
  }
  return v;
}

template <int kUpSlots>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(link_waves<kUpSlots>())))
k_links(DevPtrs d, float rho, uint32_t G) {
  __shared__ float2 lyz[2][kSliceHits];
  __shared__ uint32_t lbs[2][slice_bins<kUpSlots>()];
  // Tiles go to the XCDs (block b runs on XCD b % kXcds) in groups of G
  // consecutive tiles, group g on XCD g % kXcds: the adjacent-row runs that
  // tiles of rows r - 1 and r + 1 both stage are then read through one L2
  // (G = 1: consecutive tiles on consecutive XCDs).
  const uint32_t l = blockIdx.x / kXcds;
  const uint32_t tile = G <= 1 ? blockIdx.x : ((l / G) * kXcds + blockIdx.x % kXcds) * G + l % G;
  if (tile >= d.n_link_tiles) return;
  const uint32_t sr = d.tile_sr[tile], R = d.R, row = sr % R;
  const uint32_t a = d.row_off[sr] + (tile - d.tile_off[sr]) * kThreads;
  const uint32_t cnt = min((uint32_t)kThreads, d.row_off[sr + 1] - a);
  const uint32_t lane = threadIdx.x;
  const bool mine = lane < cnt;
  const uint32_t p = a + lane;
  if (row == 0 || row + 1 >= R) {
    if (mine) {
      d.up0[p] = -1;
      d.down0[p] = -1;
    }
    return;
  }
  const float2 h = mine ? d.syz[p] : make_float2(0.0f, 0.0f);
  const float zmin = wave_minf(mine ? h.y : INFINITY), zmax = wave_maxf(mine ? h.y : -INFINITY);
  // a non-finite or out-of-range z (flagged by K1) has no place in the z-line
  // order: such a tile searches the whole adjacent rows in global memory
  const bool stage = !__any(mine && !(fabsf(h.y) <= kMaxCoord));
  const RowConst rc = d.rows[row];
  const RowView dn = adjacent_view<slice_bins<kUpSlots>()>(d, sr - 1, zmin, zmax, rc.wz_dn, stage, lyz[0], lbs[0]);
  const RowView up = adjacent_view<slice_bins<kUpSlots>()>(d, sr + 1, zmin, zmax, rc.wz_up, stage, lyz[1], lbs[1]);
  __syncthreads();
  if (mine) link_hit<kUpSlots>(d, p, h, dn, up, rc, rho);
}

}  // namespace

void launch_links(const DevPtrs& d, uint32_t, hipStream_t s) {
  if (d.n_link_tiles == 0) return;
  // group size: as set, or one contiguous eighth of the tiles per XCD
  const uint32_t n = d.n_link_tiles;
  const uint32_t G = d.k2_group == kLinkGroupEighth ? (n + kXcds - 1) / kXcds : std::max<uint32_t>(1u, d.k2_group);
  const uint64_t groups = (n + (uint64_t)G - 1) / G;
  const uint32_t blocks = G == 1 ? n : (uint32_t)((groups + kXcds - 1) / kXcds * kXcds * G);   // every group slot
  if (d.k2_slots == 4)
    hipLaunchKernelGGL(k_links<4>, dim3(blocks), dim3(kThreads), 0, s, d, d.rho, G);
  else
    hipLaunchKernelGGL(k_links<8>, dim3(blocks), dim3(kThreads), 0, s, d, d.rho, G);
}

}  // namespace tpc
