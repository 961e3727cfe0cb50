// K2: neighbour finder -- step C2 of the tracker definition.
//
// One workgroup per (sector, row).  The two adjacent rows (r-1, r+1) are
// staged in LDS -- their (y, z) pairs and bin starts -- so every candidate
// test of the row's hits reads LDS instead of scattered L2 lines.  Rows too
// large for the LDS budget read the same arrays from global memory.  All
// window tests and the pair deviation use float32 with contraction off, in
// the order the definition writes them, so the argmin is bit-identical to any
// other evaluation of the definition.
#include "device_common.h"

namespace tpc {
namespace {

constexpr int kThreads = 256;
constexpr uint32_t kLdsRowCap = 3072;    // hits per staged row

struct RowView {
  const float2* yz;        // indexed by position - off
  const uint32_t* bs;      // bin starts (global positions), nb+1 entries
  uint32_t off;            // global sorted position of the row's first hit
  int ny, nz;
  float y_lo, inv_wy, z_lo, inv_wz;
};

// Positions [lo, hi) of candidate bins for a window around (y, z), one z-line at a time.
template <class Fn>
__device__ __forceinline__ void for_window(const RowView& v, float y, float z, float wy, float wz, Fn fn) {
#pragma clang fp contract(off)
  const float py = wy + kWinPad, pz = wz + kWinPad;
  const int iy0 = bin1(y - py, v.y_lo, v.inv_wy, v.ny), iy1 = bin1(y + py, v.y_lo, v.inv_wy, v.ny);
  const int iz0 = bin1(z - pz, v.z_lo, v.inv_wz, v.nz), iz1 = bin1(z + pz, v.z_lo, v.inv_wz, v.nz);
  for (int iz = iz0; iz <= iz1; ++iz) {
    const uint32_t lo = v.bs[iz * v.ny + iy0] - v.off, hi = v.bs[iz * v.ny + iy1 + 1] - v.off;
    for (uint32_t q = lo; q < hi; ++q) fn(q);
  }
}

__device__ __forceinline__ void row_view(const DevPtrs& d, uint32_t sr, RowView& v) {
  const uint32_t R = d.R;
  const RowConst rc = d.rows[sr % R];
  const SectorConst sc = d.secs[sr / R];
  const uint32_t dims = d.row_dims[sr];
  v.ny = (int)(dims & 0xFFFFu);
  v.nz = (int)(dims >> 16);
  v.off = d.row_off[sr];
  v.y_lo = rc.y_lo;
  v.inv_wy = rc.inv_wy;
  v.z_lo = sc.z_lo;
  v.inv_wz = sc.inv_wz;
  v.yz = d.syz + v.off;
  v.bs = d.bin_start + bin_base(d, sr);
}

// Stage a row's (y, z) and bin starts into LDS.
__device__ __forceinline__ void stage(RowView& v, uint32_t n, float2* lyz, uint32_t* lbs) {
  const uint32_t nb = (uint32_t)(v.ny * v.nz) + 1;
  for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) lyz[j] = v.yz[j];
  for (uint32_t j = threadIdx.x; j < nb; j += blockDim.x) lbs[j] = v.bs[j];
  v.yz = lyz;
  v.bs = lbs;
}

// Candidate slots per thread for the passing hits of row r+1 (mean 1.6, max 7
// on a central event); a hit with more falls back to rescanning the window.
constexpr int kUpSlots = 8;

__device__ __forceinline__ void links_row(const DevPtrs& d, uint32_t sr, const RowView& dn, const RowView& up,
                                          const RowConst& rc, float rho, uint16_t* slots) {
#pragma clang fp contract(off)
  const uint32_t a = d.row_off[sr], n = d.row_off[sr + 1] - a;
  const float t = rc.t;
  for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
    const float2 h = d.syz[a + j];
    int32_t bu = -1, bd = -1;
    float best = 0.0f;
    // passing candidates of row r+1, collected once
    int nu = 0;
    for_window(up, h.x, h.y, rc.wy_up, rc.wz_up, [&](uint32_t qu) {
      const float2 pu = up.yz[qu];
      if (!(fabsf(pu.x - h.x) <= rc.wy_up && fabsf(pu.y - h.y) <= rc.wz_up)) return;
      if (nu < kUpSlots) slots[nu] = (uint16_t)qu;
      ++nu;
    });
    if (nu == 0) {
      d.up0[a + j] = -1;
      d.down0[a + j] = -1;
      continue;
    }
    auto pair = [&](const float2 pd, int32_t gd, uint32_t qu) {
      const float2 pu = up.yz[qu];
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
    for_window(dn, h.x, h.y, rc.wy_dn, rc.wz_dn, [&](uint32_t qd) {
      const float2 pd = dn.yz[qd];
      if (!(fabsf(pd.x - h.x) <= rc.wy_dn && fabsf(pd.y - h.y) <= rc.wz_dn)) return;
      const int32_t gd = (int32_t)(dn.off + qd);
      if (nu <= kUpSlots) {
        for (int k = 0; k < nu; ++k) pair(pd, gd, slots[k]);
      } else {
        for_window(up, h.x, h.y, rc.wy_up, rc.wz_up, [&](uint32_t qu) {
          const float2 pu = up.yz[qu];
          if (fabsf(pu.x - h.x) <= rc.wy_up && fabsf(pu.y - h.y) <= rc.wz_up) pair(pd, gd, qu);
        });
      }
    });
    d.up0[a + j] = bu;
    d.down0[a + j] = bd;
  }
}

__global__ void __launch_bounds__(kThreads) k_links(DevPtrs d, uint32_t cap, float rho) {
  extern __shared__ uint32_t lds[];
  __shared__ uint16_t slots[kThreads][kUpSlots];
  const uint32_t sr = blockIdx.x;
  const uint32_t R = d.R;
  const uint32_t row = sr % R;
  const uint32_t a = d.row_off[sr], n = d.row_off[sr + 1] - a;
  if (row == 0 || row + 1 >= R) {
    for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
      d.up0[a + j] = -1;
      d.down0[a + j] = -1;
    }
    return;
  }
  if (n == 0) return;
  RowView dn, up;
  row_view(d, sr - 1, dn);
  row_view(d, sr + 1, up);
  const uint32_t nd = d.row_off[sr] - dn.off, nu = d.row_off[sr + 2] - up.off;
  // LDS layout: yz_dn[cap], yz_up[cap], bs_dn[cap+2], bs_up[cap+2]
  float2* lyz = reinterpret_cast<float2*>(lds);
  uint32_t* lbs = lds + 4 * cap;
  if (nd <= cap) stage(dn, nd, lyz, lbs);
  if (nu <= cap) stage(up, nu, lyz + cap, lbs + cap + 2);
  __syncthreads();
  links_row(d, sr, dn, up, d.rows[row], rho, slots[threadIdx.x]);
}

}  // namespace

void launch_links(const DevPtrs& d, uint32_t max_row_hits, hipStream_t s) {
  if (d.SR == 0) return;
  const uint32_t cap = max_row_hits < kLdsRowCap ? max_row_hits : kLdsRowCap;
  const size_t lds = (size_t)(4 * cap + 2 * (cap + 2)) * sizeof(uint32_t);
  hipLaunchKernelGGL(k_links, dim3(d.SR), dim3(kThreads), lds, s, d, cap, d.rho);
}

}  // namespace tpc
