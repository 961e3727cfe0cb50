// K5: tracklet constructor -- step C5 of the tracker definition.
//
// Each tracklet (chain start) walks its chain (dependent up1 gathers), seeds
// from three chain hits, fits the chain, extends outward through the row
// grids and refits inward with a fresh covariance, filling gaps and extending
// below the chain.  Two schedules compute it: the row-synchronous kernel
// (k_tracklets_rs, a wave sweeps the rows of one sector in lockstep with each
// row staged in LDS; for frames whose rows fit the stage) and the
// lane-per-tracklet pipeline (k_seed, k_up, k_sort, k_down, k_guard; any row
// size).  The helix state p[5] and packed covariance C[15] are accumulated in
// double registers (see par_t / cov_t); the per-step increments and the
// Jacobian are float32.  The transport exploits the sparsity of the Jacobian
// (6 non-trivial entries).
//
// Latency is the bound (each row step is a dependent chain: propagate ->
// grid lookup -> candidate loads -> update), so the per-row constants are
// staged in LDS, a row's grid is located with one 8-byte load, and the
// float32 step arithmetic uses the hardware reciprocal / square root (its
// rounding is relative to one row step; the results are checked against the
// FP64 definition to 1e-4 relative, not bit-exact).
//
// The per-tracklet row -> hit column lives in global memory (row-major over
// tracklets, so lanes at the same row write one coalesced segment); the
// downward pass rewrites every row in [x_ref row, outermost row] with its
// final value, which is the only range the selector reads.
//
// z precision: in a continuous-readout frame the drift coordinate reaches
// several thousand cm, where one float32 ulp is ~5e-4 cm; summed over ~150
// steps that shifts tan(lambda) by ~1e-4 relative.  Each lane therefore keeps
// the state's z relative to its start hit (zref); z_m - zref is exact in
// float32 for the hits of one track (Sterbenz), and zref is added back only
// when the result is stored.
#include <algorithm>

#include "device_common.h"

namespace tpc {
namespace {

constexpr int kThreads = 64;
// Row-synchronous schedule: two lanes per tracklet (the pair splits the
// candidate search and runs the rest of the step redundantly).
constexpr int kPair = 2;
constexpr int kTrkPerWave = kThreads / kPair;

__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }   // i >= j

// Arithmetic types of the Kalman state p and of its covariance C.  Both are
// accumulated in double: a track's covariance shrinks by up to seven orders
// of magnitude under strongly correlated updates (y, sin phi and q/pT move
// together), so a float32 recursion loses about 1e-2 of its relative
// precision, and a float32 state rounds every row's increment of sin phi and
// y into values hundreds of times larger, which shifts the fitted q/pT by
// more than 1e-4.  Everything evaluated per row step from the state (the
// increments, the Jacobian, the search window) stays in float32, where its
// rounding is relative to the step itself.
using par_t = double;
using cov_t = double;

__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float frsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fabs_(float x) { return fabsf(x); }
// double reciprocal: the float32 hardware estimate refined by one Newton step (relative error ~1e-14)
__device__ __forceinline__ double frcp(double x) {
  const double r = __builtin_amdgcn_rcpf(float(x));
  return r * (2.0 - x * r);
}
__device__ __forceinline__ double fabs_(double x) { return fabs(x); }

// native vector types: arrays of them stay in registers
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct Trk {
  par_t p[5];
  cov_t c[15];
};

// The state at the innermost hit of the inward pass, in the float32 the result is stored in.
struct Snap {
  float p[5];
  float c[15];
};
__device__ __forceinline__ Snap snap_of(const Trk& t) {
  Snap s;
#pragma unroll
  for (int q = 0; q < 5; ++q) s.p[q] = float(t.p[q]);
#pragma unroll
  for (int q = 0; q < 15; ++q) s.c[q] = float(t.c[q]);
  return s;
}

// Per-row constants used in the tracklet loop: x, half-width, y_lo, 1/(2Y).
struct RowK {
  float x, half_y, y_lo, inv_wy;
};

// asin(u)/u and d/du of it; |u| is below 0.02 for row-to-row steps.
__device__ __forceinline__ float asin_over(float u) {
  const float u2 = u * u;
  if (fabsf(u) < 0.05f) return 1.0f + u2 * (1.0f / 6.0f + u2 * (3.0f / 40.0f + u2 * (5.0f / 112.0f)));
  return asinf(u) / u;
}
__device__ __forceinline__ float asin_over_prime(float u) {
  const float u2 = u * u;
  if (fabsf(u) < 0.1f)
    return u * (1.0f / 3.0f + u2 * (3.0f / 10.0f + u2 * (15.0f / 56.0f + u2 * (35.0f / 144.0f))));
  return (u * frsqrt(1.0f - u2) - asinf(u)) / u2;
}
// Helix transport from x to x + dx with covariance; false on |sin phi| >= s_max or |u| >= 1.
// kNoExit: the failure tests do not branch (the row-synchronous waves, where a
// branch costs every lane); on false the state then holds meaningless values,
// and every caller stops the tracklet without reading it again.
//
// The increments of one row step (dy, dz, kappa*dx) and the Jacobian are
// evaluated in float32: their rounding is relative to the step, far below the
// tolerance.  They are accumulated into the state in par_t, and the covariance
// is transported in cov_t.
template <bool kNoExit>
__device__ __forceinline__ bool propagate(Trk& t, float dx, const KfConst& k) {
  using V = cov_t;
  const float s1 = float(t.p[2]), tl = float(t.p[3]), qp = float(t.p[4]);
  const float kap = k.bk * qp;
  const par_t s2p = t.p[2] + par_t(kap * dx);
  const float s2 = float(s2p);
  if (!kNoExit && !(fabsf(s1) < k.s_max)) return false;
  if (!kNoExit && !(fabsf(s2) < k.s_max)) return false;
  const float c1 = fsqrt((1.0f - s1) * (1.0f + s1));
  const float c2 = fsqrt((1.0f - s2) * (1.0f + s2));
  const float ic = frcp(c1 + c2);
  const float dy = dx * ((s1 + s2) * ic);
  const float L = fsqrt(dx * dx + dy * dy);
  const float u = 0.5f * kap * L;
  if (!kNoExit && !(fabsf(u) < 1.0f)) return false;
  const bool ok = fabsf(s1) < k.s_max && fabsf(s2) < k.s_max && fabsf(u) < 1.0f;
  const float sgn = dx >= 0.0f ? 1.0f : -1.0f;
  const float S = sgn * L * asin_over(u);
  // Jacobian entries (exact derivative of the map above)
  const float ic1 = frcp(c1), ic2 = frcp(c2);
  const float D = (1.0f + c1 * c2 + s1 * s2) * (ic * ic);
  const float ddy_ds1 = dx * D * (ic1 + ic2);
  const float ddy_dk = dx * dx * (D * ic2) * k.bk;
  const float dS_dL = sgn * frsqrt(1.0f - u * u);
  const float dS_dkap = sgn * 0.5f * L * L * asin_over_prime(u);
  const float dL_ddy = L > 0.0f ? dy * frcp(L) : 0.0f;
  const V A = ddy_ds1;                                  // F02
  const V B = ddy_dk;                                   // F04
  const V Cc = tl * dS_dL * dL_ddy * ddy_ds1;           // F12
  const V Dd = S;                                       // F13
  const V E = tl * (dS_dL * dL_ddy * ddy_dk + dS_dkap * k.bk);  // F14
  const V Fk = k.bk * dx;                               // F24
  t.p[0] += par_t(dy);
  t.p[1] += par_t(tl * S);
  t.p[2] = s2p;
  // C' = F C F^T with F = I + {02:A, 04:B, 12:Cc, 13:Dd, 14:E, 24:Fk}
  V* c = t.c;
  V M[5][5];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j) M[i][j] = i >= j ? c[tri(i, j)] : c[tri(j, i)];
  V G[5][5];   // G = F C
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    G[0][j] = M[0][j] + A * M[2][j] + B * M[4][j];
    G[1][j] = M[1][j] + Cc * M[2][j] + Dd * M[3][j] + E * M[4][j];
    G[2][j] = M[2][j] + Fk * M[4][j];
    G[3][j] = M[3][j];
    G[4][j] = M[4][j];
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) {   // C'_ij = sum_k G_ik F_jk
    const V g0 = G[i][0], g1 = G[i][1], g2 = G[i][2], g3 = G[i][3], g4 = G[i][4];
    const V r0 = g0 + A * g2 + B * g4;
    const V r1 = g1 + Cc * g2 + Dd * g3 + E * g4;
    const V r2 = g2 + Fk * g4;
    const V rr[5] = {r0, r1, r2, g3, g4};
#pragma unroll
    for (int j = 0; j <= i; ++j) c[tri(i, j)] = rr[j];
  }
  return ok;
}

// Kalman update with a measurement of (y, z).  The covariance update is the
// plain C' = C - K H C: in double it keeps far more precision than the
// parameters need (the Joseph form, which guards the positive definiteness of
// a float32 recursion, costs 40 more double operations per step).  Each
// element takes two fused multiply-adds (the sum of the two products and its
// subtraction would be three operations).
__device__ __forceinline__ void update(Trk& t, float ym, float zm, const KfConst& k, float& chi2) {
  using P = par_t;
  using V = cov_t;
  V* c = t.c;
  const V vy = k.vy, vz = k.vz;
  const V r0 = V(P(ym) - t.p[0]), r1 = V(P(zm) - t.p[1]);
  const V S00 = c[0] + vy, S01 = c[1], S11 = c[2] + vz;
  const V id = frcp(S00 * S11 - S01 * S01);
  const V I00 = S11 * id, I01 = -S01 * id, I11 = S00 * id;
  V c0[5], c1[5];   // columns 0 and 1 of C (C_i0, C_i1)
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    c0[i] = c[tri(i, 0)];
    c1[i] = i >= 1 ? c[tri(i, 1)] : c[tri(1, 0)];
  }
  V K0[5], K1[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    K0[i] = c0[i] * I00 + c1[i] * I01;
    K1[i] = c0[i] * I01 + c1[i] * I11;
    t.p[i] = fma(K0[i], r0, fma(K1[i], r1, t.p[i]));
  }
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) c[tri(i, j)] = fma(-K0[i], c0[j], fma(-K1[i], c1[j], c[tri(i, j)]));
  chi2 += float(r0 * (I00 * r0 + I01 * r1) + r1 * (I01 * r0 + I11 * r1));
}

__device__ __forceinline__ void set_c0(Trk& t, const KfConst& k) {
#pragma unroll
  for (int i = 0; i < 15; ++i) t.c[i] = cov_t(0);
  t.c[tri(0, 0)] = k.vy;
  t.c[tri(1, 1)] = k.vz;
  t.c[tri(2, 2)] = k.c0_sinphi;
  t.c[tri(3, 3)] = k.c0_tanl;
  t.c[tri(4, 4)] = k.c0_qpt;
}

// Grid search in row sr for the candidate closest to the prediction; -1 if
// none, else its position, with its (y, z) in hv.  z-lines are walked as one
// flat sequence of candidate groups per lane (see search_lds); the kGroup loads
// of a group are issued together.
constexpr int kGroup = 6;   // measured on the 32-orbit frame: 4 -> 6 is -3.7% in K5, 8 and above slower
constexpr int kGroupLds = 4;   // candidates per group of the LDS search

__device__ __forceinline__ int32_t search_m(const DevPtrs& d, uint2 meta, const RowK& rk, const SectorConst& sc,
                                            const Trk& t, const KfConst& k, float zref, float2& hv) {
  const float sy2 = float(t.c[0] + cov_t(k.vy)), sz2 = float(t.c[2] + cov_t(k.vz));
  const float wy = fminf(k.gate * fsqrt(sy2), k.cap), wz = fminf(k.gate * fsqrt(sz2), k.cap);
  const float isy = frcp(sy2), isz = frcp(sz2);
  const float yp = float(t.p[0]), zp = float(t.p[1]);          // zp relative to zref
  const float za = zref + zp;                     // absolute, for the bin range only
  const int ny = (int)(meta.y & 0xFFFFu), nz = (int)(meta.y >> 16);
  const int iy0 = bin1((yp - wy) - kWinPad, rk.y_lo, rk.inv_wy, ny);
  const int iy1 = bin1((yp + wy) + kWinPad, rk.y_lo, rk.inv_wy, ny);
  const int iz0 = bin1((za - wz) - kWinPad, sc.z_lo, sc.inv_wz, nz);
  const int iz1 = bin1((za + wz) + kWinPad, sc.z_lo, sc.inv_wz, nz);
  const uint32_t* bs = d.bin_start + meta.x;
  int32_t best = -1;
  float bd = 0.0f;
  int iz = iz0;
  uint32_t q = bs[iz * ny + iy0], hi = bs[iz * ny + iy1 + 1];
  for (;;) {
    while (q >= hi && iz < iz1) {
      ++iz;
      q = bs[iz * ny + iy0];
      hi = bs[iz * ny + iy1 + 1];
    }
    if (q >= hi) break;
    float2 h[kGroup];
#pragma unroll
    for (int j = 0; j < kGroup; ++j) h[j] = d.syz[min(q + j, hi - 1)];
#pragma unroll
    for (int j = 0; j < kGroup; ++j) {
      const float dy = h[j].x - yp, dz = (h[j].y - zref) - zp;
      if (q + j < hi && fabsf(dy) <= wy && fabsf(dz) <= wz) {
        const float dd = dy * dy * isy + dz * dz * isz;
        if (best < 0 || dd < bd) {
          best = (int32_t)(q + j);
          bd = dd;
          hv = h[j];
        }
      }
    }
    q += kGroup;
  }
  return best;
}

__device__ __forceinline__ int32_t search(const DevPtrs& d, uint32_t sr, const RowK& rk, const SectorConst& sc,
                                          const Trk& t, const KfConst& k, float zref, float2& hv) {
  return search_m(d, d.row_meta[sr], rk, sc, t, k, zref, hv);
}

// The same search over a row staged in LDS: (y, z) of the row's hits at
// yz[q - first] and its bin starts (global positions) in bs[].  It is run by the
// two lanes of a pair that carry the same tracklet: on every z-line they take
// alternate groups of kGroupLds candidates, walking the z-lines as one flat
// sequence, and then exchange their best candidates (a DPP swap inside the
// pair, no LDS round trip).  A group is read whole: its entries past the
// z-line's end (at most kGroupLds - 1, inside the stage's slack) are masked out.
// The result -- smallest deviation, ties to the smaller position -- is the same
// as a single ascending scan.
__device__ __forceinline__ int pair_swap(int v) {   // value of the other lane of the pair (quad_perm 1,0,3,2)
  return __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false);
}
__device__ __forceinline__ int32_t search_lds(const float2* yz, const uint32_t* bs, uint32_t first, uint2 meta,
                                              const RowK& rk, const SectorConst& sc, const Trk& t, const KfConst& k,
                                              float zref, uint32_t half) {
  const float sy2 = float(t.c[0] + cov_t(k.vy)), sz2 = float(t.c[2] + cov_t(k.vz));
  const float wy = fminf(k.gate * fsqrt(sy2), k.cap), wz = fminf(k.gate * fsqrt(sz2), k.cap);
  const float isy = frcp(sy2), isz = frcp(sz2);
  const float yp = float(t.p[0]), zp = float(t.p[1]);
  const float za = zref + zp;
  const int ny = (int)(meta.y & 0xFFFFu), nz = (int)(meta.y >> 16);
  const int iy0 = bin1((yp - wy) - kWinPad, rk.y_lo, rk.inv_wy, ny);
  const int iy1 = bin1((yp + wy) + kWinPad, rk.y_lo, rk.inv_wy, ny);
  const int iz0 = bin1((za - wz) - kWinPad, sc.z_lo, sc.inv_wz, nz);
  const int iz1 = bin1((za + wz) + kWinPad, sc.z_lo, sc.inv_wz, nz);
  int32_t best = -1;
  float bd = 0.0f;
  // z-lines are taken two at a time (a window almost never spans more): the
  // candidates of the pair of lines form one flat sequence -- line iz, then
  // line iz + 1, so positions ascend -- and the two lanes of a pair take
  // alternate groups of it
  for (int iz = iz0; iz <= iz1; iz += 2) {
    const int izb = iz + 1 <= iz1 ? iz + 1 : iz;
    const uint32_t lo0 = bs[iz * ny + iy0], hi0 = bs[iz * ny + iy1 + 1];
    const uint32_t lo1 = bs[izb * ny + iy0], hi1 = bs[izb * ny + iy1 + 1];
    const uint32_t n0 = hi0 - lo0, tot = n0 + (izb > iz ? hi1 - lo1 : 0u);
    for (uint32_t g0 = half * kGroupLds; g0 < tot; g0 += kPair * kGroupLds) {
      uint32_t pos[kGroupLds];
      float2 h[kGroupLds];
#pragma unroll
      for (int j = 0; j < kGroupLds; ++j) {
        const uint32_t f = g0 + j;   // past the end: at most kGroupLds - 1 entries beyond a line, masked below
        pos[j] = f < n0 ? lo0 + f : lo1 + (f - n0);
        h[j] = yz[pos[j] - first];
      }
#pragma unroll
      for (int j = 0; j < kGroupLds; ++j) {
        const float dy = h[j].x - yp, dz = (h[j].y - zref) - zp;
        if (g0 + j < tot && fabsf(dy) <= wy && fabsf(dz) <= wz) {
          const float dd = dy * dy * isy + dz * dz * isz;
          if (best < 0 || dd < bd) {
            best = (int32_t)pos[j];
            bd = dd;
          }
        }
      }
    }
  }
  // the pair's two candidates: smaller deviation, ties to the smaller position
  const int32_t ob = pair_swap(best);
  const float od = __int_as_float(pair_swap(__float_as_int(bd)));
  if (ob >= 0 && (best < 0 || od < bd || (od == bd && ob < best))) {
    best = ob;
    bd = od;
  }
  return best;
}

// Three-point seed; false on failure.
__device__ __forceinline__ bool seed3(float x0, float2 h0, float xm, float2 hm, float xl, float2 hl, const KfConst& k,
                                      Trk& t) {
  const float ax = xm - x0, ay = hm.x - h0.x, bx = xl - xm, by = hl.x - hm.x, cx = xl - x0, cy = hl.x - h0.x;
  const float cross = ax * by - ay * bx;
  const float la = sqrtf(ax * ax + ay * ay), lb = sqrtf(bx * bx + by * by), lc = sqrtf(cx * cx + cy * cy);
  if (!(la > 0.0f && lb > 0.0f && lc > 0.0f)) return false;
  const float kap = 2.0f * cross / (la * lb * lc);
  const float u = 0.5f * kap * lc;
  if (!(fabsf(u) < 1.0f)) return false;
  const float phi0 = atan2f(cy, cx) - asinf(u);
  const float s0l = lc * asin_over(u);
  float qpt = k.bk != 0.0f ? kap / k.bk : 0.0f;
  qpt = fminf(k.qpt_max, fmaxf(-k.qpt_max, qpt));
  float sp, cp;
  sincosf(phi0, &sp, &cp);
  t.p[0] = h0.x;
  t.p[1] = 0.0f;             // z relative to the start hit
  t.p[2] = sp;
  t.p[3] = (hl.y - h0.y) / s0l;
  t.p[4] = qpt;
  return cp > 0.0f && fabsf(sp) < k.s_max;
}

__device__ __forceinline__ void load_rows(const DevPtrs& d, RowK* lrows) {
  for (uint32_t r = threadIdx.x; r < d.R; r += blockDim.x) {
    const RowConst rc = d.rows[r];
    lrows[r] = RowK{rc.x, rc.half_y, rc.y_lo, rc.inv_wy};
  }
  __syncthreads();
}

// SPD guard for the stored covariance.  Near-singular fits (a short, strongly
// curved arc can correlate sin phi and q/pT at 0.99) sit within float32
// rounding of the positive-definite boundary; LDL^T with every pivot floored
// at kPivotFloor * C_kk returns them to a nearby positive-definite matrix and
// leaves every other covariance untouched (no rebuild when no pivot is low).
constexpr float kPivotFloor = 1e-5f;

__device__ __forceinline__ void spd_guard(float* c) {
  float L[5][5], D[5];
  bool fixed = false;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    float dk = c[tri(k, k)];
#pragma unroll
    for (int j = 0; j < k; ++j) dk -= L[k][j] * L[k][j] * D[j];
    const float floor_k = kPivotFloor * c[tri(k, k)];
    if (!(dk > floor_k)) {
      dk = floor_k;
      fixed = true;
    }
    D[k] = dk;
    const float idk = 1.0f / dk;
#pragma unroll
    for (int i = k + 1; i < 5; ++i) {
      float v = c[tri(i, k)];
#pragma unroll
      for (int j = 0; j < k; ++j) v -= L[i][j] * L[k][j] * D[j];
      L[i][k] = v * idk;
    }
  }
  if (!fixed) return;
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      float v = (i == j ? 1.0f : L[i][j]) * D[j];
#pragma unroll
      for (int q = 0; q < j; ++q) v += L[i][q] * L[j][q] * D[q];
      c[tri(i, j)] = v;
    }
}

template <bool kGuard>
__device__ __forceinline__ void store_tracklet(const DevPtrs& d, uint32_t i, int nh, uint32_t rin, uint32_t rout,
                                               uint32_t r0, const Snap& snap, float chi2, float zref) {
  const uint32_t T = d.tcap;
  d.tk_info[i] = nh;
  d.tk_info[T + i] = (int32_t)rin;
  d.tk_info[2 * T + i] = (int32_t)rout;
  d.tk_info[3 * T + i] = (int32_t)r0;
#pragma unroll
  for (int q = 0; q < 5; ++q) d.tk_param[(size_t)q * T + i] = q == 1 ? snap.p[q] + zref : snap.p[q];
  float c[15];
#pragma unroll
  for (int q = 0; q < 15; ++q) c[q] = snap.c[q];
  if (kGuard) spd_guard(c);
#pragma unroll
  for (int q = 0; q < 15; ++q) d.tk_cov[(size_t)q * T + i] = c[q];
  d.tk_chi2[i] = chi2;
}

// The covariance guard over every stored tracklet, one lane each (for k_down,
// whose lanes store as they finish: there the guard would cost the whole wave
// once for every group of lanes that finish together).  When the refit ran in
// bucket order its results wait in slot order (one contiguous record per
// tracklet, see kRec*), so that the refit's lanes write whole lines; the
// guard gathers each tracklet's record through the bucket slot of tracklet i
// and writes the result arrays in tracklet order.
enum : int { kRecInfo = 0, kRecParam = 4, kRecCov = 9, kRecChi2 = 24, kRecWords = 25 };

__global__ void __launch_bounds__(256) k_guard(DevPtrs d) {
  const uint32_t nt = min(d.hdr->n_starts, d.tcap), T = d.tcap;
  const bool staged = d.k5_refit_order == 0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nt; i += gridDim.x * blockDim.x) {
    if (staged) {
      if (d.tk_info[i] < 0) continue;   // no seed, or the chain fit failed: no refit record
      const uint32_t* rec = d.k5_rec + (size_t)d.k5_inv[i] * kRecWords;
      uint32_t w[kRecWords];
#pragma unroll
      for (int q = 0; q < kRecWords; ++q) w[q] = rec[q];
#pragma unroll
      for (int q = 0; q < 4; ++q) d.tk_info[(size_t)q * T + i] = (int32_t)w[kRecInfo + q];
#pragma unroll
      for (int q = 0; q < 5; ++q) d.tk_param[(size_t)q * T + i] = __int_as_float((int)w[kRecParam + q]);
      float c[15];
#pragma unroll
      for (int q = 0; q < 15; ++q) c[q] = __int_as_float((int)w[kRecCov + q]);
      spd_guard(c);
#pragma unroll
      for (int q = 0; q < 15; ++q) d.tk_cov[(size_t)q * T + i] = c[q];
      d.tk_chi2[i] = __int_as_float((int)w[kRecChi2]);
    } else {
      if (d.tk_info[i] < 1) continue;
      float c[15];
#pragma unroll
      for (int q = 0; q < 15; ++q) c[q] = d.tk_cov[(size_t)q * T + i];
      spd_guard(c);
#pragma unroll
      for (int q = 0; q < 15; ++q) d.tk_cov[(size_t)q * T + i] = c[q];
    }
  }
}

// ---------------------------------------------------------------------------
// Lane-per-tracklet schedule: k_seed, k_up, k_sort, k_down, k_guard.
//
// A wave steps as long as its longest lane.  With one loop per pass (chain
// fit, outward extension, inward refit) a wave steps through its longest
// chain fit, then its longest extension, then its longest refit, and on a
// 32-orbit frame only about 56% of the lane steps do work.  Here the chain
// fit and the outward extension run as one loop (both move outward one row
// per step, so the lanes of a wave, which hold consecutive tracklets of one
// sector and start rows close together, stay on the same rows), and the
// inward refits are regrouped by (sector, outermost row) before they run: a
// wave's lanes then start the refit on the same row and walk the same rows in
// step, and most of them stop within a few rows of each other.
//
// k_seed: one lane per tracklet walks its chain (dependent up1 gathers that
// fill the chain's rows of the row -> hit column) and builds the three-point
// seed.  It leaves the seed in tk_param, the chain's last row in
// tk_info[2T + i] and 0 (seeded) or -1 (no seed) in tk_info[i].
// k_up: chain fit and outward extension, one lane per tracklet; it hands the
// refit its start (below) and counts the tracklet in its (sector, outermost
// row) bucket.
// k_sort: bucket offsets (an exclusive scan) and a scatter of the tracklet
// indices into bucket order (the order inside a bucket does not matter: every
// tracklet's refit is independent of the others).
// k_down: the inward refit, one lane per tracklet in bucket order; stores the
// tracklet.
// k_guard: the covariance guard over every stored tracklet.
//
// Workgroups are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8),
// each with its own L2.  Tracklets (and buckets) are ordered by sector, so each
// XCD is given one contiguous eighth of them: its lanes then search the row
// grids of a few sectors only, which stay resident in that XCD's L2.
__global__ void __launch_bounds__(kThreads) k_seed(DevPtrs d, KfConst k) {
  __shared__ float lx[kMaxRows];
  const uint32_t nt = min(d.hdr->n_starts, d.tcap);
  const uint32_t R = d.R, T = d.tcap;
  // the bucket counts of k_up start at zero (the C4 row counts are not used after C4)
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < d.SR; q += gridDim.x * blockDim.x) d.row_nstart[q] = 0;
  const XcdSched sch = xcd_sched(nt);
  if (sch.first >= sch.end) return;   // the grid is sized for the tracklet capacity
  for (uint32_t r = threadIdx.x; r < R; r += blockDim.x) lx[r] = d.rows[r].x;
  __syncthreads();
  for (uint32_t vb = sch.first; vb < sch.end; vb += sch.stride) {
    const uint32_t i = vb * kThreads + threadIdx.x;
    if (i >= nt) continue;
    const uint32_t r0 = d.start_sr[i] % R;
    int32_t* H = d.tk_rowhit + i;     // row r at H[r * T]
    const int32_t p0 = (int32_t)d.start_pos[i];
    int32_t p = p0, plast = p0;
    uint32_t n = 0;
    while (p >= 0 && r0 + n < R) {   // links step one row outward, so a chain ends before row R
      H[(size_t)(r0 + n) * T] = p;
      plast = p;
      ++n;
      p = d.up1[p];
    }
    const uint32_t m = (n - 1) / 2, rl = r0 + n - 1;
    const int32_t pm = H[(size_t)(r0 + m) * T];
    Trk t;
    const bool ok = seed3(lx[r0], d.syz[p0], lx[r0 + m], d.syz[pm], lx[rl], d.syz[plast], k, t);
    if (ok) {
#pragma unroll
      for (int q = 0; q < 5; ++q) d.tk_param[(size_t)q * T + i] = float(t.p[q]);   // seed3 works in float32
    }
    d.tk_info[2 * T + i] = (int32_t)rl;
    d.tk_info[i] = ok ? 0 : -1;
  }
}

// atomicAdd(&ctr[key], 1) for every lane with `on`, one atomic per distinct
// key in the wave (many tracklets share a bucket, and the atomics of one
// address serialize); returns the lane's slot (the counter before its add).
// Called by all lanes of the wave.
__device__ __forceinline__ uint32_t wave_claim(uint32_t* ctr, uint32_t key, bool on) {
  const uint32_t lane = threadIdx.x % kWave;
  uint32_t slot = 0;
  unsigned long long todo = __ballot(on);
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const uint32_t lk = (uint32_t)__shfl((int)key, leader, kWave);
    const unsigned long long grp = __ballot(on && key == lk) & todo;
    uint32_t base = 0;
    if ((int)lane == leader) base = atomicAdd(&ctr[lk], (uint32_t)__popcll(grp));
    base = (uint32_t)__shfl((int)base, leader, kWave);
    if ((grp >> lane) & 1ull) slot = base + (uint32_t)__popcll(grp & ((1ull << lane) - 1ull));
    todo &= ~grp;
  }
  return slot;
}

// Hand-off from k_up to k_down, per tracklet i, in the rows of tk_cov (free
// until the tracklet is stored, by the lane that has read its hand-off), as
// 32-bit words at word w * T + i: 0-5 sin phi, tan lambda and q/pT at the
// outermost hit (double, low word first), 6-7 that hit's (y, z), 8 the
// outermost row, 9 the start row r0, 10 z_ref, 11 the sector.
enum : int { kHoPout = 0, kHoHit = 6, kHoRout = 8, kHoR0 = 9, kHoZref = 10, kHoSec = 11 };

__device__ __forceinline__ void put_word(const DevPtrs& d, int w, uint32_t i, uint32_t v) {
  reinterpret_cast<uint32_t*>(d.tk_cov)[(size_t)w * d.tcap + i] = v;
}
__device__ __forceinline__ uint32_t get_word(const DevPtrs& d, int w, uint32_t i) {
  return reinterpret_cast<const uint32_t*>(d.tk_cov)[(size_t)w * d.tcap + i];
}

__device__ __forceinline__ void set_priority(uint32_t rows_left, uint32_t& level) {
  const uint32_t want = (rows_left >= 75) + (rows_left >= 150) + (rows_left >= 225);
  if (want == level) return;
  level = want;
  if (want == 3) __builtin_amdgcn_s_setprio(3);
  else if (want == 2) __builtin_amdgcn_s_setprio(2);
  else if (want == 1) __builtin_amdgcn_s_setprio(1);
  else __builtin_amdgcn_s_setprio(0);
}

// Chain fit and outward extension of tracklet i (seeded); false if the chain
// fit fails, else the hand-off is written and key is its refit bucket.
__device__ __forceinline__ bool up_one(const DevPtrs& d, const KfConst& k, const RowK* lrows, uint32_t i,
                                       uint32_t& key, uint32_t& steps, uint32_t& prio) {
  const uint32_t R = d.R, T = d.tcap;
  const uint32_t sr0 = d.start_sr[i];
  const uint32_t sec = sr0 / R, srb = sec * R, r0 = sr0 - srb;
  const SectorConst sc = d.secs[sec];
  const uint32_t rl = (uint32_t)d.tk_info[2 * T + i];
  int32_t* H = d.tk_rowhit + i;     // row r at H[r * T]
  float2 ho = d.syz[d.start_pos[i]];   // the outermost hit so far
  const float zref = ho.y;
  Trk t;
#pragma unroll
  for (int q = 0; q < 5; ++q) t.p[q] = par_t(d.tk_param[(size_t)q * T + i]);
  set_c0(t, k);
  float chi2 = 0.0f, xprev = lrows[r0].x;
  par_t pout[3] = {t.p[2], t.p[3], t.p[4]};
  uint32_t rout = rl;
  int miss = 0;
  bool failed = false;
  // chain fit and outward extension, one row per iteration; while a row is
  // stepped, the chain hits' coordinates are loaded two rows ahead (their
  // indices three) and the next row's grid word one row ahead
  const int32_t hk1 = r0 + 1 <= rl ? H[(size_t)(r0 + 1) * T] : -1;
  float2 hnx = hk1 >= 0 ? d.syz[hk1] : make_float2(0.0f, 0.0f);
  int32_t hk2 = r0 + 2 <= rl ? H[(size_t)(r0 + 2) * T] : -1;
  float2 hn2 = hk2 >= 0 ? d.syz[hk2] : make_float2(0.0f, 0.0f);
  int32_t hk3 = r0 + 3 <= rl ? H[(size_t)(r0 + 3) * T] : -1;
  uint2 mnx = r0 + 1 < R && r0 + 1 > rl ? d.row_meta[srb + r0 + 1] : make_uint2(0u, 0u);
  for (uint32_t r = r0 + 1; r < R; ++r) {
    // issue priority by the rows still ahead (outward, then about as many inward): a wave far from its
    // end goes first, so fewer waves are left running alone at the end (-1.6% on the 32-orbit frame)
    set_priority(2 * (R - __builtin_amdgcn_readfirstlane(r)), prio);
    const bool chain = r <= rl;
    const float2 hc = hnx;
    const uint2 meta = mnx;
    hnx = hn2;
    hn2 = hk3 >= 0 ? d.syz[hk3] : make_float2(0.0f, 0.0f);
    hk3 = r + 3 <= rl ? H[(size_t)(r + 3) * T] : -1;
    if (r + 1 < R && r + 1 > rl) mnx = d.row_meta[srb + r + 1];
    ++steps;
    const RowK rk = lrows[r];
    const bool pok = propagate<true>(t, rk.x - xprev, k);
    xprev = rk.x;
    if (chain && !pok) {
      failed = true;
      break;
    }
    if (!chain && (!pok || fabs_(t.p[0]) > rk.half_y + k.margin)) break;
    int32_t h = 0;   // chain rows hold a hit
    float2 hm = hc;
    if (!chain) {
      h = search_m(d, meta, rk, sc, t, k, zref, hm);
      H[(size_t)r * T] = h;
    }
    if (h >= 0) {
      update(t, hm.x, hm.y - zref, k, chi2);
      if (r >= rl) {
        pout[0] = t.p[2];
        pout[1] = t.p[3];
        pout[2] = t.p[4];
        rout = r;
        ho = hm;
        miss = 0;
      }
    } else if (++miss > k.max_miss) {
      break;
    }
  }
  if (failed) {
    d.tk_info[i] = -2;   // the chain fit failed: no tracklet
    return false;
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(pout[q]);
    put_word(d, kHoPout + 2 * q, i, (uint32_t)b);
    put_word(d, kHoPout + 2 * q + 1, i, (uint32_t)(b >> 32));
  }
  put_word(d, kHoHit, i, (uint32_t)__float_as_int(ho.x));
  put_word(d, kHoHit + 1, i, (uint32_t)__float_as_int(ho.y));
  put_word(d, kHoRout, i, rout);
  put_word(d, kHoR0, i, r0);
  put_word(d, kHoZref, i, (uint32_t)__float_as_int(zref));
  put_word(d, kHoSec, i, sec);
  key = srb + rout;
  return true;
}

__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) k_up(DevPtrs d, KfConst k) {
  __shared__ RowK lrows[kMaxRows];
  const uint32_t nt = min(d.hdr->n_starts, d.tcap);
  const XcdSched sch = xcd_sched(nt);
  if (sch.first >= sch.end) return;   // the grid is sized for the tracklet capacity
  load_rows(d, lrows);
  uint32_t steps = 0, prio = 0;
  for (uint32_t vb = sch.first; vb < sch.end; vb += sch.stride) {
    const uint32_t i = vb * kThreads + threadIdx.x;
    bool on = i < nt && d.tk_info[i] >= 0;
    uint32_t key = 0;
    if (on) on = up_one(d, k, lrows, i, key, steps, prio);
    (void)wave_claim(d.row_nstart, key, on);   // count the tracklet in its refit bucket
  }
  uint32_t sum = steps;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) sum += (uint32_t)__shfl_xor((int)sum, off, kWave);
  if (threadIdx.x == 0 && sum) atomicAdd(&d.hdr->n_steps, (unsigned long long)sum);
}

// Scatter of the refit tracklets into (sector, outermost row) order; k5_off
// holds the exclusive scan of the bucket counts (total at [SR]) and serves as
// the buckets' fill cursors.
__global__ void __launch_bounds__(256) k_sort(DevPtrs d) {
  const uint32_t nt = min(d.hdr->n_starts, d.tcap), R = d.R;
  for (uint32_t b = blockIdx.x * blockDim.x; b < nt; b += gridDim.x * blockDim.x) {   // wave-uniform bounds
    const uint32_t i = b + threadIdx.x;
    const bool on = i < nt && d.tk_info[i] >= 0;
    const uint32_t key = on ? get_word(d, kHoSec, i) * R + get_word(d, kHoRout, i) : 0u;
    const uint32_t slot = wave_claim(d.k5_off, key, on);
    if (on) {
      d.k5_perm[slot] = i;
      d.k5_inv[i] = slot;
    }
  }
}

__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) k_down(DevPtrs d, KfConst k) {
  __shared__ RowK lrows[kMaxRows];
  // the state at each lane's innermost hit so far, in the float32 it is stored
  // in (in LDS rather than registers: four waves per SIMD instead of three)
  __shared__ f32x4 snap_s[5][kThreads];
  const uint32_t lane = threadIdx.x;
  auto save = [&](const Trk& t) {
    const Snap v = snap_of(t);
    snap_s[0][lane] = f32x4{v.p[0], v.p[1], v.p[2], v.p[3]};
#pragma unroll
    for (int q = 0; q < 4; ++q) snap_s[1 + q][lane] = f32x4{q == 0 ? v.p[4] : v.c[4 * q - 1], v.c[4 * q], v.c[4 * q + 1], v.c[4 * q + 2]};
  };
  // bucket order: the refit tracklets (the scan total; the scatter moves only
  // [0, SR)); tracklet order: every tracklet, those without a hand-off skipped
  const bool sorted = d.k5_refit_order == 0;
  const uint32_t nv = sorted ? d.k5_off[d.SR] : min(d.hdr->n_starts, d.tcap);
  const uint32_t R = d.R, T = d.tcap;
  const XcdSched sch = xcd_sched(nv);
  if (sch.first >= sch.end) return;   // the grid is sized for the tracklet capacity
  load_rows(d, lrows);
  uint32_t steps = 0, prio = 0;
  for (uint32_t vb = sch.first; vb < sch.end; vb += sch.stride) {
    const uint32_t j = vb * kThreads + threadIdx.x;
    if (j >= nv || (!sorted && d.tk_info[j] < 0)) continue;
    const uint32_t i = sorted ? d.k5_perm[j] : j;
    Trk t;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const unsigned long long b = (unsigned long long)get_word(d, kHoPout + 2 * q, i) |
                                   ((unsigned long long)get_word(d, kHoPout + 2 * q + 1, i) << 32);
      t.p[2 + q] = __longlong_as_double((long long)b);
    }
    const float hy = __int_as_float((int)get_word(d, kHoHit, i)), hz = __int_as_float((int)get_word(d, kHoHit + 1, i));
    const uint32_t rout = get_word(d, kHoRout, i), r0 = get_word(d, kHoR0, i);
    const float zref = __int_as_float((int)get_word(d, kHoZref, i));
    const uint32_t sec = get_word(d, kHoSec, i), srb = sec * R;
    const SectorConst sc = d.secs[sec];
    int32_t* H = d.tk_rowhit + i;     // row r at H[r * T]
    // inward refit from the outermost hit, fresh covariance
    t.p[0] = hy;
    t.p[1] = hz - zref;
    set_c0(t, k);
    float chi2 = 0.0f;
    int nh = 1;
    save(t);
    uint32_t rin = rout;
    float xprev = lrows[rout].x;
    int miss = 0;
    // the outward pass's row -> hit entries are loaded three rows ahead and
    // their coordinates two rows ahead, the next row's grid word one row ahead
    auto known = [&](int r) { return r >= (int)r0 && r >= 0 ? H[(size_t)r * T] : -1; };
    int32_t hA = known((int)rout - 1), hB = known((int)rout - 2), hC = known((int)rout - 3);
    float2 vA = hA >= 0 ? d.syz[hA] : make_float2(0.0f, 0.0f);
    float2 vB = hB >= 0 ? d.syz[hB] : make_float2(0.0f, 0.0f);
    uint2 mA = rout >= 1 ? d.row_meta[srb + rout - 1] : make_uint2(0u, 0u);
    for (int r = (int)rout - 1; r >= 0; --r) {
      set_priority(2 * (uint32_t)__builtin_amdgcn_readfirstlane(r), prio);
      const int32_t hk = hA;
      const float2 vk = vA;
      const uint2 meta = mA;
      hA = hB;
      vA = vB;
      hB = hC;
      vB = hC >= 0 ? d.syz[hC] : make_float2(0.0f, 0.0f);
      hC = known(r - 3);
      if (r >= 1) mA = d.row_meta[srb + (uint32_t)r - 1];
      const RowK rk = lrows[r];
      ++steps;
      if (!propagate<true>(t, rk.x - xprev, k)) break;
      xprev = rk.x;
      const bool below = (uint32_t)r < r0;
      if (below && fabs_(t.p[0]) > rk.half_y + k.margin) break;
      int32_t h = hk;
      float2 hm = vk;
      if (h < 0) h = search_m(d, meta, rk, sc, t, k, zref, hm);
      // the row's entry changes only where the refit searched: below the start
      // row (never written before) or in a gap the outward pass left
      if (below || h != hk) H[(size_t)r * T] = h;
      if (h >= 0) {
        update(t, hm.x, hm.y - zref, k, chi2);
        ++nh;
        save(t);
        rin = (uint32_t)r;
        if (below) miss = 0;
      } else if (below && ++miss > k.max_miss) {
        break;
      }
    }
    Snap snap;
    const f32x4 w0 = snap_s[0][lane];
    snap.p[0] = w0.x;
    snap.p[1] = w0.y;
    snap.p[2] = w0.z;
    snap.p[3] = w0.w;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const f32x4 w = snap_s[1 + q][lane];
      if (q == 0) snap.p[4] = w.x;
      else snap.c[4 * q - 1] = w.x;
      snap.c[4 * q] = w.y;
      snap.c[4 * q + 1] = w.z;
      snap.c[4 * q + 2] = w.w;
    }
    if (sorted) {   // the record at the tracklet's bucket slot: consecutive lanes, consecutive records
      uint32_t* rec = d.k5_rec + (size_t)j * kRecWords;
      rec[kRecInfo] = (uint32_t)nh;
      rec[kRecInfo + 1] = rin;
      rec[kRecInfo + 2] = rout;
      rec[kRecInfo + 3] = r0;
#pragma unroll
      for (int q = 0; q < 5; ++q) rec[kRecParam + q] = (uint32_t)__float_as_int(q == 1 ? snap.p[q] + zref : snap.p[q]);
#pragma unroll
      for (int q = 0; q < 15; ++q) rec[kRecCov + q] = (uint32_t)__float_as_int(snap.c[q]);
      rec[kRecChi2] = (uint32_t)__float_as_int(chi2);
    } else {
      store_tracklet<false>(d, i, nh, rin, rout, r0, snap, chi2, zref);
    }
  }
  uint32_t sum = steps;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) sum += (uint32_t)__shfl_xor((int)sum, off, kWave);
  if (threadIdx.x == 0 && sum) atomicAdd(&d.hdr->n_steps, (unsigned long long)sum);
}

// ---------------------------------------------------------------------------
// Row-synchronous schedule ("coalesced row-grid reads").  A wave takes up to
// 32 tracklets of ONE sector, two lanes per tracklet: the pair splits each
// candidate search and runs the rest of the step redundantly, which shortens
// the wave's per-row instruction stream (the longest waves' instruction issue
// bounds this kernel: a central event's waves are all resident, 2-3 per SIMD,
// and the SIMD favours those with the most rows still to step through).  After
// each pair has walked its chain and built its seed, the wave sweeps the rows
// in lockstep -- outward, then inward --
// and at every row stages that row's (y, z) and bin starts in LDS with one
// coalesced load shared by all lanes; the loads for the next row are issued
// before the current row's Kalman step and land in registers while it runs.
// Every search and every measurement read then hits LDS, which takes the
// dependent global-memory round trips out of the per-row critical path.  Rows
// larger than the stage fall back to global-memory search for that row.
//
// The stage is filled with 16-byte loads that every lane issues
// unconditionally: the (y, z) pairs from the even index at or below the row's
// first hit, the bin starts from the multiple of four at or below the row's
// first bin (both arrays carry padding at their ends, so reads past a row stay
// inside the allocation).  A load whose slot lies past the row re-reads the
// first one; the stage entries it fills are never used.
constexpr int kStageHits = 320;
constexpr int kStageBins = kStageHits + 2;                       // nBins + 1 <= N_r + 1
constexpr int kPreYz = 3;   // float4 loads per lane: 2 hits each
constexpr int kPreBs = 2;   // uint4 loads per lane: 4 bin starts each
// alignment slack (1), whole-group reads past a z-line (kGroupLds - 1)
static_assert(kPreYz * kThreads * 2 >= kStageHits + 1 + kGroupLds - 1, "yz stage too small");
static_assert(kPreBs * kThreads * 4 >= kStageBins + 3, "bin stage too small");

struct Stage {
  uint32_t first;   // global index of stage entry 0 (even, <= the row's first hit)
  uint32_t boff;    // stage index of the row's bin 0
  uint2 meta;
  RowK rk;
  bool fits;
};


struct Prefetch {
  f32x4 yz[kPreYz];
  u32x4 bs[kPreBs];
  Stage st;
};

__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, off, kWave));
  return v;
}
__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off, kWave));
  return v;
}

// Issue the loads of sector row r (wave-uniform) into registers.  The row's
// offsets and grid word come from the wave's LDS copy of the sector's row
// table, so no load here waits on another; only the 64-entry chunks the row
// needs are loaded (a scalar decision), each lane from an index clamped into
// the row, so the loads need no per-lane predication.
// Issue priority of a wave from the rows it still has to step through (a
// longest-remaining-first order for the waves that share a SIMD); `level`
// holds the wave's current setting, so the instruction is issued on changes only.
__device__ __forceinline__ float uniform_f(float v) {
  return __int_as_float((int)__builtin_amdgcn_readfirstlane((uint32_t)__float_as_int(v)));
}
template <bool kAllFit>
__device__ __forceinline__ void prefetch_row(const DevPtrs& d, const RowK* lrows, const uint32_t* roff_s,
                                             const uint2* meta_s, uint32_t r, Prefetch& pf) {
  const uint32_t lane = threadIdx.x;
  const uint32_t a = __builtin_amdgcn_readfirstlane(roff_s[r]);
  const uint32_t n = __builtin_amdgcn_readfirstlane(roff_s[r + 1]) - a;
  const uint2 meta = meta_s[r];
  pf.st.meta = make_uint2(__builtin_amdgcn_readfirstlane(meta.x), __builtin_amdgcn_readfirstlane(meta.y));
  const RowK rk = lrows[r];   // the row's constants, for the step that uses the stage
  pf.st.rk = RowK{uniform_f(rk.x), uniform_f(rk.half_y), uniform_f(rk.y_lo), uniform_f(rk.inv_wy)};
  pf.st.fits = kAllFit || n <= (uint32_t)kStageHits;
  const uint32_t ybase = a & ~1u, ycnt = a + n - ybase;
  pf.st.first = ybase;
  const uint32_t bbase = pf.st.meta.x & ~3u;
  pf.st.boff = pf.st.meta.x - bbase;
  if (!pf.st.fits) return;
  const f32x4* ysrc = reinterpret_cast<const f32x4*>(d.syz + ybase);
#pragma unroll
  for (int m = 0; m < kPreYz; ++m) {
    const uint32_t q = lane + m * kThreads;   // pair q holds entries 2q, 2q + 1
    pf.yz[m] = ysrc[2 * q < ycnt ? q : 0];
  }
  const uint32_t bcnt = pf.st.boff + (pf.st.meta.y & 0xFFFFu) * (pf.st.meta.y >> 16) + 1;   // every row has a grid
  const u32x4* bsrc = reinterpret_cast<const u32x4*>(d.bin_start + bbase);
#pragma unroll
  for (int m = 0; m < kPreBs; ++m) {
    const uint32_t q = lane + m * kThreads;   // quad q holds entries 4q .. 4q + 3
    pf.bs[m] = bsrc[4 * q < bcnt ? q : 0];
  }
}

// Write prefetched registers to the LDS stage (call between two barriers).
__device__ __forceinline__ void commit_row(const Prefetch& pf, f32x4* yz4_s, u32x4* bs4_s, Stage& st) {
  const uint32_t lane = threadIdx.x;
  st = pf.st;
  if (!st.fits) return;
#pragma unroll
  for (int m = 0; m < kPreYz; ++m) yz4_s[lane + m * kThreads] = pf.yz[m];
#pragma unroll
  for (int m = 0; m < kPreBs; ++m) bs4_s[lane + m * kThreads] = pf.bs[m];
}

// Three waves per SIMD (<= 168 VGPRs) keep every wave of a central event
// resident at once.  The double-precision state then spills about 40 VGPRs
// to scratch; measured on a central event this is faster than two waves per
// SIMD without spills (0.86 against 1.09 ms).
template <bool kAllFit>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3))) k_tracklets_rs(DevPtrs d, KfConst k) {
  __shared__ RowK lrows[kMaxRows];
  __shared__ f32x4 yz4_s[kPreYz * kThreads];   // the staged row: (y, z) pairs
  __shared__ u32x4 bs4_s[kPreBs * kThreads];   // and its bin starts
  const float2* yz_s = reinterpret_cast<const float2*>(yz4_s);
  const uint32_t* bs_s = reinterpret_cast<const uint32_t*>(bs4_s);
  __shared__ uint32_t roff_s[kMaxRows + 1];   // the current sector's row offsets
  __shared__ uint2 meta_s[kMaxRows];          // and grid words
  const uint32_t R = d.R, T = d.tcap, S = d.S;
  const uint32_t lane = threadIdx.x;
  const uint32_t W = d.wave_off[S];
  // XCD-contiguous ranges of waves (one wave per block, waves ordered by sector)
  const uint32_t per = (W + kXcds - 1) / kXcds;
  const uint32_t xcd = blockIdx.x % kXcds;
  const uint32_t vend = min(W, (xcd + 1) * per);
  // the grid is sized for the tracklet capacity; blocks without a wave leave at once
  if (xcd * per + blockIdx.x / kXcds >= vend) return;
  load_rows(d, lrows);
  unsigned long long my_steps = 0;
  uint32_t prio = 0;   // s_setprio level of this wave (waves start at 0)
  for (uint32_t v = xcd * per + blockIdx.x / kXcds; v < vend; v += gridDim.x / kXcds) {
    // sector of wave v: last s with wave_off[s] <= v
    uint32_t lo = 0, hi = S;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) / 2;
      if (d.wave_off[mid] <= v) lo = mid; else hi = mid;
    }
    const uint32_t sec = lo, srb = sec * R;
    const uint32_t ts = min(d.row_start_off[srb], T), te = min(d.row_start_off[srb + R], T);
    const uint32_t half = lane & 1u;   // both lanes of a pair compute the same tracklet and store identical values
    const uint32_t i = ts + (v - d.wave_off[sec]) * kTrkPerWave + (lane >> 1);
    const SectorConst sc = d.secs[sec];
    int32_t* H = d.tk_rowhit + i;
    __syncthreads();   // the previous wave's last reads of the row table are done
    for (uint32_t q = lane; q <= R; q += kThreads) {
      roff_s[q] = d.row_off[srb + q];
      if (q < R) meta_s[q] = d.row_meta[srb + q];
    }
    __syncthreads();
    // ---- per lane: chain walk and seed ----
    bool ok = i < te;
    uint32_t r0 = 0, rl = 0, n = 0;
    float zref = 0.0f, chi2 = 0.0f, xprev = 0.0f;
    Trk t;
    if (ok) {
      const uint32_t sr0 = d.start_sr[i];
      r0 = sr0 % R;
      int32_t p = (int32_t)d.start_pos[i];
      int32_t plast = p;
      while (p >= 0 && r0 + n < R) {
        H[(size_t)(r0 + n) * T] = p;
        plast = p;
        ++n;
        p = d.up1[p];
      }
      const uint32_t m = (n - 1) / 2;
      rl = r0 + n - 1;
      const int32_t pm = H[(size_t)(r0 + m) * T];
      const float2 h0 = d.syz[d.start_pos[i]];
      zref = h0.y;
      if (seed3(lrows[r0].x, h0, lrows[r0 + m].x, d.syz[pm], lrows[rl].x, d.syz[plast], k, t)) {
        set_c0(t, k);
        xprev = lrows[r0].x;
      } else {
        d.tk_info[i] = -1;
        ok = false;
      }
    }
    uint32_t steps = ok ? n - 1 : 0;
    // ---- outward sweep ----
    bool up = ok, failed = false;
    par_t pout[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) pout[q] = t.p[q];
    uint32_t rout = rl;
    int miss = 0;
    Stage st;
    Prefetch pf;
    uint32_t r = __builtin_amdgcn_readfirstlane(wave_min(up ? r0 + 1 : R));   // wave-uniform from here on
    if (r < R) {
      prefetch_row<kAllFit>(d, lrows, roff_s, meta_s, r, pf);
      commit_row(pf, yz4_s, bs4_s, st);
      __syncthreads();
    }
    int32_t hnext = (up && r <= rl && r > r0) ? H[(size_t)r * T] : -1;
    // Drain every load issued so far (the sector constants, the first row, the
    // chain hit) before the loop: the compiler's wait counters are tracked per
    // register across the back edge, and a value still pending from before the
    // loop would otherwise make every iteration wait for all its loads --
    // including the prefetch of the next row, which should overlap the step.
    __builtin_amdgcn_s_waitcnt(0);
    while (r < R && __any(up)) {
      set_priority(2 * R - r, prio);   // the rest of this sweep, then (about) the whole inward sweep
      if (r + 1 < R) prefetch_row<kAllFit>(d, lrows, roff_s, meta_s, r + 1, pf);
      const int32_t hchain = hnext;
      hnext = (up && r + 1 <= rl && r + 1 > r0) ? H[(size_t)(r + 1) * T] : -1;
      if (up && r > r0) {
        // flags instead of nested branches: a lane that stops here keeps
        // nothing of this step (its state is not read again)
        const RowK rk = st.rk;
        const bool chain = r <= rl;
        steps += chain ? 0u : 1u;
        const bool pok = propagate<true>(t, rk.x - xprev, k);
        xprev = rk.x;
        failed = failed || (!pok && chain);
        const bool go = pok && (chain || fabs_(t.p[0]) <= rk.half_y + k.margin);
        up = go;
        int32_t h = hchain;
        if (go && !chain) {
          float2 unused;
          h = (kAllFit || st.fits) ? search_lds(yz_s, bs_s + st.boff, st.first, st.meta, rk, sc, t, k, zref, half)
                                   : search(d, srb + r, rk, sc, t, k, zref, unused);
          H[(size_t)r * T] = h;
        }
        if (go && h >= 0) {
          const float2 hm = (kAllFit || st.fits) ? yz_s[(uint32_t)h - st.first] : d.syz[h];
          update(t, hm.x, hm.y - zref, k, chi2);
          if (r >= rl) {
#pragma unroll
            for (int q = 0; q < 5; ++q) pout[q] = t.p[q];
            rout = r;
            miss = 0;
          }
        }
        const bool missed = go && h < 0;
        miss += missed ? 1 : 0;
        up = up && !(missed && miss > k.max_miss);
      }
      __syncthreads();
      if (r + 1 < R) commit_row(pf, yz4_s, bs4_s, st);
      __syncthreads();
      ++r;
    }
    if (failed) {
      d.tk_info[i] = -2;
      ok = false;
    }
    // ---- inward sweep from each lane's outermost hit, fresh covariance ----
    bool down = ok;
    int nh = 1;
    Snap snap;
    uint32_t rin = rout;
    if (down) {
      const float2 ho = d.syz[H[(size_t)rout * T]];
#pragma unroll
      for (int q = 2; q < 5; ++q) t.p[q] = pout[q];
      t.p[0] = ho.x;
      t.p[1] = ho.y - zref;
      set_c0(t, k);
      chi2 = 0.0f;
      snap = snap_of(t);
      xprev = lrows[rout].x;
      miss = 0;
    }
    int32_t rr = (int32_t)__builtin_amdgcn_readfirstlane(wave_max(down ? rout : 0)) - 1;
    if (rr >= 0) {
      prefetch_row<kAllFit>(d, lrows, roff_s, meta_s, (uint32_t)rr, pf);
      commit_row(pf, yz4_s, bs4_s, st);
      __syncthreads();
    }
    hnext = (down && rr >= (int32_t)r0 && rr < (int32_t)rout) ? H[(size_t)rr * T] : -1;
    __builtin_amdgcn_s_waitcnt(0);   // as before the outward sweep
    while (rr >= 0 && __any(down)) {
      set_priority((uint32_t)rr, prio);
      if (rr > 0) prefetch_row<kAllFit>(d, lrows, roff_s, meta_s, (uint32_t)rr - 1, pf);
      const int32_t hrow = hnext;
      hnext = (down && rr - 1 >= (int32_t)r0 && rr - 1 < (int32_t)rout) ? H[(size_t)(rr - 1) * T] : -1;
      if (down && rr < (int32_t)rout) {
        const RowK rk = st.rk;   // flags instead of nested branches, as in the outward sweep
        ++steps;
        const bool pok = propagate<true>(t, rk.x - xprev, k);
        xprev = rk.x;
        const bool below = (uint32_t)rr < r0;
        const bool go = pok && !(below && fabs_(t.p[0]) > rk.half_y + k.margin);
        down = go;
        int32_t h = below ? -1 : hrow;
        if (go && h < 0) {
          float2 unused;
          h = (kAllFit || st.fits) ? search_lds(yz_s, bs_s + st.boff, st.first, st.meta, rk, sc, t, k, zref, half)
                                   : search(d, srb + (uint32_t)rr, rk, sc, t, k, zref, unused);
        }
        if (go && (below || h != hrow)) H[(size_t)rr * T] = h;   // changed only where the refit searched
        if (go && h >= 0) {
          const float2 hm = (kAllFit || st.fits) ? yz_s[(uint32_t)h - st.first] : d.syz[h];
          update(t, hm.x, hm.y - zref, k, chi2);
          ++nh;
          snap = snap_of(t);
          rin = (uint32_t)rr;
          if (below) miss = 0;
        }
        const bool missed = go && below && h < 0;
        miss += missed ? 1 : 0;
        down = down && !(missed && miss > k.max_miss);
      }
      __syncthreads();
      if (rr > 0) commit_row(pf, yz4_s, bs4_s, st);
      __syncthreads();
      --rr;
    }
    if (ok) {
      store_tracklet<true>(d, i, nh, rin, rout, r0, snap, chi2, zref);
      if (half == 0) my_steps += steps;
    }
  }
  if (my_steps) atomicAdd(&d.hdr->n_steps, my_steps);
}

// Waves of the row-synchronous schedule: ceil(tracklets of sector s / 32) per
// sector, prefix-summed (one block).
__global__ void __launch_bounds__(1024) k_waves(DevPtrs d) {
  __shared__ uint32_t wsum[1024 / kWave];
  const uint32_t S = d.S, R = d.R, T = d.tcap;
  const uint32_t per = (S + blockDim.x - 1) / blockDim.x;
  const uint32_t s0 = min(S, threadIdx.x * per), s1 = min(S, s0 + per);
  uint32_t sum = 0;
  for (uint32_t s = s0; s < s1; ++s) {
    const uint32_t a = min(d.row_start_off[s * R], T), b = min(d.row_start_off[(s + 1) * R], T);
    sum += (b - a + kTrkPerWave - 1) / kTrkPerWave;
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan<uint32_t>(sum, wsum, &total);
  for (uint32_t s = s0; s < s1; ++s) {
    d.wave_off[s] = run;
    const uint32_t a = min(d.row_start_off[s * R], T), b = min(d.row_start_off[(s + 1) * R], T);
    run += (b - a + kTrkPerWave - 1) / kTrkPerWave;
  }
  if (threadIdx.x == 0) d.wave_off[S] = total;
}

}  // namespace

void launch_tracklets(const DevPtrs& d, const KfConst& k, uint32_t max_row_hits, hipStream_t s) {
  if (d.tcap == 0) return;
  const bool rowsync = d.k5_mode == 2 || (d.k5_mode == 0 && max_row_hits <= (uint32_t)kStageHits);
  if (rowsync) {
    hipLaunchKernelGGL(k_waves, dim3(1), dim3(1024), 0, s, d);
    uint32_t blocks = (d.tcap + kTrkPerWave - 1) / kTrkPerWave + d.S;
    if (blocks > 16384) blocks = 16384;
    if (max_row_hits <= (uint32_t)kStageHits)   // every row is staged: the kernel carries no global-memory search
      hipLaunchKernelGGL(k_tracklets_rs<true>, dim3(xcd_grid(blocks)), dim3(kThreads), 0, s, d, k);
    else
      hipLaunchKernelGGL(k_tracklets_rs<false>, dim3(xcd_grid(blocks)), dim3(kThreads), 0, s, d, k);
    return;
  }
  uint32_t blocks = (d.tcap + kThreads - 1) / kThreads;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_seed, dim3(xcd_grid(blocks)), dim3(kThreads), 0, s, d, k);
  hipLaunchKernelGGL(k_up, dim3(xcd_grid(blocks)), dim3(kThreads), 0, s, d, k);
  const uint32_t sort_blocks = std::min<uint32_t>((d.tcap + 255) / 256, 4096);
  if (d.k5_refit_order == 0) {
    launch_scan_u32(d.row_nstart, d.k5_off, d.SR, d.scan_blocks, s);
    hipLaunchKernelGGL(k_sort, dim3(sort_blocks), dim3(256), 0, s, d);
  }
  hipLaunchKernelGGL(k_down, dim3(xcd_grid(blocks)), dim3(kThreads), 0, s, d, k);
  hipLaunchKernelGGL(k_guard, dim3(sort_blocks), dim3(256), 0, s, d);
}

}  // namespace tpc
