// K7-K9: sector merger and merged-chain refit -- steps C8 and C9 of the
// tracker definition, on the C7 tracks of a completed request.
//
// A particle that crosses a sector edge leaves one track segment per sector.
// C8 links a segment a to a segment b of the neighbouring sector on the same
// side when a's state, rotated into b's frame and propagated to b's x_ref,
// lands within fixed windows of b's state, b starting at a larger radius;
// each segment keeps its best successor (smallest position score) and each
// its best predecessor, and a link needs both.  C9 refits every chain of two
// or more segments with one inward Kalman pass over all its clusters.
//
//   k_merge_ranges  first track of each sector (tracks are in sector order)
//   k_merge_match   one thread per segment a: the tracks of the two
//                   neighbouring sectors; tan(lambda) and q/pT are invariants
//                   of the rotation and the propagation, so their windows are
//                   tested first; survivors are rotated and propagated in
//                   double.  Best successor kept locally; best predecessor by
//                   a 64-bit atomicMin of (score as float bits, a).
//   k_merge_link    mutual best -> next[a]; predecessor flags
//   k_merge_count   per chain head: segments and clusters (scans follow)
//   k_merge_emit    per chain head: merged cluster list, and the refit (state
//                   and covariance in double) or the C5 result of a single
//                   segment
#include "device_common.h"

namespace tpc {
namespace {

constexpr int kThreads = 256;
constexpr int kSide = 18;

__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }

struct MTrack {
  uint32_t sector;
  int32_t phys;
  double x, p[5];
  double r_in;
};

__device__ __forceinline__ MTrack load_track(const DevPtrs& d, const MergeArgs& m, uint32_t t) {
  MTrack a;
  a.sector = d.out_sector[t];
  a.phys = m.phys[a.sector];
  a.x = d.out_xref[t];
#pragma unroll
  for (int q = 0; q < 5; ++q) a.p[q] = d.out_param[(size_t)t * 5 + q];
  a.r_in = sqrt(a.x * a.x + a.p[0] * a.p[0]);
  return a;
}

// Helix transport of the state only (the map of C5), in double.
__device__ __forceinline__ double asin_over_d(double u) {
  const double u2 = u * u;
  if (fabs(u) < 1e-2) return 1.0 + u2 * (1.0 / 6.0 + u2 * (3.0 / 40.0 + u2 * (5.0 / 112.0 + u2 * (35.0 / 1152.0))));
  return asin(u) / u;
}
__device__ __forceinline__ double asin_over_prime_d(double u) {
  const double u2 = u * u;
  if (fabs(u) < 1e-2) return u * (1.0 / 3.0 + u2 * (3.0 / 10.0 + u2 * (15.0 / 56.0 + u2 * (35.0 / 144.0))));
  return (u / sqrt(1.0 - u2) - asin(u)) / u2;
}

// x1 -> x2 with the exact Jacobian F (sparse entries A..Fk) when cov is given.
__device__ bool prop_d(double* p, double x1, double x2, double bk, double smax, double* c) {
  const double dx = x2 - x1;
  const double s1 = p[2], tl = p[3], kap = bk * p[4];
  if (!(fabs(s1) < smax)) return false;
  const double s2 = s1 + kap * dx;
  if (!(fabs(s2) < smax)) return false;
  const double c1 = sqrt((1.0 - s1) * (1.0 + s1)), c2 = sqrt((1.0 - s2) * (1.0 + s2));
  const double dy = dx * ((s1 + s2) / (c1 + c2));
  const double L = sqrt(dx * dx + dy * dy);
  const double u = 0.5 * kap * L;
  if (!(fabs(u) < 1.0)) return false;
  const double sgn = dx >= 0.0 ? 1.0 : -1.0;
  const double S = sgn * L * asin_over_d(u);
  if (c) {
    const double D = (1.0 + c1 * c2 + s1 * s2) / ((c1 + c2) * (c1 + c2));
    const double A = dx * D * (1.0 / c1 + 1.0 / c2);
    const double B = dx * (D / c2) * bk * dx;
    const double dS_dL = sgn / sqrt(1.0 - u * u);
    const double dS_dkap = sgn * 0.5 * L * L * asin_over_prime_d(u);
    const double dL_ddy = L > 0.0 ? dy / L : 0.0;
    const double Cc = tl * dS_dL * dL_ddy * A;
    const double Dd = S;
    const double E = tl * (dS_dL * dL_ddy * B + dS_dkap * bk);
    const double Fk = bk * dx;
    double M[5][5], G[3][5];
    for (int i = 0; i < 5; ++i)
      for (int j = 0; j < 5; ++j) M[i][j] = i >= j ? c[tri(i, j)] : c[tri(j, i)];
    for (int j = 0; j < 5; ++j) {
      G[0][j] = M[0][j] + A * M[2][j] + B * M[4][j];
      G[1][j] = M[1][j] + Cc * M[2][j] + Dd * M[3][j] + E * M[4][j];
      G[2][j] = M[2][j] + Fk * M[4][j];
    }
    // C' = G F^T on the lower triangle (rows 3, 4 of F are those of the identity)
    for (int i = 0; i < 5; ++i) {
      const double g0 = i < 3 ? G[i][0] : M[i][0], g1 = i < 3 ? G[i][1] : M[i][1], g2 = i < 3 ? G[i][2] : M[i][2];
      const double g3 = i < 3 ? G[i][3] : M[i][3], g4 = i < 3 ? G[i][4] : M[i][4];
      const double rr[5] = {g0 + A * g2 + B * g4, g1 + Cc * g2 + Dd * g3 + E * g4, g2 + Fk * g4, g3, g4};
      for (int j = 0; j <= i; ++j) c[tri(i, j)] = rr[j];
    }
  }
  p[0] += dy;
  p[1] += tl * S;
  p[2] = s2;
  return true;
}

// Rotation into the frame turned by the angle with cosine cd and sine sd, at
// the same point in space; first-order covariance onto the new plane x' = const.
__device__ bool rotate_d(double& x, double* p, double cd, double sd, double bk, double* c) {
  const double s = p[2], cs = sqrt((1.0 - s) * (1.0 + s));
  const double s2 = s * cd - cs * sd, c2 = cs * cd + s * sd;
  if (!(c2 > 0.0)) return false;
  const double x2 = x * cd + p[0] * sd;
  const double y2 = -x * sd + p[0] * cd;
  if (c) {
    // J = I except J00 = cs/c2, J10 = -tanl sd/c2, J20 = -bk qpt sd, J22 = c2/cs
    const double j00 = cs / c2, j10 = -p[3] * sd / c2, j20 = -bk * p[4] * sd, j22 = c2 / cs;
    double M[5][5];
    for (int i = 0; i < 5; ++i)
      for (int j = 0; j < 5; ++j) M[i][j] = i >= j ? c[tri(i, j)] : c[tri(j, i)];
    double G[5][5];   // G = J M
    for (int j = 0; j < 5; ++j) {
      G[0][j] = j00 * M[0][j];
      G[1][j] = j10 * M[0][j] + M[1][j];
      G[2][j] = j20 * M[0][j] + j22 * M[2][j];
      G[3][j] = M[3][j];
      G[4][j] = M[4][j];
    }
    for (int i = 0; i < 5; ++i) {   // C' = G J^T
      const double rr[5] = {G[i][0] * j00, G[i][0] * j10 + G[i][1], G[i][0] * j20 + G[i][2] * j22, G[i][3], G[i][4]};
      for (int j = 0; j <= i; ++j) c[tri(i, j)] = rr[j];
    }
  }
  x = x2;
  p[0] = y2;
  p[2] = s2;
  return true;
}

// Kalman update of (y, z), Joseph form, in double.
__device__ void update_d(double* p, double* c, double ym, double zm, double vy, double vz, double& chi2) {
  const double r0 = ym - p[0], r1 = zm - p[1];
  const double S00 = c[0] + vy, S01 = c[1], S11 = c[2] + vz;
  const double det = S00 * S11 - S01 * S01;
  const double I00 = S11 / det, I01 = -S01 / det, I11 = S00 / det;
  double c0[5], c1[5], K0[5], K1[5];
  for (int i = 0; i < 5; ++i) {
    c0[i] = c[tri(i, 0)];
    c1[i] = i >= 1 ? c[tri(i, 1)] : c[1];
  }
  for (int i = 0; i < 5; ++i) {
    K0[i] = c0[i] * I00 + c1[i] * I01;
    K1[i] = c0[i] * I01 + c1[i] * I11;
    p[i] += K0[i] * r0 + K1[i] * r1;
  }
  double P[5][5];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) P[i][j] = (i >= j ? c[tri(i, j)] : c[tri(j, i)]) - K0[i] * c0[j] - K1[i] * c1[j];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j <= i; ++j)
      c[tri(i, j)] = P[i][j] + (K0[i] * vy - P[i][0]) * K0[j] + (K1[i] * vz - P[i][1]) * K1[j];
  chi2 += r0 * (I00 * r0 + I01 * r1) + r1 * (I01 * r0 + I11 * r1);
}

__device__ __forceinline__ uint32_t n_tracks(const DevPtrs& d) { return min(d.hdr->n_tracks, d.max_tracks); }

// Neighbour of physical sector ph one step (+1 / -1) along its side's ring.
__device__ __forceinline__ int32_t neighbour(int32_t ph, int step) {
  const int32_t side = ph / kSide, i = ph % kSide;
  return side * kSide + (i + step + kSide) % kSide;
}

__global__ void __launch_bounds__(kThreads) k_merge_init(DevPtrs d, MergeArgs m, uint32_t nt) {
  const uint32_t a = blockIdx.x * kThreads + threadIdx.x;
  if (a >= nt) return;
  m.pred_key[a] = ~0ull;
  m.has_pred[a] = 0u;
}

__global__ void __launch_bounds__(kThreads) k_merge_ranges(DevPtrs d, MergeArgs m) {
  const uint32_t s = blockIdx.x * kThreads + threadIdx.x;
  if (s > d.S) return;
  // first track of sector s: lower bound of s in the sorted track sectors
  uint32_t lo = 0, hi = n_tracks(d);
  while (lo < hi) {
    const uint32_t mid = (lo + hi) / 2;
    if (d.out_sector[mid] < s) lo = mid + 1; else hi = mid;
  }
  m.sec_first[s] = lo;
  if (s < d.S) {
    // the run's sector holding each physical neighbour (-1 if absent from the frame)
    const int32_t ph = m.phys[s];
    for (int k = 0; k < 2; ++k) {
      int32_t hit = -1;
      if (ph >= 0) {
        const int32_t want = neighbour(ph, k == 0 ? -1 : 1);
        for (uint32_t q = 0; q < d.S; ++q)
          if (m.phys[q] == want) { hit = (int32_t)q; break; }
      }
      m.nbr[2 * s + k] = hit;
    }
  }
}

__global__ void __launch_bounds__(kThreads) k_merge_match(DevPtrs d, MergeArgs m, KfConst k) {
  const uint32_t nt = n_tracks(d);
  const uint32_t a = blockIdx.x * kThreads + threadIdx.x;
  if (a >= nt) return;
  const MTrack ta = load_track(d, m, a);
  int32_t best = -1;
  double best_s = 0.0;
  if (ta.phys >= 0) {
    for (int side = 0; side < 2; ++side) {
      const int32_t nb = m.nbr[2 * ta.sector + side];
      if (nb < 0) continue;
      const int step = side == 0 ? -1 : 1;
      const double cd = m.cos20, sd = step * m.sin20;
      const uint32_t b0 = m.sec_first[nb], b1 = m.sec_first[nb + 1];
      for (uint32_t b = b0; b < b1; ++b) {
        // rotation and propagation keep tan(lambda) and q/pT: their windows first
        const float tlb = d.out_param[(size_t)b * 5 + 3], qb = d.out_param[(size_t)b * 5 + 4];
        if (!(fabs(ta.p[3] - (double)tlb) <= m.dtanl && fabs(ta.p[4] - (double)qb) <= m.dqpt)) continue;
        const MTrack tb = load_track(d, m, b);
        if (!(tb.r_in > ta.r_in)) continue;
        double x = ta.x, q[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) q[i] = ta.p[i];
        if (!rotate_d(x, q, cd, sd, m.bk, nullptr)) continue;
        if (!prop_d(q, x, tb.x, m.bk, m.s_max, nullptr)) continue;
        const double dy = q[0] - tb.p[0], dz = q[1] - tb.p[1];
        if (!(fabs(dy) <= m.dy && fabs(dz) <= m.dz && fabs(q[2] - tb.p[2]) <= m.dsinphi)) continue;
        const double cyy = d.out_cov[(size_t)b * 15 + 0], czz = d.out_cov[(size_t)b * 15 + 2];
        const double sc = dy * dy / (cyy + m.vy) + dz * dz / (czz + m.vz);
        if (best < 0 || sc < best_s || (sc == best_s && (int32_t)b < best)) {
          best = (int32_t)b;
          best_s = sc;
        }
        const unsigned long long key = ((unsigned long long)__float_as_uint((float)sc) << 32) | a;
        atomicMin(&m.pred_key[b], key);
      }
    }
  }
  m.succ[a] = best;
}

__global__ void __launch_bounds__(kThreads) k_merge_link(DevPtrs d, MergeArgs m) {
  const uint32_t nt = n_tracks(d);
  const uint32_t a = blockIdx.x * kThreads + threadIdx.x;
  if (a >= nt) return;
  const int32_t b = m.succ[a];
  const bool link = b >= 0 && (uint32_t)(m.pred_key[b] & 0xFFFFFFFFull) == a;
  m.next[a] = link ? b : -1;
  if (link) m.has_pred[b] = 1u;
}

// Per track: 1 if it heads a chain (for the scan of chain indices), and at
// each head the chain's cluster count (for the scan of cluster offsets).
__global__ void __launch_bounds__(kThreads) k_merge_count(DevPtrs d, MergeArgs m) {
  const uint32_t nt = n_tracks(d);
  const uint32_t a = blockIdx.x * kThreads + threadIdx.x;
  if (a >= nt) return;
  const bool head = m.has_pred[a] == 0u;
  m.head_flag[a] = head ? 1u : 0u;
  uint32_t n = 0;
  if (head)
    for (int32_t t = (int32_t)a; t >= 0; t = m.next[t]) n += d.out_first[t + 1] - d.out_first[t];
  m.chain_clusters[a] = n;
}

// Row of input cluster id inside sector s (upper bound in the sector's row offsets).
__device__ __forceinline__ uint32_t row_of(const DevPtrs& d, uint32_t s, uint32_t id) {
  uint32_t lo = 0, hi = d.R;   // first row r with row_off[s*R + r + 1] > id
  while (lo < hi) {
    const uint32_t mid = (lo + hi) / 2;
    if (d.row_off[s * d.R + mid + 1] <= id) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ void __launch_bounds__(kThreads) k_merge_emit(DevPtrs d, MergeArgs m, KfConst k) {
  const uint32_t nt = n_tracks(d);
  const uint32_t a = blockIdx.x * kThreads + threadIdx.x;
  if (a >= nt || m.head_flag[a] == 0u) return;
  const uint32_t c = m.head_scan[a];   // chain index
  uint32_t o = m.cl_scan[a];
  m.heads[c] = a;
  m.first[c] = o;
  int32_t last = (int32_t)a, nseg = 0;
  for (int32_t t = (int32_t)a; t >= 0; t = m.next[t]) {
    for (uint32_t j = d.out_first[t]; j < d.out_first[t + 1]; ++j) m.clusters[o++] = d.out_clusters[j];
    m.head_of[t] = a;
    last = t;
    ++nseg;
  }
  if (c + 1 == m.head_scan[nt]) m.first[c + 1] = o;
  double P[5], C[15];
  double chi2 = d.out_chi2[a];
  const uint32_t ncl = o - m.first[c];
  int32_t ndf = 2 * (int32_t)ncl - 5;
#pragma unroll
  for (int q = 0; q < 5; ++q) P[q] = d.out_param[(size_t)a * 5 + q];
#pragma unroll
  for (int q = 0; q < 15; ++q) C[q] = d.out_cov[(size_t)a * 15 + q];
  if (nseg > 1) {
    // inward pass over the chain's clusters, from the outermost one of the last segment
    const double vy = m.vy, vz = m.vz;
    int32_t seg = last;
    uint32_t j = d.out_first[seg + 1] - 1;
    uint32_t sec = d.out_sector[seg];
    uint32_t id = d.out_clusters[j];
    uint32_t row = row_of(d, sec, id);
    double p[5], cv[15];
    double x = d.out_xref[seg];
#pragma unroll
    for (int q = 0; q < 5; ++q) p[q] = d.out_param[(size_t)seg * 5 + q];
    bool ok = prop_d(p, x, d.rows[row].x, m.bk, m.s_max, nullptr);
    double ch = 0.0;
    if (ok) {
      x = d.rows[row].x;
      p[0] = d.y[id];
      p[1] = d.z[id];
#pragma unroll
      for (int q = 0; q < 15; ++q) cv[q] = 0.0;
      cv[0] = vy;
      cv[2] = vz;
      cv[5] = m.c0_sinphi;
      cv[9] = m.c0_tanl;
      cv[14] = m.c0_qpt;
      // walk back: earlier clusters of this segment, then the previous segments
      for (;;) {
        if (j > d.out_first[seg]) {
          --j;
        } else {
          // previous segment in the chain: the one whose next is seg
          int32_t pv = (int32_t)a;
          while (m.next[pv] != seg) pv = m.next[pv];
          const int step = (m.phys[d.out_sector[pv]] % kSide - m.phys[sec] % kSide + kSide) % kSide == 1 ? 1 : -1;
          if (!rotate_d(x, p, m.cos20, step * m.sin20, m.bk, cv)) { ok = false; break; }
          seg = pv;
          sec = d.out_sector[seg];
          j = d.out_first[seg + 1] - 1;
        }
        id = d.out_clusters[j];
        row = row_of(d, sec, id);
        if (!prop_d(p, x, d.rows[row].x, m.bk, m.s_max, cv)) { ok = false; break; }
        x = d.rows[row].x;
        update_d(p, cv, d.y[id], d.z[id], vy, vz, ch);
        if (seg == (int32_t)a && j == d.out_first[a]) break;
      }
    }
    if (ok) {
#pragma unroll
      for (int q = 0; q < 5; ++q) P[q] = p[q];
#pragma unroll
      for (int q = 0; q < 15; ++q) C[q] = cv[q];
      chi2 = ch;
    } else {
      ndf = -1;
    }
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) m.param[(size_t)c * 5 + q] = (float)P[q];
#pragma unroll
  for (int q = 0; q < 15; ++q) m.cov[(size_t)c * 15 + q] = (float)C[q];
  m.chi2[c] = (float)chi2;
  m.ndf[c] = ndf;
  m.nseg[c] = nseg;
}

}  // namespace

void launch_merge(const DevPtrs& d, const MergeArgs& m, const KfConst& k, uint32_t nt, hipStream_t s) {
  const uint32_t g = (nt + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_merge_ranges, dim3((d.S + 1 + kThreads - 1) / kThreads), dim3(kThreads), 0, s, d, m);
  if (g == 0) return;
  hipLaunchKernelGGL(k_merge_init, dim3(g), dim3(kThreads), 0, s, d, m, nt);
  hipLaunchKernelGGL(k_merge_match, dim3(g), dim3(kThreads), 0, s, d, m, k);
  hipLaunchKernelGGL(k_merge_link, dim3(g), dim3(kThreads), 0, s, d, m);
  hipLaunchKernelGGL(k_merge_count, dim3(g), dim3(kThreads), 0, s, d, m);
  launch_scan_u32(m.head_flag, m.head_scan, nt, d.scan_blocks, s);
  launch_scan_u32(m.chain_clusters, m.cl_scan, nt, d.scan_blocks, s);
  hipLaunchKernelGGL(k_merge_emit, dim3(g), dim3(kThreads), 0, s, d, m, k);
}

}  // namespace tpc
