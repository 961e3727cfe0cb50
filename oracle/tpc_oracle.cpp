// FP64 reference tracker (test infrastructure only; see tpc_oracle.h).
//
// Plain, single-threaded C++.  Build with -O2 -ffp-contract=off so that the
// float32 decisions (C1 bin, C2 window and deviation, C6 owned fraction) are
// evaluated with one IEEE rounding per written operation, exactly as stated.
#include "tpc_oracle.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

constexpr double kCB = 0.00299792458;   // GeV / (T cm)
constexpr float kWinPad = 0.01f;        // cm added to search ranges before binning

// asin(u)/u and its derivative, evaluated stably for small |u|.
double asin_over(double u) {
  if (std::fabs(u) < 1e-2) {
    double u2 = u * u;
    return 1.0 + u2 * (1.0 / 6.0 + u2 * (3.0 / 40.0 + u2 * (5.0 / 112.0 + u2 * (35.0 / 1152.0))));
  }
  return std::asin(u) / u;
}
double asin_over_prime(double u) {
  if (std::fabs(u) < 1e-2) {
    double u2 = u * u;
    return u * (1.0 / 3.0 + u2 * (3.0 / 10.0 + u2 * (15.0 / 56.0 + u2 * (35.0 / 144.0))));
  }
  return (u / std::sqrt(1.0 - u * u) - std::asin(u)) / (u * u);
}

// packed lower triangle index (i >= j): 00,10,11,20,21,22,...
inline int tri(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

void unpack(const double* c15, double C[5][5]) {
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) C[i][j] = c15[tri(i, j)];
}
void pack(const double C[5][5], double* c15) {
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j <= i; ++j) c15[tri(i, j)] = 0.5 * (C[i][j] + C[j][i]);
}

// Helix transport, exact map and its exact Jacobian (definition C5, propagation).
int propagate(const double* p, double x1, double x2, double bk, double smax, double* q, double F[5][5]) {
  const double dx = x2 - x1;
  const double s1 = p[2], tl = p[3], k = p[4];
  const double kap = bk * k;
  if (!(std::fabs(s1) < smax)) return 1;
  const double s2 = s1 + kap * dx;
  if (!(std::fabs(s2) < smax)) return 1;
  const double c1 = std::sqrt((1.0 - s1) * (1.0 + s1));
  const double c2 = std::sqrt((1.0 - s2) * (1.0 + s2));
  const double T = (s1 + s2) / (c1 + c2);
  const double dy = dx * T;
  const double L = std::sqrt(dx * dx + dy * dy);
  const double u = 0.5 * kap * L;
  if (!(std::fabs(u) < 1.0)) return 1;
  const double sgn = dx >= 0.0 ? 1.0 : -1.0;
  const double S = sgn * L * asin_over(u);
  q[0] = p[0] + dy;
  q[1] = p[1] + tl * S;
  q[2] = s2;
  q[3] = tl;
  q[4] = k;
  if (F) {
    for (int i = 0; i < 5; ++i)
      for (int j = 0; j < 5; ++j) F[i][j] = (i == j) ? 1.0 : 0.0;
    const double D = (1.0 + c1 * c2 + s1 * s2) / ((c1 + c2) * (c1 + c2));
    const double ddy_ds1 = dx * D * (1.0 / c1 + 1.0 / c2);
    const double ddy_dk = dx * (D / c2) * bk * dx;
    const double dS_dL = sgn / std::sqrt(1.0 - u * u);
    const double dS_dkap = sgn * 0.5 * L * L * asin_over_prime(u);
    const double dL_ddy = L > 0.0 ? dy / L : 0.0;
    const double dS_ds1 = dS_dL * dL_ddy * ddy_ds1;
    const double dS_dk = dS_dL * dL_ddy * ddy_dk + dS_dkap * bk;
    F[0][2] = ddy_ds1;
    F[0][4] = ddy_dk;
    F[1][2] = tl * dS_ds1;
    F[1][3] = S;
    F[1][4] = tl * dS_dk;
    F[2][4] = bk * dx;
  }
  return 0;
}

void transport_cov(double* c15, const double F[5][5]) {
  double C[5][5], T[5][5], R[5][5];
  unpack(c15, C);
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) {
      double s = 0.0;
      for (int k = 0; k < 5; ++k) s += F[i][k] * C[k][j];
      T[i][j] = s;
    }
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) {
      double s = 0.0;
      for (int k = 0; k < 5; ++k) s += T[i][k] * F[j][k];
      R[i][j] = s;
    }
  pack(R, c15);
}

// Kalman update with measurement of (y, z), Joseph form.
void kf_update(double* p, double* c15, double ym, double zm, double vy, double vz, double* chi2) {
  double C[5][5];
  unpack(c15, C);
  const double r0 = ym - p[0], r1 = zm - p[1];
  const double S00 = C[0][0] + vy, S01 = C[1][0], S11 = C[1][1] + vz;
  const double det = S00 * S11 - S01 * S01;
  const double I00 = S11 / det, I01 = -S01 / det, I11 = S00 / det;
  double K[5][2];
  for (int i = 0; i < 5; ++i) {
    K[i][0] = C[i][0] * I00 + C[i][1] * I01;
    K[i][1] = C[i][0] * I01 + C[i][1] * I11;
  }
  for (int i = 0; i < 5; ++i) p[i] += K[i][0] * r0 + K[i][1] * r1;
  double A[5][5];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) A[i][j] = (i == j ? 1.0 : 0.0) - (j == 0 ? K[i][0] : 0.0) - (j == 1 ? K[i][1] : 0.0);
  double T[5][5], R[5][5];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) {
      double s = 0.0;
      for (int k = 0; k < 5; ++k) s += A[i][k] * C[k][j];
      T[i][j] = s;
    }
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) {
      double s = 0.0;
      for (int k = 0; k < 5; ++k) s += T[i][k] * A[j][k];
      R[i][j] = s + K[i][0] * vy * K[j][0] + K[i][1] * vz * K[j][1];
    }
  pack(R, c15);
  if (chi2) *chi2 += r0 * (I00 * r0 + I01 * r1) + r1 * (I01 * r0 + I11 * r1);
}

void grid_dims(uint32_t n, int k, int64_t ly, int64_t lz, int* ny, int* nz) {
  int64_t B = std::max<int64_t>(1, (int64_t)n / k);
  int64_t q = (B * ly) / lz;
  int64_t s = (int64_t)std::sqrt((double)q);
  while (s * s > q) --s;
  while ((s + 1) * (s + 1) <= q) ++s;
  if (s < 1) s = 1;
  if (s > B) s = B;
  *ny = (int)s;
  *nz = (int)std::max<int64_t>(1, B / s);
}

// One coordinate's bin: float32 round-to-nearest, one rounding per operation.
int bin1(float v, float lo, float inv_w, int n) {
  float a = v - lo;
  float b = (float)n * inv_w;
  float u = a * b;
  if (!(u >= 0.0f)) u = 0.0f;
  if (u > (float)(n - 1)) u = (float)(n - 1);
  return (int)u;
}

struct RowC {      // per-row constants derived from the geometry (float32 where a decision uses them)
  double X, Y;
  float y_lo, inv_wy;
  int64_t ly;
  float t, wy_up, wz_up, wy_dn, wz_dn, dmax;
};

}  // namespace

struct orc_run {
  orc_config cfg;
  uint32_t S, R;
  std::vector<uint32_t> off;                 // row offsets
  const double* y;
  const double* z;
  std::vector<float> zlo, zhi, inv_wz;
  std::vector<int64_t> lz;
  std::vector<RowC> rc;
  float rho;
  double bk;
  // C1
  std::vector<uint32_t> sorted_id;
  std::vector<double> sy, sz;                // FP64 coordinates at sorted positions
  std::vector<float> fy, fz;                 // float32 coordinates at sorted positions
  std::vector<uint32_t> bin_start, dims;
  // C2/C3
  std::vector<int32_t> up0, down0, up1, down1;
  // C4
  std::vector<uint32_t> starts, start_row;   // sorted position, (sector*R+row)
  // C5
  std::vector<int32_t> tk_rowhit, tk_nhits, tk_xref;
  std::vector<double> tk_param, tk_cov, tk_chi2;
  // C6
  std::vector<uint32_t> trk_tracklet, trk_first, trk_clusters;
};

namespace {

uint32_t bin_base(const orc_run* r, uint32_t sr) { return r->off[sr] + 2u * sr; }

// All sorted positions of row sr whose hits may lie in [ylo, yhi] x [zlo, zhi].
template <class Fn>
void for_range(const orc_run* r, uint32_t sr, float ylo, float yhi, float zlo, float zhi, Fn fn) {
  const uint32_t s = sr / r->R, row = sr % r->R;
  const RowC& c = r->rc[row];
  const int ny = r->dims[sr] & 0xFFFF, nz = r->dims[sr] >> 16;
  const int iy0 = bin1(ylo, c.y_lo, c.inv_wy, ny), iy1 = bin1(yhi, c.y_lo, c.inv_wy, ny);
  const int iz0 = bin1(zlo, r->zlo[s], r->inv_wz[s], nz), iz1 = bin1(zhi, r->zlo[s], r->inv_wz[s], nz);
  const uint32_t base = bin_base(r, sr);
  for (int iz = iz0; iz <= iz1; ++iz) {
    uint32_t a = r->bin_start[base + (uint32_t)(iz * ny + iy0)];
    uint32_t b = r->bin_start[base + (uint32_t)(iz * ny + iy1 + 1)];
    for (uint32_t p = a; p < b; ++p) fn(p);
  }
}

void set_c0(const orc_config& c, double* C) {
  for (int i = 0; i < 15; ++i) C[i] = 0.0;
  C[tri(0, 0)] = c.sigma_y * c.sigma_y;
  C[tri(1, 1)] = c.sigma_z * c.sigma_z;
  C[tri(2, 2)] = c.c0_sinphi;
  C[tri(3, 3)] = c.c0_tanl;
  C[tri(4, 4)] = c.c0_qpt;
}

int seed3(const orc_config& cfg, double bk, double x0, double y0, double z0, double xm, double ym, double xl,
          double yl, double zl, double* p) {
  const double ax = xm - x0, ay = ym - y0, bx = xl - xm, by = yl - ym, cx = xl - x0, cy = yl - y0;
  const double cross = ax * by - ay * bx;
  const double la = std::sqrt(ax * ax + ay * ay), lb = std::sqrt(bx * bx + by * by), lc = std::sqrt(cx * cx + cy * cy);
  if (!(la > 0.0 && lb > 0.0 && lc > 0.0)) return 1;
  const double kap = 2.0 * cross / (la * lb * lc);
  const double u = 0.5 * kap * lc;
  if (!(std::fabs(u) < 1.0)) return 1;
  const double phi0 = std::atan2(cy, cx) - std::asin(u);
  const double s0l = lc * asin_over(u);
  double qpt = bk != 0.0 ? kap / bk : 0.0;
  qpt = std::min(cfg.seed_qpt_max, std::max(-cfg.seed_qpt_max, qpt));
  p[0] = y0;
  p[1] = z0;
  p[2] = std::sin(phi0);
  p[3] = (zl - z0) / s0l;
  p[4] = qpt;
  if (!(std::cos(phi0) > 0.0) || !(std::fabs(p[2]) < cfg.s_max)) return 1;
  return 0;
}

// Grid search in row sr around (yp, zp) with variances (sy2, sz2); C5.3 rule.
int32_t search(const orc_run* r, uint32_t sr, double yp, double zp, double sy2, double sz2) {
  const orc_config& c = r->cfg;
  const double wy = std::min(c.gate_nsigma * std::sqrt(sy2), c.win_cap);
  const double wz = std::min(c.gate_nsigma * std::sqrt(sz2), c.win_cap);
  const float ylo = (float)(yp - wy) - kWinPad, yhi = (float)(yp + wy) + kWinPad;
  const float zlo = (float)(zp - wz) - kWinPad, zhi = (float)(zp + wz) + kWinPad;
  int32_t best = -1;
  double bd = 0.0;
  for_range(r, sr, ylo, yhi, zlo, zhi, [&](uint32_t p) {
    const double dy = r->sy[p] - yp, dz = r->sz[p] - zp;
    if (!(std::fabs(dy) <= wy && std::fabs(dz) <= wz)) return;
    const double d = dy * dy / sy2 + dz * dz / sz2;
    if (best < 0 || d < bd || (d == bd && (int32_t)p < best)) {
      best = (int32_t)p;
      bd = d;
    }
  });
  return best;
}

struct Track5 {
  double p[5];
  double C[15];
};

bool prop_step(const orc_run* r, Track5& t, double x1, double x2) {
  double q[5], F[5][5];
  if (propagate(t.p, x1, x2, r->bk, r->cfg.s_max, q, F)) return false;
  std::memcpy(t.p, q, sizeof q);
  transport_cov(t.C, F);
  return true;
}

// C5 for start index i.
void construct_one(orc_run* r, uint32_t i) {
  const orc_config& c = r->cfg;
  const uint32_t R = r->R;
  const uint32_t sr0 = r->start_row[i];
  const uint32_t sec = sr0 / R, r0 = sr0 % R;
  const uint32_t srb = sec * R;
  int32_t* hit = &r->tk_rowhit[(size_t)i * R];
  for (uint32_t k = 0; k < R; ++k) hit[k] = -1;
  r->tk_nhits[i] = 0;
  // chain walk
  std::vector<int32_t> chain;
  for (int32_t p = (int32_t)r->starts[i]; p >= 0; p = r->up1[p]) chain.push_back(p);
  const uint32_t n = (uint32_t)chain.size();
  const uint32_t m = (n - 1) / 2;
  const uint32_t rl = r0 + n - 1;
  Track5 t;
  const double vy = c.sigma_y * c.sigma_y, vz = c.sigma_z * c.sigma_z;
  if (seed3(c, r->bk, r->rc[r0].X, r->sy[chain[0]], r->sz[chain[0]], r->rc[r0 + m].X, r->sy[chain[m]],
            r->rc[rl].X, r->sy[chain[n - 1]], r->sz[chain[n - 1]], t.p)) {
    r->tk_nhits[i] = -1;
    return;
  }
  set_c0(c, t.C);
  hit[r0] = chain[0];
  for (uint32_t j = 1; j < n; ++j) {     // C5.2: chain hits, no gating
    if (!prop_step(r, t, r->rc[r0 + j - 1].X, r->rc[r0 + j].X)) {
      r->tk_nhits[i] = -2;
      return;
    }
    kf_update(t.p, t.C, r->sy[chain[j]], r->sz[chain[j]], vy, vz, nullptr);
    hit[r0 + j] = chain[j];
  }
  // C5.3: extend upward
  double pout[5];
  std::memcpy(pout, t.p, sizeof pout);
  uint32_t rout = rl;
  int miss = 0;
  for (uint32_t row = rl + 1; row < R; ++row) {
    if (!prop_step(r, t, r->rc[row - 1].X, r->rc[row].X)) break;
    if (std::fabs(t.p[0]) > r->rc[row].Y + c.edge_margin) break;
    int32_t h = search(r, srb + row, t.p[0], t.p[1], t.C[tri(0, 0)] + vy, t.C[tri(1, 1)] + vz);
    if (h >= 0) {
      kf_update(t.p, t.C, r->sy[h], r->sz[h], vy, vz, nullptr);
      hit[row] = h;
      std::memcpy(pout, t.p, sizeof pout);
      rout = row;
      miss = 0;
    } else if (++miss > c.max_miss) {
      break;
    }
  }
  // C5.4: downward refit from the outermost hit with a fresh covariance
  std::vector<int32_t> fin(R, -1);
  // the outermost hit itself is the prior for (y, z), like the seed's first hit
  std::memcpy(t.p, pout, sizeof pout);
  t.p[0] = r->sy[hit[rout]];
  t.p[1] = r->sz[hit[rout]];
  set_c0(c, t.C);
  double chi2 = 0.0;
  fin[rout] = hit[rout];
  int nh = 1;
  Track5 snap = t;
  uint32_t rin = rout;
  miss = 0;
  for (int row = (int)rout - 1; row >= 0; --row) {
    if (!prop_step(r, t, r->rc[row + 1].X, r->rc[row].X)) break;
    const bool below = (uint32_t)row < r0;
    if (below && std::fabs(t.p[0]) > r->rc[row].Y + c.edge_margin) break;
    int32_t h = hit[row];
    if (h < 0) h = search(r, srb + row, t.p[0], t.p[1], t.C[tri(0, 0)] + vy, t.C[tri(1, 1)] + vz);
    if (h >= 0) {
      kf_update(t.p, t.C, r->sy[h], r->sz[h], vy, vz, &chi2);
      fin[row] = h;
      ++nh;
      snap = t;
      rin = (uint32_t)row;
      if (below) miss = 0;
    } else if (below && ++miss > c.max_miss) {
      break;
    }
  }
  // C5.5
  for (uint32_t k = 0; k < R; ++k) hit[k] = fin[k];
  r->tk_nhits[i] = nh;
  r->tk_xref[i] = (int32_t)rin;
  std::memcpy(&r->tk_param[(size_t)i * 5], snap.p, 5 * sizeof(double));
  std::memcpy(&r->tk_cov[(size_t)i * 15], snap.C, 15 * sizeof(double));
  r->tk_chi2[i] = chi2;
}

}  // namespace

extern "C" {

orc_run* orc_run_create(const orc_config* cfg, uint32_t n_sectors, const uint32_t* row_offsets, const double* y,
                        const double* z, const float* sector_z_lo, const float* sector_z_hi) {
  orc_run* r = new orc_run();
  r->cfg = *cfg;
  r->S = n_sectors;
  r->R = (uint32_t)cfg->n_rows;
  const uint32_t SR = r->S * r->R;
  r->off.assign(row_offsets, row_offsets + SR + 1);
  r->y = y;
  r->z = z;
  r->bk = -kCB * cfg->bz;
  const double ry = cfg->sigma_y / cfg->sigma_z;
  r->rho = (float)(ry * ry);
  r->rc.resize(r->R);
  for (uint32_t k = 0; k < r->R; ++k) {
    RowC& c = r->rc[k];
    c.X = cfg->row_x[k];
    c.Y = cfg->row_half_y[k];
    c.y_lo = (float)(-c.Y);
    c.inv_wy = (float)(1.0 / (2.0 * c.Y));
    c.ly = (int64_t)std::ceil(20.0 * c.Y);
    c.t = c.wy_up = c.wz_up = c.wy_dn = c.wz_dn = c.dmax = 0.0f;
    if (k >= 1 && k + 1 < r->R) {
      const double du = cfg->row_x[k + 1] - cfg->row_x[k];
      const double dd = cfg->row_x[k] - cfg->row_x[k - 1];
      const double t = dd / (dd + du);
      c.t = (float)t;
      c.wy_up = (float)(cfg->win_a_y * du + cfg->win_b_y);
      c.wz_up = (float)(cfg->win_a_z * du + cfg->win_b_z);
      c.wy_dn = (float)(cfg->win_a_y * dd + cfg->win_b_y);
      c.wz_dn = (float)(cfg->win_a_z * dd + cfg->win_b_z);
      const double n2 = cfg->link_nsigma * cfg->link_nsigma;
      const double s2 = cfg->sigma_y * cfg->sigma_y;
      c.dmax = (float)((n2 * s2) * ((1.0 + t * t) + (1.0 - t) * (1.0 - t)));
    }
  }
  r->zlo.resize(r->S);
  r->zhi.resize(r->S);
  r->inv_wz.resize(r->S);
  r->lz.resize(r->S);
  for (uint32_t s = 0; s < r->S; ++s) {
    r->zlo[s] = sector_z_lo[s];
    r->zhi[s] = sector_z_hi[s];
    const double w = (double)sector_z_hi[s] - (double)sector_z_lo[s];
    r->inv_wz[s] = (float)(1.0 / w);
    r->lz[s] = (int64_t)std::ceil(10.0 * w);
  }
  return r;
}

void orc_run_destroy(orc_run* r) { delete r; }

// A run holding only given tracklets, for step C6 on its own: cluster ids
// equal sorted positions, one sector.
orc_run* orc_run_from_tracklets(const orc_config* cfg, uint32_t n_clusters, uint64_t n_tracklets, const int32_t* nhits,
                                const uint32_t* start_pos, const int32_t* rowhit) {
  orc_run* r = new orc_run();
  r->cfg = *cfg;
  r->S = 1;
  r->R = (uint32_t)cfg->n_rows;
  r->off.assign(r->R + 1, 0);
  r->off[r->R] = n_clusters;
  r->y = r->z = nullptr;
  r->sorted_id.resize(n_clusters);
  for (uint32_t i = 0; i < n_clusters; ++i) r->sorted_id[i] = i;
  r->starts.assign(start_pos, start_pos + n_tracklets);
  r->tk_nhits.assign(nhits, nhits + n_tracklets);
  r->tk_rowhit.assign(rowhit, rowhit + n_tracklets * r->R);
  return r;
}

// C1: per (sector, row) grid dimensions, bins and stable counting order.
int orc_run_grid(orc_run* r) {
  const uint32_t SR = r->S * r->R, N = r->off[SR];
  r->sorted_id.assign(N, 0);
  r->sy.assign(N, 0.0);
  r->sz.assign(N, 0.0);
  r->fy.assign(N, 0.0f);
  r->fz.assign(N, 0.0f);
  r->bin_start.assign((size_t)N + 2 * SR, 0xFFFFFFFFu);
  r->dims.assign(SR, 0);
  std::vector<uint32_t> idx, key;
  for (uint32_t sr = 0; sr < SR; ++sr) {
    const uint32_t s = sr / r->R, row = sr % r->R;
    const uint32_t a = r->off[sr], nr = r->off[sr + 1] - a;
    const RowC& c = r->rc[row];
    int ny, nz;
    grid_dims(nr, r->cfg.grid_hits_per_bin, c.ly, r->lz[s], &ny, &nz);
    r->dims[sr] = (uint32_t)ny | ((uint32_t)nz << 16);
    idx.resize(nr);
    key.resize(nr);
    for (uint32_t j = 0; j < nr; ++j) {
      const float fy = (float)r->y[a + j], fz = (float)r->z[a + j];
      const int iy = bin1(fy, c.y_lo, c.inv_wy, ny);
      const int iz = bin1(fz, r->zlo[s], r->inv_wz[s], nz);
      key[j] = (uint32_t)(iz * ny + iy);
      idx[j] = j;
    }
    std::stable_sort(idx.begin(), idx.end(), [&](uint32_t u, uint32_t v) { return key[u] < key[v]; });
    const uint32_t nb = (uint32_t)(ny * nz);
    const uint32_t base = bin_base(r, sr);
    uint32_t j = 0;
    for (uint32_t b = 0; b <= nb; ++b) {
      while (j < nr && key[idx[j]] < b) ++j;
      r->bin_start[base + b] = a + j;
    }
    for (uint32_t j2 = 0; j2 < nr; ++j2) {
      const uint32_t p = a + j2, id = a + idx[j2];
      r->sorted_id[p] = id;
      r->sy[p] = r->y[id];
      r->sz[p] = r->z[id];
      r->fy[p] = (float)r->y[id];
      r->fz[p] = (float)r->z[id];
    }
  }
  return 0;
}

}  // extern "C"

namespace {

// C2 + C3.  The decisions of C2 are taken in float32 (as the definition
// fixes them) unless fp64 is set: then windows, cut and deviation are
// evaluated in double from the same coordinates, which shows how far the
// float32 rule departs from an FP64 one (only at near-ties).
int links_impl(orc_run* r, bool fp64) {
  const uint32_t SR = r->S * r->R, N = r->off[SR], R = r->R;
  const orc_config& cfg = r->cfg;
  r->up0.assign(N, -1);
  r->down0.assign(N, -1);
  std::vector<uint32_t> U, D;
  const double rho64 = (cfg.sigma_y / cfg.sigma_z) * (cfg.sigma_y / cfg.sigma_z);
  for (uint32_t sr = 0; sr < SR; ++sr) {
    const uint32_t row = sr % R;
    if (row == 0 || row + 1 >= R) continue;
    const RowC& c = r->rc[row];
    // double-precision constants of the row (used when fp64)
    const double du = cfg.row_x[row + 1] - cfg.row_x[row], dd = cfg.row_x[row] - cfg.row_x[row - 1];
    const double t64 = dd / (dd + du);
    const double wyu = cfg.win_a_y * du + cfg.win_b_y, wzu = cfg.win_a_z * du + cfg.win_b_z;
    const double wyd = cfg.win_a_y * dd + cfg.win_b_y, wzd = cfg.win_a_z * dd + cfg.win_b_z;
    const double dmax64 = (cfg.link_nsigma * cfg.link_nsigma * cfg.sigma_y * cfg.sigma_y) *
                          ((1.0 + t64 * t64) + (1.0 - t64) * (1.0 - t64));
    for (uint32_t p = r->off[sr]; p < r->off[sr + 1]; ++p) {
      const float yh = r->fy[p], zh = r->fz[p];
      const double yh64 = r->sy[p], zh64 = r->sz[p];
      auto in_up = [&](uint32_t q) {
        if (fp64) return std::fabs(r->sy[q] - yh64) <= wyu && std::fabs(r->sz[q] - zh64) <= wzu;
        const float dy = r->fy[q] - yh, dz = r->fz[q] - zh;
        return std::fabs(dy) <= c.wy_up && std::fabs(dz) <= c.wz_up;
      };
      auto in_dn = [&](uint32_t q) {
        if (fp64) return std::fabs(r->sy[q] - yh64) <= wyd && std::fabs(r->sz[q] - zh64) <= wzd;
        const float dy = r->fy[q] - yh, dz = r->fz[q] - zh;
        return std::fabs(dy) <= c.wy_dn && std::fabs(dz) <= c.wz_dn;
      };
      U.clear();
      D.clear();
      for_range(r, sr + 1, yh - (c.wy_up + kWinPad), yh + (c.wy_up + kWinPad), zh - (c.wz_up + kWinPad),
                zh + (c.wz_up + kWinPad), [&](uint32_t q) {
                  if (in_up(q)) U.push_back(q);
                });
      if (U.empty()) continue;
      for_range(r, sr - 1, yh - (c.wy_dn + kWinPad), yh + (c.wy_dn + kWinPad), zh - (c.wz_dn + kWinPad),
                zh + (c.wz_dn + kWinPad), [&](uint32_t q) {
                  if (in_dn(q)) D.push_back(q);
                });
      int32_t bu = -1, bd = -1;
      double best = 0.0;
      for (uint32_t d : D)
        for (uint32_t u : U) {
          double dev;
          if (fp64) {
            const double yp = r->sy[d] + t64 * (r->sy[u] - r->sy[d]);
            const double zp = r->sz[d] + t64 * (r->sz[u] - r->sz[d]);
            const double ey = yh64 - yp, ez = zh64 - zp;
            dev = ey * ey + rho64 * (ez * ez);
            if (!(dev <= dmax64)) continue;
          } else {
            const float yp = r->fy[d] + c.t * (r->fy[u] - r->fy[d]);
            const float zp = r->fz[d] + c.t * (r->fz[u] - r->fz[d]);
            const float ey = yh - yp, ez = zh - zp;
            const float devf = ey * ey + r->rho * (ez * ez);
            if (!(devf <= c.dmax)) continue;
            dev = devf;
          }
          if (bu < 0 || dev < best || (dev == best && ((int32_t)u < bu || ((int32_t)u == bu && (int32_t)d < bd)))) {
            best = dev;
            bu = (int32_t)u;
            bd = (int32_t)d;
          }
        }
      r->up0[p] = bu;
      r->down0[p] = bd;
    }
  }
  r->up1.assign(N, -1);
  r->down1.assign(N, -1);
  for (uint32_t h = 0; h < N; ++h) {
    const int32_t u = r->up0[h], d = r->down0[h];
    if (u >= 0 && r->down0[u] == (int32_t)h) r->up1[h] = u;
    if (d >= 0 && r->up0[d] == (int32_t)h) r->down1[h] = d;
  }
  return 0;
}

}  // namespace

extern "C" {

int orc_run_links(orc_run* r) { return links_impl(r, false); }
int orc_run_links_fp64(orc_run* r) { return links_impl(r, true); }

// C4: chain starts in ascending sorted position (= sector, row, grid order).
int orc_run_starts(orc_run* r) {
  const uint32_t SR = r->S * r->R;
  r->starts.clear();
  r->start_row.clear();
  for (uint32_t sr = 0; sr < SR; ++sr)
    for (uint32_t h = r->off[sr]; h < r->off[sr + 1]; ++h) {
      const int32_t u = r->up1[h];
      if (r->down1[h] == -1 && u >= 0 && r->up1[u] >= 0) {
        r->starts.push_back(h);
        r->start_row.push_back(sr);
      }
    }
  const size_t T = r->starts.size();
  r->tk_rowhit.assign(T * r->R, -1);
  r->tk_nhits.assign(T, 0);
  r->tk_xref.assign(T, -1);
  r->tk_param.assign(T * 5, 0.0);
  r->tk_cov.assign(T * 15, 0.0);
  r->tk_chi2.assign(T, 0.0);
  return 0;
}

int orc_run_construct(orc_run* r, const uint32_t* which, uint64_t n_which) {
  const uint64_t T = r->starts.size();
  if (!which) {
    for (uint64_t i = 0; i < T; ++i) construct_one(r, (uint32_t)i);
  } else {
    for (uint64_t k = 0; k < n_which; ++k)
      if (which[k] < T) construct_one(r, which[k]);
  }
  return 0;
}

// C6 + C7.
int orc_run_select(orc_run* r) {
  const uint32_t SR = r->S * r->R, N = r->off[SR], R = r->R;
  const uint64_t T = r->starts.size();
  const int minh = r->cfg.min_tracklet_hits;
  std::vector<uint64_t> W(N, 0);
  auto key = [&](uint64_t i) {
    return ((uint64_t)(uint32_t)r->tk_nhits[i] << 32) | (uint64_t)(0xFFFFFFFFu - r->starts[i]);
  };
  for (uint64_t i = 0; i < T; ++i) {
    if (r->tk_nhits[i] < minh) continue;
    const uint64_t k = key(i);
    for (uint32_t row = 0; row < R; ++row) {
      const int32_t h = r->tk_rowhit[i * R + row];
      if (h >= 0) W[h] = std::max(W[h], k);
    }
  }
  r->trk_tracklet.clear();
  r->trk_first.assign(1, 0);
  r->trk_clusters.clear();
  for (uint64_t i = 0; i < T; ++i) {
    if (r->tk_nhits[i] < minh) continue;
    const uint64_t k = key(i);
    uint32_t owned = 0;
    for (uint32_t row = 0; row < R; ++row) {
      const int32_t h = r->tk_rowhit[i * R + row];
      if (h >= 0 && W[h] == k) ++owned;
    }
    const float need = (float)r->cfg.min_owned_frac * (float)r->tk_nhits[i];
    if ((int)owned < r->cfg.min_track_hits || !((float)owned >= need)) continue;
    r->trk_tracklet.push_back((uint32_t)i);
    for (uint32_t row = 0; row < R; ++row) {
      const int32_t h = r->tk_rowhit[i * R + row];
      if (h >= 0 && W[h] == k) r->trk_clusters.push_back(r->sorted_id[h]);
    }
    r->trk_first.push_back((uint32_t)r->trk_clusters.size());
  }
  return 0;
}

// ---------------------------------------------------------------------------
// C8 sector merger and C9 refit of merged chains (on the C7 tracks of a run).
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

constexpr double kPi = 3.14159265358979323846;

// Rotation of a state at x from the frame of azimuth a into the frame of
// azimuth a + d, at the same point in space, with its first-order Jacobian on
// the new plane x' = const through that point (C8.1).  Fails unless the track
// moves outward in the new frame (cos phi' > 0).
bool rotate(double x, const double* p, double d, double bk, double* xo, double* q, double J[5][5]) {
  const double cd = std::cos(d), sd = std::sin(d);
  const double s = p[2], c = std::sqrt((1.0 - s) * (1.0 + s));
  const double s2 = s * cd - c * sd, c2 = c * cd + s * sd;   // sin, cos of phi - d
  if (!(c2 > 0.0)) return false;
  *xo = x * cd + p[0] * sd;
  q[0] = -x * sd + p[0] * cd;
  q[1] = p[1];
  q[2] = s2;
  q[3] = p[3];
  q[4] = p[4];
  if (J) {
    for (int i = 0; i < 5; ++i)
      for (int j = 0; j < 5; ++j) J[i][j] = (i == j) ? 1.0 : 0.0;
    J[0][0] = c / c2;
    J[1][0] = -p[3] * sd / c2;
    J[2][0] = -bk * p[4] * sd;
    J[2][2] = c2 / c;
  }
  return true;
}

double radius_of(double x, double y) { return std::sqrt(x * x + y * y); }

struct MergeTrack {
  uint32_t sector;       // index in the run
  int32_t phys;          // physical sector 0..35, -1: no neighbours
  double x;              // x_ref
  double p[5], C[15];
  double r_in;           // global radius of the innermost point
  uint32_t first, n;     // clusters in trk_clusters
};

}  // namespace

struct orc_merge {
  std::vector<int32_t> next, prev, head;       // per track: successor, predecessor, chain head
  std::vector<uint32_t> heads;                 // chain heads in ascending track index
  std::vector<double> param, cov, chi2;        // per head: refit result (single-segment chains: C5 result)
  std::vector<int32_t> ndf, nseg;
  std::vector<uint32_t> first, clusters;       // per head: merged cluster list (input ids, chain order)
};

namespace {

// C8.2 match score of t followed by u (both tracks of the run); false if no match.
bool match_pair(const orc_run* r, const MergeTrack& a, const MergeTrack& b, double* score) {
  const orc_config& c = r->cfg;
  if (!(b.r_in > a.r_in)) return false;
  const int side_a = a.phys / 18, side_b = b.phys / 18;
  if (side_a != side_b) return false;
  const int ia = a.phys % 18, ib = b.phys % 18;
  int step = ib - ia;
  if (step == 17) step = -1;
  if (step == -17) step = 1;
  if (step != 1 && step != -1) return false;
  double xr, q[5];
  if (!rotate(a.x, a.p, step * (20.0 * kPi / 180.0), r->bk, &xr, q, nullptr)) return false;
  double q2[5];
  if (propagate(q, xr, b.x, r->bk, c.s_max, q2, nullptr)) return false;
  const double dy = q2[0] - b.p[0], dz = q2[1] - b.p[1];
  if (!(std::fabs(dy) <= c.merge_dy && std::fabs(dz) <= c.merge_dz && std::fabs(q2[2] - b.p[2]) <= c.merge_dsinphi &&
        std::fabs(q2[3] - b.p[3]) <= c.merge_dtanl && std::fabs(q2[4] - b.p[4]) <= c.merge_dqpt))
    return false;
  *score = dy * dy / (b.C[tri(0, 0)] + c.sigma_y * c.sigma_y) + dz * dz / (b.C[tri(1, 1)] + c.sigma_z * c.sigma_z);
  return true;
}

}  // namespace

extern "C" {

orc_merge* orc_merge_run(orc_run* r, const int32_t* sector_phys) {
  orc_merge* m = new orc_merge();
  const orc_config& c = r->cfg;
  const uint32_t R = r->R, nt = (uint32_t)r->trk_tracklet.size();
  std::vector<MergeTrack> T(nt);
  for (uint32_t k = 0; k < nt; ++k) {
    const uint32_t i = r->trk_tracklet[k];
    MergeTrack& t = T[k];
    t.sector = r->start_row[i] / R;
    t.phys = sector_phys ? sector_phys[t.sector] : -1;
    t.x = r->rc[r->tk_xref[i]].X;
    std::memcpy(t.p, &r->tk_param[(size_t)i * 5], 5 * sizeof(double));
    std::memcpy(t.C, &r->tk_cov[(size_t)i * 15], 15 * sizeof(double));
    t.r_in = radius_of(t.x, t.p[0]);
    t.first = r->trk_first[k];
    t.n = r->trk_first[k + 1] - r->trk_first[k];
  }
  // C8.3 mutual best: each track's best successor and best predecessor
  std::vector<int32_t> succ(nt, -1), pred(nt, -1);
  std::vector<double> s_succ(nt, 0.0), s_pred(nt, 0.0);
  for (uint32_t a = 0; a < nt; ++a) {
    if (T[a].phys < 0) continue;
    for (uint32_t b = 0; b < nt; ++b) {
      if (b == a || T[b].phys < 0) continue;
      double sc;
      if (!match_pair(r, T[a], T[b], &sc)) continue;
      if (succ[a] < 0 || sc < s_succ[a] || (sc == s_succ[a] && (int32_t)b < succ[a])) {
        succ[a] = (int32_t)b;
        s_succ[a] = sc;
      }
      if (pred[b] < 0 || sc < s_pred[b] || (sc == s_pred[b] && (int32_t)a < pred[b])) {
        pred[b] = (int32_t)a;
        s_pred[b] = sc;
      }
    }
  }
  m->next.assign(nt, -1);
  m->prev.assign(nt, -1);
  for (uint32_t a = 0; a < nt; ++a)
    if (succ[a] >= 0 && pred[succ[a]] == (int32_t)a) {
      m->next[a] = succ[a];
      m->prev[succ[a]] = (int32_t)a;
    }
  // C9 chains from their heads, refit of chains of two or more segments
  std::vector<int32_t> pos_of(r->sorted_id.size());
  for (uint32_t p = 0; p < r->sorted_id.size(); ++p) pos_of[r->sorted_id[p]] = (int32_t)p;
  m->head.assign(nt, -1);
  m->first.assign(1, 0);
  const double vy = c.sigma_y * c.sigma_y, vz = c.sigma_z * c.sigma_z;
  for (uint32_t h = 0; h < nt; ++h) {
    if (m->prev[h] >= 0) continue;
    std::vector<uint32_t> chain;
    for (int32_t k = (int32_t)h; k >= 0; k = m->next[k]) {
      chain.push_back((uint32_t)k);
      m->head[k] = (int32_t)h;
    }
    m->heads.push_back(h);
    m->nseg.push_back((int32_t)chain.size());
    for (uint32_t k : chain)
      for (uint32_t j = 0; j < T[k].n; ++j) m->clusters.push_back(r->trk_clusters[T[k].first + j]);
    m->first.push_back((uint32_t)m->clusters.size());
    double P[5], Cv[15], chi2 = 0.0;
    int ndf = 2 * (int)(m->first.back() - m->first[m->first.size() - 2]) - 5;
    std::memcpy(P, T[h].p, sizeof P);
    std::memcpy(Cv, T[h].C, sizeof Cv);
    chi2 = r->tk_chi2[r->trk_tracklet[h]];
    if (chain.size() > 1) {
      // the clusters of the chain (each segment's own clusters, ascending row) with row and position
      struct Hit { uint32_t seg, row; int32_t pos; };
      std::vector<Hit> hits;
      for (uint32_t k : chain)
        for (uint32_t j = 0; j < T[k].n; ++j) {
          const uint32_t id = r->trk_clusters[T[k].first + j];
          const uint32_t sr = (uint32_t)(std::upper_bound(r->off.begin(), r->off.end(), id) - r->off.begin()) - 1;
          hits.push_back(Hit{k, sr % R, pos_of[id]});
        }
      // hits are in chain order, ascending row inside a segment; walk them backwards
      const MergeTrack& last = T[chain.back()];
      double q[5], x = last.x;
      std::memcpy(q, last.p, sizeof q);
      const Hit& ho = hits.back();
      double q2[5];
      bool ok = propagate(q, x, r->rc[ho.row].X, r->bk, c.s_max, q2, nullptr) == 0;
      if (ok) {
        std::memcpy(q, q2, sizeof q);
        q[0] = r->sy[ho.pos];
        q[1] = r->sz[ho.pos];
        x = r->rc[ho.row].X;
        Track5 t;
        std::memcpy(t.p, q, sizeof q);
        set_c0(c, t.C);
        chi2 = 0.0;
        uint32_t seg = ho.seg;
        for (int k = (int)hits.size() - 2; k >= 0 && ok; --k) {
          const Hit& hh = hits[k];
          if (hh.seg != seg) {   // into the previous segment's frame
            const int dphys = T[hh.seg].phys % 18 - T[seg].phys % 18;
            int step = dphys;
            if (step == 17) step = -1;
            if (step == -17) step = 1;
            double xr, qr[5], J[5][5];
            ok = rotate(x, t.p, step * (20.0 * kPi / 180.0), r->bk, &xr, qr, J);
            if (!ok) break;
            std::memcpy(t.p, qr, sizeof qr);
            transport_cov(t.C, J);
            x = xr;
            seg = hh.seg;
          }
          ok = prop_step(r, t, x, r->rc[hh.row].X);
          if (!ok) break;
          x = r->rc[hh.row].X;
          kf_update(t.p, t.C, r->sy[hh.pos], r->sz[hh.pos], vy, vz, &chi2);
        }
        if (ok) {
          std::memcpy(P, t.p, sizeof P);
          std::memcpy(Cv, t.C, sizeof Cv);
        }
      }
      if (!ok) ndf = -1;
    }
    for (int q = 0; q < 5; ++q) m->param.push_back(P[q]);
    for (int q = 0; q < 15; ++q) m->cov.push_back(Cv[q]);
    m->chi2.push_back(chi2);
    m->ndf.push_back(ndf);
  }
  return m;
}

void orc_merge_destroy(orc_merge* m) { delete m; }

uint64_t orc_merge_get(orc_merge* m, int what, void* dst, uint64_t cap) {
  const void* src = nullptr;
  uint64_t bytes = 0;
  switch (what) {
#define ORC_MCASE(id, vec)                      \
  case id:                                      \
    src = m->vec.data();                        \
    bytes = m->vec.size() * sizeof(m->vec[0]);  \
    break;
    ORC_MCASE(ORC_M_NEXT, next)
    ORC_MCASE(ORC_M_HEAD, head)
    ORC_MCASE(ORC_M_HEADS, heads)
    ORC_MCASE(ORC_M_NSEG, nseg)
    ORC_MCASE(ORC_M_PARAM, param)
    ORC_MCASE(ORC_M_COV, cov)
    ORC_MCASE(ORC_M_CHI2, chi2)
    ORC_MCASE(ORC_M_NDF, ndf)
    ORC_MCASE(ORC_M_FIRST, first)
    ORC_MCASE(ORC_M_CLUSTERS, clusters)
#undef ORC_MCASE
    default:
      return 0;
  }
  if (dst && src) std::memcpy(dst, src, std::min(cap, bytes));
  return bytes;
}

int orc_rotate(double x, const double* p_in, double d, double bz, double* x_out, double* p_out, double* J) {
  double Jm[5][5];
  if (!rotate(x, p_in, d, -kCB * bz, x_out, p_out, Jm)) return 1;
  if (J)
    for (int i = 0; i < 5; ++i)
      for (int j = 0; j < 5; ++j) J[i * 5 + j] = Jm[i][j];
  return 0;
}

uint64_t orc_get(orc_run* r, int what, void* dst, uint64_t cap) {
  const void* src = nullptr;
  uint64_t bytes = 0;
  uint64_t sizes[4];
  switch (what) {
#define ORC_CASE(id, vec)                       \
  case id:                                      \
    src = r->vec.data();                        \
    bytes = r->vec.size() * sizeof(r->vec[0]);  \
    break;
    ORC_CASE(ORC_SORTED_ID, sorted_id)
    ORC_CASE(ORC_BIN_START, bin_start)
    ORC_CASE(ORC_ROW_DIMS, dims)
    ORC_CASE(ORC_UP0, up0)
    ORC_CASE(ORC_DOWN0, down0)
    ORC_CASE(ORC_UP1, up1)
    ORC_CASE(ORC_DOWN1, down1)
    ORC_CASE(ORC_STARTS, starts)
    ORC_CASE(ORC_TK_ROWHIT, tk_rowhit)
    ORC_CASE(ORC_TK_NHITS, tk_nhits)
    ORC_CASE(ORC_TK_PARAM, tk_param)
    ORC_CASE(ORC_TK_COV, tk_cov)
    ORC_CASE(ORC_TK_XREF_ROW, tk_xref)
    ORC_CASE(ORC_TK_CHI2, tk_chi2)
    ORC_CASE(ORC_TRK_TRACKLET, trk_tracklet)
    ORC_CASE(ORC_TRK_FIRST, trk_first)
    ORC_CASE(ORC_TRK_CLUSTERS, trk_clusters)
#undef ORC_CASE
    case ORC_SIZES:
      sizes[0] = r->off[r->S * r->R];
      sizes[1] = r->starts.size();
      sizes[2] = r->trk_tracklet.size();
      sizes[3] = r->trk_clusters.size();
      src = sizes;
      bytes = sizeof sizes;
      break;
    default:
      return 0;
  }
  if (dst && src) std::memcpy(dst, src, std::min(cap, bytes));
  return bytes;
}

int orc_propagate(const double* p_in, double x1, double x2, double bz, double s_max, double* p_out, double* F) {
  double Fm[5][5];
  const int rc = propagate(p_in, x1, x2, -kCB * bz, s_max, p_out, Fm);
  if (F && rc == 0)
    for (int i = 0; i < 5; ++i)
      for (int j = 0; j < 5; ++j) F[i * 5 + j] = Fm[i][j];
  return rc;
}

int orc_propagate_cov(const double* p_in, const double* c_in, double x1, double x2, double bz, double s_max,
                      double* p_out, double* c_out) {
  double Fm[5][5];
  const int rc = propagate(p_in, x1, x2, -kCB * bz, s_max, p_out, Fm);
  if (rc) return rc;
  for (int i = 0; i < 15; ++i) c_out[i] = c_in[i];
  transport_cov(c_out, Fm);
  return 0;
}

void orc_kf_update(double* p, double* C, double ym, double zm, double vy, double vz, double* chi2) {
  kf_update(p, C, ym, zm, vy, vz, chi2);
}

int orc_seed(const orc_config* cfg, double x0, double y0, double z0, double xm, double ym, double xl, double yl,
             double zl, double* p_out) {
  return seed3(*cfg, -kCB * cfg->bz, x0, y0, z0, xm, ym, xl, yl, zl, p_out);
}

void orc_bin(float y, float z, float y_lo, float inv_wy, float z_lo, float inv_wz, int ny, int nz, int* iy, int* iz) {
  *iy = bin1(y, y_lo, inv_wy, ny);
  *iz = bin1(z, z_lo, inv_wz, nz);
}

void orc_grid_dims(uint32_t n_hits, int k, int64_t ly_mm, int64_t lz_mm, int* ny, int* nz) {
  grid_dims(n_hits, k, ly_mm, lz_mm, ny, nz);
}

}  // extern "C"
