// Track-model compression oracle, steps C10 and C11 (definition in tpc_codec.h).
// TEST INFRASTRUCTURE ONLY: see tpc_codec.h.
//
// Written as the definition reads, one track and one cluster at a time.  The
// float32 steps are float32 operations in the stated order; the build turns
// floating-point contraction off, so no multiply-add is fused.
#include "tpc_codec.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace {

constexpr double kCB = 0.00299792458;   // GeV / (T cm)
constexpr int16_t kEscape = -32768;

// Row of input cluster id: the (sector, row) slot whose offsets contain it.
uint32_t row_of(uint64_t id, const uint32_t* row_offsets, uint32_t n_sr, int32_t n_rows) {
  const uint32_t* hi = std::upper_bound(row_offsets, row_offsets + n_sr + 1, (uint32_t)id);
  const uint32_t sr = (uint32_t)(hi - row_offsets) - 1;
  return sr % (uint32_t)n_rows;
}

// Model prediction at row radius xr for one axis: c0 + u * (c1 + u * c2), u = xr - x_ref, float32.
float predict(float xr, float x_ref, float c0, float c1, float c2) {
  const float u = xr - x_ref;
  const float inner = c1 + u * c2;
  const float outer = u * inner;
  return c0 + outer;
}

}  // namespace

extern "C" {

int orc_codec_coef(const float* param, double bz, float* coef) {
  const double y = param[0], z = param[1], s = param[2], T = param[3], qpt = param[4];
  if (!(std::fabs(s) < 1.0)) return 1;
  const double kappa = (-kCB * bz) * qpt;
  const double c = std::sqrt(1.0 - s * s);
  const double ic = 1.0 / c;
  const double ic3 = ic * ic * ic;
  coef[0] = (float)y;
  coef[1] = (float)(s * ic);
  coef[2] = (float)(0.5 * kappa * ic3);
  coef[3] = (float)z;
  coef[4] = (float)(T * ic);
  coef[5] = (float)(((0.5 * T) * s) * kappa * ic3);
  return 0;
}

uint64_t orc_codec_encode(int32_t n_rows, const double* row_x, double bz, float q_y, float q_z, uint32_t n_tracks,
                          const uint32_t* first, const uint32_t* ids, const float* x_ref, const float* param,
                          uint64_t n_clusters, const float* y, const float* z, const uint32_t* row_offsets,
                          uint32_t n_sr, float* coef, uint8_t* row, int16_t* code, float* raw, uint8_t* un_row,
                          float* un_yz, uint64_t* n_unassigned) {
  const float inv_qy = (float)(1.0 / (double)q_y), inv_qz = (float)(1.0 / (double)q_z);
  std::vector<char> on_track(n_clusters, 0);
  uint64_t escaped = 0;
  for (uint32_t t = 0; t < n_tracks; ++t) {
    float* a = coef + 6 * (size_t)t;
    if (orc_codec_coef(param + 5 * (size_t)t, bz, a) != 0) {
      for (int q = 0; q < 6; ++q) a[q] = 0.0f;   // no model: every cluster of the track is escaped
    }
    const bool model = std::fabs(param[5 * (size_t)t + 2]) < 1.0f;
    for (uint32_t j = first[t]; j < first[t + 1]; ++j) {
      const uint32_t id = ids[j];
      on_track[id] = 1;
      const uint32_t r = row_of(id, row_offsets, n_sr, n_rows);
      row[j] = (uint8_t)r;
      const float xr = (float)row_x[r];
      const float py = predict(xr, x_ref[t], a[0], a[1], a[2]);
      const float pz = predict(xr, x_ref[t], a[3], a[4], a[5]);
      const float vy = (y[id] - py) * inv_qy;
      const float vz = (z[id] - pz) * inv_qz;
      raw[2 * (size_t)j] = 0.0f;
      raw[2 * (size_t)j + 1] = 0.0f;
      if (model && std::fabs(vy) <= 32767.0f && std::fabs(vz) <= 32767.0f) {
        code[2 * (size_t)j] = (int16_t)std::rint(vy);
        code[2 * (size_t)j + 1] = (int16_t)std::rint(vz);
      } else {
        code[2 * (size_t)j] = kEscape;
        code[2 * (size_t)j + 1] = 0;
        raw[2 * (size_t)j] = y[id];
        raw[2 * (size_t)j + 1] = z[id];
        ++escaped;
      }
    }
  }
  uint64_t nu = 0;
  for (uint64_t id = 0; id < n_clusters; ++id) {
    if (on_track[id]) continue;
    un_row[nu] = (uint8_t)row_of(id, row_offsets, n_sr, n_rows);
    un_yz[2 * nu] = y[id];
    un_yz[2 * nu + 1] = z[id];
    ++nu;
  }
  *n_unassigned = nu;
  return escaped;
}

void orc_codec_decode(int32_t n_rows, const double* row_x, float q_y, float q_z, uint32_t n_tracks,
                      const uint32_t* first, const float* x_ref, const float* coef, const uint8_t* row,
                      const int16_t* code, const float* raw, float* y_out, float* z_out) {
  (void)n_rows;
  for (uint32_t t = 0; t < n_tracks; ++t) {
    const float* a = coef + 6 * (size_t)t;
    for (uint32_t j = first[t]; j < first[t + 1]; ++j) {
      if (code[2 * (size_t)j] == kEscape) {
        y_out[j] = raw[2 * (size_t)j];
        z_out[j] = raw[2 * (size_t)j + 1];
        continue;
      }
      const float xr = (float)row_x[row[j]];
      const float py = predict(xr, x_ref[t], a[0], a[1], a[2]);
      const float pz = predict(xr, x_ref[t], a[3], a[4], a[5]);
      const float dy = (float)code[2 * (size_t)j] * q_y;
      const float dz = (float)code[2 * (size_t)j + 1] * q_z;
      y_out[j] = py + dy;
      z_out[j] = pz + dz;
    }
  }
}

}  // extern "C"
