/*
 * Reference ("oracle") for track-model compression of TPC clusters, steps C10
 * (encoding) and C11 (decoding).
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of this directory: nothing on the
 * product path links, loads or calls it; it shares no code with the HIP
 * library.
 *
 * The paper names TPC data compression as the farm's main task (abstract;
 * Introduction and its table of processing shares) and the track-model
 * decoding as a step ported to the GPU (section on the differences between
 * online and offline processing), but it does not give the format.  This project's
 * definition (the same text is in the library's public header):
 *
 * C10 encoding, per track t of a frame (C7 output: parameters p = (y, z,
 *   sin phi, tan lambda, q/pT) at x_ref, float32 as stored, clusters in
 *   ascending row order):
 *   model coefficients in double, rounded to float32 once:
 *     kappa = (-0.00299792458 * Bz) * (q/pT);  c = sqrt(1 - s*s);  ic = 1 / c;
 *     ic3 = ic * ic * ic;
 *     a0 = y, a1 = s * ic, a2 = 0.5 * kappa * ic3,
 *     b0 = z, b1 = T * ic, b2 = ((0.5 * T) * s) * kappa * ic3
 *   (the second-order expansion of the helix around x_ref in u = x - x_ref);
 *   for each cluster (row r, input coordinates y_m, z_m), in float32, every
 *   operation rounded, no fused multiply-add:
 *     u = X_r - x_ref (X_r = float32(row radius));
 *     p_y = a0 + u * (a1 + u * a2);  p_z = b0 + u * (b1 + u * b2);
 *     v_y = (y_m - p_y) * inv_qy with inv_qy = float32(1 / q_y) (double
 *     division, rounded); likewise v_z;
 *     if |v_y| <= 32767 and |v_z| <= 32767: k_y = rint(v_y), k_z = rint(v_z)
 *     (round half to even), else the cluster is escaped: k_y = -32768 and its
 *     raw (y_m, z_m) is stored.
 *   A track with |sin phi| >= 1 has no model (C5 keeps |sin phi| below
 *   s_max, so this does not occur in practice): its coefficients are 0 and
 *   every cluster of it is escaped.
 *   The stream holds, per track, x_ref and the six coefficients, and per
 *   cluster its row (8 bits) and (k_y, k_z) (16 bits each); clusters on no
 *   track are stored raw (row, y, z) in input order.
 * C11 decoding: y = p_y + k_y * q_y, z = p_z + k_z * q_z (float32, rounded,
 *   no fused multiply-add; q as float32); escaped and unassigned clusters are
 *   their raw values.
 */
#ifndef TPC_CODEC_ORACLE_H
#define TPC_CODEC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Model coefficients (a0, a1, a2, b0, b1, b2) of a track from its stored
 * float32 parameters.  Returns 1 if |sin phi| >= 1 (no model), else 0. */
int orc_codec_coef(const float* param, double bz, float* coef);

/* C10 over a frame.  Tracks: first[n_tracks + 1] offsets into ids (input
 * cluster indices), x_ref[n_tracks], param[5 * n_tracks].  Clusters: y, z in
 * input order; row_offsets[n_sr + 1] (n_sr = sectors * n_rows) give each
 * cluster's (sector, row).  Outputs: coef[6 * n_tracks];
 * row[n_track_clusters]; code[2 * n_track_clusters]; raw[2 * n_track_clusters]
 * (escaped clusters' (y, z), other entries 0); un_row[n_clusters],
 * un_yz[2 * n_clusters] (clusters on no track, input order).  Returns the
 * number of escaped clusters; *n_unassigned receives the unassigned count. */
uint64_t orc_codec_encode(int32_t n_rows, const double* row_x, double bz, float q_y, float q_z, uint32_t n_tracks,
                          const uint32_t* first, const uint32_t* ids, const float* x_ref, const float* param,
                          uint64_t n_clusters, const float* y, const float* z, const uint32_t* row_offsets,
                          uint32_t n_sr, float* coef, uint8_t* row, int16_t* code, float* raw, uint8_t* un_row,
                          float* un_yz, uint64_t* n_unassigned);

/* C11: decodes the track clusters of a stream (tracks in order, clusters in
 * stream order) into y_out, z_out [n_track_clusters]. */
void orc_codec_decode(int32_t n_rows, const double* row_x, float q_y, float q_z, uint32_t n_tracks,
                      const uint32_t* first, const float* x_ref, const float* coef, const uint8_t* row,
                      const int16_t* code, const float* raw, float* y_out, float* z_out);

#ifdef __cplusplus
}
#endif
#endif
