/*
 * tpc_tracker.h -- C ABI of the MI355X TPC sector track finder.
 *
 * What it computes.  The paper (arXiv:2502.09138, Introduction and Tables 1-3)
 * identifies TPC processing, dominated by track finding on clusters, as the
 * step that takes essentially all of ALICE's synchronous reconstruction time
 * and the GPU-offloaded part of the asynchronous one; it does not spell the
 * algorithm out.  This library implements per-sector track finding on TPC
 * clusters as a cellular-automaton neighbour search over pad rows followed
 * by Kalman-filter tracklet construction along helices, defined here step by
 * step (C1..C7).  Every number below is an input or a stated rule; nothing is
 * taken from any other implementation.
 *
 * Notation: S sectors, R pad rows (row r at radius X_r, sector half-width Y_r),
 * N clusters; (y, z) are sector-local coordinates in cm (z may be a drift
 * coordinate).  Clusters arrive sector-major, row-major: the clusters of
 * sector s, row r are [row_offsets[s*R+r], row_offsets[s*R+r+1]); a cluster's
 * index in the input arrays is its input id.  "Sorted position" p is the index
 * into the per-row grid order of C1 (rows keep their input ranges).
 *
 * C1  Grid (per sector s, row r, N_r hits).  Integer dims:
 *       Ly = ceil(20*Y_r) [mm], Lz = ceil(10*((double)z_hi_s - (double)z_lo_s)) [mm],
 *       B = max(1, N_r / K), nY = clamp(isqrt(B*Ly / Lz), 1, B), nZ = max(1, B / nY)
 *     (integer divisions, K = grid_hits_per_bin).  Bin of a hit, float32
 *     round-to-nearest, one rounding per operation, no contraction:
 *       u = (y - y_lo) * ((float)nY * inv_wy);  u = 0 if !(u >= 0);
 *       u = nY-1 if u > nY-1;  iy = (int)u     (same for z with z_lo, inv_wz, nZ)
 *     with y_lo = (float)(-Y_r), inv_wy = (float)(1/(2*Y_r)),
 *     inv_wz = (float)(1/((double)z_hi - (double)z_lo)); bin = iz*nY + iy.
 *     Sorted order of a row: ascending (bin, input id) -- a stable counting
 *     sort.  bin_start of row (s,r) lives at offset row_offsets[s*R+r] + 2*(s*R+r),
 *     nBins+1 entries holding sorted positions.
 * C2  Neighbour finder (rows 1..R-2).  du = X_{r+1}-X_r, dd = X_r-X_{r-1},
 *     t = (float)(dd/(dd+du)), W_y(d) = (float)(a_y*d + b_y), W_z likewise,
 *     Dmax = (float)((n^2*sigma_y^2) * ((1 + t^2) + (1-t)^2)) (double, then
 *     rounded), rho = (float)((sigma_y/sigma_z)^2).  For hit h: U = hits u in
 *     row r+1 with |y_u-y_h| <= W_y(du) and |z_u-z_h| <= W_z(du); D likewise in
 *     row r-1 with dd.  For (d,u) in D x U, in float32 as written:
 *       yp = y_d + t*(y_u-y_d); zp = z_d + t*(z_u-z_d);
 *       ey = y_h-yp; ez = z_h-zp; dev = ey*ey + rho*(ez*ez)
 *     Keep dev <= Dmax; choose the smallest (dev, pos_u, pos_d).  up0/down0 =
 *     sorted positions or -1.  Rows 0 and R-1 get no links.
 * C3  Cleaner: up1[h] = up0[h] if down0[up0[h]] == h else -1; down1[h] =
 *     down0[h] if up0[down0[h]] == h else -1 (evaluated on the C2 snapshot).
 * C4  Starts: down1[h] == -1 and up1[h] >= 0 and up1[up1[h]] >= 0; listed in
 *     ascending sorted position (= sector, row, grid order).  The start index
 *     in this list identifies the tracklet; startPos = its sorted position.
 * C5  Tracklet constructor (one per start; state p = (y, z, sin phi, tan
 *     lambda, q/pT) at x; kappa = -c_B*Bz*q/pT, c_B = 0.00299792458):
 *     Propagation x1 -> x2: fail if |s1| >= s_max; s2 = s1 + kappa*dx; fail if
 *       |s2| >= s_max; y2 = y1 + dx*(s1+s2)/(c1+c2) with c = sqrt(1-s^2);
 *       chord L = sqrt(dx^2+dy^2); u = kappa*L/2 (fail if |u| >= 1);
 *       ds = sign(dx)*L*asin(u)/u; z2 = z1 + tanl*ds.  Covariance C <- F C F^T
 *       with F the exact derivative of this map; no process noise.
 *     Update with (y_m, z_m), V = diag(sigma_y^2, sigma_z^2): standard gain,
 *       chi2 += r^T S^-1 r.
 *     Seed: chain h0..h_{n-1} along up1; points (X, y) of h0, h_m (m = (n-1)/2),
 *       h_{n-1}; kappa = 2(a x b)/(|a||b||c|) (a = Pm-P0, b = Pl-Pm, c = Pl-P0);
 *       u = kappa|c|/2 (fail if |u| >= 1); phi0 = atan2(c_y, c_x) - asin(u);
 *       tanl = (z_l - z_0)/(|c| asin(u)/u); q/pT = kappa/(-c_B*Bz) (0 if Bz = 0)
 *       clamped to +-seed_qpt_max; fail unless cos(phi0) > 0 and
 *       |sin phi0| < s_max.  p = (y0, z0, sin phi0, tanl, q/pT) at X_{r0},
 *       C = C0 = diag(sigma_y^2, sigma_z^2, c0_sinphi, c0_tanl, c0_qpt).
 *     Chain fit: propagate row by row and update with h1..h_{n-1} (no gate).
 *     Upward: for rows above the chain: propagate (stop on failure); stop if
 *       |y| > Y_r + edge_margin; search; update on a hit, else count a miss and
 *       stop after max_miss+1 consecutive misses.  Search in row r: window
 *       w = min(g*sqrt(C_yy+sigma_y^2), cap) in y (same in z); candidate
 *       minimising dy^2/(C_yy+sigma_y^2) + dz^2/(C_zz+sigma_z^2), ties by
 *       smaller sorted position.
 *     Downward refit: from the outermost hit row r_out with p from the
 *       upward pass, (y, z) set to that hit's coordinates and C = C0; for rows
 *       r_out-1 .. 0: propagate (stop on failure); below the start row r0
 *       stop if |y| > Y_r + edge_margin; use the row's hit from the upward
 *       pass without a gate, else search; count misses only below r0.
 *     Result: hits of the downward pass; p, C at x_ref = X of the innermost
 *       hit; chi2 of the downward pass; ndf = 2*nHits - 5.  Valid if
 *       nHits >= min_tracklet_hits.
 * C6  Selector: key = (nHits << 32) | (0xFFFFFFFF - startPos).  W[hit] = max
 *     key over valid tracklets holding the hit.  Owned = hits with W == key.
 *     Emit the tracklet as a track if owned >= min_track_hits and (float)owned
 *     >= (float)min_owned_frac * (float)nHits (float32).
 * C7  Output: tracks in ascending startPos (hence by sector); cluster lists are
 *     input ids of the owned hits in ascending row; parameters are the C5
 *     result at x_ref.
 * C8  Sector merger (tracks of sectors whose physical numbers are given:
 *     0..17 one side, 18..35 the other, 20 degrees apart, neighbours one step
 *     apart on the same side).  Rotation of a state at x into the frame
 *     turned by d, same point in space: x' = x cos d + y sin d, y' = -x sin d
 *     + y cos d, phi' = phi - d (fail unless cos phi' > 0), z, tan lambda,
 *     q/pT unchanged; covariance by the first-order Jacobian onto the plane
 *     x' = const (dy'/dy = cos phi / cos phi', dz'/dy = -tanl sin d / cos
 *     phi', dsin phi'/dy = -kappa sin d, dsin phi'/dsin phi = cos phi' /
 *     cos phi).  Track b (sector of a's neighbour) may follow track a if b's
 *     innermost point lies at a larger radius sqrt(x_ref^2 + y^2) than a's,
 *     and a's state, rotated into b's frame and propagated to b's x_ref,
 *     differs from b's by at most merge_dy, merge_dz, merge_dsinphi,
 *     merge_dtanl, merge_dqpt; score = dy^2/(C_b,yy + sigma_y^2) +
 *     dz^2/(C_b,zz + sigma_z^2).  Each a keeps its best successor and each b
 *     its best predecessor (smallest score, ties to the smaller track index);
 *     a -> b is linked when both agree.  Chains start at tracks without a
 *     predecessor, in ascending track order.
 * C9  Refit of a chain of two or more segments: from the outermost cluster of
 *     its last segment (state: that segment's C5 result propagated there, y
 *     and z set to the cluster, C = C0) inward over every cluster of the
 *     chain (each segment's own clusters, descending row), rotating the state
 *     and covariance into the previous segment's frame where the chain
 *     crosses a sector edge; result at the innermost cluster of the first
 *     segment, chi2 of the pass, ndf = 2*nClusters - 5 (-1 if a rotation or
 *     propagation fails; the chain then keeps its first segment's result).
 * C10 Track-model encoding (the paper names TPC data compression as the
 *     farm's main task -- abstract; Introduction and its table of processing
 *     shares -- and the track-model decoding as a step moved to the GPU --
 *     section on online and offline processing -- without giving a format;
 *     this is the project's definition).  Per C7 track (parameters p = (y, z,
 *     s = sin phi, T = tan lambda, q/pT) at x_ref as stored, float32), model
 *     coefficients computed in double and rounded to float32 once:
 *       kappa = (-c_B * Bz) * q/pT, c = sqrt(1 - s*s), ic = 1/c, ic3 = ic*ic*ic,
 *       a = (y, s*ic, 0.5*kappa*ic3), b = (z, T*ic, ((0.5*T)*s)*kappa*ic3)
 *     (the helix to second order in u = x - x_ref; |s| >= 1: all zero and
 *     every cluster of the track escaped).  Per track cluster (row r, input
 *     (y_m, z_m)), float32, each operation rounded, no fused multiply-add:
 *       u = X_r - x_ref; p_y = a0 + u*(a1 + u*a2), p_z likewise with b;
 *       v_y = (y_m - p_y) * float32(1/q_y), v_z likewise;
 *       if |v_y| <= 32767 and |v_z| <= 32767: (k_y, k_z) = (rint(v_y),
 *       rint(v_z)) (half to even), else k_y = TPC_CODEC_ESCAPE, k_z = 0 and
 *       (y_m, z_m) stored raw.
 *     Clusters on no track are stored raw (row, y, z) in input order.
 * C11 Decoding: y = p_y + k_y*q_y, z = p_z + k_z*q_z (float32, rounded, no
 *     fused multiply-add); escaped and unassigned clusters are their raw
 *     values.  A decoded cluster lies within q/2 (plus float32 rounding) of
 *     the encoded one.
 *
 * Floating point: C1, C2 and the C6 fraction test are exact float32
 * definitions (bit-identical results expected).  C5 runs in float32 on the
 * GPU; its results agree with an FP64 evaluation of the same steps within
 * rounding, and a search decision may differ only when two candidates (or a
 * candidate and a window edge) are within rounding of each other.
 *
 * Threading: a tracker is used by one host thread at a time.  One request is
 * in flight per tracker: tpc_track_timeframe returns TPC_E_BUSY until the
 * previous request has been released.
 */
#ifndef TPC_TRACKER_H
#define TPC_TRACKER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TPC_ABI_VERSION 3u
#define TPC_MAX_ROWS 255
#define TPC_MAX_ROW_HITS 65535u       /* clusters per (sector, row) */
#define TPC_MAX_COORD 16384.0f        /* |y|, |z| bound (cm) for exact grid searches */

typedef int32_t tpc_status;
enum {
  TPC_OK = 0,
  TPC_E_INVAL = -1,      /* bad argument or configuration; nothing was enqueued */
  TPC_E_NOMEM = -2,      /* allocation failed */
  TPC_E_DEVICE = -3,     /* HIP runtime error */
  TPC_E_CAPACITY = -4,   /* a capacity was exceeded (see error_flags); results discarded */
  TPC_E_NOTREADY = -5,   /* non-blocking get on a request still running */
  TPC_E_INPUT = -6,      /* non-finite or out-of-range cluster coordinate */
  TPC_E_BUSY = -7        /* previous request not yet released */
};

/* device-side error flags reported in tpc_tracks.error_flags */
enum {
  TPC_ERR_NONFINITE = 1u,          /* a y or z is NaN/Inf or |.| > TPC_MAX_COORD */
  TPC_ERR_TRACKLET_OVERFLOW = 2u,  /* more starts than max_tracklets */
  TPC_ERR_TRACK_OVERFLOW = 4u,     /* more tracks than max_tracks */
  TPC_ERR_CLUSTER_OVERFLOW = 8u    /* more track clusters than max_track_clusters */
};

typedef struct tpc_tracker tpc_tracker;

typedef struct {
  uint32_t abi_version;            /* TPC_ABI_VERSION */
  int32_t n_rows;                  /* R, 3..TPC_MAX_ROWS */
  const double* row_x;             /* [n_rows] pad-row radius X_r (cm), strictly increasing; copied at create */
  const double* row_half_y;        /* [n_rows] sector half-width Y_r (cm), > 0; copied at create */
  double bz_tesla;                 /* solenoid field */
  double sigma_y, sigma_z;         /* cluster resolution (cm), > 0 */
  /* cuts (C1..C6) */
  int32_t grid_hits_per_bin;       /* K >= 1 */
  double win_a_y, win_b_y, win_a_z, win_b_z;   /* neighbour windows W(d) = a*d + b (cm) */
  double link_nsigma;              /* n in Dmax */
  double s_max;                    /* |sin phi| limit, (0, 1) */
  double seed_qpt_max;             /* |q/pT| clamp of the seed (1/GeV) */
  double c0_sinphi, c0_tanl, c0_qpt;           /* initial variances */
  double gate_nsigma, win_cap, edge_margin;    /* search gate g, window cap (cm), edge margin (cm) */
  int32_t max_miss, min_tracklet_hits, min_track_hits;
  double min_owned_frac;
  /* C8 merger windows on (segment propagated into the next sector) - (segment found there):
   * |dy|, |dz| (cm), |d sin phi|, |d tan lambda|, |d q/pT| (1/GeV) */
  double merge_dy, merge_dz, merge_dsinphi, merge_dtanl, merge_dqpt;
  /* schedule of the tracklet kernel (results are identical):
   * 0 = automatic, 1 = one lane per tracklet with per-lane grid gathers,
   * 2 = row-synchronous waves with the row grid staged in LDS */
  int32_t tracklet_schedule;
  /* capacities (device workspace is sized from these) */
  uint32_t max_sectors;
  uint64_t max_clusters;           /* < 2^31 */
  uint64_t max_tracklets;          /* 0 = max_clusters / 4 */
  uint64_t max_tracks;             /* 0 = max_tracklets */
  uint64_t max_track_clusters;     /* 0 = max_clusters */
  /* device and memory */
  int32_t device;                  /* HIP device ordinal */
  void* stream;                    /* hipStream_t to enqueue on; NULL = a stream owned by the tracker */
  void* workspace;                 /* device memory >= tpc_workspace_bytes(cfg), 256-byte aligned, owned by
                                      the caller and kept alive until destroy; NULL = tracker allocates */
  uint64_t workspace_bytes;
} tpc_tracker_config;

/* Fills every field with the library defaults (geometry pointers NULL). */
void tpc_default_config(tpc_tracker_config* cfg);

/* Device bytes the tracker needs for cfg (0 if cfg is invalid).  Host only. */
uint64_t tpc_workspace_bytes(const tpc_tracker_config* cfg);

/* Validates cfg (TPC_E_INVAL before any device call), then selects the
 * device, uploads the constant tables (the float32 constants of C1, C2 and
 * C5 derived in double from the geometry and cuts) and carves the workspace. */
tpc_status tpc_tracker_create(const tpc_tracker_config* cfg, tpc_tracker** out);
void tpc_tracker_destroy(tpc_tracker* t);

/* Per-request workspaces (a server carving workspaces out of one budgeted
 * pool).  tpc_workspace_bytes_for: device bytes a binding for at most
 * max_clusters / max_sectors needs on tracker t (tracklet, track and track-
 * cluster capacities follow the defaults for max_clusters, limited by t's
 * create-time ones); 0 if the capacities exceed those t was created with.
 * tpc_tracker_bind_workspace: moves t onto caller-owned device memory of
 * workspace_bytes (>= tpc_workspace_bytes_for, 256-byte aligned) with those
 * capacities; later requests are limited to them.  Allowed only between
 * requests (TPC_E_BUSY while one is in flight); a workspace the tracker had
 * allocated itself is freed.  The caller keeps the memory alive, and does
 * not reuse it, until the next bind, a release of the last request on it,
 * or destroy.  Costs one small host-to-device copy on the tracker's stream
 * (the row constants).  TPC_E_INVAL for a NULL or misaligned workspace, too
 * few bytes, or capacities beyond the create-time ones. */
uint64_t tpc_workspace_bytes_for(const tpc_tracker* t, uint64_t max_clusters, uint32_t max_sectors);
tpc_status tpc_tracker_bind_workspace(tpc_tracker* t, void* workspace, uint64_t workspace_bytes,
                                      uint64_t max_clusters, uint32_t max_sectors);

enum { TPC_IN_DEVICE = 0u, TPC_IN_HOST = 1u };

typedef struct {
  uint32_t n_sectors;              /* 1..max_sectors */
  uint32_t n_rows;                 /* must equal the config's n_rows */
  const uint32_t* row_offsets;     /* HOST [n_sectors*n_rows+1], starts at 0, non-decreasing, ends at n_clusters */
  const float* y;                  /* [n_clusters] sector-local y (cm) */
  const float* z;                  /* [n_clusters] z or drift coordinate (cm) */
  const uint16_t* charge;          /* [n_clusters] or NULL; carried, not read by tracking */
  uint64_t n_clusters;             /* <= max_clusters */
  const float* sector_z_lo;        /* HOST [n_sectors] grid z range per sector; z_hi > z_lo */
  const float* sector_z_hi;
  uint32_t flags;                  /* TPC_IN_DEVICE: y/z are device pointers, borrowed until the request
                                      completes; TPC_IN_HOST: host arrays, copied before return */
} tpc_timeframe;

/* Enqueues C1..C7 (defined above: the TPC track finding that the paper's
 * Introduction and Tables 1-3 place at the core of the GPU workload) for one
 * time frame on the tracker's stream and returns at once.  Errors in the
 * host-side validation return TPC_E_INVAL and enqueue nothing; device-side
 * errors are reported by tpc_get_tracks. */
tpc_status tpc_track_timeframe(tpc_tracker* t, const tpc_timeframe* tf, uint64_t* request_id);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same as
 * tpc_track_timeframe, but the request's whole device workspace is carved
 * from one fixed array of TPC_SCRATCH_BYTES per device inside the library,
 * not from the tracker's own workspace, and the call allocates nothing (no
 * hipMalloc, hipFree or allocating library routine).  Frames whose workspace
 * (tpc_workspace_bytes_for their cluster and sector counts) exceeds the array
 * are rejected with TPC_E_INVAL and a message; that is about 0.85M clusters
 * at the default capacities (about 300 B per cluster).  The array is shared by
 * every tracker on the device and keeps the last request's contents: requests
 * that overlap on one device race, so issue the next one only after the
 * previous one was released.  Results are read with tpc_get_tracks (host
 * copies) or tpc_get_tracks_device (views into the array, valid until the next
 * call of this function on the device).  A later tpc_track_timeframe runs on
 * the tracker's own workspace again. */
#define TPC_SCRATCH_BYTES (256ull << 20)
tpc_status tpc_track_timeframe_scratch(tpc_tracker* t, const tpc_timeframe* tf, uint64_t* request_id);

typedef struct {
  uint32_t n_tracks;
  uint64_t n_track_clusters;
  const uint32_t* track_sector;    /* [n_tracks] */
  const uint32_t* track_start;     /* [n_tracks] startPos (sorted position of the start hit) */
  const uint32_t* track_first;     /* [n_tracks+1] offsets into cluster_ids */
  const uint32_t* cluster_ids;     /* [n_track_clusters] input ids, ascending row within a track */
  const float* x_ref;              /* [n_tracks] cm */
  const float* param;              /* [n_tracks*5] y, z, sin phi, tan lambda, q/pT at x_ref */
  const float* cov;                /* [n_tracks*15] lower triangle row-major: 00,10,11,20,21,22,... */
  const float* chi2;               /* [n_tracks] */
  const int32_t* ndf;              /* [n_tracks] */
  uint32_t error_flags;            /* TPC_ERR_* */
  uint32_t n_tracklets;            /* number of starts (C4) */
  uint64_t n_steps;                /* row steps taken by the C5 lanes (work measure) */
} tpc_tracks;

/* Waits for (blocking != 0) or polls the request and fills *out with views of
 * tracker-owned host memory, valid until tpc_release or destroy.  Returns
 * TPC_E_NOTREADY when polling a running request, TPC_E_INPUT/TPC_E_CAPACITY
 * when the device reported an error (out->error_flags set, no tracks). */
tpc_status tpc_get_tracks(tpc_tracker* t, uint64_t request_id, int32_t blocking, tpc_tracks* out);

/* Same as tpc_get_tracks, but the array pointers are DEVICE memory of the
 * tracker's workspace (nothing is copied to the host; the counts and flags
 * come from the completed request).  Valid until tpc_release or destroy; read
 * them on the tracker's stream or after the call returns. */
tpc_status tpc_get_tracks_device(tpc_tracker* t, uint64_t request_id, int32_t blocking, tpc_tracks* out);

/* C8 + C9 on the tracks of a completed request (before its release): links
 * track segments across the edges between neighbouring sectors and refits the
 * merged chains.  sector_phys: HOST [n_sectors of the request], the physical
 * sector number (0..35) of each of the frame's sectors, -1 for a sector with
 * no neighbours (an independent chunk); NULL = none has neighbours.  Runs on
 * the tracker's stream and waits for it; *out receives views of tracker-owned
 * host memory, valid until tpc_release or destroy: per input track its
 * successor (-1) and chain head, per chain (in ascending head order) the head
 * track, segment count, merged cluster list (input ids: the segments' lists in
 * chain order) and the refit state at the innermost cluster (a single
 * segment's chain: its C5 result).  TPC_E_INVAL for an unknown request or a
 * sector number out of range; TPC_E_CAPACITY if the request had failed. */
typedef struct {
  uint32_t n_tracks;               /* tracks of the request */
  uint32_t n_chains;
  uint64_t n_chain_clusters;
  const int32_t* next;             /* [n_tracks] */
  const uint32_t* head_of;         /* [n_tracks] */
  const uint32_t* heads;           /* [n_chains] */
  const int32_t* nseg;             /* [n_chains] */
  const uint32_t* first;           /* [n_chains+1] offsets into clusters */
  const uint32_t* clusters;        /* [n_chain_clusters] input ids */
  const float* param;              /* [n_chains*5] y, z, sin phi, tan lambda, q/pT at the head's x_ref */
  const float* cov;                /* [n_chains*15] */
  const float* chi2;               /* [n_chains] */
  const int32_t* ndf;              /* [n_chains] */
} tpc_merged;
tpc_status tpc_merge_sectors(tpc_tracker* t, uint64_t request_id, const int32_t* sector_phys, tpc_merged* out);

/* ---- C10 / C11: track-model compression ---- */
#define TPC_CODEC_ESCAPE (-32768)

/* A compressed frame.  All arrays are DEVICE memory owned by the caller:
 * coef [6*n_tracks] (a0, a1, a2, b0, b1, b2 per track), x_ref [n_tracks],
 * first [n_tracks+1] (offsets of each track's clusters), row [n_track_clusters]
 * (pad row), code [2*n_track_clusters] (k_y, k_z), raw [2*n_track_clusters]
 * ((y, z) of escaped clusters, 0 elsewhere), un_row [n_unassigned] and un_yz
 * [2*n_unassigned] (clusters on no track, input order; the encoder needs room
 * for n_clusters of the frame). */
typedef struct {
  float* coef;
  float* x_ref;
  uint32_t* first;
  uint8_t* row;
  int16_t* code;
  float* raw;
  uint8_t* un_row;
  float* un_yz;
} tpc_codec_stream;

typedef struct {
  uint32_t n_tracks;
  uint64_t n_track_clusters;
  uint64_t n_unassigned;
  uint64_t n_escaped;
} tpc_codec_counts;

/* C10 on the tracks of a completed request (before its release; the request's
 * input arrays must still hold the clusters).  q_y, q_z: residual quanta (cm,
 * finite, > 0).  Runs on the tracker's stream and waits for it; *counts
 * receives the stream's sizes.  The stream arrays are sized by the caller from
 * the request's track counts (tpc_get_tracks) and the frame's cluster count.
 * Uses the request's workspace for flags (its C2 and C6 intermediates are
 * overwritten).  TPC_E_INVAL for an unknown request, bad quanta or NULL
 * arrays; TPC_E_INPUT/TPC_E_CAPACITY if the request failed. */
tpc_status tpc_encode_tracks(tpc_tracker* t, uint64_t request_id, float q_y, float q_z, const tpc_codec_stream* out,
                             tpc_codec_counts* counts);

/* C11: decodes a stream (device arrays, counts as returned by the encoder,
 * the same quanta) into DEVICE arrays y_out, z_out, row_out of
 * n_track_clusters + n_unassigned entries: the track clusters in stream
 * order, then the unassigned ones.  Needs only the tracker's geometry (no
 * request); runs on the tracker's stream and waits for it. */
tpc_status tpc_decode_tracks(tpc_tracker* t, const tpc_codec_stream* in, const tpc_codec_counts* counts, float q_y,
                             float q_z, float* y_out, float* z_out, uint8_t* row_out);

/* Waits for the request and frees its slot. */
tpc_status tpc_release(tpc_tracker* t, uint64_t request_id);

/* Message of the last error on the calling thread ("" if none). */
const char* tpc_last_error(void);

/* ---- introspection (tests, profiling) ---- */
enum {
  TPC_DBG_SORTED_ID = 1,   /* u32 [N] */
  TPC_DBG_SORTED_YZ,       /* f32 [2N] (y, z) pairs */
  TPC_DBG_BIN_START,       /* u32 [N + 2*S*R] (only nBins+1 entries per row defined) */
  TPC_DBG_ROW_DIMS,        /* u32 [S*R] nY | nZ << 16 */
  TPC_DBG_UP0, TPC_DBG_DOWN0, TPC_DBG_UP1, TPC_DBG_DOWN1,   /* i32 [N] */
  TPC_DBG_STARTS,          /* u32 [T] */
  TPC_DBG_TK_ROWHIT,       /* i32 [R*max_tracklets] row-major; only rows [xref_row, out_row] defined */
  TPC_DBG_TK_INFO,         /* i32 [4*T]: nHits (<0: seed/propagation failure), xref_row, out_row, start row */
  TPC_DBG_TK_PARAM,        /* f32 [5*T] parameter-major: param k of tracklet i at [k*max_tracklets + i] */
  TPC_DBG_TK_COV,          /* f32 [15*max_tracklets] same layout */
  TPC_DBG_TK_CHI2          /* f32 [T] */
};
/* Copies an intermediate of the last completed request to host memory;
 * *bytes receives the full size.  Waits for the request. */
tpc_status tpc_debug_copy(tpc_tracker* t, int32_t what, void* host_dst, uint64_t cap_bytes, uint64_t* bytes);

/* Selects the tracklet-constructor schedule for later requests (same meaning
 * as tpc_tracker_config.tracklet_schedule: 0 auto, 1 one lane per tracklet with
 * global-memory searches, 2 row-synchronous waves with LDS-staged rows).  All
 * schedules compute the same step C5; they differ in memory traffic and
 * speed, which is what a shape-class autotuner chooses between.  Returns
 * TPC_E_INVAL for other values or while a request is in flight. */
tpc_status tpc_set_tracklet_schedule(tpc_tracker* t, int32_t schedule);

/* Tuning knobs for later requests (results are identical under every
 * setting; they change speed only, which is what a shape-class autotuner
 * chooses between):
 *   TPC_KNOB_TRACKLET_SCHEDULE  0 auto, 1 lane-per-tracklet pipeline, 2
 *                               row-synchronous (as tpc_set_tracklet_schedule)
 *   TPC_KNOB_SELECT_TILE_ROWS   0 auto (4 rows, fewer where a block would need
 *                               more than 48 KB of LDS); 1, 2, 4: rows per C6
 *                               selector tile, reduced to the largest power of
 *                               two whose blocks fit 48 KB of LDS (none: the
 *                               global-memory selector); -1: the global-memory
 *                               selector
 *   TPC_KNOB_REFIT_ORDER        0 the lane-per-tracklet pipeline refits in
 *                               (sector, outermost row) order, 1 in tracklet
 *                               order
 *   TPC_KNOB_LINK_SLOTS         0 auto (8), 4 or 8: C2 up-row candidates held
 *                               per hit before the pair search falls back to
 *                               rescanning the window
 *   TPC_KNOB_LINK_GROUP         0 auto (64), 1..4096: consecutive C2 tiles
 *                               (64 hits each) given to one XCD before the
 *                               next XCD's group (1 deals them out one by
 *                               one); -1: one contiguous eighth per XCD
 *   TPC_KNOB_SELECT_THREADS     0 auto (512), 256, 512 or 1024: workgroup size
 *                               of the C6 selector's tile kernels
 * TPC_E_INVAL for an unknown knob or value, or while a request is in flight. */
enum {
  TPC_KNOB_TRACKLET_SCHEDULE = 1,
  TPC_KNOB_SELECT_TILE_ROWS = 2,
  TPC_KNOB_REFIT_ORDER = 3,
  TPC_KNOB_LINK_SLOTS = 4,
  TPC_KNOB_LINK_GROUP = 5,
  TPC_KNOB_SELECT_THREADS = 6
};
tpc_status tpc_set_knob(tpc_tracker* t, int32_t knob, int32_t value);

/* Per-pass timing with HIP events on the tracker's stream, for later requests.
 * pass_mask: bit p times pass p (TPC_N_PASSES passes, in the order below);
 * 0 turns timing off, TPC_TIME_ALL_PASSES times every pass; TPC_E_INVAL for
 * bits beyond the passes.  Each timed pass costs up to two event records on
 * the stream, so a caller that needs one pass's time should time that pass
 * alone. */
#define TPC_N_PASSES 6     /* K1 grid, K2 neighbours, K3/K4 clean+starts, K5 tracklets, K6 select, output */
#define TPC_TIME_ALL_PASSES 0x3F
tpc_status tpc_set_timing(tpc_tracker* t, int32_t pass_mask);
/* Milliseconds of each pass of the last completed request; -1 for a pass
 * that was not timed.  TPC_E_INVAL if timing was off for that request. */
tpc_status tpc_get_pass_times(tpc_tracker* t, float* ms, int32_t n);

#ifdef __cplusplus
}
#endif
#endif /* TPC_TRACKER_H */
