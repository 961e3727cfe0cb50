/*
 * FP64 reference tracker ("oracle") for TPC per-sector track finding.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or
 * calls this code; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the HIP library: both receive the same geometry and cut values as plain
 * numbers and each derives what it needs on its own.
 *
 * The paper (Introduction; Tables 1-3) places TPC track finding at the core
 * of the GPU workload but does not spell the algorithm out, so this oracle
 * implements the project's written definition, steps C1..C7:
 *   C1 per-row grid sort, C2 neighbour finder, C3 neighbour cleaner,
 *   C4 start-hit finder, C5 tracklet constructor (helix + Kalman filter),
 *   C6 tracklet selector, C7 canonical output.
 * Everything is FP64 and single-threaded, except the decisions that the
 * definition fixes in float32 (bin index, neighbour windows and pair
 * deviation, owned-fraction test): those are evaluated with float32
 * round-to-nearest operations in the stated order, so both implementations
 * take them in the same precision.
 */
#ifndef TPC_ORACLE_H
#define TPC_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n_rows;
  const double* row_x;        /* [n_rows] pad-row centre, cm */
  const double* row_half_y;   /* [n_rows] sector half-width at the row, cm */
  double bz;                  /* Tesla */
  double sigma_y, sigma_z;    /* cm */
  int32_t grid_hits_per_bin;
  double win_a_y, win_b_y, win_a_z, win_b_z;
  double link_nsigma;
  double s_max;
  double seed_qpt_max;
  double c0_sinphi, c0_tanl, c0_qpt;
  double gate_nsigma, win_cap, edge_margin;
  int32_t max_miss, min_tracklet_hits, min_track_hits;
  double min_owned_frac;
  /* C8 merger windows: |dy|, |dz| (cm), |d sin phi|, |d tan lambda|, |d q/pT| (1/GeV) */
  double merge_dy, merge_dz, merge_dsinphi, merge_dtanl, merge_dqpt;
} orc_config;

typedef struct orc_run orc_run;

/* Borrowed input; y/z are FP64 (the float32 entry converts exactly). */
orc_run* orc_run_create(const orc_config* cfg, uint32_t n_sectors, const uint32_t* row_offsets,
                        const double* y, const double* z, const float* sector_z_lo,
                        const float* sector_z_hi);
void orc_run_destroy(orc_run* r);

/* A run that holds only the given tracklets (T of them): nHits (<
 * min_tracklet_hits = not valid), start positions, and rows ([T*n_rows],
 * sorted positions, -1 = no hit), for step C6 on its own; cluster ids equal
 * sorted positions.  Call orc_run_select on it. */
orc_run* orc_run_from_tracklets(const orc_config* cfg, uint32_t n_clusters, uint64_t n_tracklets,
                                const int32_t* nhits, const uint32_t* start_pos, const int32_t* rowhit);

int orc_run_grid(orc_run* r);                 /* C1 */
int orc_run_links(orc_run* r);                /* C2 + C3 */
/* C2 + C3 with the C2 windows, cut and deviation evaluated in double instead
 * of the float32 the definition fixes (to show where the two differ). */
int orc_run_links_fp64(orc_run* r);
int orc_run_starts(orc_run* r);               /* C4 */
/* C5 on the listed start indices (NULL = all starts). */
int orc_run_construct(orc_run* r, const uint32_t* which, uint64_t n_which);
int orc_run_select(orc_run* r);               /* C6 + C7, needs all tracklets */

enum {
  ORC_SORTED_ID = 1,      /* u32 [N] input id at each sorted position */
  ORC_BIN_START,          /* u32 [N + 2*S*R] per row at N_r-offset + 2*row, nBins+1 used */
  ORC_ROW_DIMS,           /* u32 [S*R] nY | nZ << 16 */
  ORC_UP0, ORC_DOWN0, ORC_UP1, ORC_DOWN1,   /* i32 [N] sorted positions, -1 none */
  ORC_STARTS,             /* u32 [T] sorted positions of start hits, canonical order */
  ORC_TK_ROWHIT,          /* i32 [T*R] tracklet-major */
  ORC_TK_NHITS,           /* i32 [T] (0 = not constructed, <0 failure code) */
  ORC_TK_PARAM,           /* f64 [T*5] */
  ORC_TK_COV,             /* f64 [T*15] */
  ORC_TK_XREF_ROW,        /* i32 [T] */
  ORC_TK_CHI2,            /* f64 [T] */
  ORC_TRK_TRACKLET,       /* u32 [n_tracks] tracklet index of each track */
  ORC_TRK_FIRST,          /* u32 [n_tracks+1] */
  ORC_TRK_CLUSTERS,       /* u32 [total] input ids, ascending row */
  ORC_SIZES               /* u64 [4] N, T, n_tracks, n_track_clusters */
};
/* Copies the array into dst (cap bytes); returns the bytes the array holds. */
uint64_t orc_get(orc_run* r, int what, void* dst, uint64_t cap);

/* C8 sector merger + C9 refit on the C7 tracks of a run (after orc_run_select).
 * sector_phys[S]: physical sector (0..17 A side, 18..35 C side) of each of the
 * run's sectors, or -1 for a sector with no neighbours (independent chunks);
 * NULL = no sector has neighbours (nothing merges). */
typedef struct orc_merge orc_merge;
orc_merge* orc_merge_run(orc_run* r, const int32_t* sector_phys);
void orc_merge_destroy(orc_merge* m);
enum {
  ORC_M_NEXT = 1,        /* i32 [n_tracks] successor track (-1 none) */
  ORC_M_HEAD,            /* i32 [n_tracks] head of the track's chain */
  ORC_M_HEADS,           /* u32 [n_merged] chain heads, ascending */
  ORC_M_NSEG,            /* i32 [n_merged] segments per chain */
  ORC_M_PARAM,           /* f64 [n_merged*5] refit (chains of >= 2) or C5 result */
  ORC_M_COV,             /* f64 [n_merged*15] */
  ORC_M_CHI2,            /* f64 [n_merged] */
  ORC_M_NDF,             /* i32 [n_merged] 2*nClusters-5, -1 if the refit failed */
  ORC_M_FIRST,           /* u32 [n_merged+1] */
  ORC_M_CLUSTERS         /* u32 [...] input ids, chain order, ascending row in a segment */
};
uint64_t orc_merge_get(orc_merge* m, int what, void* dst, uint64_t cap);

/* ---- unit-level entry points used by the pins ---- */
/* Rotation of a state at x into the frame turned by d (radians), same point in
 * space; J is the 5x5 Jacobian onto the new plane x' = const.  1 if the track
 * does not move outward in the new frame. */
int orc_rotate(double x, const double* p_in, double d, double bz, double* x_out, double* p_out, double* J);
/* Helix transport of p=(y,z,sinphi,tanl,qpt) from x1 to x2; F is 5x5 row-major.
 * Returns 0 on success, 1 if |sinphi| >= s_max at either end. */
int orc_propagate(const double* p_in, double x1, double x2, double bz, double s_max,
                  double* p_out, double* F);
/* Same transport applied to a packed covariance as well: C' = F C F^T. */
int orc_propagate_cov(const double* p_in, const double* c_in, double x1, double x2, double bz, double s_max,
                      double* p_out, double* c_out);
/* One Kalman update with measurement (ym, zm), variances (vy, vz).  C packed lower
 * triangle (15).  Joseph form.  Adds r^T S^-1 r to *chi2. */
void orc_kf_update(double* p, double* C, double ym, double zm, double vy, double vz, double* chi2);
/* Three-point seed; returns 0 ok, 1 if no circle through the points. */
int orc_seed(const orc_config* cfg, double x0, double y0, double z0, double xm, double ym,
             double xl, double yl, double zl, double* p_out);
/* Grid bin (iy, iz) of one hit, float32 definition. */
void orc_bin(float y, float z, float y_lo, float inv_wy, float z_lo, float inv_wz, int ny, int nz,
             int* iy, int* iz);
void orc_grid_dims(uint32_t n_hits, int k, int64_t ly_mm, int64_t lz_mm, int* ny, int* nz);

#ifdef __cplusplus
}
#endif
#endif
