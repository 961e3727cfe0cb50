// Internal layout shared by the host runtime and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tpc {

constexpr int kMaxRows = 255;
constexpr float kMaxCoord = 16384.0f;   // |y|, |z| beyond this (or non-finite) is flagged as bad input
constexpr float kWinPad = 0.01f;    // cm added to a search window before binning (covers rounding)
constexpr int kPasses = 6;
constexpr uint32_t kLinkTile = 64;    // hits per K2 tile (one wave)
constexpr uint32_t kPackHits = 1024;  // K1: consecutive rows sorted by one workgroup up to this many hits
constexpr uint32_t kPackRows = 32;    // and this many rows
constexpr uint32_t kLinkGroupEighth = 0xFFFFFFFFu;   // K2 group size: one contiguous eighth of the tiles per XCD

// Per pad row: float32 constants used by C1, C2 and C5 (computed in double on the host, rounded once).
struct RowConst {
  float x, half_y, y_lo, inv_wy;
  float t, wy_up, wz_up, wy_dn;
  float wz_dn, dmax;
  int32_t ly;          // ceil(20 * Y_r), mm
  int32_t pad;
};

// Per sector of the current request.
struct SectorConst {
  float z_lo, inv_wz;
  int32_t lz;          // mm
  int32_t pad;
};

// Scalar constants of C5/C6 in float32.
struct KfConst {
  float bk;            // -c_B * Bz
  float s_max, qpt_max;
  float vy, vz;        // sigma^2
  float c0_sinphi, c0_tanl, c0_qpt;
  float gate, cap, margin;
  float rho;
  float min_owned_frac;
  int32_t max_miss, min_tracklet_hits, min_track_hits;
  int32_t grid_k;
  int32_t n_rows;
};

// Device result header (copied to pinned host memory at the end of a request).
struct ResultHeader {
  uint32_t n_starts;       // C4 count (may exceed capacity; see flags)
  uint32_t error_flags;
  uint32_t n_tracks;
  uint32_t pad0;
  uint64_t n_track_clusters;
  uint64_t n_steps;        // row steps taken by all tracklet lanes (C5 work measure)
  uint32_t codec_escaped;  // clusters the last C10 encoding stored raw
  uint32_t codec_unassigned;  // clusters on no track in the last C10 encoding (host copy of the scan total)
};

// All device pointers of one request.
struct DevPtrs {
  // inputs
  const uint32_t* row_off;   // [SR+1]
  const float* y;
  const float* z;
  const RowConst* rows;      // [R]
  const SectorConst* secs;   // [S]
  // C1
  const uint32_t* pack_first;   // [n_packs + 1] first (sector, row) slot of each K1 pack, then SR
  uint32_t* row_dims;        // [SR]
  uint2* row_meta;           // [SR] (bin_start offset of the row, dims) for one-load grid lookups
  uint32_t* bin_start;       // [N + 2SR]
  float2* syz;               // [N]
  uint32_t* sid;             // [N]
  // C2/C3/C4
  int32_t* up0;
  int32_t* down0;
  int32_t* up1;
  int32_t* down1;
  uint8_t* sflag;            // [N] start flag
  uint32_t* row_nstart;      // [SR]
  uint32_t* row_start_off;   // [SR+1] exclusive scan
  uint32_t* start_pos;       // [Tcap]
  uint32_t* start_sr;        // [Tcap]
  uint32_t* wave_off;        // [S+1] row-synchronous K5: first wave of each sector
  const uint32_t* tile_off;  // [SR+1] K2: first tile of each row (ceil(N_r / kLinkTile) tiles per row)
  uint32_t* tile_sr;         // [tiles] K2: row of each tile (written by K1)
  // C5
  int32_t* tk_rowhit;        // [R * Tcap]
  int32_t* tk_info;          // [4 * Tcap]: nHits, r_in, r_out, r0
  float* tk_param;           // [5 * Tcap]
  float* tk_cov;             // [15 * Tcap]
  float* tk_chi2;            // [Tcap]
  uint32_t* k5_off;          // [SR+1] lane-per-tracklet K5: refit bucket offsets (sector, outermost row)
  uint32_t* k5_perm;         // [Tcap] tracklets in bucket order
  uint32_t* k5_inv;          // [Tcap] bucket slot of each tracklet
  uint32_t* k5_rec;          // [25 * Tcap] refit results in slot order (one record per tracklet)
  // C6
  uint32_t* W;               // [N] ownership word (32-bit key) per sorted position
  uint8_t* own_part;         // [R * Tcap] owned hits of a tracklet per selector tile (then prefixes)
  unsigned long long* tk_pack;   // [Tcap] (owned << 32) | accepted
  unsigned long long* tk_scan;   // [Tcap + 1] exclusive scan of tk_pack
  uint32_t* acc_list;        // [max_tracks] tracklet of each track (track order)
  // outputs
  uint32_t* out_sector;
  uint32_t* out_start;
  uint32_t* out_first;       // [max_tracks + 1]
  uint32_t* out_clusters;
  float* out_xref;
  float* out_param;          // [5 * max_tracks] track-major
  float* out_cov;            // [15 * max_tracks]
  float* out_chi2;
  int32_t* out_ndf;
  // scratch for scans
  unsigned long long* scan_blocks;   // [kScanMaxBlocks]
  ResultHeader* hdr;
  // sizes
  int32_t grid_k;
  float rho;                 // (sigma_y / sigma_z)^2, float32
  int32_t k5_mode;           // 0 auto, 1 lane-per-tracklet pipeline, 2 row-synchronous
  int32_t k5_refit_order;    // 0 (sector, outermost row) buckets, 1 tracklet order
  int32_t k2_slots;          // K2 up-candidate slots per lane: 4 or 8 (0 = 8)
  uint32_t k2_group;         // K2 tiles per XCD group (1: round robin, kLinkGroupEighth: an eighth of the tiles)
  uint32_t k6_threads;       // workgroup size of the K6 tile kernels: 256, 512 or 1024
  uint32_t S, R, SR, N;
  uint32_t tcap;
  uint32_t tile_cap;         // LDS words of one selector tile (max hits in a sector's row block)
  uint32_t n_link_tiles;     // K2 tiles of this request
  uint32_t n_packs;          // K1 row packs of this request
  uint32_t max_tracks;
  uint64_t max_track_clusters;
};

// C8/C9 sector merger on the tracks of a completed request (all in the workspace).
struct MergeArgs {
  const int32_t* phys;                 // [S] physical sector of each of the frame's sectors, -1: no neighbours
  int32_t* nbr;                        // [2S] frame sector of the -1 / +1 neighbour, -1 if absent
  uint32_t* sec_first;                 // [S+1] first track of each sector
  int32_t* succ;                       // [MT] best successor
  unsigned long long* pred_key;        // [MT] (score bits << 32) | best predecessor
  int32_t* next;                       // [MT] linked successor, -1 none
  uint32_t* has_pred;                  // [MT]
  uint32_t* head_flag;                 // [MT]
  uint32_t* head_scan;                 // [MT+1] chain index of each head
  uint32_t* chain_clusters;            // [MT] clusters of the chain (at heads)
  uint32_t* cl_scan;                   // [MT+1]
  uint32_t* heads;                     // [MT] per chain: head track
  uint32_t* head_of;                   // [MT] per track: its chain's head
  uint32_t* first;                     // [MT+1] per chain: first merged cluster
  uint32_t* clusters;                  // [MC] merged cluster lists
  float* param;                        // [5 MT] per chain, track-major
  float* cov;                          // [15 MT]
  float* chi2;                         // [MT]
  int32_t* ndf;                        // [MT] -1: refit failed
  int32_t* nseg;                       // [MT]
  double cos20, sin20;                 // the rotation between neighbouring sectors
  double bk, s_max;                    // -c_B * Bz and the |sin phi| limit, in double
  double vy, vz, c0_sinphi, c0_tanl, c0_qpt;   // measurement and initial variances, in double
  double dy, dz, dsinphi, dtanl, dqpt; // C8 windows
};

// C10 track-model encoding of a completed request's tracks.
struct CodecArgs {
  // the request's tracks (C7 outputs in the workspace) and clusters
  const float* param;          // [5 * n_tracks] track-major
  const float* xref_in;        // [n_tracks]
  const uint32_t* first_in;    // [n_tracks + 1]
  const uint32_t* clusters;    // [n_cl] input cluster ids
  uint32_t n_tracks;
  uint64_t n_cl;
  const uint32_t* row_off;     // [SR + 1] input-order row offsets
  uint32_t SR, R, N;
  const RowConst* rows;        // [R] (x)
  const float* y;              // [N] input coordinates
  const float* z;
  double bk;                   // -c_B * Bz
  float inv_qy, inv_qz;        // float32(1 / q)
  // stream (caller's device arrays)
  float* coef;                 // [6 * n_tracks]
  float* x_ref;                // [n_tracks]
  uint32_t* first;             // [n_tracks + 1]
  uint8_t* row;                // [n_cl]
  int16_t* code;               // [2 * n_cl]
  float* raw;                  // [2 * n_cl]
  uint8_t* un_row;             // [N]
  float* un_yz;                // [2 * N]
  // workspace scratch
  uint32_t* unf;               // [N] 1 = on no track
  uint32_t* row_cnt;           // [SR] clusters on no track per (sector, row)
  uint32_t* row_pos;           // [SR + 1] exclusive scan of row_cnt
  uint32_t* n_escaped;
};

// C11 decoding of a stream into cluster arrays.
struct DecodeArgs {
  const float* coef;
  const float* x_ref;
  const uint32_t* first;
  const uint8_t* row;
  const int16_t* code;
  const float* raw;
  const uint8_t* un_row;
  const float* un_yz;
  uint32_t n_tracks;
  uint64_t n_cl, n_un;
  const RowConst* rows;
  float q_y, q_z;
  float* y_out;                // [n_cl + n_un]
  float* z_out;
  uint8_t* row_out;
};

constexpr int kScanBlock = 1024;                   // elements per scan block (256 threads x 4)
constexpr int kScanMaxBlocks = 8192;               // supports scans of up to 8M elements

// ---- launch wrappers (each in its own .hip file) ----
void launch_grid(const DevPtrs& d, uint32_t max_row_hits, uint32_t max_pack_hits, hipStream_t s);
void launch_links(const DevPtrs& d, uint32_t max_row_hits, hipStream_t s);
void launch_clean_starts(const DevPtrs& d, uint32_t max_row_hits, hipStream_t s);
void launch_tracklets(const DevPtrs& d, const KfConst& k, uint32_t max_row_hits, hipStream_t s);
void launch_select(const DevPtrs& d, const KfConst& k, uint32_t tile_rows, hipStream_t s);
void launch_merge(const DevPtrs& d, const MergeArgs& m, const KfConst& k, uint32_t n_tracks, hipStream_t s);
void launch_codec_encode(const CodecArgs& a, unsigned long long* scan_blocks, hipStream_t s);
void launch_codec_decode(const DecodeArgs& a, hipStream_t s);
// exclusive scans; n read from *n_dev when n_dev != nullptr (then n_max bounds the grid)
void launch_scan_u32(const uint32_t* in, uint32_t* out, uint32_t n, unsigned long long* blocks, hipStream_t s);
void launch_scan_u64(const unsigned long long* in, unsigned long long* out, const uint32_t* n_dev, uint32_t n_max,
                     unsigned long long* blocks, hipStream_t s);

}  // namespace tpc
