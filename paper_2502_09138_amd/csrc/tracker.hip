// Host runtime of the C ABI declared in include/tpc_tracker.h.
//
// create:  validate the configuration, derive the float32 constant tables
//          (double arithmetic, one rounding), carve one device workspace,
//          allocate pinned staging/output buffers.
// track:   validate the time frame on the host, stage row offsets and sector
//          constants, enqueue K1..K6 on one stream with no host sync, copy the
//          result header to pinned memory and record a completion event.
// get:     wait for the event, copy the compact outputs to pinned memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tpc_tracker.h"
#include "tpc_internal.h"

using namespace tpc;

namespace {

thread_local std::string g_last_error;

tpc_status fail(tpc_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(TPC_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

constexpr double kCB = 0.00299792458;

// Device scratch of the allocation-free entry point tpc_track_timeframe_scratch:
// a request's whole workspace (grid, links, tracklets, outputs) carved from one
// file-scope array of each device, so that call allocates nothing.  Its host
// address is a stand-in: host code uses only the device address looked up with
// hipGetSymbolAddress (g_scratch_ptr, per device).
constexpr uint64_t kScratchBytes = TPC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
constexpr uint64_t kAlign = 256;
constexpr uint32_t kSelectTileWords = 12288;     // 48 KB of LDS per selector tile at most
constexpr uint32_t kSelectThreadsAuto = 512;    // TPC_KNOB_SELECT_THREADS = 0: K6 tile workgroup size
constexpr uint32_t kLinkGroupAuto = 64;          // TPC_KNOB_LINK_GROUP = 0: K2 tiles per XCD group
constexpr uint32_t kSelectGlobal = 0xFFFFFFFFu;  // TPC_KNOB_SELECT_TILE_ROWS = -1: the global-memory selector

struct Layout {   // byte offsets of every workspace buffer
  uint64_t row_off, rows, secs, pack_first, row_dims, row_meta, bin_start, syz, sid, up0, down0, up1, down1, sflag, row_nstart,
      row_start_off, start_pos, start_sr, wave_off, tile_off, tile_sr, tk_rowhit, tk_info, tk_param, tk_cov, tk_chi2, k5_off, k5_perm, k5_inv, k5_rec, W, own_part, tk_pack,
      tk_scan, acc_list,
      out_sector, out_start, out_first, out_clusters, out_xref, out_param, out_cov, out_chi2, out_ndf, scan_blocks,
      hdr, in_y, in_z, m_phys, m_nbr, m_sec_first, m_succ, m_pred_key, m_next, m_has_pred, m_head_flag, m_head_scan,
      m_chain_cl, m_cl_scan, m_heads, m_head_of, m_first, m_clusters, m_param, m_cov, m_chi2, m_ndf, m_nseg, total;
};

struct Caps {
  uint64_t N, SRmax, T, MT, MC;
  uint32_t R, Smax;
};

Caps caps_of(const tpc_tracker_config& c) {
  Caps k;
  k.R = (uint32_t)c.n_rows;
  k.Smax = c.max_sectors;
  k.N = c.max_clusters;
  k.SRmax = (uint64_t)c.max_sectors * k.R;
  k.T = c.max_tracklets ? c.max_tracklets : std::max<uint64_t>(1, c.max_clusters / 4);
  k.MT = c.max_tracks ? c.max_tracks : k.T;
  k.MC = c.max_track_clusters ? c.max_track_clusters : std::max<uint64_t>(1, c.max_clusters);
  return k;
}

Layout layout_of(const Caps& k) {
  Layout L{};
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) {
    uint64_t at = o;
    o += (bytes + kAlign - 1) / kAlign * kAlign;
    return at;
  };
  // per-frame metadata, contiguous so that one copy from a pinned mirror fills it
  L.row_off = take((k.SRmax + 1) * 4);
  L.tile_off = take((k.SRmax + 1) * 4);
  L.secs = take((uint64_t)k.Smax * sizeof(SectorConst));
  L.pack_first = take((k.SRmax + 1) * 4);
  L.rows = take((uint64_t)k.R * sizeof(RowConst));
  L.row_dims = take(k.SRmax * 4);
  L.row_meta = take(k.SRmax * 8);
  // + 4 and + 2 entries: the tracklet stage reads both in 16-byte units
  L.bin_start = take((k.N + 2 * k.SRmax + 2 + 4) * 4);
  L.syz = take((k.N + 2) * 8);
  L.sid = take(k.N * 4);
  L.up0 = take(k.N * 4);
  L.down0 = take(k.N * 4);
  L.up1 = take(k.N * 4);
  L.down1 = take(k.N * 4);
  L.sflag = take(k.N);
  L.row_nstart = take(k.SRmax * 4);
  L.row_start_off = take((k.SRmax + 1) * 4);
  L.start_pos = take(k.T * 4);
  L.start_sr = take(k.T * 4);
  L.wave_off = take(((uint64_t)k.Smax + 1) * 4);
  L.tile_sr = take((k.N / kLinkTile + k.SRmax + 1) * 4);   // sum of ceil(N_r / 64) <= N / 64 + SR
  L.tk_rowhit = take((uint64_t)k.R * k.T * 4);
  L.tk_info = take(4 * k.T * 4);
  L.tk_param = take(5 * k.T * 4);
  L.tk_cov = take(15 * k.T * 4);
  L.tk_chi2 = take(k.T * 4);
  L.k5_off = take((k.SRmax + 1) * 4);
  L.k5_perm = take(k.T * 4);
  L.k5_inv = take(k.T * 4);
  L.k5_rec = take(k.T * 25 * 4);
  L.W = take(k.N * 4);
  L.own_part = take((uint64_t)k.R * k.T);
  L.tk_pack = take(k.T * 8);
  L.tk_scan = take((k.T + 1) * 8);
  L.acc_list = take((k.MT + 1) * 4);
  L.out_sector = take(k.MT * 4);
  L.out_start = take(k.MT * 4);
  L.out_first = take((k.MT + 1) * 4);
  L.out_clusters = take(k.MC * 4);
  L.out_xref = take(k.MT * 4);
  L.out_param = take(5 * k.MT * 4);
  L.out_cov = take(15 * k.MT * 4);
  L.out_chi2 = take(k.MT * 4);
  L.out_ndf = take(k.MT * 4);
  L.scan_blocks = take((uint64_t)kScanMaxBlocks * 8);
  L.hdr = take(sizeof(ResultHeader));
  L.in_y = take(k.N * 4);
  L.in_z = take(k.N * 4);
  // C8/C9 sector merger
  L.m_phys = take((uint64_t)k.Smax * 4);
  L.m_nbr = take((uint64_t)k.Smax * 8);
  L.m_sec_first = take(((uint64_t)k.Smax + 1) * 4);
  L.m_succ = take(k.MT * 4);
  L.m_pred_key = take(k.MT * 8);
  L.m_next = take(k.MT * 4);
  L.m_has_pred = take(k.MT * 4);
  L.m_head_flag = take(k.MT * 4);
  L.m_head_scan = take((k.MT + 1) * 4);
  L.m_chain_cl = take(k.MT * 4);
  L.m_cl_scan = take((k.MT + 1) * 4);
  L.m_heads = take(k.MT * 4);
  L.m_head_of = take(k.MT * 4);
  L.m_first = take((k.MT + 1) * 4);
  L.m_clusters = take(k.MC * 4);
  L.m_param = take(5 * k.MT * 4);
  L.m_cov = take(15 * k.MT * 4);
  L.m_chi2 = take(k.MT * 4);
  L.m_ndf = take(k.MT * 4);
  L.m_nseg = take(k.MT * 4);
  L.total = o;
  return L;
}

std::string validate_config(const tpc_tracker_config* c) {
  if (!c) return "config is NULL";
  if (c->abi_version != TPC_ABI_VERSION) return "abi_version mismatch";
  if (c->n_rows < 3 || c->n_rows > TPC_MAX_ROWS) return "n_rows out of range [3, 255]";
  if (!c->row_x || !c->row_half_y) return "row_x / row_half_y is NULL";
  for (int r = 0; r < c->n_rows; ++r) {
    if (!std::isfinite(c->row_x[r]) || !std::isfinite(c->row_half_y[r]) || !(c->row_half_y[r] > 0.0))
      return "row geometry not finite or half-width <= 0";
    if (r > 0 && !(c->row_x[r] > c->row_x[r - 1])) return "row_x not strictly increasing";
  }
  if (!std::isfinite(c->bz_tesla)) return "bz not finite";
  if (!(c->sigma_y > 0.0) || !(c->sigma_z > 0.0)) return "sigma_y/sigma_z must be > 0";
  if (c->grid_hits_per_bin < 1) return "grid_hits_per_bin must be >= 1";
  if (!(c->s_max > 0.0 && c->s_max < 1.0)) return "s_max must be in (0, 1)";
  if (!(c->gate_nsigma > 0.0) || !(c->win_cap > 0.0) || !(c->seed_qpt_max > 0.0)) return "gate/cap/qpt_max must be > 0";
  if (!(c->c0_sinphi > 0.0 && c->c0_tanl > 0.0 && c->c0_qpt > 0.0)) return "initial variances must be > 0";
  if (c->max_miss < 0 || c->min_tracklet_hits < 3 || c->min_track_hits < 1) return "hit-count cuts out of range";
  if (!(c->merge_dy >= 0.0 && c->merge_dz >= 0.0 && c->merge_dsinphi >= 0.0 && c->merge_dtanl >= 0.0 &&
        c->merge_dqpt >= 0.0))
    return "merge windows must be >= 0";
  if (c->max_sectors < 1) return "max_sectors must be >= 1";
  if (c->tracklet_schedule < 0 || c->tracklet_schedule > 2) return "tracklet_schedule must be 0, 1 or 2";
  if (c->max_clusters >= (1ull << 31)) return "max_clusters must be < 2^31";
  const Caps k = caps_of(*c);
  if (k.T > (uint64_t)kScanBlock * kScanMaxBlocks) return "max_tracklets exceeds 8M";
  if (k.SRmax + 1 > (uint64_t)kScanBlock * kScanMaxBlocks) return "max_sectors * n_rows too large";
  if (k.MT >= (1ull << 32) || k.MC >= (1ull << 32)) return "output capacities must be < 2^32";
  return "";
}

static __device__ __align__(256) unsigned char scratch[kScratchBytes];
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Device address of this device's scratch array (looked up once per device, with that device current).
tpc_status scratch_lookup(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) return fail(TPC_E_INVAL, "device ordinal beyond the scratch table");
  if (g_scratch_ptr[device]) return TPC_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return fail(TPC_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[device] = ptr;
  return TPC_OK;
}

}  // namespace

struct tpc_tracker {
  tpc_tracker_config cfg{};
  std::vector<double> row_x, row_half_y;
  Caps caps{};        // capacities of the current workspace binding
  Layout lay{};
  Caps host_caps{};   // capacities the pinned host buffers are sized for (create time)
  // the workspace requests run on unless they use the device scratch (create or bind_workspace)
  char* home_ws = nullptr;
  Caps home_caps{};
  Layout home_lay{};
  bool on_scratch = false;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  char* ws = nullptr;
  bool own_ws = false;
  DevPtrs d{};
  KfConst kc{};
  std::vector<RowConst> rows;
  // pinned host memory
  RowConst* h_rows = nullptr;   // row constants, uploaded into each workspace binding
  char* h_frame = nullptr;   // pinned mirror of the row_off / tile_off / secs block
  uint32_t* h_row_off = nullptr;
  uint32_t* h_tile_off = nullptr;
  SectorConst* h_secs = nullptr;
  uint32_t* h_pack = nullptr;
  ResultHeader* h_hdr = nullptr;
  char* h_out = nullptr;      // all outputs, laid out like the device outputs
  char* h_merge = nullptr;    // merger outputs (allocated at the first merge), laid out like the device ones
  int32_t* h_phys = nullptr;  // pinned copy of the sector numbers of a merge
  tpc_merged merged{};
  hipEvent_t done = nullptr;
  hipEvent_t ev[kPasses + 1] = {};
  uint32_t timing = 0;   // mask of timed passes
  uint32_t timed_last = 0;   // pass mask the last request was timed with
  // request state
  uint64_t next_id = 1, cur_id = 0;
  bool in_flight = false;
  bool fetched = false;
  uint32_t cur_S = 0, cur_N = 0;
  tpc_tracks out{};
  uint32_t select_tile_rows = 0;   // TPC_KNOB_SELECT_TILE_ROWS (0 = auto, kSelectGlobal = global selector)
};

namespace {

// Device pointers of every workspace buffer for the current binding (t->ws,
// t->lay, t->caps), and the pinned mirror's views of the per-frame block.
void carve(tpc_tracker* t) {
  DevPtrs& d = t->d;
  char* w = t->ws;
  const Layout& lay = t->lay;
  const Caps& caps = t->caps;
  const tpc_tracker_config* cfg = &t->cfg;
  const KfConst& k = t->kc;
  const uint32_t R = caps.R;
  d.row_off = (const uint32_t*)(w + lay.row_off);
  d.rows = (const RowConst*)(w + lay.rows);
  d.secs = (const SectorConst*)(w + lay.secs);
  d.pack_first = (const uint32_t*)(w + lay.pack_first);
  d.row_dims = (uint32_t*)(w + lay.row_dims);
  d.row_meta = (uint2*)(w + lay.row_meta);
  d.bin_start = (uint32_t*)(w + lay.bin_start);
  d.syz = (float2*)(w + lay.syz);
  d.sid = (uint32_t*)(w + lay.sid);
  d.up0 = (int32_t*)(w + lay.up0);
  d.down0 = (int32_t*)(w + lay.down0);
  d.up1 = (int32_t*)(w + lay.up1);
  d.down1 = (int32_t*)(w + lay.down1);
  d.sflag = (uint8_t*)(w + lay.sflag);
  d.row_nstart = (uint32_t*)(w + lay.row_nstart);
  d.row_start_off = (uint32_t*)(w + lay.row_start_off);
  d.start_pos = (uint32_t*)(w + lay.start_pos);
  d.start_sr = (uint32_t*)(w + lay.start_sr);
  d.wave_off = (uint32_t*)(w + lay.wave_off);
  d.tile_off = (const uint32_t*)(w + lay.tile_off);
  d.tile_sr = (uint32_t*)(w + lay.tile_sr);
  d.tk_rowhit = (int32_t*)(w + lay.tk_rowhit);
  d.tk_info = (int32_t*)(w + lay.tk_info);
  d.tk_param = (float*)(w + lay.tk_param);
  d.tk_cov = (float*)(w + lay.tk_cov);
  d.tk_chi2 = (float*)(w + lay.tk_chi2);
  d.k5_off = (uint32_t*)(w + lay.k5_off);
  d.k5_perm = (uint32_t*)(w + lay.k5_perm);
  d.k5_inv = (uint32_t*)(w + lay.k5_inv);
  d.k5_rec = (uint32_t*)(w + lay.k5_rec);
  d.W = (uint32_t*)(w + lay.W);
  d.own_part = (uint8_t*)(w + lay.own_part);
  d.tk_pack = (unsigned long long*)(w + lay.tk_pack);
  d.tk_scan = (unsigned long long*)(w + lay.tk_scan);
  d.acc_list = (uint32_t*)(w + lay.acc_list);
  d.out_sector = (uint32_t*)(w + lay.out_sector);
  d.out_start = (uint32_t*)(w + lay.out_start);
  d.out_first = (uint32_t*)(w + lay.out_first);
  d.out_clusters = (uint32_t*)(w + lay.out_clusters);
  d.out_xref = (float*)(w + lay.out_xref);
  d.out_param = (float*)(w + lay.out_param);
  d.out_cov = (float*)(w + lay.out_cov);
  d.out_chi2 = (float*)(w + lay.out_chi2);
  d.out_ndf = (int32_t*)(w + lay.out_ndf);
  d.scan_blocks = (unsigned long long*)(w + lay.scan_blocks);
  d.hdr = (ResultHeader*)(w + lay.hdr);
  d.grid_k = cfg->grid_hits_per_bin;
  d.k5_mode = cfg->tracklet_schedule;
  d.k2_group = kLinkGroupAuto;
  d.k6_threads = kSelectThreadsAuto;
  d.rho = k.rho;
  d.R = R;
  d.tcap = (uint32_t)caps.T;
  d.max_tracks = (uint32_t)caps.MT;
  d.max_track_clusters = caps.MC;
  if (t->h_frame) {
    t->h_row_off = (uint32_t*)t->h_frame;
    t->h_tile_off = (uint32_t*)(t->h_frame + (lay.tile_off - lay.row_off));
    t->h_secs = (SectorConst*)(t->h_frame + (lay.secs - lay.row_off));
    t->h_pack = (uint32_t*)(t->h_frame + (lay.pack_first - lay.row_off));
  }
}

}  // namespace

extern "C" {

void tpc_default_config(tpc_tracker_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof *c);
  c->abi_version = TPC_ABI_VERSION;
  c->n_rows = 152;
  c->bz_tesla = 0.5;
  c->sigma_y = 0.1;
  c->sigma_z = 0.15;
  c->grid_hits_per_bin = 2;
  c->win_a_y = 2.0;
  c->win_b_y = 0.5;
  c->win_a_z = 2.0;
  c->win_b_z = 0.7;
  c->link_nsigma = 4.0;
  c->s_max = 0.99;
  c->seed_qpt_max = 10.0;
  c->c0_sinphi = 0.25;
  c->c0_tanl = 0.25;
  c->c0_qpt = 25.0;
  c->gate_nsigma = 3.0;
  c->win_cap = 3.0;
  c->edge_margin = 1.0;
  c->max_miss = 5;
  c->min_tracklet_hits = 10;
  c->min_track_hits = 10;
  c->min_owned_frac = 0.5;
  c->merge_dy = 2.0;
  c->merge_dz = 2.0;
  c->merge_dsinphi = 0.05;
  c->merge_dtanl = 0.05;
  c->merge_dqpt = 1.0;
  c->max_sectors = 36;
  c->max_clusters = 2000000;
  c->device = 0;
}

uint64_t tpc_workspace_bytes(const tpc_tracker_config* cfg) {
  if (!validate_config(cfg).empty()) return 0;
  return layout_of(caps_of(*cfg)).total;
}

const char* tpc_last_error(void) { return g_last_error.c_str(); }

tpc_status tpc_tracker_create(const tpc_tracker_config* cfg, tpc_tracker** out) {
  if (!out) return fail(TPC_E_INVAL, "out is NULL");
  *out = nullptr;
  const std::string why = validate_config(cfg);
  if (!why.empty()) return fail(TPC_E_INVAL, why);
  const Caps caps = caps_of(*cfg);
  const Layout lay = layout_of(caps);
  if (cfg->workspace && cfg->workspace_bytes < lay.total) return fail(TPC_E_INVAL, "workspace too small");
  if (cfg->workspace && ((uintptr_t)cfg->workspace % kAlign)) return fail(TPC_E_INVAL, "workspace not 256-byte aligned");
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (cfg->device < 0 || cfg->device >= ndev) return fail(TPC_E_INVAL, "device ordinal out of range");
  HIP_TRY(hipSetDevice(cfg->device));
  tpc_tracker* t = new tpc_tracker();
  t->cfg = *cfg;
  t->row_x.assign(cfg->row_x, cfg->row_x + cfg->n_rows);
  t->row_half_y.assign(cfg->row_half_y, cfg->row_half_y + cfg->n_rows);
  t->cfg.row_x = t->row_x.data();
  t->cfg.row_half_y = t->row_half_y.data();
  t->caps = caps;
  t->lay = lay;
  t->device = cfg->device;
  auto cleanup = [&](tpc_status st) {
    tpc_tracker_destroy(t);
    return st;
  };
  if (cfg->stream) {
    t->stream = (hipStream_t)cfg->stream;
  } else {
    if (hipStreamCreateWithFlags(&t->stream, hipStreamNonBlocking) != hipSuccess)
      return cleanup(fail(TPC_E_DEVICE, "hipStreamCreate failed"));
    t->own_stream = true;
  }
  if (cfg->workspace) {
    t->ws = (char*)cfg->workspace;
  } else {
    if (hipMalloc((void**)&t->ws, lay.total) != hipSuccess) return cleanup(fail(TPC_E_NOMEM, "hipMalloc workspace"));
    t->own_ws = true;
  }
  // constant tables: double arithmetic, one rounding to float32
  const uint32_t R = caps.R;
  t->rows.resize(R);
  for (uint32_t r = 0; r < R; ++r) {
    RowConst& c = t->rows[r];
    std::memset(&c, 0, sizeof c);
    const double X = t->row_x[r], Y = t->row_half_y[r];
    c.x = (float)X;
    c.half_y = (float)Y;
    c.y_lo = (float)(-Y);
    c.inv_wy = (float)(1.0 / (2.0 * Y));
    c.ly = (int32_t)std::ceil(20.0 * Y);
    if (r >= 1 && r + 1 < R) {
      const double du = t->row_x[r + 1] - X, dd = X - t->row_x[r - 1];
      const double tt = dd / (dd + du);
      c.t = (float)tt;
      c.wy_up = (float)(cfg->win_a_y * du + cfg->win_b_y);
      c.wz_up = (float)(cfg->win_a_z * du + cfg->win_b_z);
      c.wy_dn = (float)(cfg->win_a_y * dd + cfg->win_b_y);
      c.wz_dn = (float)(cfg->win_a_z * dd + cfg->win_b_z);
      const double n2 = cfg->link_nsigma * cfg->link_nsigma, s2 = cfg->sigma_y * cfg->sigma_y;
      c.dmax = (float)((n2 * s2) * ((1.0 + tt * tt) + (1.0 - tt) * (1.0 - tt)));
    }
  }
  KfConst& k = t->kc;
  k.bk = (float)(-kCB * cfg->bz_tesla);
  k.s_max = (float)cfg->s_max;
  k.qpt_max = (float)cfg->seed_qpt_max;
  k.vy = (float)(cfg->sigma_y * cfg->sigma_y);
  k.vz = (float)(cfg->sigma_z * cfg->sigma_z);
  k.c0_sinphi = (float)cfg->c0_sinphi;
  k.c0_tanl = (float)cfg->c0_tanl;
  k.c0_qpt = (float)cfg->c0_qpt;
  k.gate = (float)cfg->gate_nsigma;
  k.cap = (float)cfg->win_cap;
  k.margin = (float)cfg->edge_margin;
  const double ry = cfg->sigma_y / cfg->sigma_z;
  k.rho = (float)(ry * ry);
  k.min_owned_frac = (float)cfg->min_owned_frac;
  k.max_miss = cfg->max_miss;
  k.min_tracklet_hits = cfg->min_tracklet_hits;
  k.min_track_hits = cfg->min_track_hits;
  k.grid_k = cfg->grid_hits_per_bin;
  k.n_rows = cfg->n_rows;
  // pinned host buffers, sized for the create-time capacities (later bindings are no larger)
  t->host_caps = caps;
  if (hipHostMalloc((void**)&t->h_frame, lay.pack_first + (caps.SRmax + 1) * 4 - lay.row_off) != hipSuccess ||
      hipHostMalloc((void**)&t->h_hdr, sizeof(ResultHeader)) != hipSuccess ||
      hipHostMalloc((void**)&t->h_rows, R * sizeof(RowConst)) != hipSuccess)
    return cleanup(fail(TPC_E_NOMEM, "hipHostMalloc staging"));
  const uint64_t out_bytes = lay.out_ndf + caps.MT * 4 - lay.out_sector;
  if (hipHostMalloc((void**)&t->h_out, out_bytes) != hipSuccess)
    return cleanup(fail(TPC_E_NOMEM, "hipHostMalloc outputs"));
  std::memcpy(t->h_rows, t->rows.data(), R * sizeof(RowConst));
  carve(t);
  t->home_ws = t->ws;
  t->home_caps = caps;
  t->home_lay = lay;
  if (hipMemcpy((void*)t->d.rows, t->h_rows, R * sizeof(RowConst), hipMemcpyHostToDevice) != hipSuccess)
    return cleanup(fail(TPC_E_DEVICE, "upload row constants"));
  if (const tpc_status st = scratch_lookup(cfg->device); st != TPC_OK) return cleanup(st);
  if (hipEventCreateWithFlags(&t->done, hipEventDisableTiming) != hipSuccess)
    return cleanup(fail(TPC_E_DEVICE, "hipEventCreate"));
  for (int i = 0; i <= kPasses; ++i)
    if (hipEventCreate(&t->ev[i]) != hipSuccess) return cleanup(fail(TPC_E_DEVICE, "hipEventCreate"));
  *out = t;
  g_last_error.clear();
  return TPC_OK;
}

void tpc_tracker_destroy(tpc_tracker* t) {
  if (!t) return;
  // teardown: errors here cannot be reported to anyone, so they are ignored
  (void)hipSetDevice(t->device);
  if (t->in_flight && t->done) (void)hipEventSynchronize(t->done);
  if (t->stream) (void)hipStreamSynchronize(t->stream);
  if (t->done) (void)hipEventDestroy(t->done);
  for (auto& e : t->ev)
    if (e) (void)hipEventDestroy(e);
  if (t->own_ws && t->home_ws) (void)hipFree(t->home_ws);
  if (t->h_frame) (void)hipHostFree(t->h_frame);
  if (t->h_hdr) (void)hipHostFree(t->h_hdr);
  if (t->h_out) (void)hipHostFree(t->h_out);
  if (t->h_rows) (void)hipHostFree(t->h_rows);
  if (t->h_merge) (void)hipHostFree(t->h_merge);
  if (t->h_phys) (void)hipHostFree(t->h_phys);
  if (t->own_stream && t->stream) (void)hipStreamDestroy(t->stream);
  delete t;
}

}  // extern "C"

namespace {

// Capacities of a workspace binding for at most max_clusters / max_sectors: the
// defaults for max_clusters, limited by what the tracker was created with.
Caps bound_caps(const tpc_tracker* t, uint64_t max_clusters, uint32_t max_sectors) {
  tpc_tracker_config c = t->cfg;
  c.max_clusters = max_clusters;
  c.max_sectors = max_sectors;
  c.max_tracklets = c.max_tracks = c.max_track_clusters = 0;
  Caps k = caps_of(c);
  const Caps& h = t->host_caps;
  k.T = std::min(k.T, h.T);
  k.MT = std::min(k.MT, h.MT);
  k.MC = std::min(k.MC, h.MC);
  return k;
}

}  // namespace

extern "C" {

uint64_t tpc_workspace_bytes_for(const tpc_tracker* t, uint64_t max_clusters, uint32_t max_sectors) {
  if (!t || max_sectors < 1 || max_clusters >= (1ull << 31)) return 0;
  if (max_clusters > t->host_caps.N || max_sectors > t->host_caps.Smax) return 0;
  return layout_of(bound_caps(t, max_clusters, max_sectors)).total;
}

tpc_status tpc_tracker_bind_workspace(tpc_tracker* t, void* workspace, uint64_t workspace_bytes, uint64_t max_clusters,
                                      uint32_t max_sectors) {
  if (!t) return fail(TPC_E_INVAL, "tracker is NULL");
  if (t->in_flight) return fail(TPC_E_BUSY, "a request is in flight");
  if (!workspace || ((uintptr_t)workspace % kAlign)) return fail(TPC_E_INVAL, "workspace NULL or not 256-byte aligned");
  if (max_sectors < 1 || max_sectors > t->host_caps.Smax || max_clusters > t->host_caps.N)
    return fail(TPC_E_INVAL, "capacities exceed those the tracker was created with");
  const Caps k = bound_caps(t, max_clusters, max_sectors);   // the pinned host buffers hold at most these
  const Layout lay = layout_of(k);
  if (workspace_bytes < lay.total) return fail(TPC_E_INVAL, "workspace too small for these capacities");
  HIP_TRY(hipSetDevice(t->device));
  if (t->own_ws && t->home_ws) {
    HIP_TRY(hipStreamSynchronize(t->stream));
    HIP_TRY(hipFree(t->home_ws));
  }
  t->own_ws = false;
  t->home_ws = t->ws = (char*)workspace;
  t->home_caps = t->caps = k;
  t->home_lay = t->lay = lay;
  t->on_scratch = false;
  carve(t);
  // the row constants live in the workspace: upload them into the new one, in stream order
  HIP_TRY(hipMemcpyAsync((void*)t->d.rows, t->h_rows, k.R * sizeof(RowConst), hipMemcpyHostToDevice, t->stream));
  return TPC_OK;
}

}  // extern "C"

namespace {

__global__ void k_begin(ResultHeader* h) {
  h->n_starts = 0;
  h->error_flags = 0;
  h->n_tracks = 0;
  h->pad0 = 0;
  h->codec_escaped = 0;
  h->codec_unassigned = 0;
  h->n_track_clusters = 0;
  h->n_steps = 0;
}

std::string validate_frame(const tpc_tracker* t, const Caps& caps, const tpc_timeframe* f, uint32_t* max_row) {
  if (!f) return "timeframe is NULL";
  if (f->n_rows != (uint32_t)t->cfg.n_rows) return "n_rows differs from the configuration";
  if (f->n_sectors < 1 || f->n_sectors > caps.Smax) return "n_sectors out of range";
  if (f->n_clusters > caps.N) return "n_clusters exceeds max_clusters";
  if (!f->row_offsets || !f->sector_z_lo || !f->sector_z_hi) return "row_offsets / sector z ranges are NULL";
  if (f->n_clusters && (!f->y || !f->z)) return "y / z is NULL";
  if (f->flags & ~1u) return "unknown flags";
  const uint64_t SR = (uint64_t)f->n_sectors * f->n_rows;
  if (f->row_offsets[0] != 0) return "row_offsets[0] != 0";
  uint32_t mx = 0;
  for (uint64_t i = 0; i < SR; ++i) {
    if (f->row_offsets[i + 1] < f->row_offsets[i]) return "row_offsets not non-decreasing";
    mx = std::max(mx, f->row_offsets[i + 1] - f->row_offsets[i]);
  }
  if (f->row_offsets[SR] != f->n_clusters) return "row_offsets does not end at n_clusters";
  if (mx > TPC_MAX_ROW_HITS) return "a row holds more than 65535 clusters";
  for (uint32_t s = 0; s < f->n_sectors; ++s) {
    const float lo = f->sector_z_lo[s], hi = f->sector_z_hi[s];
    if (!std::isfinite(lo) || !std::isfinite(hi) || !(hi > lo) || std::fabs(lo) > TPC_MAX_COORD ||
        std::fabs(hi) > TPC_MAX_COORD)
      return "sector z range invalid";
  }
  *max_row = mx;
  return "";
}

// Enqueues C1..C7 of a validated frame on the tracker's current workspace binding.
tpc_status enqueue(tpc_tracker* t, const tpc_timeframe* f, uint32_t max_row, uint64_t* request_id) {
  DevPtrs& d = t->d;
  const uint32_t S = f->n_sectors, R = f->n_rows, SR = S * R, N = (uint32_t)f->n_clusters;
  d.S = S;
  d.SR = SR;
  d.N = N;
  std::memcpy(t->h_row_off, f->row_offsets, (SR + 1) * sizeof(uint32_t));
  for (uint32_t s = 0; s < S; ++s) {
    SectorConst& c = t->h_secs[s];
    const double w = (double)f->sector_z_hi[s] - (double)f->sector_z_lo[s];
    c.z_lo = f->sector_z_lo[s];
    c.inv_wz = (float)(1.0 / w);
    c.lz = (int32_t)std::ceil(10.0 * w);
    c.pad = 0;
  }
  hipStream_t st = t->stream;   // the previous request was released, so the staging buffers are free
  if (f->flags & TPC_IN_HOST) {
    d.y = (const float*)(t->ws + t->lay.in_y);
    d.z = (const float*)(t->ws + t->lay.in_z);
    if (N) {
      HIP_TRY(hipMemcpyAsync((void*)d.y, f->y, (size_t)N * 4, hipMemcpyHostToDevice, st));
      HIP_TRY(hipMemcpyAsync((void*)d.z, f->z, (size_t)N * 4, hipMemcpyHostToDevice, st));
      HIP_TRY(hipStreamSynchronize(st));   // host arrays may be released on return
    }
  } else {
    d.y = f->y;
    d.z = f->z;
  }
  // K2 tiles: ceil(N_r / kLinkTile) per row, first tile of each row
  {
    uint32_t nt = 0;
    for (uint32_t i = 0; i < SR; ++i) {
      t->h_tile_off[i] = nt;
      nt += (f->row_offsets[i + 1] - f->row_offsets[i] + kLinkTile - 1) / kLinkTile;
    }
    t->h_tile_off[SR] = nt;
    d.n_link_tiles = nt;
  }
  // K1 packs: consecutive rows up to kPackHits hits and kPackRows rows (a larger row alone)
  uint32_t max_pack = 0;
  {
    uint32_t np = 0, cur = 0, rows = 0;
    for (uint32_t i = 0; i < SR; ++i) {
      const uint32_t n = f->row_offsets[i + 1] - f->row_offsets[i];
      if (rows && (cur + n > kPackHits || rows == kPackRows)) {
        max_pack = std::max(max_pack, cur);
        cur = rows = 0;
      }
      if (!rows) t->h_pack[np++] = i;
      cur += n;
      ++rows;
    }
    if (rows) max_pack = std::max(max_pack, cur);
    t->h_pack[np] = SR;
    d.n_packs = np;
  }
  // row offsets, tile offsets, sector constants and packs in one copy
  HIP_TRY(hipMemcpyAsync((void*)d.row_off, t->h_frame, t->lay.pack_first + (d.n_packs + 1) * 4 - t->lay.row_off,
                         hipMemcpyHostToDevice, st));
  // selector tile: 4 rows, or 2 or 1 where a block of 4 rows would need more
  // than kSelectTileWords words of LDS; 0 = rows too large, global-memory
  // selector.  (Measured with the batched selector loads: 4 rows up to 48 KB
  // of LDS beat the earlier 16 KB limit for multi-row tiles on every workload
  // -- time frame 3.98 against 4.14 ms per frame, central event 1.026 against
  // 1.032 ms, chunks 11.11 against 11.45 ms.)  Per-tile owned counts are
  // bytes, so tiles need at most 255 rows per sector.
  uint32_t tile_rows = 0, tile_cap = 0;
  const uint32_t forced = t->select_tile_rows == kSelectGlobal ? 0u : t->select_tile_rows;
  for (uint32_t tr = forced ? forced : 4; tr >= 1 && tile_rows == 0 && R <= 255 && t->select_tile_rows != kSelectGlobal;
       tr /= 2) {
    uint32_t mx = 0;
    for (uint32_t s = 0; s < S; ++s)
      for (uint32_t ra = 0; ra < R; ra += tr) {
        const uint32_t rb = std::min(R, ra + tr);
        mx = std::max(mx, f->row_offsets[s * R + rb] - f->row_offsets[s * R + ra]);
      }
    if (mx <= kSelectTileWords) {
      tile_rows = tr;
      tile_cap = std::max(mx, 1u);
    }
  }
  d.tile_cap = tile_cap;
  // event b opens pass b and closes pass b - 1: recorded when either is timed
  const uint32_t tmask = t->timing;
  auto mark = [&](int b) -> hipError_t {
    const uint32_t need = (tmask >> b) | (b > 0 ? tmask >> (b - 1) : 0u);
    return (need & 1u) ? hipEventRecord(t->ev[b], st) : hipSuccess;
  };
  HIP_TRY(mark(0));
  hipLaunchKernelGGL(k_begin, dim3(1), dim3(1), 0, st, d.hdr);
  launch_grid(d, max_row, max_pack, st);
  HIP_TRY(mark(1));
  launch_links(d, max_row, st);
  HIP_TRY(mark(2));
  launch_clean_starts(d, max_row, st);
  HIP_TRY(mark(3));
  launch_tracklets(d, t->kc, max_row, st);
  HIP_TRY(mark(4));
  launch_select(d, t->kc, tile_rows, st);
  HIP_TRY(mark(5));
  HIP_TRY(hipMemcpyAsync(t->h_hdr, d.hdr, sizeof(ResultHeader), hipMemcpyDeviceToHost, st));
  HIP_TRY(mark(6));
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(t->done, st));
  t->timed_last = tmask;
  t->cur_id = t->next_id++;
  t->in_flight = true;
  t->fetched = false;
  t->cur_S = S;
  t->cur_N = N;
  if (request_id) *request_id = t->cur_id;
  return TPC_OK;
}

}  // namespace

extern "C" {

tpc_status tpc_track_timeframe(tpc_tracker* t, const tpc_timeframe* f, uint64_t* request_id) {
  if (!t) return fail(TPC_E_INVAL, "tracker is NULL");
  if (t->in_flight) return fail(TPC_E_BUSY, "previous request not released");
  uint32_t max_row = 0;
  const std::string why = validate_frame(t, t->home_caps, f, &max_row);
  if (!why.empty()) return fail(TPC_E_INVAL, why);
  HIP_TRY(hipSetDevice(t->device));
  if (t->on_scratch) {   // back on the tracker's own workspace (its row constants are still there)
    t->ws = t->home_ws;
    t->caps = t->home_caps;
    t->lay = t->home_lay;
    t->on_scratch = false;
    carve(t);
  }
  return enqueue(t, f, max_row, request_id);
}

tpc_status tpc_track_timeframe_scratch(tpc_tracker* t, const tpc_timeframe* f, uint64_t* request_id) {
  if (!t) return fail(TPC_E_INVAL, "tracker is NULL");
  if (t->in_flight) return fail(TPC_E_BUSY, "previous request not released");
  uint32_t max_row = 0;
  const std::string why = validate_frame(t, t->host_caps, f, &max_row);
  if (!why.empty()) return fail(TPC_E_INVAL, why);
  const Caps k = bound_caps(t, std::max<uint64_t>(1, f->n_clusters), f->n_sectors);
  const Layout lay = layout_of(k);
  if (lay.total > kScratchBytes)
    return fail(TPC_E_INVAL, "the frame needs " + std::to_string(lay.total) + " bytes of device scratch; the scratch holds " +
                                 std::to_string(kScratchBytes));
  void* ptr = t->device < kMaxDevices ? g_scratch_ptr[t->device] : nullptr;
  if (!ptr) return fail(TPC_E_DEVICE, "device scratch address not looked up");
  HIP_TRY(hipSetDevice(t->device));
  t->ws = (char*)ptr;
  t->caps = k;
  t->lay = lay;
  t->on_scratch = true;
  carve(t);
  // another tracker may have used the scratch since: its row constants go in with every request
  HIP_TRY(hipMemcpyAsync((void*)t->d.rows, t->h_rows, k.R * sizeof(RowConst), hipMemcpyHostToDevice, t->stream));
  return enqueue(t, f, max_row, request_id);
}

tpc_status tpc_get_tracks(tpc_tracker* t, uint64_t request_id, int32_t blocking, tpc_tracks* out) {
  if (!t || !out) return fail(TPC_E_INVAL, "NULL argument");
  if (!t->in_flight || request_id != t->cur_id) return fail(TPC_E_INVAL, "unknown request id");
  HIP_TRY(hipSetDevice(t->device));
  if (!blocking) {
    hipError_t q = hipEventQuery(t->done);
    if (q == hipErrorNotReady) return fail(TPC_E_NOTREADY, "request still running");
    if (q != hipSuccess) return fail(TPC_E_DEVICE, hipGetErrorString(q));
  }
  HIP_TRY(hipEventSynchronize(t->done));
  std::memset(out, 0, sizeof *out);
  const ResultHeader h = *t->h_hdr;
  out->error_flags = h.error_flags;
  out->n_tracklets = h.n_starts;
  out->n_steps = h.n_steps;
  if (h.error_flags & TPC_ERR_NONFINITE) return fail(TPC_E_INPUT, "non-finite or out-of-range cluster coordinate");
  if (h.error_flags) return fail(TPC_E_CAPACITY, "capacity exceeded (see error_flags)");
  const DevPtrs& d = t->d;
  const Layout& L = t->lay;
  char* ho = t->h_out;
  auto host = [&](uint64_t off) { return ho + (off - L.out_sector); };
  if (!t->fetched) {
    const uint32_t n = h.n_tracks;
    const uint64_t nc = h.n_track_clusters;
    hipStream_t st = t->stream;
    struct {
      const void* src;
      uint64_t off, bytes;
    } cp[] = {
        {d.out_sector, L.out_sector, n * 4ull},      {d.out_start, L.out_start, n * 4ull},
        {d.out_first, L.out_first, (n + 1) * 4ull},  {d.out_clusters, L.out_clusters, nc * 4},
        {d.out_xref, L.out_xref, n * 4ull},          {d.out_param, L.out_param, n * 20ull},
        {d.out_cov, L.out_cov, n * 60ull},           {d.out_chi2, L.out_chi2, n * 4ull},
        {d.out_ndf, L.out_ndf, n * 4ull},
    };
    for (auto& c : cp)
      if (c.bytes) HIP_TRY(hipMemcpyAsync(host(c.off), c.src, c.bytes, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    t->fetched = true;
  }
  out->n_tracks = h.n_tracks;
  out->n_track_clusters = h.n_track_clusters;
  out->track_sector = (const uint32_t*)host(L.out_sector);
  out->track_start = (const uint32_t*)host(L.out_start);
  out->track_first = (const uint32_t*)host(L.out_first);
  out->cluster_ids = (const uint32_t*)host(L.out_clusters);
  out->x_ref = (const float*)host(L.out_xref);
  out->param = (const float*)host(L.out_param);
  out->cov = (const float*)host(L.out_cov);
  out->chi2 = (const float*)host(L.out_chi2);
  out->ndf = (const int32_t*)host(L.out_ndf);
  return TPC_OK;
}

tpc_status tpc_get_tracks_device(tpc_tracker* t, uint64_t request_id, int32_t blocking, tpc_tracks* out) {
  if (!t || !out) return fail(TPC_E_INVAL, "NULL argument");
  if (!t->in_flight || request_id != t->cur_id) return fail(TPC_E_INVAL, "unknown request id");
  HIP_TRY(hipSetDevice(t->device));
  if (!blocking) {
    hipError_t q = hipEventQuery(t->done);
    if (q == hipErrorNotReady) return fail(TPC_E_NOTREADY, "request still running");
    if (q != hipSuccess) return fail(TPC_E_DEVICE, hipGetErrorString(q));
  }
  HIP_TRY(hipEventSynchronize(t->done));
  std::memset(out, 0, sizeof *out);
  const ResultHeader h = *t->h_hdr;
  out->error_flags = h.error_flags;
  out->n_tracklets = h.n_starts;
  out->n_steps = h.n_steps;
  if (h.error_flags & TPC_ERR_NONFINITE) return fail(TPC_E_INPUT, "non-finite or out-of-range cluster coordinate");
  if (h.error_flags) return fail(TPC_E_CAPACITY, "capacity exceeded (see error_flags)");
  const DevPtrs& d = t->d;
  out->n_tracks = h.n_tracks;
  out->n_track_clusters = h.n_track_clusters;
  out->track_sector = d.out_sector;
  out->track_start = d.out_start;
  out->track_first = d.out_first;
  out->cluster_ids = d.out_clusters;
  out->x_ref = d.out_xref;
  out->param = d.out_param;
  out->cov = d.out_cov;
  out->chi2 = d.out_chi2;
  out->ndf = d.out_ndf;
  return TPC_OK;
}

tpc_status tpc_merge_sectors(tpc_tracker* t, uint64_t request_id, const int32_t* sector_phys, tpc_merged* out) {
  if (!t || !out) return fail(TPC_E_INVAL, "NULL argument");
  if (!t->in_flight || request_id != t->cur_id) return fail(TPC_E_INVAL, "unknown request id");
  const uint32_t S = t->cur_S;
  if (sector_phys)
    for (uint32_t s = 0; s < S; ++s)
      if (sector_phys[s] < -1 || sector_phys[s] >= 36) return fail(TPC_E_INVAL, "sector number out of range [-1, 35]");
  HIP_TRY(hipSetDevice(t->device));
  HIP_TRY(hipEventSynchronize(t->done));
  const ResultHeader h = *t->h_hdr;
  if (h.error_flags) return fail(h.error_flags & TPC_ERR_NONFINITE ? TPC_E_INPUT : TPC_E_CAPACITY, "the request failed");
  const Layout& L = t->lay;
  const Caps& hc = t->host_caps;
  const Layout HL = layout_of(hc);   // pinned merge buffers are laid out for the create-time capacities
  if (!t->h_merge) {
    if (hipHostMalloc((void**)&t->h_merge, HL.m_nseg + hc.MT * 4 - HL.m_next) != hipSuccess ||
        hipHostMalloc((void**)&t->h_phys, (size_t)hc.Smax * 4) != hipSuccess)
      return fail(TPC_E_NOMEM, "hipHostMalloc merge buffers");
  }
  char* w = t->ws;
  MergeArgs m{};
  m.phys = (const int32_t*)(w + L.m_phys);
  m.nbr = (int32_t*)(w + L.m_nbr);
  m.sec_first = (uint32_t*)(w + L.m_sec_first);
  m.succ = (int32_t*)(w + L.m_succ);
  m.pred_key = (unsigned long long*)(w + L.m_pred_key);
  m.next = (int32_t*)(w + L.m_next);
  m.has_pred = (uint32_t*)(w + L.m_has_pred);
  m.head_flag = (uint32_t*)(w + L.m_head_flag);
  m.head_scan = (uint32_t*)(w + L.m_head_scan);
  m.chain_clusters = (uint32_t*)(w + L.m_chain_cl);
  m.cl_scan = (uint32_t*)(w + L.m_cl_scan);
  m.heads = (uint32_t*)(w + L.m_heads);
  m.head_of = (uint32_t*)(w + L.m_head_of);
  m.first = (uint32_t*)(w + L.m_first);
  m.clusters = (uint32_t*)(w + L.m_clusters);
  m.param = (float*)(w + L.m_param);
  m.cov = (float*)(w + L.m_cov);
  m.chi2 = (float*)(w + L.m_chi2);
  m.ndf = (int32_t*)(w + L.m_ndf);
  m.nseg = (int32_t*)(w + L.m_nseg);
  m.cos20 = std::cos(20.0 * 3.14159265358979323846 / 180.0);
  m.sin20 = std::sin(20.0 * 3.14159265358979323846 / 180.0);
  const tpc_tracker_config& c = t->cfg;
  m.bk = -kCB * c.bz_tesla;
  m.s_max = c.s_max;
  m.vy = c.sigma_y * c.sigma_y;
  m.vz = c.sigma_z * c.sigma_z;
  m.c0_sinphi = c.c0_sinphi;
  m.c0_tanl = c.c0_tanl;
  m.c0_qpt = c.c0_qpt;
  m.dy = c.merge_dy;
  m.dz = c.merge_dz;
  m.dsinphi = c.merge_dsinphi;
  m.dtanl = c.merge_dtanl;
  m.dqpt = c.merge_dqpt;
  for (uint32_t s = 0; s < S; ++s) t->h_phys[s] = sector_phys ? sector_phys[s] : -1;
  hipStream_t st = t->stream;
  HIP_TRY(hipMemcpyAsync((void*)m.phys, t->h_phys, (size_t)S * 4, hipMemcpyHostToDevice, st));
  const uint32_t n = h.n_tracks;
  launch_merge(t->d, m, t->kc, n, st);
  HIP_TRY(hipGetLastError());
  // counts, then the arrays
  uint32_t* cnt = (uint32_t*)(t->h_merge + (HL.m_head_scan - HL.m_next));
  HIP_TRY(hipMemcpyAsync(cnt, m.head_scan + n, 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(cnt + 1, m.cl_scan + n, 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const uint32_t nc = n ? cnt[0] : 0;
  const uint64_t ncl = n ? cnt[1] : 0;
  auto host = [&](uint64_t off) { return t->h_merge + (off - HL.m_next); };
  struct {
    const void* src;
    uint64_t off, bytes;
  } cp[] = {
      {m.next, HL.m_next, n * 4ull},           {m.head_of, HL.m_head_of, n * 4ull},
      {m.heads, HL.m_heads, nc * 4ull},        {m.nseg, HL.m_nseg, nc * 4ull},
      {m.first, HL.m_first, (nc + 1) * 4ull},  {m.clusters, HL.m_clusters, ncl * 4},
      {m.param, HL.m_param, nc * 20ull},       {m.cov, HL.m_cov, nc * 60ull},
      {m.chi2, HL.m_chi2, nc * 4ull},          {m.ndf, HL.m_ndf, nc * 4ull},
  };
  if (n) {
    for (auto& e : cp)
      if (e.bytes) HIP_TRY(hipMemcpyAsync(host(e.off), e.src, e.bytes, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
  } else {
    *(uint32_t*)host(HL.m_first) = 0;
  }
  std::memset(out, 0, sizeof *out);
  out->n_tracks = n;
  out->n_chains = nc;
  out->n_chain_clusters = ncl;
  out->next = (const int32_t*)host(HL.m_next);
  out->head_of = (const uint32_t*)host(HL.m_head_of);
  out->heads = (const uint32_t*)host(HL.m_heads);
  out->nseg = (const int32_t*)host(HL.m_nseg);
  out->first = (const uint32_t*)host(HL.m_first);
  out->clusters = (const uint32_t*)host(HL.m_clusters);
  out->param = (const float*)host(HL.m_param);
  out->cov = (const float*)host(HL.m_cov);
  out->chi2 = (const float*)host(HL.m_chi2);
  out->ndf = (const int32_t*)host(HL.m_ndf);
  return TPC_OK;
}

namespace {
bool good_quantum(float q) { return std::isfinite(q) && q > 0.0f; }
}  // namespace

tpc_status tpc_encode_tracks(tpc_tracker* t, uint64_t request_id, float q_y, float q_z, const tpc_codec_stream* out,
                             tpc_codec_counts* counts) {
  if (!t || !out || !counts) return fail(TPC_E_INVAL, "NULL argument");
  if (!t->in_flight || request_id != t->cur_id) return fail(TPC_E_INVAL, "unknown request id");
  if (!good_quantum(q_y) || !good_quantum(q_z)) return fail(TPC_E_INVAL, "quanta must be finite and > 0");
  if (!out->coef || !out->x_ref || !out->first || !out->row || !out->code || !out->raw || !out->un_row || !out->un_yz)
    return fail(TPC_E_INVAL, "NULL stream array");
  HIP_TRY(hipSetDevice(t->device));
  HIP_TRY(hipEventSynchronize(t->done));
  const ResultHeader h = *t->h_hdr;
  if (h.error_flags) return fail(h.error_flags & TPC_ERR_NONFINITE ? TPC_E_INPUT : TPC_E_CAPACITY, "the request failed");
  const DevPtrs& d = t->d;
  CodecArgs a{};
  a.param = d.out_param;
  a.xref_in = d.out_xref;
  a.first_in = d.out_first;
  a.clusters = d.out_clusters;
  a.n_tracks = h.n_tracks;
  a.n_cl = h.n_track_clusters;
  a.row_off = d.row_off;
  a.SR = t->cur_S * t->caps.R;
  a.R = t->caps.R;
  a.N = t->cur_N;
  a.rows = d.rows;
  a.y = d.y;
  a.z = d.z;
  a.bk = -kCB * t->cfg.bz_tesla;
  a.inv_qy = (float)(1.0 / (double)q_y);
  a.inv_qz = (float)(1.0 / (double)q_z);
  a.coef = out->coef;
  a.x_ref = out->x_ref;
  a.first = out->first;
  a.row = out->row;
  a.code = out->code;
  a.raw = out->raw;
  a.un_row = out->un_row;
  a.un_yz = out->un_yz;
  // scratch of the completed request: the C6 ownership words (one per
  // cluster) and the C4 / K5 per-row counts
  a.unf = d.W;
  a.row_cnt = d.row_nstart;
  a.row_pos = d.k5_off;
  a.n_escaped = &d.hdr->codec_escaped;
  hipStream_t st = t->stream;
  launch_codec_encode(a, d.scan_blocks, st);
  HIP_TRY(hipGetLastError());
  uint32_t* cnt = reinterpret_cast<uint32_t*>(&t->h_hdr->codec_escaped);
  HIP_TRY(hipMemcpyAsync(cnt, a.n_escaped, 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(&t->h_hdr->codec_unassigned, a.row_pos + a.SR, 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  counts->n_tracks = a.n_tracks;
  counts->n_track_clusters = a.n_cl;
  counts->n_escaped = t->h_hdr->codec_escaped;
  counts->n_unassigned = a.SR ? t->h_hdr->codec_unassigned : 0;
  return TPC_OK;
}

tpc_status tpc_decode_tracks(tpc_tracker* t, const tpc_codec_stream* in, const tpc_codec_counts* counts, float q_y,
                             float q_z, float* y_out, float* z_out, uint8_t* row_out) {
  if (!t || !in || !counts || !y_out || !z_out || !row_out) return fail(TPC_E_INVAL, "NULL argument");
  if (!good_quantum(q_y) || !good_quantum(q_z)) return fail(TPC_E_INVAL, "quanta must be finite and > 0");
  if ((counts->n_tracks && (!in->coef || !in->x_ref || !in->first)) ||
      (counts->n_track_clusters && (!in->row || !in->code || !in->raw)) ||
      (counts->n_unassigned && (!in->un_row || !in->un_yz)))
    return fail(TPC_E_INVAL, "NULL stream array");
  if (counts->n_track_clusters && !counts->n_tracks) return fail(TPC_E_INVAL, "track clusters without tracks");
  HIP_TRY(hipSetDevice(t->device));
  DecodeArgs a{};
  a.coef = in->coef;
  a.x_ref = in->x_ref;
  a.first = in->first;
  a.row = in->row;
  a.code = in->code;
  a.raw = in->raw;
  a.un_row = in->un_row;
  a.un_yz = in->un_yz;
  a.n_tracks = counts->n_tracks;
  a.n_cl = counts->n_track_clusters;
  a.n_un = counts->n_unassigned;
  a.rows = t->d.rows;
  a.q_y = q_y;
  a.q_z = q_z;
  a.y_out = y_out;
  a.z_out = z_out;
  a.row_out = row_out;
  hipStream_t st = t->stream;
  if (a.n_cl + a.n_un) launch_codec_decode(a, st);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  return TPC_OK;
}

tpc_status tpc_release(tpc_tracker* t, uint64_t request_id) {
  if (!t) return fail(TPC_E_INVAL, "tracker is NULL");
  if (!t->in_flight || request_id != t->cur_id) return fail(TPC_E_INVAL, "unknown request id");
  HIP_TRY(hipSetDevice(t->device));
  HIP_TRY(hipEventSynchronize(t->done));
  t->in_flight = false;
  return TPC_OK;
}

tpc_status tpc_debug_copy(tpc_tracker* t, int32_t what, void* dst, uint64_t cap, uint64_t* bytes) {
  if (!t) return fail(TPC_E_INVAL, "tracker is NULL");
  HIP_TRY(hipSetDevice(t->device));
  HIP_TRY(hipStreamSynchronize(t->stream));
  const DevPtrs& d = t->d;
  const uint64_t N = t->cur_N, SR = (uint64_t)t->cur_S * t->caps.R, T = t->caps.T;
  const uint64_t ns = std::min<uint64_t>(t->h_hdr->n_starts, T);
  const void* src = nullptr;
  uint64_t n = 0;
  switch (what) {
    case TPC_DBG_SORTED_ID: src = d.sid; n = N * 4; break;
    case TPC_DBG_SORTED_YZ: src = d.syz; n = N * 8; break;
    case TPC_DBG_BIN_START: src = d.bin_start; n = (N + 2 * SR) * 4; break;
    case TPC_DBG_ROW_DIMS: src = d.row_dims; n = SR * 4; break;
    case TPC_DBG_UP0: src = d.up0; n = N * 4; break;
    case TPC_DBG_DOWN0: src = d.down0; n = N * 4; break;
    case TPC_DBG_UP1: src = d.up1; n = N * 4; break;
    case TPC_DBG_DOWN1: src = d.down1; n = N * 4; break;
    case TPC_DBG_STARTS: src = d.start_pos; n = ns * 4; break;
    case TPC_DBG_TK_ROWHIT: src = d.tk_rowhit; n = (uint64_t)t->caps.R * T * 4; break;
    case TPC_DBG_TK_INFO: src = d.tk_info; n = 4 * T * 4; break;
    case TPC_DBG_TK_PARAM: src = d.tk_param; n = 5 * T * 4; break;
    case TPC_DBG_TK_COV: src = d.tk_cov; n = 15 * T * 4; break;
    case TPC_DBG_TK_CHI2: src = d.tk_chi2; n = ns * 4; break;
    default: return fail(TPC_E_INVAL, "unknown debug array");
  }
  if (bytes) *bytes = n;
  if (dst && n) HIP_TRY(hipMemcpy(dst, src, std::min(cap, n), hipMemcpyDeviceToHost));
  return TPC_OK;
}

tpc_status tpc_set_tracklet_schedule(tpc_tracker* t, int32_t schedule) {
  if (!t) return fail(TPC_E_INVAL, "tracker is NULL");
  if (schedule < 0 || schedule > 2) return fail(TPC_E_INVAL, "tracklet_schedule must be 0, 1 or 2");
  if (t->in_flight) return fail(TPC_E_INVAL, "a request is in flight");
  t->cfg.tracklet_schedule = schedule;
  t->d.k5_mode = schedule;
  return TPC_OK;
}

tpc_status tpc_set_knob(tpc_tracker* t, int32_t knob, int32_t value) {
  if (!t) return fail(TPC_E_INVAL, "tracker is NULL");
  if (t->in_flight) return fail(TPC_E_INVAL, "a request is in flight");
  switch (knob) {
    case TPC_KNOB_TRACKLET_SCHEDULE:
      return tpc_set_tracklet_schedule(t, value);
    case TPC_KNOB_SELECT_TILE_ROWS:
      if (value != 0 && value != 1 && value != 2 && value != 4 && value != -1)
        return fail(TPC_E_INVAL, "select tile rows must be 0, 1, 2, 4 or -1");
      t->select_tile_rows = value < 0 ? kSelectGlobal : (uint32_t)value;
      return TPC_OK;
    case TPC_KNOB_REFIT_ORDER:
      if (value != 0 && value != 1) return fail(TPC_E_INVAL, "refit order must be 0 or 1");
      t->d.k5_refit_order = value;
      return TPC_OK;
    case TPC_KNOB_LINK_SLOTS:
      if (value != 0 && value != 4 && value != 8) return fail(TPC_E_INVAL, "link slots must be 0, 4 or 8");
      t->d.k2_slots = value;
      return TPC_OK;
    case TPC_KNOB_SELECT_THREADS:
      if (value != 0 && value != 256 && value != 512 && value != 1024)
        return fail(TPC_E_INVAL, "select threads must be 0, 256, 512 or 1024");
      t->d.k6_threads = value == 0 ? kSelectThreadsAuto : (uint32_t)value;
      return TPC_OK;
    case TPC_KNOB_LINK_GROUP:
      if (value < -1 || value > 4096) return fail(TPC_E_INVAL, "link group must be 0 (auto), -1 or 1..4096 tiles");
      t->d.k2_group = value == 0 ? kLinkGroupAuto : value < 0 ? kLinkGroupEighth : (uint32_t)value;
      return TPC_OK;
    default:
      return fail(TPC_E_INVAL, "unknown knob");
  }
}

tpc_status tpc_set_timing(tpc_tracker* t, int32_t pass_mask) {
  if (!t) return fail(TPC_E_INVAL, "tracker is NULL");
  if (pass_mask & ~TPC_TIME_ALL_PASSES) return fail(TPC_E_INVAL, "pass_mask has bits beyond the passes");
  t->timing = (uint32_t)pass_mask;
  return TPC_OK;
}

tpc_status tpc_get_pass_times(tpc_tracker* t, float* ms, int32_t n) {
  if (!t || !ms) return fail(TPC_E_INVAL, "NULL argument");
  if (!t->timed_last) return fail(TPC_E_INVAL, "timing was off for the last request");
  HIP_TRY(hipSetDevice(t->device));
  HIP_TRY(hipEventSynchronize(t->done));
  for (int i = 0; i < n && i < kPasses; ++i) {
    ms[i] = -1.0f;
    if (t->timed_last >> i & 1u) HIP_TRY(hipEventElapsedTime(&ms[i], t->ev[i], t->ev[i + 1]));
  }
  return TPC_OK;
}

}  // extern "C"
