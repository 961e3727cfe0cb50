"""Python binding of the C ABI in include/tpc_tracker.h (argument marshalling only).

Every step of the tracking runs in the HIP library ``libtpc_tracker.so``; this
module only fills the C structs, hands over device pointers, and copies the
returned views into numpy arrays.  PyTorch supplies device memory (the
workspace and the cluster arrays) and the HIP stream.  There is no fallback:
if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

from .config import TrackerConfig

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtpc_tracker.so")

TPC_ABI_VERSION = 3
TPC_OK, TPC_E_INVAL, TPC_E_NOMEM, TPC_E_DEVICE, TPC_E_CAPACITY, TPC_E_NOTREADY, TPC_E_INPUT, TPC_E_BUSY = \
    0, -1, -2, -3, -4, -5, -6, -7
TPC_IN_DEVICE, TPC_IN_HOST = 0, 1
TPC_ERR_NONFINITE, TPC_ERR_TRACKLET_OVERFLOW, TPC_ERR_TRACK_OVERFLOW, TPC_ERR_CLUSTER_OVERFLOW = 1, 2, 4, 8
(TPC_DBG_SORTED_ID, TPC_DBG_SORTED_YZ, TPC_DBG_BIN_START, TPC_DBG_ROW_DIMS, TPC_DBG_UP0, TPC_DBG_DOWN0, TPC_DBG_UP1,
 TPC_DBG_DOWN1, TPC_DBG_STARTS, TPC_DBG_TK_ROWHIT, TPC_DBG_TK_INFO, TPC_DBG_TK_PARAM, TPC_DBG_TK_COV,
 TPC_DBG_TK_CHI2) = range(1, 15)
N_PASSES = 6
PASS_NAMES = ("grid", "neighbours", "clean+starts", "tracklets", "select", "output")


class TrackerError(RuntimeError):
    def __init__(self, status, msg, error_flags=0):
        super().__init__(f"tpc status {status}: {msg}" + (f" (error_flags {error_flags:#x})" if error_flags else ""))
        self.status = status
        self.error_flags = error_flags


class _Config(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("n_rows", C.c_int32),
        ("row_x", C.POINTER(C.c_double)), ("row_half_y", C.POINTER(C.c_double)),
        ("bz_tesla", C.c_double), ("sigma_y", C.c_double), ("sigma_z", C.c_double),
        ("grid_hits_per_bin", C.c_int32),
        ("win_a_y", C.c_double), ("win_b_y", C.c_double), ("win_a_z", C.c_double), ("win_b_z", C.c_double),
        ("link_nsigma", C.c_double), ("s_max", C.c_double), ("seed_qpt_max", C.c_double),
        ("c0_sinphi", C.c_double), ("c0_tanl", C.c_double), ("c0_qpt", C.c_double),
        ("gate_nsigma", C.c_double), ("win_cap", C.c_double), ("edge_margin", C.c_double),
        ("max_miss", C.c_int32), ("min_tracklet_hits", C.c_int32), ("min_track_hits", C.c_int32),
        ("min_owned_frac", C.c_double),
        ("merge_dy", C.c_double), ("merge_dz", C.c_double), ("merge_dsinphi", C.c_double),
        ("merge_dtanl", C.c_double), ("merge_dqpt", C.c_double),
        ("tracklet_schedule", C.c_int32),
        ("max_sectors", C.c_uint32), ("max_clusters", C.c_uint64), ("max_tracklets", C.c_uint64),
        ("max_tracks", C.c_uint64), ("max_track_clusters", C.c_uint64),
        ("device", C.c_int32), ("stream", C.c_void_p), ("workspace", C.c_void_p), ("workspace_bytes", C.c_uint64),
    ]


class _Frame(C.Structure):
    _fields_ = [
        # pointer fields as plain addresses (the C side sees the same layout)
        ("n_sectors", C.c_uint32), ("n_rows", C.c_uint32), ("row_offsets", C.c_void_p),
        ("y", C.c_void_p), ("z", C.c_void_p), ("charge", C.c_void_p), ("n_clusters", C.c_uint64),
        ("sector_z_lo", C.c_void_p), ("sector_z_hi", C.c_void_p), ("flags", C.c_uint32),
    ]


class _Tracks(C.Structure):
    _fields_ = [
        ("n_tracks", C.c_uint32), ("n_track_clusters", C.c_uint64),
        ("track_sector", C.POINTER(C.c_uint32)), ("track_start", C.POINTER(C.c_uint32)),
        ("track_first", C.POINTER(C.c_uint32)), ("cluster_ids", C.POINTER(C.c_uint32)),
        ("x_ref", C.POINTER(C.c_float)), ("param", C.POINTER(C.c_float)), ("cov", C.POINTER(C.c_float)),
        ("chi2", C.POINTER(C.c_float)), ("ndf", C.POINTER(C.c_int32)),
        ("error_flags", C.c_uint32), ("n_tracklets", C.c_uint32), ("n_steps", C.c_uint64),
    ]


class _Merged(C.Structure):
    _fields_ = [
        ("n_tracks", C.c_uint32), ("n_chains", C.c_uint32), ("n_chain_clusters", C.c_uint64),
        ("next", C.POINTER(C.c_int32)), ("head_of", C.POINTER(C.c_uint32)), ("heads", C.POINTER(C.c_uint32)),
        ("nseg", C.POINTER(C.c_int32)), ("first", C.POINTER(C.c_uint32)), ("clusters", C.POINTER(C.c_uint32)),
        ("param", C.POINTER(C.c_float)), ("cov", C.POINTER(C.c_float)), ("chi2", C.POINTER(C.c_float)),
        ("ndf", C.POINTER(C.c_int32)),
    ]


class _CodecStream(C.Structure):
    _fields_ = [("coef", C.c_void_p), ("x_ref", C.c_void_p), ("first", C.c_void_p), ("row", C.c_void_p),
                ("code", C.c_void_p), ("raw", C.c_void_p), ("un_row", C.c_void_p), ("un_yz", C.c_void_p)]


class _CodecCounts(C.Structure):
    _fields_ = [("n_tracks", C.c_uint32), ("n_track_clusters", C.c_uint64), ("n_unassigned", C.c_uint64),
                ("n_escaped", C.c_uint64)]


TPC_CODEC_ESCAPE = -32768
# tuning knobs (tpc_set_knob)
KNOBS = {"schedule": 1, "select_tile_rows": 2, "refit_order": 3, "link_slots": 4, "link_group": 5,
         "select_threads": 6}
CODEC_FIELDS = ("coef", "x_ref", "first", "row", "code", "raw", "un_row", "un_yz")

EXPORTED = ("tpc_default_config", "tpc_workspace_bytes", "tpc_tracker_create", "tpc_tracker_destroy",
            "tpc_workspace_bytes_for", "tpc_tracker_bind_workspace", "tpc_track_timeframe_scratch",
            "tpc_track_timeframe", "tpc_get_tracks", "tpc_get_tracks_device", "tpc_release", "tpc_last_error", "tpc_debug_copy",
            "tpc_set_timing", "tpc_get_pass_times", "tpc_set_tracklet_schedule", "tpc_merge_sectors",
            "tpc_encode_tracks", "tpc_decode_tracks", "tpc_set_knob")

_lib = None


def load():
    """Load libtpc_tracker.so (built by ``paper_2502_09138_amd.build``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                           "(python -m paper_2502_09138_amd.build)")
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    L.tpc_default_config.argtypes = [P(_Config)]
    L.tpc_workspace_bytes.restype = C.c_uint64
    L.tpc_workspace_bytes.argtypes = [P(_Config)]
    L.tpc_tracker_create.restype = C.c_int32
    L.tpc_tracker_create.argtypes = [P(_Config), P(C.c_void_p)]
    L.tpc_tracker_destroy.argtypes = [C.c_void_p]
    L.tpc_workspace_bytes_for.restype = C.c_uint64
    L.tpc_workspace_bytes_for.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32]
    L.tpc_tracker_bind_workspace.restype = C.c_int32
    L.tpc_tracker_bind_workspace.argtypes = [C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint64, C.c_uint32]
    L.tpc_track_timeframe.restype = C.c_int32
    L.tpc_track_timeframe.argtypes = [C.c_void_p, P(_Frame), P(C.c_uint64)]
    L.tpc_track_timeframe_scratch.restype = C.c_int32
    L.tpc_track_timeframe_scratch.argtypes = [C.c_void_p, P(_Frame), P(C.c_uint64)]
    L.tpc_get_tracks.restype = C.c_int32
    L.tpc_get_tracks.argtypes = [C.c_void_p, C.c_uint64, C.c_int32, P(_Tracks)]
    L.tpc_get_tracks_device.restype = C.c_int32
    L.tpc_get_tracks_device.argtypes = [C.c_void_p, C.c_uint64, C.c_int32, P(_Tracks)]
    L.tpc_merge_sectors.restype = C.c_int32
    L.tpc_merge_sectors.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, P(_Merged)]
    L.tpc_encode_tracks.restype = C.c_int32
    L.tpc_encode_tracks.argtypes = [C.c_void_p, C.c_uint64, C.c_float, C.c_float, P(_CodecStream), P(_CodecCounts)]
    L.tpc_decode_tracks.restype = C.c_int32
    L.tpc_decode_tracks.argtypes = [C.c_void_p, P(_CodecStream), P(_CodecCounts), C.c_float, C.c_float, C.c_void_p,
                                    C.c_void_p, C.c_void_p]
    L.tpc_release.restype = C.c_int32
    L.tpc_release.argtypes = [C.c_void_p, C.c_uint64]
    L.tpc_last_error.restype = C.c_char_p
    L.tpc_debug_copy.restype = C.c_int32
    L.tpc_debug_copy.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_uint64, P(C.c_uint64)]
    L.tpc_set_tracklet_schedule.restype = C.c_int32
    L.tpc_set_tracklet_schedule.argtypes = [C.c_void_p, C.c_int32]
    L.tpc_set_knob.restype = C.c_int32
    L.tpc_set_knob.argtypes = [C.c_void_p, C.c_int32, C.c_int32]
    L.tpc_set_timing.restype = C.c_int32
    L.tpc_set_timing.argtypes = [C.c_void_p, C.c_int32]
    L.tpc_get_pass_times.restype = C.c_int32
    L.tpc_get_pass_times.argtypes = [C.c_void_p, P(C.c_float), C.c_int32]
    _lib = L
    return L


def _check(st, error_flags=0):
    if st != TPC_OK:
        raise TrackerError(st, load().tpc_last_error().decode(), error_flags)


def make_config(cfg: TrackerConfig, *, max_clusters, max_sectors=36, max_tracklets=0, max_tracks=0,
                max_track_clusters=0, device=0, tracklet_schedule=0):
    """Fill the C config struct; returns (struct, keep-alive arrays)."""
    c = _Config()
    load().tpc_default_config(C.byref(c))
    row_x = np.ascontiguousarray(cfg.row_x, np.float64)
    row_half_y = np.ascontiguousarray(cfg.row_half_y, np.float64)
    c.n_rows = len(row_x)
    c.row_x = row_x.ctypes.data_as(C.POINTER(C.c_double))
    c.row_half_y = row_half_y.ctypes.data_as(C.POINTER(C.c_double))
    c.bz_tesla = cfg.bz
    for f in ("sigma_y", "sigma_z", "grid_hits_per_bin", "win_a_y", "win_b_y", "win_a_z", "win_b_z", "link_nsigma",
              "s_max", "seed_qpt_max", "c0_sinphi", "c0_tanl", "c0_qpt", "gate_nsigma", "win_cap", "edge_margin",
              "max_miss", "min_tracklet_hits", "min_track_hits", "min_owned_frac", "merge_dy", "merge_dz",
              "merge_dsinphi", "merge_dtanl", "merge_dqpt"):
        setattr(c, f, getattr(cfg, f))
    c.max_sectors = max_sectors
    c.max_clusters = max_clusters
    c.max_tracklets = max_tracklets
    c.max_tracks = max_tracks
    c.max_track_clusters = max_track_clusters
    c.device = device
    c.tracklet_schedule = tracklet_schedule
    return c, (row_x, row_half_y)


@dataclasses.dataclass
class Tracks:
    n_tracklets: int
    error_flags: int
    sector: np.ndarray
    start: np.ndarray
    first: np.ndarray
    cluster_ids: np.ndarray
    x_ref: np.ndarray
    param: np.ndarray     # [n, 5]
    cov: np.ndarray       # [n, 15]
    chi2: np.ndarray
    ndf: np.ndarray

    @property
    def n_tracks(self):
        return len(self.sector)


class Tracker:
    """One tracker on one GPU; workspace and stream come from torch."""

    def __init__(self, cfg: TrackerConfig | None = None, *, max_clusters, max_sectors=36, max_tracklets=0,
                 max_tracks=0, max_track_clusters=0, device=0, stream=None, tracklet_schedule=0, workspace=None):
        """``workspace``: optional (device address, bytes) of caller-owned memory to create the
        tracker on (256-byte aligned, at least ``workspace_bytes`` of the configuration); by
        default torch allocates it."""
        import torch
        self._torch = torch
        L = load()
        cfg = cfg or TrackerConfig()
        self.cfg = cfg
        self.R = len(cfg.row_x)
        self.device = torch.device("cuda", device)
        c, self._keep = make_config(cfg, max_clusters=max_clusters, max_sectors=max_sectors,
                                    max_tracklets=max_tracklets, max_tracks=max_tracks,
                                    max_track_clusters=max_track_clusters, device=device,
                                    tracklet_schedule=tracklet_schedule)
        nbytes = L.tpc_workspace_bytes(C.byref(c))
        if nbytes == 0:
            raise TrackerError(TPC_E_INVAL, "invalid tracker configuration")
        if workspace is not None and int(workspace[1]) >= nbytes:
            self._ws = None
            c.workspace = int(workspace[0])
        else:
            self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            c.workspace = (self._ws.data_ptr() + 255) // 256 * 256
        c.workspace_bytes = nbytes
        # the tracker's own stream (default priority); each submit orders it after torch's current stream
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self._ready = torch.cuda.Event()   # reused to order each submit after torch's current stream
        c.stream = self.stream.cuda_stream
        self._h = C.c_void_p()
        _check(L.tpc_tracker_create(C.byref(c), C.byref(self._h)))
        self.workspace_bytes = nbytes
        self._inputs = None

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().tpc_tracker_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- requests ----
    def submit(self, y, z, row_offsets, z_lo, z_hi, *, host=False, scratch=False):
        """Enqueue one time frame; y/z are CUDA float32 tensors (or numpy with host=True).  scratch=True
        uses the allocation-free entry point (the library's fixed device scratch array)."""
        row_offsets = np.ascontiguousarray(row_offsets, np.uint32)
        z_lo = np.ascontiguousarray(z_lo, np.float32)
        z_hi = np.ascontiguousarray(z_hi, np.float32)
        f = _Frame()
        f.n_rows = self.R
        f.n_sectors = (len(row_offsets) - 1) // self.R
        f.row_offsets = row_offsets.ctypes.data
        f.n_clusters = int(row_offsets[-1])
        f.sector_z_lo = z_lo.ctypes.data
        f.sector_z_hi = z_hi.ctypes.data
        if host:
            y = np.ascontiguousarray(y, np.float32)
            z = np.ascontiguousarray(z, np.float32)
            f.y, f.z = y.ctypes.data, z.ctypes.data
            f.flags = TPC_IN_HOST
        else:
            assert y.is_cuda and z.is_cuda and y.dtype == self._torch.float32 and z.dtype == self._torch.float32
            assert y.is_contiguous() and z.is_contiguous()
            # ordered after the work that produced y and z; the tensors stay referenced
            # (self._inputs) until release(), which waits for the request, so the
            # caching allocator cannot hand their memory out while the kernels read it
            self._ready.record(self._torch.cuda.current_stream(self.device))
            self.stream.wait_event(self._ready)
            f.y, f.z = y.data_ptr(), z.data_ptr()
            f.flags = TPC_IN_DEVICE
        rid = C.c_uint64()
        entry = load().tpc_track_timeframe_scratch if scratch else load().tpc_track_timeframe
        _check(entry(self._h, C.byref(f), C.byref(rid)))
        # borrowed until the request completes; set only once the request is accepted, so a
        # rejected submit (busy, invalid) leaves the in-flight request's inputs referenced
        self._inputs = (y, z, row_offsets, z_lo, z_hi)
        self._n_clusters = {rid.value: int(f.n_clusters)}
        return rid.value

    def get(self, rid, blocking=True, copy=True):
        """The tracks of request rid, copied to the tracker's pinned host buffers by the library.
        copy=True returns numpy arrays of their own; copy=False returns views of the pinned buffers,
        valid until release(rid) (the next request overwrites them)."""
        t = _Tracks()
        st = load().tpc_get_tracks(self._h, rid, 1 if blocking else 0, C.byref(t))
        if st == TPC_E_NOTREADY:
            return None
        _check(st, t.error_flags)
        n, nc = t.n_tracks, t.n_track_clusters

        def arr(ptr, count, dt):
            if count == 0:
                return np.zeros(0, dt)
            return np.ctypeslib.as_array(ptr, shape=(count,)).astype(dt, copy=copy)

        return Tracks(n_tracklets=t.n_tracklets, error_flags=t.error_flags,
                      sector=arr(t.track_sector, n, np.uint32), start=arr(t.track_start, n, np.uint32),
                      first=arr(t.track_first, n + 1, np.uint32), cluster_ids=arr(t.cluster_ids, nc, np.uint32),
                      x_ref=arr(t.x_ref, n, np.float32), param=arr(t.param, 5 * n, np.float32).reshape(n, 5),
                      cov=arr(t.cov, 15 * n, np.float32).reshape(n, 15), chi2=arr(t.chi2, n, np.float32),
                      ndf=arr(t.ndf, n, np.int32))

    def get_device(self, rid):
        """Wait for the request; counts plus device addresses of the output arrays (no copy)."""
        t = _Tracks()
        _check(load().tpc_get_tracks_device(self._h, rid, 1, C.byref(t)))
        addr = lambda p: C.cast(p, C.c_void_p).value or 0
        return dict(n_tracks=t.n_tracks, n_track_clusters=t.n_track_clusters, n_tracklets=t.n_tracklets,
                    n_steps=t.n_steps, error_flags=t.error_flags, cluster_ids=addr(t.cluster_ids),
                    track_first=addr(t.track_first), param=addr(t.param), cov=addr(t.cov))

    def get_counts(self, rid):
        """Wait for the request; returns dict(n_tracks, n_track_clusters, n_tracklets, n_steps, error_flags)."""
        t = _Tracks()
        _check(load().tpc_get_tracks(self._h, rid, 1, C.byref(t)))
        return dict(n_tracks=t.n_tracks, n_track_clusters=t.n_track_clusters, n_tracklets=t.n_tracklets,
                    n_steps=t.n_steps, error_flags=t.error_flags)

    def merge(self, rid, sector_phys=None):
        """C8 + C9 on the tracks of completed request rid (before release); sector_phys[s] = physical
        sector 0..35 of the frame's sector s (-1 or None: no neighbours).  Returns a dict of arrays."""
        sp = None if sector_phys is None else np.ascontiguousarray(sector_phys, np.int32)
        m = _Merged()
        _check(load().tpc_merge_sectors(self._h, rid, None if sp is None else sp.ctypes.data, C.byref(m)))
        n, nc, ncl = m.n_tracks, m.n_chains, m.n_chain_clusters

        def arr(ptr, count, dt):
            if count == 0:
                return np.zeros(0, dt)
            return np.ctypeslib.as_array(ptr, shape=(count,)).astype(dt, copy=True)

        return dict(next=arr(m.next, n, np.int32), head_of=arr(m.head_of, n, np.uint32),
                    heads=arr(m.heads, nc, np.uint32), nseg=arr(m.nseg, nc, np.int32),
                    first=arr(m.first, nc + 1, np.uint32), clusters=arr(m.clusters, ncl, np.uint32),
                    param=arr(m.param, 5 * nc, np.float32).reshape(nc, 5),
                    cov=arr(m.cov, 15 * nc, np.float32).reshape(nc, 15), chi2=arr(m.chi2, nc, np.float32),
                    ndf=arr(m.ndf, nc, np.int32))

    def encode(self, rid, q_y, q_z):
        """C10 on the tracks of completed request rid (before release): the compressed stream as a dict of
        device tensors (the arrays of tpc_codec_stream, cut to their counts) plus the counts."""
        torch = self._torch
        t = self.get_counts(rid)
        nt, nc, n = int(t["n_tracks"]), int(t["n_track_clusters"]), self._n_clusters[rid]
        dev = self.device
        st = dict(coef=torch.empty(6 * max(nt, 1), dtype=torch.float32, device=dev),
                  x_ref=torch.empty(max(nt, 1), dtype=torch.float32, device=dev),
                  first=torch.empty(nt + 1, dtype=torch.int32, device=dev),
                  row=torch.empty(max(nc, 1), dtype=torch.uint8, device=dev),
                  code=torch.empty(2 * max(nc, 1), dtype=torch.int16, device=dev),
                  raw=torch.empty(2 * max(nc, 1), dtype=torch.float32, device=dev),
                  un_row=torch.empty(max(n, 1), dtype=torch.uint8, device=dev),
                  un_yz=torch.empty(2 * max(n, 1), dtype=torch.float32, device=dev))
        s = _CodecStream(*[st[k].data_ptr() for k in CODEC_FIELDS])
        c = _CodecCounts()
        # the tensors were allocated on torch's current stream: order the tracker's stream after it
        self._ready.record(torch.cuda.current_stream(self.device))
        self.stream.wait_event(self._ready)
        _check(load().tpc_encode_tracks(self._h, rid, float(q_y), float(q_z), C.byref(s), C.byref(c)))
        nu = int(c.n_unassigned)
        out = dict(coef=st["coef"][:6 * nt].view(nt, 6), x_ref=st["x_ref"][:nt], first=st["first"],
                   row=st["row"][:nc], code=st["code"][:2 * nc].view(nc, 2), raw=st["raw"][:2 * nc].view(nc, 2),
                   un_row=st["un_row"][:nu], un_yz=st["un_yz"][:2 * nu].view(nu, 2))
        counts = dict(n_tracks=int(c.n_tracks), n_track_clusters=int(c.n_track_clusters), n_unassigned=nu,
                      n_escaped=int(c.n_escaped))
        return out, counts

    def decode(self, stream, counts, q_y, q_z):
        """C11: (y, z, row) device tensors of a stream's clusters (track clusters in stream order, then the
        unassigned ones)."""
        torch = self._torch
        n = counts["n_track_clusters"] + counts["n_unassigned"]
        y = torch.empty(max(n, 1), dtype=torch.float32, device=self.device)
        z = torch.empty_like(y)
        row = torch.empty(max(n, 1), dtype=torch.uint8, device=self.device)
        for k in CODEC_FIELDS:
            t = stream[k]
            assert t.is_cuda and t.is_contiguous(), k
        s = _CodecStream(*[stream[k].data_ptr() if stream[k].numel() else 0 for k in CODEC_FIELDS])
        c = _CodecCounts(counts["n_tracks"], counts["n_track_clusters"], counts["n_unassigned"], counts["n_escaped"])
        self._ready.record(torch.cuda.current_stream(self.device))
        self.stream.wait_event(self._ready)
        _check(load().tpc_decode_tracks(self._h, C.byref(s), C.byref(c), float(q_y), float(q_z), y.data_ptr(),
                                        z.data_ptr(), row.data_ptr()))
        return y[:n], z[:n], row[:n]

    def track_and_merge(self, y, z, row_offsets, z_lo, z_hi, sector_phys, *, host=False):
        """One frame through C1..C9: (tracks, merged chains)."""
        rid = self.submit(y, z, row_offsets, z_lo, z_hi, host=host)
        try:
            return self.get(rid), self.merge(rid, sector_phys)
        finally:
            self.release(rid)

    def release(self, rid):
        _check(load().tpc_release(self._h, rid))
        self._inputs = None

    def track(self, y, z, row_offsets, z_lo, z_hi, *, host=False, scratch=False):
        rid = self.submit(y, z, row_offsets, z_lo, z_hi, host=host, scratch=scratch)
        try:
            return self.get(rid)
        finally:
            self.release(rid)

    def track_to_host(self, y, z, row_offsets, z_lo, z_hi, consume):
        """Tracks one frame and calls consume(tracks) on views of the pinned host copy of its outputs
        (no further copy), before the request is released; returns what consume returns."""
        rid = self.submit(y, z, row_offsets, z_lo, z_hi)
        try:
            return consume(self.get(rid, copy=False))
        finally:
            self.release(rid)

    def track_event(self, ev, host=False):
        if host:
            return self.track(ev.y, ev.z, ev.row_offsets, ev.sector_z_lo, ev.sector_z_hi, host=True)
        torch = self._torch
        y = torch.from_numpy(ev.y).to(self.device)
        z = torch.from_numpy(ev.z).to(self.device)
        return self.track(y, z, ev.row_offsets, ev.sector_z_lo, ev.sector_z_hi)

    # ---- per-request workspaces ----
    def workspace_bytes_for(self, max_clusters, max_sectors):
        """Device bytes of a workspace binding for these capacities (0 if beyond the create-time ones)."""
        return int(load().tpc_workspace_bytes_for(self._h, int(max_clusters), int(max_sectors)))

    def bind_workspace(self, address, nbytes, max_clusters, max_sectors):
        """Move the tracker onto caller-owned device memory at ``address`` (256-byte aligned) sized for
        the given capacities; the caller keeps that memory alive while requests run on it."""
        _check(load().tpc_tracker_bind_workspace(self._h, C.c_void_p(int(address)), int(nbytes), int(max_clusters),
                                                 int(max_sectors)))
        self._ws = None   # the create-time workspace is no longer used

    # ---- introspection ----
    def debug(self, what, dtype):
        L = load()
        n = C.c_uint64()
        _check(L.tpc_debug_copy(self._h, what, None, 0, C.byref(n)))
        out = np.empty(n.value // np.dtype(dtype).itemsize, dtype)
        if n.value:
            _check(L.tpc_debug_copy(self._h, what, out.ctypes.data, n.value, C.byref(n)))
        return out

    def set_knobs(self, **knobs):
        """Tuning knobs for later requests (results identical under every setting): schedule (0 auto,
        1 lane-per-tracklet pipeline, 2 row-synchronous), select_tile_rows (0 auto, 1, 2, 4, -1 global),
        refit_order (0 bucket order, 1 tracklet order), link_slots (0 auto, 4, 8), link_group (0 auto,
        1..4096 consecutive K2 tiles per XCD group, -1 an eighth of the tiles per XCD), select_threads (0 auto,
        256, 512, 1024: workgroup size of the K6 tile kernels)."""
        for name, value in knobs.items():
            if name not in KNOBS:
                raise ValueError(f"unknown knob {name}")
            _check(load().tpc_set_knob(self._h, KNOBS[name], int(value)))

    def set_tracklet_schedule(self, schedule):
        """0 auto, 1 one lane per tracklet, 2 row-synchronous (applies to later requests)."""
        _check(load().tpc_set_tracklet_schedule(self._h, int(schedule)))

    def set_timing(self, on=True, passes=None):
        """Time every pass (or only the named ones, e.g. ("tracklets",)) of later requests."""
        mask = 0
        if on:
            names = PASS_NAMES if passes is None else passes
            for n in names:
                mask |= 1 << PASS_NAMES.index(n)
        _check(load().tpc_set_timing(self._h, mask))

    def pass_times(self):
        """Milliseconds of the timed passes of the last request, by pass name."""
        ms = (C.c_float * N_PASSES)()
        _check(load().tpc_get_pass_times(self._h, ms, N_PASSES))
        return {n: float(v) for n, v in zip(PASS_NAMES, ms) if v >= 0.0}
