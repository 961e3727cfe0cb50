"""ctypes front end of the FP64 reference tracker (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
import this module.  The library it loads (``liboracle.so``) is built from
``tpc_oracle.cpp`` (steps C1..C9) and ``tpc_codec.cpp`` (C10/C11, track-model
compression) by :func:`build`; it shares no code with the HIP path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

ORC_SORTED_ID, ORC_BIN_START, ORC_ROW_DIMS, ORC_UP0, ORC_DOWN0, ORC_UP1, ORC_DOWN1, ORC_STARTS, \
    ORC_TK_ROWHIT, ORC_TK_NHITS, ORC_TK_PARAM, ORC_TK_COV, ORC_TK_XREF_ROW, ORC_TK_CHI2, \
    ORC_TRK_TRACKLET, ORC_TRK_FIRST, ORC_TRK_CLUSTERS, ORC_SIZES = range(1, 19)


def build(force=True):
    """Compile liboracle.so with g++ (-O2, no FP contraction)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    srcs = [os.path.join(HERE, "tpc_oracle.cpp"), os.path.join(HERE, "tpc_codec.cpp")]
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                           "-shared", "-Wall", "-o", tmp, *srcs])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Cfg(C.Structure):
    _fields_ = [
        ("n_rows", C.c_int32), ("row_x", C.POINTER(C.c_double)), ("row_half_y", C.POINTER(C.c_double)),
        ("bz", C.c_double), ("sigma_y", C.c_double), ("sigma_z", C.c_double),
        ("grid_hits_per_bin", C.c_int32),
        ("win_a_y", C.c_double), ("win_b_y", C.c_double), ("win_a_z", C.c_double), ("win_b_z", C.c_double),
        ("link_nsigma", C.c_double), ("s_max", C.c_double), ("seed_qpt_max", C.c_double),
        ("c0_sinphi", C.c_double), ("c0_tanl", C.c_double), ("c0_qpt", C.c_double),
        ("gate_nsigma", C.c_double), ("win_cap", C.c_double), ("edge_margin", C.c_double),
        ("max_miss", C.c_int32), ("min_tracklet_hits", C.c_int32), ("min_track_hits", C.c_int32),
        ("min_owned_frac", C.c_double),
        ("merge_dy", C.c_double), ("merge_dz", C.c_double), ("merge_dsinphi", C.c_double),
        ("merge_dtanl", C.c_double), ("merge_dqpt", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        vp, u32p, dp, fp = C.c_void_p, C.POINTER(C.c_uint32), C.POINTER(C.c_double), C.POINTER(C.c_float)
        L.orc_run_create.restype = vp
        L.orc_run_create.argtypes = [C.POINTER(_Cfg), C.c_uint32, u32p, dp, dp, fp, fp]
        L.orc_run_destroy.argtypes = [vp]
        i32p = C.POINTER(C.c_int32)
        L.orc_run_from_tracklets.restype = vp
        L.orc_run_from_tracklets.argtypes = [C.POINTER(_Cfg), C.c_uint32, C.c_uint64, i32p, u32p, i32p]
        for f in ("orc_run_grid", "orc_run_links", "orc_run_links_fp64", "orc_run_starts", "orc_run_select"):
            getattr(L, f).argtypes = [vp]
            getattr(L, f).restype = C.c_int
        L.orc_run_construct.argtypes = [vp, u32p, C.c_uint64]
        L.orc_merge_run.restype = vp
        L.orc_merge_run.argtypes = [vp, C.POINTER(C.c_int32)]
        L.orc_merge_destroy.argtypes = [vp]
        L.orc_merge_get.restype = C.c_uint64
        L.orc_merge_get.argtypes = [vp, C.c_int, vp, C.c_uint64]
        L.orc_rotate.restype = C.c_int
        L.orc_rotate.argtypes = [C.c_double, dp, C.c_double, C.c_double, dp, dp, dp]
        L.orc_get.restype = C.c_uint64
        L.orc_get.argtypes = [vp, C.c_int, vp, C.c_uint64]
        L.orc_propagate.restype = C.c_int
        L.orc_propagate.argtypes = [dp, C.c_double, C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_propagate_cov.restype = C.c_int
        L.orc_propagate_cov.argtypes = [dp, dp, C.c_double, C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_kf_update.argtypes = [dp, dp, C.c_double, C.c_double, C.c_double, C.c_double, dp]
        L.orc_seed.restype = C.c_int
        L.orc_seed.argtypes = [C.POINTER(_Cfg)] + [C.c_double] * 8 + [dp]
        L.orc_bin.argtypes = [C.c_float] * 6 + [C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_grid_dims.argtypes = [C.c_uint32, C.c_int, C.c_int64, C.c_int64, C.POINTER(C.c_int),
                                    C.POINTER(C.c_int)]
        u8p, i16p, u64p = C.POINTER(C.c_uint8), C.POINTER(C.c_int16), C.POINTER(C.c_uint64)
        L.orc_codec_coef.restype = C.c_int
        L.orc_codec_coef.argtypes = [fp, C.c_double, fp]
        L.orc_codec_encode.restype = C.c_uint64
        L.orc_codec_encode.argtypes = [C.c_int32, dp, C.c_double, C.c_float, C.c_float, C.c_uint32, u32p, u32p, fp, fp,
                                       C.c_uint64, fp, fp, u32p, C.c_uint32, fp, u8p, i16p, fp, u8p, fp, u64p]
        L.orc_codec_decode.argtypes = [C.c_int32, dp, C.c_float, C.c_float, C.c_uint32, u32p, fp, fp, u8p, i16p, fp,
                                       fp, fp]
        _lib = L
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(C.POINTER(t))


class Config:
    """Holds a config dict plus the ctypes struct (keeps the row arrays alive)."""

    def __init__(self, cfg: dict):
        self.d = dict(cfg)
        self.row_x = np.ascontiguousarray(cfg["row_x"], np.float64)
        self.row_half_y = np.ascontiguousarray(cfg["row_half_y"], np.float64)
        s = _Cfg()
        s.n_rows = len(self.row_x)
        s.row_x = _ptr(self.row_x, C.c_double)
        s.row_half_y = _ptr(self.row_half_y, C.c_double)
        for name, typ in _Cfg._fields_[3:]:
            setattr(s, name, typ(cfg[name]).value if typ is not C.c_int32 else int(cfg[name]))
        self.s = s


class Run:
    """One oracle run over an event (sector-major clusters)."""

    def __init__(self, cfg: dict, row_offsets, y, z, z_lo, z_hi):
        self.cfg = Config(cfg)
        self.R = self.cfg.s.n_rows
        self.row_offsets = np.ascontiguousarray(row_offsets, np.uint32)
        self.S = (len(self.row_offsets) - 1) // self.R
        self.y = np.ascontiguousarray(y, np.float64)
        self.z = np.ascontiguousarray(z, np.float64)
        self.z_lo = np.ascontiguousarray(z_lo, np.float32)
        self.z_hi = np.ascontiguousarray(z_hi, np.float32)
        self.h = lib().orc_run_create(C.byref(self.cfg.s), self.S, _ptr(self.row_offsets, C.c_uint32),
                                      _ptr(self.y, C.c_double), _ptr(self.z, C.c_double),
                                      _ptr(self.z_lo, C.c_float), _ptr(self.z_hi, C.c_float))

    @classmethod
    def from_tracklets(cls, cfg: dict, n_clusters, nhits, start_pos, rowhit):
        """A run holding only given tracklets (rowhit [T, R] sorted positions, -1 none), for C6 alone."""
        self = cls.__new__(cls)
        self.cfg = Config(cfg)
        self.R = self.cfg.s.n_rows
        self._keep = (np.ascontiguousarray(nhits, np.int32), np.ascontiguousarray(start_pos, np.uint32),
                      np.ascontiguousarray(rowhit, np.int32).reshape(-1))
        T = len(self._keep[0])
        assert len(self._keep[1]) == T and len(self._keep[2]) == T * self.R
        self.h = lib().orc_run_from_tracklets(C.byref(self.cfg.s), n_clusters, T, _ptr(self._keep[0], C.c_int32),
                                             _ptr(self._keep[1], C.c_uint32), _ptr(self._keep[2], C.c_int32))
        return self

    @classmethod
    def from_event(cls, cfg, ev, fp64=None):
        y = ev.y if fp64 is None else fp64[0]
        z = ev.z if fp64 is None else fp64[1]
        return cls(cfg, ev.row_offsets, y, z, ev.sector_z_lo, ev.sector_z_hi)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_run_destroy(self.h)
            self.h = None

    def get(self, what, dtype):
        n = lib().orc_get(self.h, what, None, 0)
        out = np.empty(n // np.dtype(dtype).itemsize, dtype)
        if n:
            lib().orc_get(self.h, what, out.ctypes.data_as(C.c_void_p), n)
        return out

    def grid(self):
        lib().orc_run_grid(self.h)
        return self

    def links(self, fp64=False):
        """C2 + C3; fp64=True evaluates the C2 decisions in double instead of float32."""
        (lib().orc_run_links_fp64 if fp64 else lib().orc_run_links)(self.h)
        return self

    def starts(self):
        lib().orc_run_starts(self.h)
        return self

    def construct(self, which=None):
        if which is None:
            lib().orc_run_construct(self.h, None, 0)
        else:
            w = np.ascontiguousarray(which, np.uint32)
            lib().orc_run_construct(self.h, _ptr(w, C.c_uint32), len(w))
        return self

    def select(self):
        lib().orc_run_select(self.h)
        return self

    def run_all(self):
        return self.grid().links().starts().construct().select()

    # ---- results ----
    def sizes(self):
        return self.get(ORC_SIZES, np.uint64)

    def result(self):
        """Dict of every array the run produced."""
        R = self.R
        T = int(self.sizes()[1])
        out = dict(
            sorted_id=self.get(ORC_SORTED_ID, np.uint32), bin_start=self.get(ORC_BIN_START, np.uint32),
            row_dims=self.get(ORC_ROW_DIMS, np.uint32), up0=self.get(ORC_UP0, np.int32),
            down0=self.get(ORC_DOWN0, np.int32), up1=self.get(ORC_UP1, np.int32),
            down1=self.get(ORC_DOWN1, np.int32), starts=self.get(ORC_STARTS, np.uint32),
            tk_rowhit=self.get(ORC_TK_ROWHIT, np.int32).reshape(T, R) if T else np.zeros((0, R), np.int32),
            tk_nhits=self.get(ORC_TK_NHITS, np.int32), tk_param=self.get(ORC_TK_PARAM, np.float64).reshape(-1, 5),
            tk_cov=self.get(ORC_TK_COV, np.float64).reshape(-1, 15), tk_xref_row=self.get(ORC_TK_XREF_ROW, np.int32),
            tk_chi2=self.get(ORC_TK_CHI2, np.float64), trk_tracklet=self.get(ORC_TRK_TRACKLET, np.uint32),
            trk_first=self.get(ORC_TRK_FIRST, np.uint32), trk_clusters=self.get(ORC_TRK_CLUSTERS, np.uint32))
        return out


ORC_M_NEXT, ORC_M_HEAD, ORC_M_HEADS, ORC_M_NSEG, ORC_M_PARAM, ORC_M_COV, ORC_M_CHI2, ORC_M_NDF, ORC_M_FIRST, \
    ORC_M_CLUSTERS = range(1, 11)


def merge(run, sector_phys=None):
    """C8 sector merger + C9 refit on the C7 tracks of a finished run; returns a dict of arrays.
    sector_phys: physical sector (0..35) of each of the run's sectors, -1 = no neighbours."""
    sp = None if sector_phys is None else np.ascontiguousarray(sector_phys, np.int32)
    h = lib().orc_merge_run(run.h, None if sp is None else _ptr(sp, C.c_int32))

    def get(what, dt):
        n = lib().orc_merge_get(h, what, None, 0)
        out = np.empty(n // np.dtype(dt).itemsize, dt)
        if n:
            lib().orc_merge_get(h, what, out.ctypes.data_as(C.c_void_p), n)
        return out

    try:
        return dict(next=get(ORC_M_NEXT, np.int32), head=get(ORC_M_HEAD, np.int32), heads=get(ORC_M_HEADS, np.uint32),
                    nseg=get(ORC_M_NSEG, np.int32), param=get(ORC_M_PARAM, np.float64).reshape(-1, 5),
                    cov=get(ORC_M_COV, np.float64).reshape(-1, 15), chi2=get(ORC_M_CHI2, np.float64),
                    ndf=get(ORC_M_NDF, np.int32), first=get(ORC_M_FIRST, np.uint32),
                    clusters=get(ORC_M_CLUSTERS, np.uint32))
    finally:
        lib().orc_merge_destroy(h)


def rotate(x, p, d, bz):
    p = np.ascontiguousarray(p, np.float64)
    xo = C.c_double()
    q = np.zeros(5)
    J = np.zeros(25)
    rc = lib().orc_rotate(x, _ptr(p, C.c_double), d, bz, C.byref(xo), _ptr(q, C.c_double), _ptr(J, C.c_double))
    return rc, xo.value, q, J.reshape(5, 5)


def propagate(p, x1, x2, bz, s_max=0.99):
    p = np.ascontiguousarray(p, np.float64)
    q = np.zeros(5)
    F = np.zeros(25)
    rc = lib().orc_propagate(_ptr(p, C.c_double), x1, x2, bz, s_max, _ptr(q, C.c_double), _ptr(F, C.c_double))
    return rc, q, F.reshape(5, 5)


def propagate_cov(p, C15, x1, x2, bz, s_max=0.99):
    p = np.ascontiguousarray(p, np.float64)
    c = np.ascontiguousarray(C15, np.float64)
    q = np.zeros(5)
    c2 = np.zeros(15)
    rc = lib().orc_propagate_cov(_ptr(p, C.c_double), _ptr(c, C.c_double), x1, x2, bz, s_max,
                                 _ptr(q, C.c_double), _ptr(c2, C.c_double))
    return rc, q, c2


def kf_update(p, C15, ym, zm, vy, vz):
    p = np.array(p, np.float64)
    c = np.array(C15, np.float64)
    chi2 = C.c_double(0.0)
    lib().orc_kf_update(_ptr(p, C.c_double), _ptr(c, C.c_double), ym, zm, vy, vz, C.byref(chi2))
    return p, c, chi2.value


def seed(cfg: dict, x0, y0, z0, xm, ym, xl, yl, zl):
    c = Config(cfg)
    p = np.zeros(5)
    rc = lib().orc_seed(C.byref(c.s), x0, y0, z0, xm, ym, xl, yl, zl, _ptr(p, C.c_double))
    return rc, p


def bin_of(y, z, y_lo, inv_wy, z_lo, inv_wz, ny, nz):
    iy, iz = C.c_int(), C.c_int()
    lib().orc_bin(y, z, y_lo, inv_wy, z_lo, inv_wz, ny, nz, C.byref(iy), C.byref(iz))
    return iy.value, iz.value


def grid_dims(n, k, ly, lz):
    ny, nz = C.c_int(), C.c_int()
    lib().orc_grid_dims(n, k, ly, lz, C.byref(ny), C.byref(nz))
    return ny.value, nz.value


def unpack_cov(c15):
    """Packed lower triangle (00,10,11,20,...) -> symmetric 5x5."""
    M = np.zeros((5, 5))
    k = 0
    for i in range(5):
        for j in range(i + 1):
            M[i, j] = M[j, i] = c15[k]
            k += 1
    return M


# ---- C10/C11: track-model compression (tpc_codec.h) ----
CODEC_ESCAPE = -32768


def codec_coef(param, bz):
    """Model coefficients (a0, a1, a2, b0, b1, b2) of one track from its float32 parameters; None if no model."""
    p = np.ascontiguousarray(param, np.float32)
    out = np.zeros(6, np.float32)
    rc = lib().orc_codec_coef(_ptr(p, C.c_float), float(bz), _ptr(out, C.c_float))
    return None if rc else out


def codec_encode(row_x, bz, q_y, q_z, first, ids, x_ref, param, y, z, row_offsets):
    """C10 over a frame's tracks (arrays as tpc_tracks holds them); returns a dict with the stream."""
    row_x = np.ascontiguousarray(row_x, np.float64)
    first = np.ascontiguousarray(first, np.uint32)
    ids = np.ascontiguousarray(ids, np.uint32)
    x_ref = np.ascontiguousarray(x_ref, np.float32)
    param = np.ascontiguousarray(param, np.float32).reshape(-1)
    y = np.ascontiguousarray(y, np.float32)
    z = np.ascontiguousarray(z, np.float32)
    ro = np.ascontiguousarray(row_offsets, np.uint32)
    nt, nc, n = len(first) - 1, len(ids), len(y)
    coef = np.zeros(6 * nt, np.float32)
    row = np.zeros(nc, np.uint8)
    code = np.zeros(2 * nc, np.int16)
    raw = np.zeros(2 * nc, np.float32)
    un_row = np.zeros(n, np.uint8)
    un_yz = np.zeros(2 * n, np.float32)
    nu = C.c_uint64(0)
    esc = lib().orc_codec_encode(len(row_x), _ptr(row_x, C.c_double), float(bz), float(q_y), float(q_z), nt,
                                 _ptr(first, C.c_uint32), _ptr(ids, C.c_uint32), _ptr(x_ref, C.c_float),
                                 _ptr(param, C.c_float), n, _ptr(y, C.c_float), _ptr(z, C.c_float),
                                 _ptr(ro, C.c_uint32), len(ro) - 1, _ptr(coef, C.c_float), _ptr(row, C.c_uint8),
                                 _ptr(code, C.c_int16), _ptr(raw, C.c_float), _ptr(un_row, C.c_uint8),
                                 _ptr(un_yz, C.c_float), C.byref(nu))
    k = int(nu.value)
    return dict(coef=coef.reshape(-1, 6), x_ref=x_ref, first=first, row=row, code=code.reshape(-1, 2),
                raw=raw.reshape(-1, 2), un_row=un_row[:k], un_yz=un_yz[:2 * k].reshape(-1, 2), n_escaped=int(esc))


def codec_decode(row_x, q_y, q_z, stream):
    """C11: (y, z) of the track clusters of a stream, in stream order."""
    row_x = np.ascontiguousarray(row_x, np.float64)
    first = np.ascontiguousarray(stream["first"], np.uint32)
    coef = np.ascontiguousarray(stream["coef"], np.float32).reshape(-1)
    x_ref = np.ascontiguousarray(stream["x_ref"], np.float32)
    row = np.ascontiguousarray(stream["row"], np.uint8)
    code = np.ascontiguousarray(stream["code"], np.int16).reshape(-1)
    raw = np.ascontiguousarray(stream["raw"], np.float32).reshape(-1)
    nc = len(row)
    yo = np.zeros(nc, np.float32)
    zo = np.zeros(nc, np.float32)
    lib().orc_codec_decode(len(row_x), _ptr(row_x, C.c_double), float(q_y), float(q_z), len(first) - 1,
                           _ptr(first, C.c_uint32), _ptr(x_ref, C.c_float), _ptr(coef, C.c_float),
                           _ptr(row, C.c_uint8), _ptr(code, C.c_int16), _ptr(raw, C.c_float),
                           _ptr(yo, C.c_float), _ptr(zo, C.c_float))
    return yo, zo
