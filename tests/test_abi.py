"""C ABI: the library loads, exports every declared entry point, and validates
configurations on the host before touching a device (CPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2502_09138_amd import tracker as trk
from paper_2502_09138_amd.config import default_config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "tpc_tracker.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tpc_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(trk.LIB_PATH):
        from paper_2502_09138_amd import build
        build.build()
    return trk.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 11
    assert set(names) == set(trk.EXPORTED)
    for n in names:
        assert hasattr(lib, n), n


def test_defaults_match_python_config(lib):
    c = trk._Config()
    lib.tpc_default_config(C.byref(c))
    py = default_config()
    assert c.abi_version == trk.TPC_ABI_VERSION and c.n_rows == 152
    assert c.bz_tesla == py.bz
    for f in ("sigma_y", "sigma_z", "grid_hits_per_bin", "win_a_y", "win_b_y", "win_a_z", "win_b_z", "link_nsigma",
              "s_max", "seed_qpt_max", "c0_sinphi", "c0_tanl", "c0_qpt", "gate_nsigma", "win_cap", "edge_margin",
              "max_miss", "min_tracklet_hits", "min_track_hits", "min_owned_frac", "merge_dy", "merge_dz",
              "merge_dsinphi", "merge_dtanl", "merge_dqpt"):
        assert getattr(c, f) == getattr(py, f), f


def test_workspace_bytes_and_validation(lib):
    cfg = default_config()
    c, keep = trk.make_config(cfg, max_clusters=100000)
    n = lib.tpc_workspace_bytes(C.byref(c))
    assert n > 100000 * 40
    c2, keep2 = trk.make_config(cfg, max_clusters=200000)
    assert lib.tpc_workspace_bytes(C.byref(c2)) > n
    bad = [("sigma_y", 0.0), ("s_max", 1.0), ("grid_hits_per_bin", 0), ("n_rows", 2), ("abi_version", 99),
           ("max_clusters", 1 << 31), ("max_tracklets", 1 << 24), ("min_tracklet_hits", 2)]
    for field, val in bad:
        c3, k3 = trk.make_config(cfg, max_clusters=1000)
        setattr(c3, field, val)
        assert lib.tpc_workspace_bytes(C.byref(c3)) == 0, field
        h = C.c_void_p()
        assert lib.tpc_tracker_create(C.byref(c3), C.byref(h)) == trk.TPC_E_INVAL, field
        assert lib.tpc_last_error() != b""
    # non-increasing rows
    c4, k4 = trk.make_config(cfg, max_clusters=1000)
    rx = np.array(k4[0])
    rx[5] = rx[4]
    c4.row_x = rx.ctypes.data_as(C.POINTER(C.c_double))
    assert lib.tpc_workspace_bytes(C.byref(c4)) == 0


def test_null_arguments_rejected(lib):
    assert lib.tpc_tracker_create(None, None) == trk.TPC_E_INVAL
    assert lib.tpc_track_timeframe(None, None, None) == trk.TPC_E_INVAL
    assert lib.tpc_release(None, 1) == trk.TPC_E_INVAL
    assert lib.tpc_set_tracklet_schedule(None, 1) == trk.TPC_E_INVAL
    assert lib.tpc_encode_tracks(None, 1, 0.01, 0.01, None, None) == trk.TPC_E_INVAL
    assert lib.tpc_decode_tracks(None, None, None, 0.01, 0.01, None, None, None) == trk.TPC_E_INVAL
    assert lib.tpc_set_knob(None, 1, 0) == trk.TPC_E_INVAL


def test_rejected_submit_keeps_the_inflight_inputs(monkeypatch):
    """A submit that the library rejects (here: busy) must not drop the references
    that keep the in-flight request's input arrays alive."""
    class FakeLib:
        def tpc_track_timeframe(self, h, f, rid):
            return trk.TPC_E_BUSY

        def tpc_last_error(self):
            return b"previous request not released"

    monkeypatch.setattr(trk, "_lib", FakeLib())
    t = trk.Tracker.__new__(trk.Tracker)
    t.R = 152
    t._h = C.c_void_p(1)
    inflight = object()
    t._inputs = inflight
    y = np.zeros(4, np.float32)
    offs = np.zeros(153, np.uint32)
    offs[-1] = 4
    with pytest.raises(trk.TrackerError) as ex:
        t.submit(y, y, offs, [0.0], [250.0], host=True)
    assert ex.value.status == trk.TPC_E_BUSY
    assert t._inputs is inflight
    t._h = C.c_void_p()
