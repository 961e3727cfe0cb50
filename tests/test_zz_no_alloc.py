"""The allocation-free entry point tpc_track_timeframe_scratch against
tpc_track_timeframe: identical outputs on two calls in a row (the second on a
smaller frame), on device and host inputs; frames beyond the scratch array are
rejected; the tracker's own workspace is used again afterwards."""
import numpy as np
import pytest

from paper_2502_09138_amd import synth
from paper_2502_09138_amd.config import default_config

pytestmark = pytest.mark.gpu
FIELDS = ("sector", "start", "first", "cluster_ids", "x_ref", "param", "cov", "chi2", "ndf")


def _same(a, b, label):
    assert a.n_tracklets == b.n_tracklets, label
    for k in FIELDS:
        np.testing.assert_array_equal(getattr(a, k), getattr(b, k), err_msg=f"{label} {k}")


def test_scratch_entry_matches_the_workspace_entry():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_09138_amd.tracker import Tracker, TrackerError, TPC_E_INVAL
    dev = torch.device("cuda", 0)
    big = synth.pp_time_frame(seed=51, n_orbits=3)               # ~0.3M clusters, 36 sectors
    small = synth.single_sector(seed=2)                          # ~27k clusters, one sector
    print("case: scratch entry, pp frame", big.n_clusters, "then single sector", small.n_clusters, flush=True)
    tr = Tracker(default_config(), max_clusters=2_000_000, max_sectors=36)
    ref = tr.track_event(big), tr.track_event(small)
    for k, ev in enumerate((big, small)):                        # two scratch calls in a row, the second smaller
        y = torch.from_numpy(ev.y).to(dev)
        z = torch.from_numpy(ev.z).to(dev)
        got = tr.track(y, z, ev.row_offsets, ev.sector_z_lo, ev.sector_z_hi, scratch=True)
        print("scratch call", k, "tracks", got.n_tracks, "reference", ref[k].n_tracks, flush=True)
        assert got.n_tracks > 50
        _same(ref[k], got, f"scratch call {k}")
    got = tr.track(small.y, small.z, small.row_offsets, small.sector_z_lo, small.sector_z_hi, host=True, scratch=True)
    _same(ref[1], got, "scratch, host input")
    _same(ref[0], tr.track_event(big), "own workspace again")  # back on the tracker's workspace
    # a frame whose workspace exceeds the array is rejected before anything is enqueued
    huge = synth.central_event(seed=2)
    with pytest.raises(TrackerError) as ex:
        tr.track(huge.y, huge.z, huge.row_offsets, huge.sector_z_lo, huge.sector_z_hi, host=True, scratch=True)
    assert ex.value.status == TPC_E_INVAL and "scratch" in str(ex.value)
    _same(ref[1], tr.track(small.y, small.z, small.row_offsets, small.sector_z_lo, small.sector_z_hi, host=True,
                           scratch=True), "scratch after a rejected frame")
    tr.close()
