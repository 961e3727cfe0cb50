"""Batched frames versus one request per sector (CPU: merge logic and shape
classes; GPU: identical results, schedule autotuner)."""
import numpy as np
import pytest

from paper_2502_09138_amd import batching, synth
from paper_2502_09138_amd.config import default_config
from paper_2502_09138_amd.tracker import Tracks

R = synth.N_ROWS


def _tracks(n, n_cl, sector=0, seed=0):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(10, 20, n)
    first = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32)
    return Tracks(n_tracklets=3 * n, error_flags=0, sector=np.full(n, sector, np.uint32),
                  start=np.sort(rng.integers(0, n_cl, n)).astype(np.uint32), first=first,
                  cluster_ids=rng.integers(0, n_cl, int(first[-1])).astype(np.uint32),
                  x_ref=rng.random(n).astype(np.float32), param=rng.random((n, 5)).astype(np.float32),
                  cov=rng.random((n, 15)).astype(np.float32), chi2=rng.random(n).astype(np.float32),
                  ndf=rng.integers(10, 50, n).astype(np.int32))


def test_merge_rebases_sectors_offsets_and_ids():
    a, b = _tracks(4, 100, seed=1), _tracks(3, 50, seed=2)
    b.error_flags = 2
    m = batching.merge_sector_tracks([(0, 0, a), (5, 100, b)])
    assert m.n_tracks == 7 and m.n_tracklets == 21 and m.error_flags == 2
    assert list(m.sector) == [0] * 4 + [5] * 3
    np.testing.assert_array_equal(m.start, np.concatenate([a.start, b.start + 100]))
    np.testing.assert_array_equal(m.first, np.concatenate([a.first, b.first[1:] + a.first[-1]]))
    np.testing.assert_array_equal(m.cluster_ids, np.concatenate([a.cluster_ids, b.cluster_ids + 100]))
    # track k's clusters are unchanged apart from the base
    for k in range(3):
        got = m.cluster_ids[m.first[4 + k]:m.first[5 + k]]
        np.testing.assert_array_equal(got, b.cluster_ids[b.first[k]:b.first[k + 1]] + 100)
    np.testing.assert_array_equal(m.param, np.concatenate([a.param, b.param]))


def test_sector_spans_and_shape_class():
    ev = synth.single_sector(seed=1)
    ro = np.concatenate([ev.row_offsets, ev.row_offsets[1:] + ev.row_offsets[-1]]).astype(np.uint32)
    spans = batching.sector_spans(ro)
    assert [(s, a, b) for s, a, b, _ in spans] == [(0, 0, ev.n_clusters), (1, ev.n_clusters, 2 * ev.n_clusters)]
    np.testing.assert_array_equal(spans[1][3], ev.row_offsets)
    c1 = batching.shape_class(ev.row_offsets)
    c2 = batching.shape_class(ro)
    assert c1[1:] == c2[1:] and c2[0] == c1[0] + 1


@pytest.mark.gpu
def test_per_sector_requests_match_the_batched_frame():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_09138_amd.tracker import Tracker
    ev = synth.uneven_chunks(chunks=[0, 3, 7, 11, 40, 41, 90, 200])
    dev = torch.device("cuda", 0)
    y = torch.from_numpy(ev.y).to(dev)
    z = torch.from_numpy(ev.z).to(dev)
    tr = Tracker(default_config(), max_clusters=ev.n_clusters, max_sectors=ev.n_sectors)
    try:
        for schedule in (1, 2):
            tr.set_tracklet_schedule(schedule)
            whole = tr.track(y, z, ev.row_offsets, ev.sector_z_lo, ev.sector_z_hi)
            per = batching.track_per_sector(tr, y, z, ev.row_offsets, ev.sector_z_lo, ev.sector_z_hi)
            print("schedule", schedule, "tracks", whole.n_tracks, per.n_tracks, flush=True)
            assert whole.n_tracks > 100 and whole.error_flags == 0
            for k in ("sector", "start", "first", "cluster_ids", "x_ref", "param", "cov", "chi2", "ndf"):
                np.testing.assert_array_equal(getattr(per, k), getattr(whole, k), err_msg=k)
            assert per.n_tracklets == whole.n_tracklets
    finally:
        tr.close()


class _TimedTracker:
    """Stands in for a Tracker in the tuner: each knob setting has a fixed total pass time."""

    def __init__(self, ms_of):
        self.ms_of, self.knobs = ms_of, {}

    def set_timing(self, on):
        pass

    def set_knobs(self, **knobs):
        self.knobs = dict(knobs)

    def submit(self, *frame):
        return 1

    def get_device(self, rid):
        return {}

    def release(self, rid):
        pass

    def pass_times(self):
        return {"tracklets": self.ms_of(self.knobs)}


def test_tuner_keeps_the_incumbent_within_the_tie_fraction():
    """A knob value replaces the one chosen so far only if faster by more than the tie fraction."""
    space = {"a": (0, 1, 2), "b": (0, 1)}
    times = {(0, 0): 10.0, (1, 0): 9.98, (2, 0): 9.0, (2, 1): 8.99}
    tr = _TimedTracker(lambda k: times.get((k["a"], k["b"]), 20.0))
    ro = np.zeros(R + 1, np.uint32)
    c = batching.ScheduleTuner(tr, space=space, repeats=1, tie=0.005).choose(None, None, ro, None, None)
    assert c == {"a": 2, "b": 0}            # 9.98 ties with 10.0; 9.0 wins; 8.99 ties with 9.0
    c = batching.ScheduleTuner(tr, space=space, repeats=1, tie=0.0).choose(None, None, ro, None, None)
    assert c == {"a": 2, "b": 1}            # without the tie rule the strict minimum wins
    cands = ({"a": 0, "b": 0}, {"a": 1, "b": 0})
    assert batching.ScheduleTuner(tr, candidates=cands, repeats=1).choose(None, None, ro, None, None) == cands[0]


@pytest.mark.gpu
def test_schedule_tuner_caches_per_shape_class(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_09138_amd.tracker import Tracker
    ev = synth.central_event(seed=2).sector_slice(list(range(6)))
    dev = torch.device("cuda", 0)
    y = torch.from_numpy(ev.y).to(dev)
    z = torch.from_numpy(ev.z).to(dev)
    tr = Tracker(default_config(), max_clusters=ev.n_clusters, max_sectors=ev.n_sectors)
    try:
        path = str(tmp_path / "tune.json")
        tuner = batching.ScheduleTuner(tr, candidates=(1, 2), cache_path=path)
        c1 = tuner.choose(y, z, ev.row_offsets, ev.sector_z_lo, ev.sector_z_hi)
        runs = tuner.tuned_runs
        assert c1 in (1, 2) and runs == 4
        c2 = tuner.choose(y, z, ev.row_offsets, ev.sector_z_lo, ev.sector_z_hi)
        assert c2 == c1 and tuner.tuned_runs == runs          # cached: no re-timing
        again = batching.ScheduleTuner(tr, candidates=(1, 2), cache_path=path)    # persisted per (arch, shape class)
        assert again.choose(y, z, ev.row_offsets, ev.sector_z_lo, ev.sector_z_hi) == c1 and again.tuned_runs == 0
        out = tr.track(y, z, ev.row_offsets, ev.sector_z_lo, ev.sector_z_hi)
        assert out.n_tracks > 100 and out.error_flags == 0
    finally:
        tr.close()


@pytest.mark.gpu
def test_every_knob_setting_gives_identical_results():
    """The tuner's knobs change speed only: every setting of schedule x selector tile rows x refit
    order x K2 slots x K2 XCD grouping x selector workgroup size gives bit-identical outputs (six sectors of the 32-orbit frame: rows beyond the
    row-synchronous stage; the central event's first four sectors: rows within it)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_09138_amd.tracker import Tracker
    dev = torch.device("cuda", 0)
    for name, ev in (("time_frame sectors 0-5", synth.time_frame(seed=3).sector_slice(range(6))),
                     ("central_event sectors 0-3", synth.central_event(seed=2).sector_slice(range(4)))):
        print("case:", name, "N=", ev.n_clusters, flush=True)
        y = torch.from_numpy(ev.y).to(dev)
        z = torch.from_numpy(ev.z).to(dev)
        tr = Tracker(default_config(), max_clusters=ev.n_clusters, max_sectors=ev.n_sectors)
        try:
            ref = None
            for knobs in batching.knob_grid():
                tr.set_knobs(**knobs)
                out = tr.track(y, z, ev.row_offsets, ev.sector_z_lo, ev.sector_z_hi)
                assert out.error_flags == 0 and out.n_tracks > 100
                if ref is None:
                    ref = out
                    continue
                for k in ("sector", "start", "first", "cluster_ids", "x_ref", "param", "cov", "chi2", "ndf"):
                    a, b = getattr(out, k), getattr(ref, k)
                    if k in ("param", "cov", "chi2", "x_ref"):
                        a, b = a.view(np.int32), b.view(np.int32)
                    assert np.array_equal(a, b), (name, knobs, k)
        finally:
            tr.close()


@pytest.mark.gpu
def test_knob_tuner_sweeps_the_grid_once_per_shape_class(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_09138_amd.tracker import Tracker
    ev = synth.uneven_chunks(chunks=[0, 3, 7, 11, 40, 41, 90, 200])
    dev = torch.device("cuda", 0)
    y = torch.from_numpy(ev.y).to(dev)
    z = torch.from_numpy(ev.z).to(dev)
    tr = Tracker(default_config(), max_clusters=ev.n_clusters, max_sectors=ev.n_sectors)
    try:
        grid = batching.knob_grid()
        tuner = batching.ScheduleTuner(tr, candidates=grid, repeats=1, cache_path=str(tmp_path / "knobs.json"))
        choice = tuner.choose(y, z, ev.row_offsets, ev.sector_z_lo, ev.sector_z_hi)
        print("knob choice", choice, flush=True)
        assert choice in grid and tuner.tuned_runs == len(grid)
        assert tuner.choose(y, z, ev.row_offsets, ev.sector_z_lo, ev.sector_z_hi) == choice
        assert tuner.tuned_runs == len(grid)
        # one knob at a time: every value of each knob once, the others at their best so far
        coord = batching.ScheduleTuner(tr, repeats=1)
        c = coord.choose(y, z, ev.row_offsets, ev.sector_z_lo, ev.sector_z_hi)
        space = batching.KNOB_SPACE
        print("coordinate choice", c, "runs", coord.tuned_runs, flush=True)
        assert set(c) == set(space) and all(c[k] in v for k, v in space.items())
        assert coord.tuned_runs == 1 + sum(len(v) - 1 for v in space.values())
    finally:
        tr.close()


@pytest.mark.gpu
def test_knobs_reject_unknown_values():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_09138_amd.tracker import Tracker, TrackerError, TPC_E_INVAL
    tr = Tracker(default_config(), max_clusters=1000, max_sectors=1)
    try:
        for knobs in ({"schedule": 3}, {"select_tile_rows": 3}, {"select_tile_rows": 8}, {"refit_order": 2},
                      {"link_slots": 6}, {"link_group": -2}, {"link_group": 4097}, {"select_threads": 128},
                      {"select_threads": 2048}):
            with pytest.raises(TrackerError) as e:
                tr.set_knobs(**knobs)
            assert e.value.status == TPC_E_INVAL, knobs
        with pytest.raises(ValueError):
            tr.set_knobs(waves=4)
        tr.set_knobs(schedule=0, select_tile_rows=-1, refit_order=1, link_slots=4, link_group=-1)   # all accepted
        tr.set_knobs(link_group=4096, select_threads=1024)
        tr.set_knobs(link_group=0)
    finally:
        tr.close()
