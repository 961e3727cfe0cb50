"""Batched frames versus one request per sector, and a schedule autotuner.

The default path is the batched one: one request carries every sector (or
independent chunk) of a frame, and each pass is a single launch over all of
them, with the work split on the device by (sector, row), (row, 64-hit tile),
(sector, block of rows) and (sector, range of tracklets).  ``track_per_sector``
is the plain alternative it is measured against: one request per sector, issued
back to back on the same tracker.  The two give identical results: sectors are
independent and every output is in canonical (sector, start position) order, so
the per-sector outputs, re-based to frame numbering, concatenate to the batched
output.

``ScheduleTuner`` picks the tracklet-constructor schedule (one lane per
tracklet with global-memory searches, or row-synchronous waves with LDS-staged
rows) per shape class of frame by timing each candidate on the first frame of
the class, and caches the choice per (GPU architecture, shape class).
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

from .tracker import Tracks

N_ROWS = 152


def merge_sector_tracks(parts) -> Tracks:
    """Concatenate per-sector Tracks; ``parts`` = [(sector, first cluster index, Tracks)] in sector order."""
    if not parts:
        raise ValueError("no sectors")
    first = [np.zeros(1, np.uint32)]
    run = 0
    cols = {k: [] for k in ("sector", "start", "cluster_ids", "x_ref", "param", "cov", "chi2", "ndf")}
    n_tracklets, flags = 0, 0
    for s, base, t in parts:
        cols["sector"].append(t.sector + np.uint32(s))
        cols["start"].append(t.start + np.uint32(base))
        cols["cluster_ids"].append(t.cluster_ids + np.uint32(base))
        first.append(t.first[1:] + np.uint32(run))
        run += int(t.first[-1]) if len(t.first) else 0
        for k in ("x_ref", "param", "cov", "chi2", "ndf"):
            cols[k].append(getattr(t, k))
        n_tracklets += t.n_tracklets
        flags |= t.error_flags
    cat = {k: np.concatenate(v) for k, v in cols.items()}
    return Tracks(n_tracklets=n_tracklets, error_flags=flags, sector=cat["sector"], start=cat["start"],
                  first=np.concatenate(first), cluster_ids=cat["cluster_ids"], x_ref=cat["x_ref"],
                  param=cat["param"].reshape(-1, 5), cov=cat["cov"].reshape(-1, 15), chi2=cat["chi2"],
                  ndf=cat["ndf"])


def sector_spans(row_offsets, n_rows=N_ROWS):
    """(sector, first cluster, end cluster, sector-local row offsets) for every sector."""
    ro = np.asarray(row_offsets, np.uint32)
    S = (len(ro) - 1) // n_rows
    out = []
    for s in range(S):
        a, b = int(ro[s * n_rows]), int(ro[(s + 1) * n_rows])
        out.append((s, a, b, (ro[s * n_rows:(s + 1) * n_rows + 1] - np.uint32(a)).astype(np.uint32)))
    return out


def track_per_sector(tracker, y, z, row_offsets, z_lo, z_hi, n_rows=N_ROWS) -> Tracks:
    """Plain path: one request per sector (device tensors are sliced, not copied)."""
    parts = []
    z_lo = np.asarray(z_lo, np.float32)
    z_hi = np.asarray(z_hi, np.float32)
    for s, a, b, ro in sector_spans(row_offsets, n_rows):
        t = tracker.track(y[a:b], z[a:b], ro, z_lo[s:s + 1], z_hi[s:s + 1])
        parts.append((s, a, t))
    return merge_sector_tracks(parts)


def shape_class(row_offsets, n_rows=N_ROWS):
    """Coarse shape of a frame: sector count and largest / mean row occupancy (powers of two)."""
    ro = np.asarray(row_offsets, np.int64)
    n = np.diff(ro)
    S = (len(ro) - 1) // n_rows
    mx = int(n.max()) if len(n) else 0
    mean = float(n.mean()) if len(n) else 0.0
    b = lambda v: 0 if v <= 1 else int(math.ceil(math.log2(v)))
    return (b(S), b(mx), b(mean))


# Values of each tuning knob (Tracker.set_knobs), the one the tuner starts from first: the automatic
# setting, except for the K2 grouping, which starts from the grouping with the least HBM traffic.
KNOB_SPACE = {"schedule": (1, 2), "select_tile_rows": (0, 2, 4, -1), "refit_order": (0, 1), "link_slots": (8, 4),
              "link_group": (-1, 64, 1, 512), "select_threads": (512, 256, 1024)}


def knob_grid(space=None):
    """Every combination of the knob values (the refit order only for the lane-per-tracklet schedule)."""
    space = dict(KNOB_SPACE if space is None else space)
    out = [{}]
    for name, values in space.items():
        nxt = []
        for c in out:
            for v in values:
                if name == "refit_order" and c.get("schedule") == 2 and v != values[0]:
                    continue
                nxt.append(dict(c, **{name: v}))
        out = nxt
    return out


class ScheduleTuner:
    """Chooses the tracker's knobs per (architecture, shape class) on the first frame of the class and
    caches the choice, optionally in a JSON file.  With ``candidates`` (knob dicts or plain schedule
    numbers) every candidate is timed; without, the knobs of ``space`` are tuned one at a time, each over
    its values with the others at their best so far (every setting timed once at most).  A setting's
    time is the sum of all passes (HIP events), best of ``repeats``; a setting replaces the one chosen
    so far (the earlier candidate, or the knob's first value) only if it is faster by more than the
    fraction ``tie``, so run-to-run noise does not decide between equals."""

    def __init__(self, tracker, candidates=None, repeats=2, cache_path=None, arch=None, space=None, tie=0.005):
        self.tracker = tracker
        self.candidates = None if candidates is None else \
            tuple(c if isinstance(c, dict) else {"schedule": int(c)} for c in candidates)
        self.space = dict(KNOB_SPACE if space is None else space)
        self.repeats = repeats
        self.tie = tie
        self.cache_path = cache_path
        self.arch = arch or "gfx950"
        self.cache = {}
        self.timings = {}
        self.tuned_runs = 0
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = {tuple(json.loads(k)): v for k, v in json.load(f).items()}

    def key(self, row_offsets):
        return (self.arch,) + shape_class(row_offsets)

    def _time(self, key, knobs, frame):
        tag = json.dumps(knobs, sort_keys=True)
        if (key, tag) not in self.timings:
            tr = self.tracker
            tr.set_knobs(**knobs)
            ms = float("inf")
            for _ in range(self.repeats):
                rid = tr.submit(*frame)
                tr.get_device(rid)
                ms = min(ms, sum(tr.pass_times().values()))
                tr.release(rid)
                self.tuned_runs += 1
            self.timings[(key, tag)] = ms
        return self.timings[(key, tag)]

    def _pick(self, key, settings, frame):
        """The first setting, replaced by any later one faster by more than the tie fraction."""
        best, t_best = None, None
        for c in settings:
            t = self._time(key, c, frame)
            if best is None or t < t_best * (1.0 - self.tie):
                best, t_best = c, t
        return best

    def choose(self, y, z, row_offsets, z_lo, z_hi):
        """The best knob setting for this frame's shape class (applied to the tracker); with plain
        schedule candidates, the schedule number."""
        key = self.key(row_offsets)
        frame = (y, z, row_offsets, z_lo, z_hi)
        if key not in self.cache:
            tr = self.tracker
            tr.set_timing(True)
            if self.candidates is not None:
                best = self._pick(key, self.candidates, frame)
            else:
                best = {k: v[0] for k, v in self.space.items()}
                for name, values in self.space.items():
                    best = self._pick(key, [dict(best, **{name: v}) for v in values], frame)
            tr.set_timing(False)
            self.cache[key] = best
            if self.cache_path:
                with open(self.cache_path, "w") as f:
                    json.dump({json.dumps(list(k)): v for k, v in self.cache.items()}, f)
        choice = self.cache[key]
        self.tracker.set_knobs(**choice)
        return choice["schedule"] if set(choice) == {"schedule"} else choice
