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


def knob_grid(schedules=(1, 2), tile_rows=(0, 2, 4, -1), refit_orders=(0, 1)):
    """Every knob setting to sweep: the refit order matters only for the lane-per-tracklet schedule."""
    out = []
    for s in schedules:
        for r in tile_rows:
            for o in (refit_orders if s == 1 else (0,)):
                out.append({"schedule": s, "select_tile_rows": r, "refit_order": o})
    return out


class ScheduleTuner:
    """Chooses the tracker's knobs per (architecture, shape class) by timing every candidate setting on
    the first frame of the class (all passes, HIP events, best of ``repeats``); the choice is cached,
    optionally in a JSON file.  Candidates are knob dicts (see ``Tracker.set_knobs``) or plain schedule
    numbers."""

    def __init__(self, tracker, candidates=(1, 2), repeats=2, cache_path=None, arch=None):
        self.tracker = tracker
        self.candidates = tuple(c if isinstance(c, dict) else {"schedule": int(c)} for c in candidates)
        self.repeats = repeats
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

    def choose(self, y, z, row_offsets, z_lo, z_hi):
        """The best knob setting for this frame's shape class (applied to the tracker); with plain
        schedule candidates, the schedule number."""
        key = self.key(row_offsets)
        if key not in self.cache:
            tr = self.tracker
            best, best_ms = None, float("inf")
            tr.set_timing(True)
            for cand in self.candidates:
                tr.set_knobs(**cand)
                ms = float("inf")
                for _ in range(self.repeats):
                    rid = tr.submit(y, z, row_offsets, z_lo, z_hi)
                    tr.get_device(rid)
                    ms = min(ms, sum(tr.pass_times().values()))
                    tr.release(rid)
                    self.tuned_runs += 1
                self.timings[(key, json.dumps(cand, sort_keys=True))] = ms
                if ms < best_ms:
                    best, best_ms = cand, ms
            tr.set_timing(False)
            self.cache[key] = best
            if self.cache_path:
                with open(self.cache_path, "w") as f:
                    json.dump({json.dumps(list(k)): v for k, v in self.cache.items()}, f)
        choice = self.cache[key]
        self.tracker.set_knobs(**choice)
        return choice["schedule"] if set(choice) == {"schedule"} else choice
