"""Serving loop: time frames arriving on a trace, served from several tracker slots.

A slot is one tracker with its own HIP stream and workspace, sized for the
largest frame the server admits.  The number of slots follows from an HBM
budget (budget // workspace bytes of one slot, at most ``max_slots``).
Requests wait in FIFO order; whenever a slot is free the oldest arrived request
is submitted on it, so up to ``slots`` frames are in flight on different streams
and their kernels overlap on the GPU.  A request's latency runs from its arrival
time on the trace to the moment its tracks are in host memory
(tpc_get_tracks returned).  With one slot this is the plain path: one frame at
a time, in arrival order.

Trace: Poisson arrivals; each request draws a frame from a pool of device-resident
frames (pp-like frames and heavy-ion frames of several sizes).  The pool is
reused, so the GPU does the full work of every request.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from .config import default_config
from .tracker import Tracker


@dataclasses.dataclass
class Frame:
    name: str
    kind: str                  # "pp" or "hi"
    y: object                  # device tensors
    z: object
    row_offsets: np.ndarray
    z_lo: np.ndarray
    z_hi: np.ndarray

    @property
    def n_clusters(self):
        return int(self.row_offsets[-1])


def make_pool(device, pp_seeds=(50, 51, 52), pp_orbits=2, hi_orbits=((60, 2), (61, 4), (62, 8)), log=None):
    """Device-resident frame pool: pp-like frames (650 kHz, Poisson(12) tracks per collision) and 50 kHz heavy-ion
    frames of the listed (seed, orbits)."""
    import torch
    from . import synth
    pool = []

    def add(ev, name, kind):
        pool.append(Frame(name, kind, torch.from_numpy(ev.y).to(device), torch.from_numpy(ev.z).to(device),
                          np.asarray(ev.row_offsets, np.uint32), np.asarray(ev.sector_z_lo, np.float32),
                          np.asarray(ev.sector_z_hi, np.float32)))
        if log:
            log(f"pool: {name} {ev.n_clusters} clusters")

    for s in pp_seeds:
        add(synth.pp_time_frame(seed=s, n_orbits=pp_orbits), f"pp(seed={s}, orbits={pp_orbits})", "pp")
    for s, o in hi_orbits:
        add(synth.time_frame(seed=s, n_orbits=o), f"pbpb(seed={s}, orbits={o})", "hi")
    return pool


def make_trace(pool, rate_hz, duration_s, pp_fraction=0.8, seed=5):
    """Poisson arrivals over ``duration_s``; returns [(arrival seconds, pool index)]."""
    rng = np.random.default_rng(seed)
    n = rng.poisson(rate_hz * duration_s)
    t = np.sort(rng.uniform(0.0, duration_s, n))
    pp = [i for i, f in enumerate(pool) if f.kind == "pp"]
    hi = [i for i, f in enumerate(pool) if f.kind == "hi"]
    kinds = rng.random(n) < pp_fraction
    idx = np.where(kinds, rng.choice(pp, n) if pp else rng.choice(hi, n), rng.choice(hi, n) if hi else rng.choice(pp, n))
    return list(zip(t.tolist(), idx.tolist()))


class Server:
    def __init__(self, max_clusters, max_sectors=36, slots=6, hbm_budget_bytes=200 << 30, cfg=None):
        cfg = cfg or default_config()
        probe = Tracker(cfg, max_clusters=max_clusters, max_sectors=max_sectors)
        per_slot = probe.workspace_bytes
        n = max(1, min(slots, hbm_budget_bytes // per_slot))
        self.trackers = [probe] + [Tracker(cfg, max_clusters=max_clusters, max_sectors=max_sectors)
                                   for _ in range(n - 1)]
        self.max_clusters = max_clusters
        self.workspace_bytes = per_slot * n

    @property
    def slots(self):
        return len(self.trackers)

    def close(self):
        for t in self.trackers:
            t.close()

    def run(self, pool, trace, keep_outputs=False, idle_sleep=20e-6):
        """Serve the trace in real time; returns per-request records (and outputs if asked)."""
        for f in pool:
            if f.n_clusters > self.max_clusters:
                raise ValueError(f"frame {f.name} exceeds the slot capacity")
        n = len(trace)
        rec = [None] * n
        outs = [None] * n if keep_outputs else None
        queue = collections.deque()
        busy = {}                       # slot -> (request, rid, submit time)
        free = list(range(self.slots))
        nxt, done = 0, 0
        t0 = time.perf_counter()
        while done < n:
            now = time.perf_counter() - t0
            while nxt < n and trace[nxt][0] <= now:
                queue.append(nxt)
                nxt += 1
            while free and queue:
                q = queue.popleft()
                s = free.pop()
                f = pool[trace[q][1]]
                rid = self.trackers[s].submit(f.y, f.z, f.row_offsets, f.z_lo, f.z_hi)
                busy[s] = (q, rid, time.perf_counter() - t0)
            progressed = False
            for s in list(busy):
                q, rid, ts = busy[s]
                out = self.trackers[s].get(rid, blocking=False)
                if out is None:
                    continue
                te = time.perf_counter() - t0
                self.trackers[s].release(rid)
                del busy[s]
                free.append(s)
                f = pool[trace[q][1]]
                rec[q] = dict(arrival=trace[q][0], submit=ts, done=te, latency=te - trace[q][0],
                              service=te - ts, clusters=f.n_clusters, kind=f.kind, tracks=out.n_tracks,
                              flags=out.error_flags)
                if keep_outputs:
                    outs[q] = out
                done += 1
                progressed = True
            if not progressed and not (free and queue):
                wait = (trace[nxt][0] - (time.perf_counter() - t0)) if (nxt < n and not busy) else idle_sleep
                time.sleep(max(0.0, min(wait, 1e-3)))
        wall = time.perf_counter() - t0
        return rec, outs, wall


def summarize(rec, wall, duration_s):
    lat = np.array([r["latency"] for r in rec]) * 1e3
    cl = sum(r["clusters"] for r in rec)
    last_arrival = max(r["arrival"] for r in rec)
    return {
        "requests": len(rec),
        "clusters": cl,
        "offered_clusters_per_s": cl / duration_s,
        "achieved_clusters_per_s": cl / wall,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "max_ms": float(lat.max()),
        "drain_s": wall - last_arrival,
        "errors": int(sum(1 for r in rec if r["flags"])),
    }
