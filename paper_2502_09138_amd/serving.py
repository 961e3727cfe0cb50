"""Serving loop: time frames arriving on a trace, admitted by an HBM budget.

Continuous batching over tracker slots.  A slot is one tracker with its own
HIP stream and pinned host buffers; it holds no device memory of its own
between requests.  The device memory is one pool of ``hbm_budget_bytes``
(grids, links, tracklet state and outputs of every request in flight live
there), carved per request: a request needs ``tpc_workspace_bytes_for`` its
own cluster count, and it is admitted -- in arrival order -- once a slot is
free and its bytes fit in what the requests in flight leave of the budget.
Its workspace is returned to the pool when its tracks have been copied to the
host.  Requests that arrive while others run are admitted as slots and memory
free up, and their kernels overlap on the device.

The plain path it is measured against is one frame at a time in arrival order,
each tracked as one request per sector (the per-sector launches).

A request's latency runs from its arrival time on the trace to the moment its
tracks are in host memory.  A request whose tracking fails (capacity, input) is
released, its status recorded, and the loop goes on.

Trace: Poisson arrivals; 70% pp-like frames of 1-4 orbits (650 kHz pile-up,
Poisson(12) tracks per collision) and 30% heavy-ion frames of 1-32 orbits
(50 kHz, the time-frame recipe).  Frames come from a device-resident pool:
every pp orbit count has its own frame; heavy-ion orbit counts are grouped in
powers of two (1, 2, 3-4, 5-8, 9-16, 17-32), each served by the frame with the
group's largest orbit count, which never understates the work.
"""
from __future__ import annotations

import bisect
import collections
import dataclasses
import time

import numpy as np

from .config import default_config
from .tracker import Tracker, TrackerError

ALIGN = 256
N_ROWS = 152
PP_ORBITS = (1, 2, 3, 4)
HI_ORBIT_FRAMES = (1, 2, 4, 8, 16, 32)


@dataclasses.dataclass
class Frame:
    name: str
    kind: str                  # "pp" or "hi"
    orbits: int
    y: object                  # device tensors
    z: object
    row_offsets: np.ndarray
    z_lo: np.ndarray
    z_hi: np.ndarray

    @property
    def n_clusters(self):
        return int(self.row_offsets[-1])

    @property
    def n_sectors(self):
        return (len(self.row_offsets) - 1) // N_ROWS


def make_pool(device, pp_orbits=PP_ORBITS, hi_orbits=HI_ORBIT_FRAMES, pp_seed0=50, hi_seed0=60, log=None):
    """Device-resident frame pool: one pp-like frame per orbit count in ``pp_orbits`` and one 50 kHz
    heavy-ion frame per orbit count in ``hi_orbits`` (seeds pp_seed0 + i, hi_seed0 + i)."""
    import torch
    from . import synth
    pool = []

    def add(ev, name, kind, orbits):
        pool.append(Frame(name, kind, orbits, torch.from_numpy(ev.y).to(device), torch.from_numpy(ev.z).to(device),
                          np.asarray(ev.row_offsets, np.uint32), np.asarray(ev.sector_z_lo, np.float32),
                          np.asarray(ev.sector_z_hi, np.float32)))
        if log:
            log(f"pool: {name} {ev.n_clusters} clusters")

    for i, o in enumerate(pp_orbits):
        add(synth.pp_time_frame(seed=pp_seed0 + i, n_orbits=o), f"pp(seed={pp_seed0 + i}, orbits={o})", "pp", o)
    for i, o in enumerate(hi_orbits):
        add(synth.time_frame(seed=hi_seed0 + i, n_orbits=o), f"pbpb(seed={hi_seed0 + i}, orbits={o})", "hi", o)
    return pool


def frame_for(pool, kind, orbits):
    """Index of the pool frame serving a request of this kind and orbit count: the frame of that kind
    with the smallest orbit count >= orbits (the largest one if none is)."""
    cand = sorted((f.orbits, i) for i, f in enumerate(pool) if f.kind == kind)
    if not cand:
        raise ValueError(f"no {kind} frame in the pool")
    for o, i in cand:
        if o >= orbits:
            return i
    return cand[-1][1]


def make_trace(pool, rate_hz=200.0, duration_s=10.0, pp_fraction=0.7, pp_orbits=(1, 4), hi_orbits=(1, 32), seed=5):
    """Poisson arrivals over ``duration_s``: [(arrival s, pool index, kind, orbits drawn)].  A request is pp with
    probability pp_fraction, its orbit count uniform over the inclusive range of its kind."""
    rng = np.random.default_rng(seed)
    n = int(rng.poisson(rate_hz * duration_s))
    t = np.sort(rng.uniform(0.0, duration_s, n))
    is_pp = rng.random(n) < pp_fraction
    o_pp = rng.integers(pp_orbits[0], pp_orbits[1] + 1, n)
    o_hi = rng.integers(hi_orbits[0], hi_orbits[1] + 1, n)
    out = []
    for k in range(n):
        kind, orb = ("pp", int(o_pp[k])) if is_pp[k] else ("hi", int(o_hi[k]))
        out.append((float(t[k]), frame_for(pool, kind, orb), kind, orb))
    return out


class WorkspacePool:
    """First-fit allocator of 256-byte-aligned ranges over [0, size) (host-side bookkeeping of one
    device buffer)."""

    def __init__(self, size):
        self.size = int(size) // ALIGN * ALIGN
        self.free_list = [(0, self.size)]     # sorted (offset, length), coalesced
        self.used = {}
        self.in_use = 0
        self.peak = 0

    def alloc(self, nbytes):
        need = (int(nbytes) + ALIGN - 1) // ALIGN * ALIGN
        for k, (off, ln) in enumerate(self.free_list):
            if ln >= need:
                if ln == need:
                    del self.free_list[k]
                else:
                    self.free_list[k] = (off + need, ln - need)
                self.used[off] = need
                self.in_use += need
                self.peak = max(self.peak, self.in_use)
                return off
        return None

    def free(self, off):
        ln = self.used.pop(off)
        self.in_use -= ln
        k = bisect.bisect_left(self.free_list, (off, 0))
        self.free_list.insert(k, (off, ln))
        # coalesce with the neighbours
        if k + 1 < len(self.free_list) and off + ln == self.free_list[k + 1][0]:
            self.free_list[k] = (off, ln + self.free_list[k + 1][1])
            del self.free_list[k + 1]
        if k > 0 and self.free_list[k - 1][0] + self.free_list[k - 1][1] == off:
            self.free_list[k - 1] = (self.free_list[k - 1][0], self.free_list[k - 1][1] + self.free_list[k][1])
            del self.free_list[k]


class Server:
    """Continuous-batching server over ``slots`` tracker slots and one device pool of hbm_budget_bytes."""

    def __init__(self, max_clusters, max_sectors=36, slots=6, hbm_budget_bytes=200 << 30, cfg=None, device=0):
        import torch
        cfg = cfg or default_config()
        self.device = torch.device("cuda", device)
        self.budget = int(hbm_budget_bytes) // ALIGN * ALIGN
        self.buf = torch.empty(self.budget + ALIGN, dtype=torch.uint8, device=self.device)
        self.base = (self.buf.data_ptr() + ALIGN - 1) // ALIGN * ALIGN
        self.pool = WorkspacePool(self.budget)
        # slots are created on the pool memory (nothing runs yet), so they allocate no device memory
        self.trackers = [Tracker(cfg, max_clusters=max_clusters, max_sectors=max_sectors, device=device,
                                 workspace=(self.base, self.budget)) for _ in range(max(1, int(slots)))]
        self.max_clusters = max_clusters
        self.max_sectors = max_sectors

    @property
    def slots(self):
        return len(self.trackers)

    def bytes_needed(self, frame):
        n = self.trackers[0].workspace_bytes_for(max(1, frame.n_clusters), frame.n_sectors)
        if n == 0:
            raise ValueError(f"frame {frame.name} exceeds the slot capacity")
        return n

    def close(self):
        for t in self.trackers:
            t.close()
        self.trackers = []
        self.buf = None

    def run(self, pool, trace, keep_outputs=False, idle_sleep=20e-6):
        """Serve the trace in real time; returns (per-request records, outputs if asked, wall seconds)."""
        need = [self.bytes_needed(f) for f in pool]
        for f, b in zip(pool, need):
            if b > self.budget:
                raise ValueError(f"frame {f.name} needs {b} bytes, more than the budget")
        n = len(trace)
        rec = [None] * n
        outs = [None] * n if keep_outputs else None
        queue = collections.deque()
        busy = {}                       # slot -> (request, rid, pool offset, admit time)
        free = list(range(self.slots))
        nxt, done = 0, 0
        held = set()                    # requests whose admission waited for budget while a slot was free
        t0 = time.perf_counter()
        while done < n:
            now = time.perf_counter() - t0
            while nxt < n and trace[nxt][0] <= now:
                queue.append(nxt)
                nxt += 1
            # admission in arrival order: the head waits for a slot and for its bytes
            blocked = False
            while free and queue:
                q = queue[0]
                f = pool[trace[q][1]]
                nb = need[trace[q][1]]
                off = self.pool.alloc(nb)
                if off is None:
                    held.add(q)
                    blocked = True
                    break
                queue.popleft()
                s = free.pop()
                tr = self.trackers[s]
                ta = time.perf_counter() - t0
                try:
                    tr.bind_workspace(self.base + off, nb, max(1, f.n_clusters), f.n_sectors)
                    rid = tr.submit(f.y, f.z, f.row_offsets, f.z_lo, f.z_hi)
                except TrackerError as e:
                    self.pool.free(off)
                    free.append(s)
                    rec[q] = self._record(trace[q], f, ta, time.perf_counter() - t0, None, e.status, q in held)
                    done += 1
                    continue
                busy[s] = (q, rid, off, ta)
            progressed = False
            for s in list(busy):
                q, rid, off, ta = busy[s]
                tr = self.trackers[s]
                status, out = 0, None
                try:
                    # in pinned host memory now; copied out of it only where the outputs are kept
                    out = tr.get(rid, blocking=False, copy=keep_outputs)
                    if out is None:
                        continue
                except TrackerError as e:
                    status = e.status
                te = time.perf_counter() - t0
                tr.release(rid)
                self.pool.free(off)
                del busy[s]
                free.append(s)
                f = pool[trace[q][1]]
                rec[q] = self._record(trace[q], f, ta, te, out, status, q in held)
                if keep_outputs:
                    outs[q] = out
                done += 1
                progressed = True
            if not progressed and (blocked or not (free and queue)):
                wait = (trace[nxt][0] - (time.perf_counter() - t0)) if (nxt < n and not busy) else idle_sleep
                time.sleep(max(0.0, min(wait, 1e-3)))
        wall = time.perf_counter() - t0
        self.held = len(held)
        return rec, outs, wall

    @staticmethod
    def _record(tr_entry, f, ta, te, out, status, held=False):
        arrival = tr_entry[0]
        return dict(arrival=arrival, admit=ta, done=te, latency=te - arrival, wait=ta - arrival, service=te - ta,
                    clusters=f.n_clusters, kind=f.kind, orbits=tr_entry[3] if len(tr_entry) > 3 else f.orbits,
                    tracks=out.n_tracks if out is not None else 0, status=status, held_by_budget=held)


def run_plain_per_sector(tracker, pool, trace, keep_outputs=False, deadline_s=None):
    """Plain path: one frame at a time in arrival order, each as one request per sector (blocking), on one
    tracker.  Latency from arrival to the frame's last sector in host memory.  With ``deadline_s`` the
    run stops starting new frames once that much wall time has passed (a saturated plain path would
    otherwise take arbitrarily long to drain); their records stay None."""
    from .batching import merge_sector_tracks, sector_spans
    n = len(trace)
    rec = [None] * n
    outs = [None] * n if keep_outputs else None
    t0 = time.perf_counter()
    for q, entry in enumerate(trace):
        now = time.perf_counter() - t0
        if deadline_s is not None and now > deadline_s:
            break
        if entry[0] > now:
            time.sleep(entry[0] - now)
        f = pool[entry[1]]
        ta = time.perf_counter() - t0
        status, parts = 0, []
        try:
            for s, a, b, ro in sector_spans(f.row_offsets):
                t = tracker.track(f.y[a:b], f.z[a:b], ro, f.z_lo[s:s + 1], f.z_hi[s:s + 1])
                parts.append((s, a, t))
            out = merge_sector_tracks(parts)
        except TrackerError as e:
            status, out = e.status, None
        te = time.perf_counter() - t0
        rec[q] = Server._record(entry, f, ta, te, out, status)
        if keep_outputs:
            outs[q] = out
    return rec, outs, time.perf_counter() - t0


def summarize(rec, wall, duration_s):
    """Latency percentiles and throughput over the completed requests (records that are None were not
    served: see run_plain_per_sector's deadline)."""
    n_all = len(rec)
    rec = [r for r in rec if r is not None]
    lat = np.array([r["latency"] for r in rec]) * 1e3
    cl = sum(r["clusters"] for r in rec)
    last_arrival = max(r["arrival"] for r in rec)
    kinds = {}
    for k in ("pp", "hi"):
        lk = np.array([r["latency"] for r in rec if r["kind"] == k]) * 1e3
        if len(lk):
            kinds[k] = {"requests": int(len(lk)), "p50_ms": float(np.percentile(lk, 50)),
                        "p99_ms": float(np.percentile(lk, 99))}
    return {
        "requests": n_all,
        "completed": len(rec),
        "clusters": cl,
        "offered_clusters_per_s": cl / duration_s,
        "achieved_clusters_per_s": cl / wall,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "max_ms": float(lat.max()),
        "drain_s": wall - last_arrival,
        "errors": int(sum(1 for r in rec if r["status"])),
        "held_by_budget": int(sum(1 for r in rec if r.get("held_by_budget"))),
        "by_kind": kinds,
    }
