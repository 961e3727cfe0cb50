"""Benchmark: TPC clusters/s tracked on one MI355X, time-frame latency against the plain path.

One step = steps C1..C7 over the whole workload: enqueue the time frame
(device-resident clusters), wait for it (tracks stay in HBM; the counts come
back to the host), release.  A second loop measures the same with the track
arrays copied to host memory ("e2e_host_copy").  The default workload is the
32-orbit continuous-readout time frame at 50 kHz (seeded synthetic data,
about 10M clusters in 36 sectors).

Beside the headline the line carries: per-frame latency of the plain
per-sector launches on the same frame; the 512 uneven chunks in one batched
request; a short serving trace (Poisson arrivals at 200 requests/s, 70% pp of
1-4 orbits, 30% heavy-ion of 1-32 orbits) served with continuous batching
under a 200 GB budget against the plain per-sector path; the roofline entry of
the dominant kernel; the FP64 oracle timed on the host cores on a bounded
sample, with the host CPU model.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes (see the per-pass table in the design notes)
K5_BYTES_PER_STEP = 30.0        # bin-start pair, ~2 candidate (y, z) pairs, row->hit entry
K5_BYTES_PER_TRACKLET = 700.0   # chain walk, seed reads, state/covariance/row column writes
K1_BYTES_PER_CLUSTER = 22.0     # read y, z; write sorted (y, z), id, ~2 B of bin starts
K2_BYTES_PER_CLUSTER = 18.0     # read own (y, z) + each adjacent row once + bin starts; write up0/down0


# Stored rocprofv3 figures per workload (commands and tables in profiles/): HBM bytes per launch
# (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 KiB, scaled on a 1 GiB device copy) and VALU wave
# instructions per launch (SQ_INSTS_VALU).  They hold for the kernel sources with the listed SHA-1
# digests and are reported as null once a source differs, or when the run's knob setting differs from the
# profiled one; they are not measured in this run.
PROFILE_SOURCES = (
    "paper_2502_09138_amd/csrc/tracklet.hip",
    "paper_2502_09138_amd/csrc/links.hip",
    "paper_2502_09138_amd/csrc/grid.hip",
    "paper_2502_09138_amd/csrc/device_common.h",
    "paper_2502_09138_amd/csrc/tpc_internal.h",
)
PROFILES = {
    "time_frame": {
        "digests": ("e6f5144456141a8ece92fb362dab16b7baf29c14", "c842c467a72239a1275ba70e0d941297d2d258a8",
                    "0c2bdc7fab0f213bed5c4784cc480462ad908377", "b4b103e57db5db269528a9bdae40217f2bb52ff1",
                    "9cd7cf284155efdc8f0dcaf15d9b2a7a4972b985"),
        "knobs": {"schedule": 1, "select_tile_rows": 4, "refit_order": 0, "link_slots": 4, "link_group": -1,
                  "select_threads": 1024},
        # tracklets: k_seed + k_up + k_sort + k_down + k_guard; VALU of k_up and k_down (the rest is < 5%)
        "traffic_bytes": {"tracklets": 5_473_990_000, "grid": 292_040_000, "neighbours": 182_370_000},
        "valu_insts": {"tracklets": 960_531_614, "grid": 21_682_775, "neighbours": 247_349_791},
        "files": "profiles/time_frame_hbm_traffic.md, profiles/time_frame_sq_counters.md",
    },
}
# Issue ceiling of vector instructions: 256 CUs x 4 SIMDs, one wave64 VALU instruction per SIMD every
# 4 cycles (16 lanes), at 2.4 GHz.
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def stored_profile(workload, knobs=None):
    import hashlib
    prof = PROFILES.get(workload)
    if prof is None:
        return None
    if prof.get("knobs") is not None and knobs != prof["knobs"]:
        return None   # profiled with another knob setting
    for rel, digest in zip(PROFILE_SOURCES, prof["digests"]):
        with open(os.path.join(ROOT, rel), "rb") as f:
            if hashlib.sha1(f.read()).hexdigest() != digest:
                return None
    return prof


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_workload(name):
    from paper_2502_09138_amd import synth
    if name == "central_event":
        return synth.central_event(seed=2), dict(workload="central_event", seed=2, n_primaries=8000,
                                                 secondary_frac=0.1)
    if name == "single_sector":
        return synth.single_sector(seed=1), dict(workload="single_sector", seed=1, n_tracks=200)
    if name == "time_frame":
        return synth.time_frame(seed=3), dict(workload="time_frame", seed=3, n_orbits=32, rate_khz=50)
    if name == "uneven_chunks":
        return synth.uneven_chunks(), dict(workload="uneven_chunks", seed0=1000, n_chunks=512)
    if name == "pp_frame":
        return synth.pp_time_frame(seed=50, n_orbits=2), dict(workload="pp_frame", seed=50, n_orbits=2, rate_khz=650)
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(ev, budget_s):
    """FP64 oracle, single thread, on whole sectors (cycling through the workload) until ~budget_s of CPU work."""
    from oracle import oracle
    from paper_2502_09138_amd.config import default_config
    cfg = default_config().as_dict()
    subs = []
    done_clusters, t_total, n_runs = 0, 0.0, 0
    while t_total < budget_s:
        s = n_runs % ev.n_sectors
        if len(subs) <= s:
            subs.append(ev.sector_slice([s]))
        sub = subs[s]
        t0 = time.perf_counter()
        oracle.Run.from_event(cfg, sub).run_all()
        t_total += time.perf_counter() - t0
        done_clusters += sub.n_clusters
        n_runs += 1
    passes = n_runs / ev.n_sectors
    return dict(value=done_clusters / t_total, unit="clusters/s", cores=1, kind="oracle",
                sample=f"{n_runs} whole-sector runs ({passes:.2f} passes over the workload's {ev.n_sectors} sectors, "
                       f"{done_clusters} clusters), full C1-C7, one thread, {t_total:.1f} s", seconds=t_total)


def copy_bandwidth(torch, dev, mib=1024, reps=5):
    """Device-to-device copy of a 1 GiB buffer: the HBM bandwidth a plain streaming kernel achieves."""
    a = torch.empty(mib << 20, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        b.copy_(a)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    del a, b
    return {"value": round(2.0 * (mib << 20) / (ms * 1e-3) / 1e9, 1), "unit": "GB/s",
            "note": f"read + write of a {mib} MiB device copy, mean of {reps}"}


def _oracle_sector(args):
    cfg, ro, y, z, lo, hi = args
    from oracle import oracle
    t0 = time.perf_counter()
    oracle.Run(cfg, ro, y, z, lo, hi).run_all()
    return time.perf_counter() - t0


def cpu_baseline_pool(ev, budget_s):
    """The same oracle, one sector per task on a process pool of all host cores (cores counted as the pool size)."""
    import multiprocessing as mp
    from paper_2502_09138_amd.config import default_config
    cfg = default_config().as_dict()
    cores = max(1, min(16, os.cpu_count() or 1))
    tasks = []
    for s in range(ev.n_sectors):
        sub = ev.sector_slice([s])
        tasks.append((cfg, sub.row_offsets, sub.y, sub.z, sub.sector_z_lo, sub.sector_z_hi))
    sizes = [int(t[1][-1]) for t in tasks]
    done, t_wall, passes = 0, 0.0, 0
    with mp.get_context("spawn").Pool(cores) as pool:
        pool.map(_oracle_sector, tasks[:cores])          # start-up outside the timing
        while t_wall < budget_s:
            t0 = time.perf_counter()
            pool.map(_oracle_sector, tasks, chunksize=1)
            t_wall += time.perf_counter() - t0
            done += sum(sizes)
            passes += 1
    return {"value": done / t_wall, "unit": "clusters/s", "cores": cores, "kind": "oracle",
            "sample": f"{passes} passes over the workload's {ev.n_sectors} sectors ({done} clusters), one sector per "
                      f"task on {cores} processes, {t_wall:.1f} s wall"}


def tr_schedule_rowsync(schedule, ev):
    """Which K5 kernel runs: the row-synchronous one when forced, or in auto mode when every row fits its stage."""
    if schedule in (1, 2):
        return schedule == 2
    return int(np.diff(np.asarray(ev.row_offsets, np.int64)).max()) <= 320


def serve_compare(dev, duration_s, rate_hz, slots, budget_bytes, plain_deadline_s, seed=5):
    """The serving trace (Poisson arrivals, 70% pp of 1-4 orbits, 30% heavy-ion of 1-32 orbits) run twice:
    the plain path (one frame at a time, per-sector launches) and the server (continuous batching over
    ``slots`` slots under an HBM budget).  Returns a dict for the JSON line."""
    import torch
    from paper_2502_09138_amd import serving
    from paper_2502_09138_amd.tracker import Tracker
    log("serve: generating the frame pool")
    pool = serving.make_pool(dev, log=log)
    trace = serving.make_trace(pool, rate_hz=rate_hz, duration_s=duration_s, seed=seed)
    cap = max(f.n_clusters for f in pool)
    res = {}
    tr = Tracker(max_clusters=cap)
    serving.run_plain_per_sector(tr, pool, trace[:3])                      # warm-up
    log(f"serve: plain per-sector path, {len(trace)} requests over {duration_s} s")
    rec, _, wall = serving.run_plain_per_sector(tr, pool, trace, deadline_s=plain_deadline_s)
    res["plain_per_sector"] = serving.summarize(rec, wall, duration_s)
    tr.close()
    del tr
    torch.cuda.empty_cache()
    log(f"serve: plain: {res['plain_per_sector']}")
    srv = serving.Server(max_clusters=cap, slots=slots, hbm_budget_bytes=budget_bytes)
    srv.run(pool, trace[:min(20, len(trace))])                              # warm-up on the head of the trace
    log(f"serve: served, {srv.slots} slots, budget {budget_bytes / 2**30:.0f} GiB")
    rec, _, wall = srv.run(pool, trace)
    res["served"] = dict(serving.summarize(rec, wall, duration_s), slots=srv.slots, budget_gib=budget_bytes / 2**30,
                         peak_in_use_gib=round(srv.pool.peak / 2**30, 3))
    srv.close()
    del srv
    torch.cuda.empty_cache()
    log(f"serve: served: {res['served']}")
    res["trace"] = {"rate_hz": rate_hz, "duration_s": duration_s, "requests": len(trace), "pp_fraction": 0.7,
                    "pp_orbits": "1-4", "hi_orbits": "1-32 (frames of 1, 2, 4, 8, 16, 32 orbits)", "seed": seed,
                    "pool": [f"{f.name}:{f.n_clusters}" for f in pool],
                    "plain_deadline_s": plain_deadline_s}
    return res


def serve_main(args):
    import torch
    dev = torch.device("cuda", 0)
    res = serve_compare(dev, args.serve, args.rate, args.slots, int(args.budget_gib * 2**30), args.plain_deadline)
    out = {
        "metric": "p50/p99 time-frame latency, plain per-sector launches vs continuous batching, Poisson trace",
        "value": round(res["served"]["p99_ms"], 3),
        "unit": "ms (p99, served)",
        "n_gpus": 1,
        "higher_is_better": False,
        "data": "synthetic",
        "dtype": "f32",
        "config": {"workload": "serving_trace", **res["trace"]},
        "plain_per_sector": res["plain_per_sector"],
        "served": res["served"],
    }
    print(json.dumps(out), flush=True)


def _entropy_bits(v):
    """Empirical Shannon entropy (bits per symbol) of an integer array."""
    if len(v) == 0:
        return 0.0
    _, c = np.unique(v, return_counts=True)
    p = c / c.sum()
    return float(-(p * np.log2(p)).sum())


def codec_extra(torch, tr, y, z, ev, q, reps=5):
    """C10/C11 on the frame's tracks: encode and decode times (HIP events on the tracker stream around each
    call, which waits for its kernels) and the stream's size against raw float32 (y, z)."""
    qy, qz = q
    rid = tr.submit(y, z, ev.row_offsets, ev.sector_z_lo, ev.sector_z_hi)
    try:
        tr.get_counts(rid)
        enc, dec = [], []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(tr.stream)
            stream, counts = tr.encode(rid, qy, qz)
            e1.record(tr.stream)
            e1.synchronize()
            enc.append(e0.elapsed_time(e1))
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(tr.stream)
            out = tr.decode(stream, counts, qy, qz)
            e1.record(tr.stream)
            e1.synchronize()
            dec.append(e0.elapsed_time(e1))
        code = stream["code"].cpu().numpy()
        row = stream["row"].cpu().numpy().astype(np.int32)
        first = stream["first"].cpu().numpy().astype(np.int64)
        del out
    finally:
        tr.release(rid)
    N = ev.n_clusters
    nt, nc, nu, ne = counts["n_tracks"], counts["n_track_clusters"], counts["n_unassigned"], counts["n_escaped"]
    ok = code[:, 0] != -32768
    # row steps inside a track (the first cluster of each track keeps its row)
    drow = row.copy()
    if nc:
        drow[1:] -= row[:-1]
        drow[first[:-1][first[:-1] < nc]] = row[first[:-1][first[:-1] < nc]]
    bits = _entropy_bits(code[ok, 0]) + _entropy_bits(code[ok, 1]) + _entropy_bits(drow)
    header = nt * (6 * 4 + 4 + 4)
    raw_part = ne * 8 + nu * 9
    stream_bytes = header + nc * 5 + raw_part
    entropy_bytes = header + nc * bits / 8.0 + raw_part
    raw_bytes = N * 8
    em, dm = float(np.median(enc)), float(np.median(dec))
    return {"encode_ms": round(em, 4), "decode_ms": round(dm, 4),
            "encode_clusters_per_s": round(N / (em * 1e-3), 1), "decode_clusters_per_s": round(N / (dm * 1e-3), 1),
            "q_cm": [qy, qz], "tracks": nt, "track_clusters": nc, "unassigned": nu, "escaped": ne,
            "bytes_raw_yz": raw_bytes, "bytes_stream": stream_bytes, "ratio_stream": round(raw_bytes / stream_bytes, 3),
            "entropy_bits_per_track_cluster": round(bits, 3),
            "ratio_entropy_coded_estimate": round(raw_bytes / entropy_bytes, 3),
            "note": "raw = float32 (y, z) per cluster; stream = 32 B per track + row and (k_y, k_z) per track "
                    "cluster (5 B) + 8 B per escaped + 9 B per unassigned cluster; the entropy estimate replaces "
                    "the 5 B by the empirical entropy of k_y, k_z and the row step"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="time_frame")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--schedule", type=int, default=0,
                    help="tracklet kernel schedule: 0 auto, 1 per-lane gathers, 2 row-synchronous LDS stage")
    ap.add_argument("--mode", choices=("batched", "per_sector"), default="batched",
                    help="batched: one request per frame (default); per_sector: one request per sector, the plain "
                         "baseline the batched path is compared with")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one device copy of this size first (PMC byte-counter calibration)")
    ap.add_argument("--serve", type=float, default=0.0,
                    help="instead of the plain bench: serve a Poisson trace of this many seconds on the plain "
                         "per-sector path and with continuous batching, report p50/p99 latency and clusters/s of both")
    ap.add_argument("--slots", type=int, default=6)
    ap.add_argument("--rate", type=float, default=200.0, help="trace arrival rate (requests/s)")
    ap.add_argument("--budget-gib", type=float, default=200.0, help="HBM budget of the server")
    ap.add_argument("--plain-deadline", type=float, default=30.0,
                    help="wall seconds after which the plain path stops starting new frames")
    ap.add_argument("--serve-extra", type=float, default=1.0,
                    help="seconds of serving trace in the default run's extras (0 = none)")
    ap.add_argument("--quick", action="store_true", help="headline only: no per-sector, chunk or serving extras")
    ap.add_argument("--codec", action="store_true", help="with --quick: still measure the track-model codec")
    ap.add_argument("--no-tune", dest="tune", action="store_false",
                    help="run the automatic knob setting instead of the tuned one")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2502_09138_amd", "tuning_gfx950.json"),
                    help="tuning table (knob setting per shape class); a class not in it is tuned on the spot")
    ap.add_argument("--knobs", default="", help='explicit knob setting as JSON, e.g. {"link_slots": 4}')
    ap.add_argument("--codec-q", default="0.01,0.015", help="residual quanta q_y,q_z (cm) of the codec")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (sectors and time frames "
              "shard across GPUs with no exchange, so the per-GPU figure is the one reported)", file=sys.stderr)
        sys.exit(2)

    if args.serve > 0:
        serve_main(args)
        return

    import torch
    from paper_2502_09138_amd import batching
    from paper_2502_09138_amd.config import default_config
    from paper_2502_09138_amd.tracker import Tracker

    log(f"bench: generating {args.workload}")
    ev, wl = make_workload(args.workload)
    N = ev.n_clusters
    log(f"bench: {N} clusters in {ev.n_sectors} sectors")
    dev = torch.device("cuda", 0)
    y = torch.from_numpy(ev.y).to(dev)
    z = torch.from_numpy(ev.z).to(dev)
    torch.cuda.synchronize()
    tr = Tracker(default_config(), max_clusters=N, max_sectors=ev.n_sectors, tracklet_schedule=args.schedule)
    tuning = None
    if args.knobs:
        knobs = json.loads(args.knobs)
        tr.set_knobs(**knobs)
        tuning = {"knobs": knobs, "source": "--knobs"}
    elif args.tune and args.mode == "batched" and args.schedule == 0:
        # the knob setting of this frame's shape class: from the shipped tuning table, else tuned here
        # (outside the timed region); the steps below run it
        t0 = time.perf_counter()
        tuner = batching.ScheduleTuner(tr, repeats=2, cache_path=args.tune_cache if os.path.exists(args.tune_cache)
                                       else None)
        cached = tuner.key(ev.row_offsets) in tuner.cache
        knobs = tuner.choose(y, z, ev.row_offsets, ev.sector_z_lo, ev.sector_z_hi)
        tuning = {"knobs": knobs, "source": "tuning table" if cached else "tuned", "runs": tuner.tuned_runs,
                  "seconds": round(time.perf_counter() - t0, 3),
                  "ms_by_setting": {k[1]: round(v, 4) for k, v in tuner.timings.items()}}
        log(f"bench: knobs {knobs} ({tuning['source']}, {tuner.tuned_runs} runs)")
    tr.set_timing(True)   # every pass during warm-up, to find the dominant one

    if args.calib_copy_mb:
        a = torch.empty(args.calib_copy_mb << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def step_batched():
        rid = tr.submit(y, z, ev.row_offsets, ev.sector_z_lo, ev.sector_z_hi)
        counts = tr.get_device(rid)
        passes = tr.pass_times()
        tr.release(rid)
        return counts, passes

    spans = batching.sector_spans(ev.row_offsets)
    zlo = np.asarray(ev.sector_z_lo, np.float32)
    zhi = np.asarray(ev.sector_z_hi, np.float32)

    def step_per_sector():
        counts, passes = {"n_tracks": 0, "n_tracklets": 0, "n_steps": 0}, {}
        for s, a, b, ro in spans:
            rid = tr.submit(y[a:b], z[a:b], ro, zlo[s:s + 1], zhi[s:s + 1])
            c = tr.get_device(rid)
            for k, v in tr.pass_times().items():
                passes[k] = passes.get(k, 0.0) + v
            tr.release(rid)
            for k in counts:
                counts[k] += c[k]
        return counts, passes

    step = step_batched if args.mode == "batched" else step_per_sector

    warm_acc = {}
    for _ in range(args.warmup):
        _, passes = step()
        for k, v in passes.items():
            warm_acc.setdefault(k, []).append(v)
    dominant = max(warm_acc, key=lambda k: float(np.median(warm_acc[k]))) if warm_acc else "tracklets"
    # timed loop: HIP events around the dominant pass only (each event record
    # costs stream time); the per-pass breakdown is taken afterwards
    tr.set_timing(True, passes=(dominant,))
    torch.cuda.synchronize()
    lat, pass_acc = [], {}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        counts, passes = step()
        lat.append(time.perf_counter() - s0)
        for k, v in passes.items():
            pass_acc.setdefault(k, []).append(v)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"bench: {args.steps} steps in {elapsed:.3f} s; tracks {counts['n_tracks']}, tracklets {counts['n_tracklets']}")
    dom_ms = float(np.mean(pass_acc[dominant]))
    # per-pass breakdown, every pass timed (outside the timed region)
    tr.set_timing(True)
    n_bd = max(3, args.steps // 2)
    bd_acc = {}
    for _ in range(n_bd):
        _, passes = step()
        for k, v in passes.items():
            bd_acc.setdefault(k, []).append(v)
    tr.set_timing(False)
    # end to end with the track arrays copied to pinned host memory (read there as numpy views)
    n_e2e = max(3, args.steps // 2)
    t1 = time.perf_counter()
    for _ in range(n_e2e):
        if args.mode == "batched":
            n_out = tr.track_to_host(y, z, ev.row_offsets, ev.sector_z_lo, ev.sector_z_hi, lambda t: t.n_tracks)
        else:
            n_out = batching.track_per_sector(tr, y, z, ev.row_offsets, ev.sector_z_lo, ev.sector_z_hi).n_tracks
    e2e = time.perf_counter() - t1
    assert n_out == counts["n_tracks"]

    value = N * args.steps / elapsed
    pass_ms = {k: float(np.mean(v)) for k, v in bd_acc.items()}
    pass_ms[dominant] = dom_ms   # the dominant pass as timed inside the timed loop
    sched = tuning["knobs"]["schedule"] if tuning else args.schedule
    k5_name = ("k_tracklets_rs (K5, C5)" if tr_schedule_rowsync(sched, ev)
               else "k_seed, k_up, k_sort, k_down, k_guard (K5, C5)")
    prof = stored_profile(wl["workload"], tuning["knobs"] if tuning else None)

    def roof_entry(kernel, pass_name, alg_bytes, issue_bound):
        ms = pass_ms[pass_name]
        gbs = alg_bytes / (ms * 1e-3) / 1e9
        hbm = dict(achieved=round(gbs, 2), peak=HBM_PEAK_GBS, unit="GB/s", frac=round(gbs / HBM_PEAK_GBS, 5),
                   algorithmic_bytes=round(alg_bytes))
        e = dict(kernel=kernel, kernel_ms=round(ms, 4))
        traffic = None if prof is None else prof["traffic_bytes"][pass_name]
        valu = None if prof is None else prof["valu_insts"][pass_name]
        issue = None if valu is None else valu / (ms * 1e-3) / 1e9
        if issue_bound and issue is not None:
            # limited by vector-instruction issue along dependent steps: the roofline is the issue rate
            e.update(bound="alu", achieved=round(issue, 2), peak=round(VALU_ISSUE_PEAK / 1e9, 1),
                     unit="G VALU wave-instructions/s", frac=round(issue * 1e9 / VALU_ISSUE_PEAK, 5),
                     traffic=traffic, hbm=hbm)
        else:
            e.update(bound="hbm", traffic=traffic, **hbm)
            if issue is not None:
                e["valu_issue_frac"] = round(issue * 1e9 / VALU_ISSUE_PEAK, 5)
        e["profile"] = (f"traffic and VALU counts from stored rocprofv3 runs ({prof['files']})" if prof is not None
                        else "no stored rocprofv3 profile for these kernel sources and workload: traffic null")
        return e

    k5_bytes = K5_BYTES_PER_STEP * counts["n_steps"] + K5_BYTES_PER_TRACKLET * counts["n_tracklets"]
    roof = {
        "tracklets": roof_entry(k5_name, "tracklets", k5_bytes, True),
        "grid": roof_entry("k_grid_lds (K1, C1)", "grid", K1_BYTES_PER_CLUSTER * N, False),
        "neighbours": roof_entry("k_links (K2, C2)", "neighbours", K2_BYTES_PER_CLUSTER * N, False),
    }
    roof["tracklets"]["note"] = ("Kalman steps of one tracklet depend on each other: the kernel is limited by "
                                 "instruction issue and latency, not bytes; bytes = 30 B/row step + 700 B/tracklet")
    rec = {
        "metric": "TPC clusters/sec tracked at 1 GPU + p50/p99 time-frame latency vs plain path",
        "value": round(value, 1),
        "unit": "clusters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": dict(wl, n_clusters=N, n_sectors=ev.n_sectors, n_rows=152, tracklets=counts["n_tracklets"],
                       tracks=counts["n_tracks"], tracklet_schedule=args.schedule, mode=args.mode,
                       knobs=tuning["knobs"] if tuning else "automatic"),
        "latency_ms": {"p50": round(1e3 * float(np.percentile(lat, 50)), 4),
                       "p99": round(1e3 * float(np.percentile(lat, 99)), 4)},
        "e2e_host_copy": {"value": round(N * n_e2e / e2e, 1), "unit": "clusters/s",
                          "ms_per_step": round(1e3 * e2e / n_e2e, 4), "steps": n_e2e},
        "passes_ms": {k: round(v, 4) for k, v in pass_ms.items()},
        "passes_note": (f"{dominant}: HIP events on the tracker stream over the {args.steps} timed steps; "
                        f"other passes: {n_bd} further steps with every pass timed"),
        "dominant_pass": dominant,
        "tuning": tuning,
        "roofline": roof.get(dominant, roof["tracklets"]),
        "roofline_passes": roof,
    }
    k12 = (K1_BYTES_PER_CLUSTER + K2_BYTES_PER_CLUSTER) * N / ((pass_ms["grid"] + pass_ms["neighbours"]) * 1e-3) / 1e9
    rec["k1_k2_hbm"] = {"achieved": round(k12, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(k12 / HBM_PEAK_GBS, 5),
                        "note": "grid and neighbour passes together: algorithmic bytes (22 + 18 B per cluster) over "
                                "their summed HIP-event times"}
    if not args.quick and args.mode == "batched":
        # the same frame as one request per sector (the plain path), frame latency and throughput
        ps = []
        for k in range(6):
            s0 = time.perf_counter()
            for sec, a, b, ro in spans:
                rid = tr.submit(y[a:b], z[a:b], ro, zlo[sec:sec + 1], zhi[sec:sec + 1])
                tr.get_device(rid)
                tr.release(rid)
            if k:                       # the first frame warms up the per-sector shapes
                ps.append(time.perf_counter() - s0)
        rec["per_sector_launches"] = {
            "value": round(N * len(ps) / sum(ps), 1), "unit": "clusters/s",
            "latency_ms": {"p50": round(1e3 * float(np.percentile(ps, 50)), 4),
                           "p99": round(1e3 * float(np.percentile(ps, 99)), 4)},
            "frames": len(ps), "speedup_of_batched": round(float(np.median(ps)) / (elapsed / args.steps), 2),
            "note": f"the same frame as {ev.n_sectors} requests of one sector each, issued back to back"}
        log(f"bench: per-sector launches: {rec['per_sector_launches']}")
    if (not args.quick or args.codec) and args.mode == "batched":
        rec["codec"] = codec_extra(torch, tr, y, z, ev, [float(v) for v in args.codec_q.split(",")])
        log(f"bench: codec: {rec['codec']}")
    tr.close()
    del tr, y, z
    torch.cuda.empty_cache()
    if not args.quick and args.mode == "batched" and args.workload != "uneven_chunks":
        log("bench: generating uneven_chunks")
        evc, _ = make_workload("uneven_chunks")
        yc = torch.from_numpy(evc.y).to(dev)
        zc = torch.from_numpy(evc.z).to(dev)
        trc = Tracker(default_config(), max_clusters=evc.n_clusters, max_sectors=evc.n_sectors,
                      tracklet_schedule=args.schedule)
        for _ in range(2):
            rid = trc.submit(yc, zc, evc.row_offsets, evc.sector_z_lo, evc.sector_z_hi)
            trc.get_device(rid)
            trc.release(rid)
        torch.cuda.synchronize()
        tc = []
        for _ in range(5):
            s0 = time.perf_counter()
            rid = trc.submit(yc, zc, evc.row_offsets, evc.sector_z_lo, evc.sector_z_hi)
            cc = trc.get_device(rid)
            trc.release(rid)
            tc.append(time.perf_counter() - s0)
        rec["uneven_chunks"] = {"value": round(evc.n_clusters * len(tc) / sum(tc), 1), "unit": "clusters/s",
                                "ms_per_step": round(1e3 * float(np.mean(tc)), 4), "n_clusters": evc.n_clusters,
                                "n_chunks": evc.n_sectors, "tracks": cc["n_tracks"],
                                "note": "512 sector-sized chunks of log-uniform occupancy (1k-200k), one batched request"}
        # the tuned knob setting of this shape class (tuning table, else tuned here), timed like the
        # automatic one
        tuner = batching.ScheduleTuner(trc, repeats=2, cache_path=args.tune_cache if os.path.exists(args.tune_cache)
                                       else None)
        choice = tuner.choose(yc, zc, evc.row_offsets, evc.sector_z_lo, evc.sector_z_hi)
        tt = []
        for _ in range(5):
            s0 = time.perf_counter()
            rid = trc.submit(yc, zc, evc.row_offsets, evc.sector_z_lo, evc.sector_z_hi)
            trc.get_device(rid)
            trc.release(rid)
            tt.append(time.perf_counter() - s0)
        rec["uneven_chunks"]["tuned"] = {"knobs": choice, "ms_per_step": round(1e3 * float(np.mean(tt)), 4),
                                         "tuning_runs": tuner.tuned_runs,
                                         "source": "tuning table" if tuner.tuned_runs == 0 else "tuned"}
        # the plain path: one request per chunk, back to back
        trc.set_knobs(schedule=0, select_tile_rows=0, refit_order=0)
        pc = []
        czlo = np.asarray(evc.sector_z_lo, np.float32)
        czhi = np.asarray(evc.sector_z_hi, np.float32)
        for k in range(3):
            s0 = time.perf_counter()
            for sec, a, b, ro in batching.sector_spans(evc.row_offsets):
                rid = trc.submit(yc[a:b], zc[a:b], ro, czlo[sec:sec + 1], czhi[sec:sec + 1])
                trc.get_device(rid)
                trc.release(rid)
            if k:                       # the first pass warms up the per-chunk shapes
                pc.append(time.perf_counter() - s0)
        rec["uneven_chunks"]["per_chunk_launches"] = {
            "ms_per_step": round(1e3 * float(np.mean(pc)), 4),
            "value": round(evc.n_clusters * len(pc) / sum(pc), 1), "unit": "clusters/s",
            "note": "one request per chunk (512), issued back to back (device views, as the batched step)"}
        log(f"bench: uneven_chunks: {rec['uneven_chunks']}")
        trc.close()
        del trc, yc, zc, evc
        torch.cuda.empty_cache()
    if not args.quick and args.serve_extra > 0:
        rec["serving"] = serve_compare(dev, args.serve_extra, args.rate, args.slots, int(args.budget_gib * 2**30),
                                       args.plain_deadline)
    rec["achievable_copy"] = copy_bandwidth(torch, dev)
    if not args.no_cpu_baseline:
        log("bench: timing the oracle on the host")
        cb = cpu_baseline(ev, args.cpu_budget)
        rec["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        rec["cpu_baseline"]["host_cpu"] = host_cpu()
        log("bench: timing the oracle on all host cores")
        rec["cpu_baseline_all_cores"] = cpu_baseline_pool(ev, args.cpu_budget)
    else:
        rec["cpu_baseline"] = None
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
