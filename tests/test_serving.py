"""Serving loop: trace generation and the workspace pool (CPU); results alone
versus in the mix, admission by the HBM budget and oracle parity of served
requests (GPU)."""
import numpy as np
import pytest

from paper_2502_09138_amd import serving


class _F:
    def __init__(self, kind, orbits):
        self.kind = kind
        self.orbits = orbits


POOL = [_F("pp", o) for o in (1, 2, 3, 4)] + [_F("hi", o) for o in (1, 2, 4, 8, 16, 32)]


def test_trace_is_poisson_with_the_stated_mix():
    tr = serving.make_trace(POOL, rate_hz=200.0, duration_s=50.0, seed=5)
    t = np.array([a for a, _, _, _ in tr])
    assert abs(len(tr) - 10000) < 4 * np.sqrt(10000)
    assert np.all(np.diff(t) >= 0) and t[0] >= 0 and t[-1] <= 50.0
    gaps = np.diff(t)
    assert abs(gaps.mean() * 200.0 - 1.0) < 0.05          # exponential gaps, mean 1/rate
    assert abs(np.std(gaps) / gaps.mean() - 1.0) < 0.05    # coefficient of variation 1
    kinds = np.array([k for _, _, k, _ in tr])
    assert abs((kinds == "pp").mean() - 0.7) < 0.02
    orb_pp = np.array([o for _, _, k, o in tr if k == "pp"])
    orb_hi = np.array([o for _, _, k, o in tr if k == "hi"])
    assert set(orb_pp.tolist()) == {1, 2, 3, 4}
    assert orb_hi.min() == 1 and orb_hi.max() == 32 and abs(orb_hi.mean() - 16.5) < 0.5
    for _, i, k, o in tr:                                   # served by the smallest frame covering the orbits
        f = POOL[i]
        assert f.kind == k and f.orbits >= o
        assert all(g.orbits < o for g in POOL if g.kind == k and g.orbits < f.orbits)
    assert serving.make_trace(POOL, 200.0, 50.0, seed=5) == tr   # seeded


def test_workspace_pool_first_fit_and_coalescing():
    p = serving.WorkspacePool(10 * 256)
    a = p.alloc(1)          # rounds to 256
    b = p.alloc(3 * 256)
    c = p.alloc(2 * 256)
    assert (a, b, c) == (0, 256, 1024) and p.in_use == 6 * 256
    assert p.alloc(5 * 256) is None                      # only 4 * 256 left
    p.free(b)
    assert p.alloc(4 * 256) == 1536                      # the hole of 3 does not fit 4: first fit is the tail
    p.free(a)
    p.free(c)                                            # 0..1536 coalesces into one hole
    assert p.free_list == [(0, 1536)]
    assert p.alloc(6 * 256) == 0 and p.in_use == 10 * 256
    assert p.peak == 10 * 256


def _gpu_pool(dev):
    return serving.make_pool(dev, pp_orbits=(1, 2), hi_orbits=(1, 2), log=print)


@pytest.mark.gpu
def test_results_identical_alone_and_in_the_mix():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda", 0)
    pool = _gpu_pool(dev)
    trace = serving.make_trace(pool, rate_hz=400.0, duration_s=0.5, pp_fraction=0.5, pp_orbits=(1, 2),
                               hi_orbits=(1, 2), seed=7)
    assert len(trace) > 100
    srv = serving.Server(max_clusters=max(f.n_clusters for f in pool), slots=3, hbm_budget_bytes=8 << 30)
    try:
        assert srv.slots == 3
        rec, outs, wall = srv.run(pool, trace, keep_outputs=True)
        st = serving.summarize(rec, wall, 0.5)
        print(st, flush=True)
        assert st["errors"] == 0 and st["requests"] == len(trace)
        assert srv.pool.in_use == 0 and srv.pool.peak <= srv.budget
        # the same frames alone, one at a time, on one slot with its own workspace
        from paper_2502_09138_amd.tracker import Tracker
        t0 = Tracker(max_clusters=max(f.n_clusters for f in pool))
        alone = {}
        for q, entry in enumerate(trace):
            i = entry[1]
            if i not in alone:
                f = pool[i]
                alone[i] = t0.track(f.y, f.z, f.row_offsets, f.z_lo, f.z_hi)
            a, b = alone[i], outs[q]
            for k in ("sector", "start", "first", "cluster_ids", "x_ref", "param", "cov", "chi2", "ndf"):
                np.testing.assert_array_equal(getattr(a, k), getattr(b, k), err_msg=f"request {q} {k}")
        assert len(alone) == len(pool)
        t0.close()
    finally:
        srv.close()


@pytest.mark.gpu
def test_budget_holds_requests_back():
    """A budget that fits one heavy-ion request at a time: later requests wait for
    memory although slots are free, the pool never exceeds the budget, and every
    result equals the plain per-sector path."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda", 0)
    pool = _gpu_pool(dev)
    cap = max(f.n_clusters for f in pool)
    probe = serving.Server(max_clusters=cap, slots=1, hbm_budget_bytes=4 << 30)
    need = [probe.bytes_needed(f) for f in pool]
    probe.close()
    budget = max(need) + min(need) // 2          # the largest frame leaves no room for a second one
    trace = [(0.0, int(np.argmax(need)), "hi", 2)] + [(0.0, i, f.kind, f.orbits) for i, f in enumerate(pool)] * 3
    srv = serving.Server(max_clusters=cap, slots=4, hbm_budget_bytes=budget)
    try:
        rec, outs, wall = srv.run(pool, trace, keep_outputs=True)
        st = serving.summarize(rec, wall, 1.0)
        print(st, "budget", budget, "needs", need, "peak", srv.pool.peak, flush=True)
        assert st["errors"] == 0 and st["held_by_budget"] >= 1 and srv.held >= 1
        assert srv.pool.peak <= budget and srv.pool.in_use == 0
        admits = [r["admit"] for r in rec]
        assert admits == sorted(admits)              # admitted in arrival order
        from paper_2502_09138_amd.tracker import Tracker
        t0 = Tracker(max_clusters=cap)
        plain, pouts, _ = serving.run_plain_per_sector(t0, pool, trace[:len(pool) + 1], keep_outputs=True)
        for q in range(len(pool) + 1):
            for k in ("sector", "start", "first", "cluster_ids", "x_ref", "param", "cov", "chi2", "ndf"):
                np.testing.assert_array_equal(getattr(pouts[q], k), getattr(outs[q], k), err_msg=f"request {q} {k}")
        t0.close()
    finally:
        srv.close()


@pytest.mark.gpu
def test_served_requests_match_the_oracle():
    """One served pp request and one served heavy-ion request against the FP64
    oracle on two sectors each, at the parity bars of the plain path."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import parity
    from oracle import oracle
    from paper_2502_09138_amd.config import default_config
    dev = torch.device("cuda", 0)
    pool = _gpu_pool(dev)
    pick = [next(i for i, f in enumerate(pool) if f.kind == "pp" and f.orbits == 2),
            next(i for i, f in enumerate(pool) if f.kind == "hi" and f.orbits == 2)]
    trace = [(0.0, i, pool[i].kind, pool[i].orbits) for i in pick]
    srv = serving.Server(max_clusters=max(f.n_clusters for f in pool), slots=2, hbm_budget_bytes=8 << 30)
    try:
        rec, outs, _ = srv.run(pool, trace, keep_outputs=True)
        cfg = default_config().as_dict()
        R = 152
        for q, i in enumerate(pick):
            f = pool[i]
            y, z = f.y.cpu().numpy(), f.z.cpu().numpy()
            for s in (3, 22):
                a, b = int(f.row_offsets[s * R]), int(f.row_offsets[(s + 1) * R])
                ro = (f.row_offsets[s * R:(s + 1) * R + 1] - a).astype(np.uint32)
                o = oracle.Run(cfg, ro, y[a:b], z[a:b], f.z_lo[s:s + 1], f.z_hi[s:s + 1]).run_all().result()
                st = parity.compare_tracks(outs[q], o, f.n_clusters, base=a)
                print(f.name, "sector", s, st, flush=True)
                parity.check_tracks(st)
    finally:
        srv.close()
