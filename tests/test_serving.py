"""Serving loop: trace generation (CPU) and identical results alone versus in
a mix of overlapping requests (GPU)."""
import numpy as np
import pytest

from paper_2502_09138_amd import serving


class _F:
    def __init__(self, kind):
        self.kind = kind


def test_trace_is_poisson_and_mixes_kinds():
    pool = [_F("pp"), _F("pp"), _F("hi"), _F("hi"), _F("hi")]
    tr = serving.make_trace(pool, rate_hz=200.0, duration_s=20.0, pp_fraction=0.8, seed=5)
    t = np.array([a for a, _ in tr])
    assert abs(len(tr) - 4000) < 4 * np.sqrt(4000)
    assert np.all(np.diff(t) >= 0) and t[0] >= 0 and t[-1] <= 20.0
    gaps = np.diff(t)
    assert abs(gaps.mean() * 200.0 - 1.0) < 0.05          # exponential gaps, mean 1/rate
    assert abs(np.std(gaps) / gaps.mean() - 1.0) < 0.1     # coefficient of variation 1
    kinds = np.array([pool[i].kind for _, i in tr])
    assert abs((kinds == "pp").mean() - 0.8) < 0.03
    assert serving.make_trace(pool, 200.0, 20.0, seed=5) == tr   # seeded


@pytest.mark.gpu
def test_results_identical_alone_and_in_the_mix():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda", 0)
    pool = serving.make_pool(dev, pp_seeds=(50, 51), pp_orbits=1, hi_orbits=((60, 1), (61, 2)))
    trace = serving.make_trace(pool, rate_hz=400.0, duration_s=0.5, pp_fraction=0.5, seed=7)
    assert len(trace) > 100
    srv = serving.Server(max_clusters=max(f.n_clusters for f in pool), slots=3)
    try:
        assert srv.slots == 3
        rec, outs, wall = srv.run(pool, trace, keep_outputs=True)
        st = serving.summarize(rec, wall, 0.5)
        print(st, flush=True)
        assert st["errors"] == 0 and st["requests"] == len(trace)
        # the same frames alone, one at a time, on one slot
        alone = {}
        t0 = srv.trackers[0]
        for q, (_, i) in enumerate(trace):
            if i not in alone:
                f = pool[i]
                alone[i] = t0.track(f.y, f.z, f.row_offsets, f.z_lo, f.z_hi)
            a, b = alone[i], outs[q]
            for k in ("sector", "start", "first", "cluster_ids", "x_ref", "param", "cov", "chi2", "ndf"):
                np.testing.assert_array_equal(getattr(a, k), getattr(b, k), err_msg=f"request {q} {k}")
        assert len(alone) == len(pool)
    finally:
        srv.close()
