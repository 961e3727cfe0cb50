"""Pins of the oracle's sector merger (C8) and merged-chain refit (C9) (CPU).

* C8.1 rotation: a generated particle's state in one sector frame, rotated by
  20 degrees, equals the generator's own crossing state in the neighbouring
  frame at the rotated x (independent closed form); the rotation Jacobian
  equals finite differences of rotate-then-return-to-the-plane.
* C8/C9 on noiseless particles aimed at a sector edge: every particle whose
  clusters lie in two sectors becomes one chain holding exactly its clusters,
  and the refit parameters equal the generator's helix to 1e-9.
* Invariants: links join same-side neighbouring sectors only, in increasing
  radius, at most one successor and one predecessor per track, no cycles.
* Plausibility on the central event (thresholds parity-unpinned): links join
  segments of one particle in >= 99.5% of cases.
"""
import math

import numpy as np
import pytest

from oracle import oracle
from paper_2502_09138_amd import synth

R = synth.N_ROWS
D20 = math.radians(20.0)


def test_rotation_matches_the_generator():
    rng = np.random.default_rng(3)
    part = synth._particles(rng, 40, np.exp(rng.uniform(np.log(0.3), np.log(5.0), 40)), 0.0, 0.9,
                            phi=np.deg2rad(rng.uniform(14.0, 26.0, 40)))
    a0, a1 = synth.sector_alpha(0), synth.sector_alpha(1)
    n = 0
    for i in range(40):
        X = 150.0
        ok, st0 = synth.helix_state_at_row(part, i, a0, X)
        if not ok:
            continue
        rc, x1, q, J = oracle.rotate(X, st0, D20, synth.BZ_TESLA)
        if rc:
            continue
        ok1, st1 = synth.helix_state_at_row(part, i, a1, x1)
        assert ok1
        assert np.allclose(q, st1, rtol=0, atol=1e-10), (q, st1)
        n += 1
    assert n >= 30


def test_rotation_jacobian_matches_finite_differences():
    bz = synth.BZ_TESLA
    x = 140.0
    p = np.array([12.0, 40.0, 0.3, 0.4, -0.8])
    rc, x1, q0, J = oracle.rotate(x, p, D20, bz)
    assert rc == 0
    eps = np.array([1e-4, 1e-4, 1e-6, 1e-6, 1e-6])
    for j in range(5):
        cols = []
        for sgn in (1, -1):
            pp = p.copy()
            pp[j] += sgn * eps[j]
            rc, xe, qe, _ = oracle.rotate(x, pp, D20, bz)
            rc2, qb, _ = oracle.propagate(qe, xe, x1, bz)      # back onto the plane x' = x1
            assert rc == 0 and rc2 == 0
            cols.append(qb)
        num = (cols[0] - cols[1]) / (2 * eps[j])
        assert np.allclose(J[:, j], num, rtol=1e-5, atol=1e-7), (j, J[:, j], num)


def _sector_of_tracks(ev, res):
    return np.searchsorted(ev.row_offsets[::R][1:], res["starts"][res["trk_tracklet"]], side="right")


def test_noiseless_boundary_crossers_merge_and_refit_to_truth(cfg):
    ev = synth.boundary_crossers(seed=7, smear=synth.NOISELESS)
    run = oracle.Run.from_event(cfg, ev, fp64=(ev.y_true, ev.z_true)).run_all()
    res = run.result()
    m = oracle.merge(run, [0, 1, 2])
    sec = _sector_of_tracks(ev, res)
    x = synth.row_geometry()[0]
    # particles whose clusters make tracks in two or more sectors (segments)
    first, cl = res["trk_first"], res["trk_clusters"]
    seg_of = {}
    for t in range(len(first) - 1):
        parts = np.unique(ev.particle[cl[first[t]:first[t + 1]]])
        assert len(parts) == 1
        seg_of.setdefault(int(parts[0]), []).append(t)
    split = {p for p, ts in seg_of.items() if len(set(sec[ts].tolist())) > 1}
    merged = 0
    for k, h in enumerate(m["heads"]):
        ids = m["clusters"][m["first"][k]:m["first"][k + 1]]
        parts = np.unique(ev.particle[ids])
        assert len(parts) == 1 and parts[0] >= 0
        p = int(parts[0])
        if m["nseg"][k] < 2:
            continue
        merged += 1
        own = np.concatenate([cl[first[t]:first[t + 1]] for t in seg_of[p]])
        assert sorted(ids.tolist()) == sorted(own.tolist())       # every segment of the particle, nothing else
        assert m["ndf"][k] == 2 * len(ids) - 5
        i = res["trk_tracklet"][h]
        ok, truth = synth.helix_state_at_row(ev.particles, p, synth.sector_alpha(sec[h]), x[res["tk_xref_row"][i]])
        assert ok
        assert np.all(np.abs(m["param"][k] - truth) <= 1e-9 * np.maximum(1.0, np.abs(truth))), (m["param"][k], truth)
        np.linalg.cholesky(oracle.unpack_cov(m["cov"][k]))
    assert merged >= 40 and merged == len(split), (merged, len(split))


def test_merge_invariants(cfg):
    ev = synth.boundary_crossers(seed=8)
    run = oracle.Run.from_event(cfg, ev).run_all()
    res = run.result()
    m = oracle.merge(run, [0, 1, 2])
    sec = _sector_of_tracks(ev, res)
    nxt = m["next"]
    x = synth.row_geometry()[0]
    xref = x[res["tk_xref_row"][res["trk_tracklet"]]]
    r_in = np.hypot(xref, res["tk_param"][res["trk_tracklet"]][:, 0])
    succ_of = {}
    for a, b in enumerate(nxt):
        if b < 0:
            continue
        assert abs(int(sec[a]) - int(sec[b])) == 1          # neighbouring sectors of one side
        assert r_in[b] > r_in[a]                             # outward
        assert b not in succ_of
        succ_of[b] = a
    assert len(m["heads"]) + len(succ_of) == len(nxt)       # every track is a head or has one predecessor
    assert len(m["heads"]) < len(nxt)
    # without neighbour information nothing merges
    m0 = oracle.merge(run, None)
    assert np.all(m0["next"] == -1) and len(m0["heads"]) == len(nxt)
    assert np.array_equal(m0["param"], res["tk_param"][res["trk_tracklet"]])


@pytest.mark.slow
def test_merge_purity_central_event(cfg):
    ev = synth.central_event(seed=2)
    run = oracle.Run.from_event(cfg, ev).run_all()
    res = run.result()
    m = oracle.merge(run, np.arange(36))
    first, cl = res["trk_first"], res["trk_clusters"]

    def major(t):
        p = ev.particle[cl[first[t]:first[t + 1]]]
        v, c = np.unique(p, return_counts=True)
        return v[c.argmax()]

    links = [(a, b) for a, b in enumerate(m["next"]) if b >= 0]
    same = sum(1 for a, b in links if major(a) == major(b) and major(a) >= 0)
    print("links", len(links), "same particle", same, "chains", len(m["heads"]))
    assert len(links) > 3000 and same >= 0.995 * len(links)
