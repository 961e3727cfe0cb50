"""GPU sector merger (C8) and chain refit (C9) against the oracle.

Bars: the oracle's links between tracks that both sides found (same start
position) are reproduced for >= 99.5% of links, and >= 99.5% of the GPU's links
are oracle links; every chain with the same clusters on both sides and a
successful refit on both has refit parameters within 1e-4 relative (floors as
for tracks) and covariance diagonals within 1e-3 relative; chains are valid
(every track in exactly one chain, cluster lists = the segments' lists in
chain order).  A refit fails when the state reaches |sin phi| >= s_max (a
looper near its turning point); whether that happens on a chain within
rounding of the limit can differ between the two sides, so at most 0.5% of
the compared chains may succeed on one side only.
"""
import numpy as np
import pytest

from oracle import oracle
from paper_2502_09138_amd import synth
from paper_2502_09138_amd.config import default_config

import parity

pytestmark = pytest.mark.gpu
R = synth.N_ROWS


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _compare(ev, phys, label):
    from paper_2502_09138_amd.tracker import Tracker
    cfg = default_config()
    tr = Tracker(cfg, max_clusters=ev.n_clusters, max_sectors=ev.n_sectors)
    tracks, mg = tr.track_and_merge(ev.y, ev.z, ev.row_offsets, ev.sector_z_lo, ev.sector_z_hi, phys, host=True)
    tr.close()
    run = oracle.Run.from_event(cfg.as_dict(), ev).run_all()
    res = run.result()
    mo = oracle.merge(run, phys)
    # chains are a partition of the tracks; cluster lists are the segments' lists in chain order
    n = tracks.n_tracks
    assert len(mg["next"]) == n and len(mg["heads"]) == len(mg["nseg"])
    assert np.array_equal(np.sort(np.unique(mg["head_of"])), np.sort(mg["heads"]))
    for c, h in enumerate(mg["heads"]):
        ids, t = [], int(h)
        while t >= 0:
            ids.append(tracks.cluster_ids[tracks.first[t]:tracks.first[t + 1]])
            t = int(mg["next"][t])
        assert np.array_equal(np.concatenate(ids), mg["clusters"][mg["first"][c]:mg["first"][c + 1]])
    # links: GPU track index <-> oracle track index by start position
    st_o = res["starts"][res["trk_tracklet"]].astype(np.int64)
    o_of = {int(s): k for k, s in enumerate(st_o)}
    g2o = np.array([o_of.get(int(s), -1) for s in tracks.start], np.int64)
    o_links = {(a, int(b)) for a, b in enumerate(mo["next"]) if b >= 0}
    g_links = {(int(g2o[a]), int(g2o[b])) for a, b in enumerate(mg["next"]) if b >= 0}
    both = {(a, b) for a, b in o_links if a in set(g2o.tolist()) and b in set(g2o.tolist())}
    found = len(both & g_links)
    print(label, "tracks", n, "oracle links", len(o_links), "GPU links", len(g_links), "common", found, flush=True)
    assert found >= 0.995 * len(both) and found >= 0.995 * len(g_links)
    # refit parity on chains with the same clusters
    oc = {}
    for c, h in enumerate(mo["heads"]):
        oc[int(st_o[h])] = c
    n_same = bad_p = bad_c = 0
    one_sided = []
    for c, h in enumerate(mg["heads"]):
        if mg["nseg"][c] < 2:
            continue
        k = oc.get(int(tracks.start[h]))
        if k is None or mo["nseg"][k] != mg["nseg"][c]:
            continue
        if not np.array_equal(np.sort(mg["clusters"][mg["first"][c]:mg["first"][c + 1]]),
                              np.sort(mo["clusters"][mo["first"][k]:mo["first"][k + 1]])):
            continue
        n_same += 1
        if (mg["ndf"][c] < 0) != (mo["ndf"][k] < 0):
            one_sided.append((int(h), int(mg["ndf"][c]), int(mo["ndf"][k])))
            continue
        if mg["ndf"][c] < 0:
            continue
        assert mg["ndf"][c] == mo["ndf"][k]
        po = mo["param"][k]
        dp = np.abs(mg["param"][c].astype(np.float64) - po)
        bad_p += int(np.any(dp > parity.PARAM_RTOL * np.maximum(np.abs(po), parity.FLOORS)))
        do = np.diag(parity.unpack_cov(mo["cov"][k]))
        dg = np.diag(parity.unpack_cov(mg["cov"][c].astype(np.float64)))
        bad_c += int(np.any(np.abs(dg - do) > parity.COV_RTOL * np.abs(do)))
    print(label, "merged chains compared", n_same, "beyond 1e-4", bad_p, "cov beyond 1e-3", bad_c,
          "refit failed on one side only", one_sided, flush=True)
    assert n_same > 0 and bad_p == 0 and bad_c == 0
    assert len(one_sided) <= 0.005 * n_same
    return mg


def test_merge_boundary_crossers(torch_cuda):
    ev = synth.boundary_crossers(seed=7)
    print("case: boundary_crossers seed=7 N=", ev.n_clusters, flush=True)
    mg = _compare(ev, [0, 1, 2], "boundary_crossers")
    assert (mg["nseg"] > 1).sum() >= 30


def test_merge_central_event(torch_cuda):
    ev = synth.central_event(seed=2)
    print("case: central_event seed=2 N=", ev.n_clusters, flush=True)
    _compare(ev, np.arange(36), "central_event")


def test_merge_time_frame_sectors(torch_cuda):
    ev = synth.time_frame(seed=3).sector_slice(range(6))
    print("case: time_frame seed=3 sectors 0-5 N=", ev.n_clusters, flush=True)
    _compare(ev, np.arange(6), "time_frame sectors 0-5")


def test_merge_without_neighbours_changes_nothing(torch_cuda):
    from paper_2502_09138_amd.tracker import Tracker
    ev = synth.uneven_chunks(chunks=range(6))
    tr = Tracker(default_config(), max_clusters=ev.n_clusters, max_sectors=ev.n_sectors)
    tracks, mg = tr.track_and_merge(ev.y, ev.z, ev.row_offsets, ev.sector_z_lo, ev.sector_z_hi, None, host=True)
    assert np.all(mg["next"] == -1) and len(mg["heads"]) == tracks.n_tracks
    assert np.array_equal(mg["param"], tracks.param) and np.array_equal(mg["clusters"], tracks.cluster_ids)
    tr.close()
