"""GPU track-model compression (C10) and decoding (C11) against the oracle.

The oracle encodes the GPU's own tracks (the same float32 parameters, x_ref and
cluster lists) from the same input clusters, so every part of the stream must
be bit-identical: coefficients, rows, codes, escaped raw values and the list
of clusters on no track.  Decoding on the GPU must give the oracle's decoded
values bit for bit, and each decoded cluster must lie within q/2 (plus float32
rounding) of its input.  Cases: a central event, six sectors of a 32-orbit
frame, a quantum small enough that many clusters escape, and a frame with no
tracks.
"""
import numpy as np
import pytest

from oracle import oracle
from paper_2502_09138_amd import synth
from paper_2502_09138_amd.config import default_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run(ev, q_y, q_z, label):
    from paper_2502_09138_amd.tracker import Tracker
    cfg = default_config()
    tr = Tracker(cfg, max_clusters=max(ev.n_clusters, 1), max_sectors=ev.n_sectors)
    rid = tr.submit(ev.y, ev.z, ev.row_offsets, ev.sector_z_lo, ev.sector_z_hi, host=True)
    try:
        tracks = tr.get(rid)
        stream, counts = tr.encode(rid, q_y, q_z)
        g = {k: v.cpu().numpy() for k, v in stream.items()}
        yd, zd, rd = (v.cpu().numpy() for v in tr.decode(stream, counts, q_y, q_z))
    finally:
        tr.release(rid)
        tr.close()
    o = oracle.codec_encode(cfg.row_x, cfg.bz, q_y, q_z, tracks.first, tracks.cluster_ids, tracks.x_ref,
                            tracks.param, ev.y, ev.z, ev.row_offsets)
    print(label, "tracks", counts["n_tracks"], "track clusters", counts["n_track_clusters"], "unassigned",
          counts["n_unassigned"], "escaped", counts["n_escaped"], flush=True)
    assert counts["n_tracks"] == tracks.n_tracks and counts["n_track_clusters"] == len(tracks.cluster_ids)
    assert counts["n_escaped"] == o["n_escaped"] and counts["n_unassigned"] == len(o["un_row"])
    assert np.array_equal(g["coef"].view(np.int32), o["coef"].view(np.int32))
    assert np.array_equal(g["x_ref"], o["x_ref"]) and np.array_equal(g["first"].view(np.uint32), o["first"])
    assert np.array_equal(g["row"], o["row"])
    assert np.array_equal(g["code"], o["code"])
    assert np.array_equal(g["raw"].view(np.int32), o["raw"].view(np.int32))
    assert np.array_equal(g["un_row"], o["un_row"]) and np.array_equal(g["un_yz"].view(np.int32),
                                                                      o["un_yz"].view(np.int32))
    # decoding: the oracle's values bit for bit, within half a quantum of the input
    oy, oz = oracle.codec_decode(cfg.row_x, q_y, q_z, o)
    nc = counts["n_track_clusters"]
    assert np.array_equal(yd[:nc].view(np.int32), oy.view(np.int32))
    assert np.array_equal(zd[:nc].view(np.int32), oz.view(np.int32))
    assert np.array_equal(rd[:nc], o["row"]) and np.array_equal(rd[nc:], o["un_row"])
    assert np.array_equal(yd[nc:], o["un_yz"][:, 0]) and np.array_equal(zd[nc:], o["un_yz"][:, 1])
    ids = tracks.cluster_ids
    ym, zm = ev.y[ids].astype(np.float64), ev.z[ids].astype(np.float64)
    assert np.all(np.abs(yd[:nc] - ym) <= 0.5 * q_y * (1 + 1e-5) + 4 * np.spacing(np.abs(ev.y[ids])))
    assert np.all(np.abs(zd[:nc] - zm) <= 0.5 * q_z * (1 + 1e-5) + 4 * np.spacing(np.abs(ev.z[ids])))
    return counts


def test_codec_central_event(torch_cuda):
    ev = synth.central_event(seed=2)
    print("case: central_event seed=2 N=", ev.n_clusters, flush=True)
    c = _run(ev, 0.01, 0.015, "central_event")
    assert c["n_tracks"] > 1000 and c["n_escaped"] < c["n_track_clusters"] // 100


def test_codec_time_frame_sectors(torch_cuda):
    ev = synth.time_frame(seed=3).sector_slice(range(6))
    print("case: time_frame seed=3 sectors 0-5 N=", ev.n_clusters, flush=True)
    _run(ev, 0.02, 0.02, "time_frame sectors 0-5")


def test_codec_escapes(torch_cuda):
    ev = synth.central_event(seed=2).sector_slice(range(2))
    print("case: central_event sectors 0-1, q = 2e-6 cm (escapes) N=", ev.n_clusters, flush=True)
    c = _run(ev, 2e-6, 2e-6, "escapes")
    assert c["n_escaped"] > c["n_track_clusters"] // 10


def test_codec_frame_without_tracks(torch_cuda):
    import types
    rng = np.random.default_rng(4)
    R = synth.N_ROWS
    row_x, half_y = synth.row_geometry()
    per = 5   # five scattered clusters per row: no chain of neighbours forms
    y = np.concatenate([rng.uniform(-0.9 * half_y[r], 0.9 * half_y[r], per) for r in range(R)]).astype(np.float32)
    z = rng.uniform(-240.0, 240.0, per * R).astype(np.float32)
    ev = types.SimpleNamespace(y=y, z=z, row_offsets=np.arange(0, per * R + 1, per, dtype=np.uint32),
                               sector_z_lo=np.array([-250.0], np.float32), sector_z_hi=np.array([250.0], np.float32),
                               n_clusters=per * R, n_sectors=1)
    print("case: one sector of scattered clusters N=", ev.n_clusters, flush=True)
    c = _run(ev, 0.01, 0.01, "no tracks")
    assert c["n_tracks"] == 0 and c["n_unassigned"] == ev.n_clusters


def test_codec_rejects_bad_arguments(torch_cuda):
    from paper_2502_09138_amd.tracker import Tracker, TrackerError, TPC_E_INVAL
    ev = synth.single_sector(seed=1, n_tracks=20)
    tr = Tracker(default_config(), max_clusters=ev.n_clusters, max_sectors=1)
    rid = tr.submit(ev.y, ev.z, ev.row_offsets, ev.sector_z_lo, ev.sector_z_hi, host=True)
    try:
        tr.get(rid)
        for q in (0.0, -0.01, float("nan"), float("inf")):
            with pytest.raises(TrackerError) as e:
                tr.encode(rid, q, 0.01)
            assert e.value.status == TPC_E_INVAL
        with pytest.raises(TrackerError) as e:
            tr.encode(rid + 1, 0.01, 0.01)      # not the request in flight
        assert e.value.status == TPC_E_INVAL
        stream, counts = tr.encode(rid, 0.01, 0.01)
        with pytest.raises(TrackerError) as e:
            tr.decode(stream, counts, 0.0, 0.01)
        assert e.value.status == TPC_E_INVAL
    finally:
        tr.release(rid)
        tr.close()
