"""Pins of the oracle's track-model compression (C10 encoding, C11 decoding), CPU.

* Hand-worked golden (tests/golden/c10_codec.json): coefficients of a straight
  and a curved track, the codes of three clusters (one escaped) and their
  decoded values.
* The model against the helix generator: a1, 2 a2 (b1, 2 b2) equal the first
  and second derivatives of the generated particle's y(x) (z(x)) at x_ref,
  taken by central differences of the generator's own crossing points.
* Round trip: every decoded cluster lies within q/2 (plus float32 rounding)
  of its input; escaped and unassigned clusters come back bit-exact, the
  unassigned ones in input order.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle
from paper_2502_09138_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c10_codec.json")


def _ulps(a, b):
    """Distance in float32 units in the last place (+0 and -0 are the same value)."""
    def key(v):
        i = int(np.float32(v).view(np.int32))
        return i if i >= 0 else -(i & 0x7FFFFFFF)
    return abs(key(a) - key(b))


def test_golden_coefficients_codes_and_decoding():
    g = json.load(open(GOLDEN))
    rows_x = np.array(g["rows_x"], np.float64)
    for tr in g["tracks"]:
        coef = oracle.codec_coef(tr["param"], g["bz"])
        for got, want in zip(coef, tr["coef"]):
            assert _ulps(got, want) <= 2, (tr["name"], coef, tr["coef"])
        for cl in tr["clusters"]:
            # one track with one cluster, in a frame of one sector of three rows
            ro = np.zeros(4, np.uint32)
            ro[cl["row"] + 1:] = 1
            s = oracle.codec_encode(rows_x, g["bz"], cl["q"], cl["q"], [0, 1], [0], [tr["x_ref"]], [tr["param"]],
                                    [cl["y"]], [cl["z"]], ro)
            assert s["row"][0] == cl["row"] and len(s["un_row"]) == 0
            if cl["code"] == "escape":
                assert s["code"][0, 0] == oracle.CODEC_ESCAPE and s["n_escaped"] == 1
                assert tuple(s["raw"][0]) == (np.float32(cl["y"]), np.float32(cl["z"]))
            else:
                assert tuple(s["code"][0]) == tuple(cl["code"]), (tr["name"], s["code"][0], cl["code"])
            yd, zd = oracle.codec_decode(rows_x, cl["q"], cl["q"], s)
            assert abs(float(yd[0]) - cl["decoded"][0]) <= 4e-6 * max(1.0, abs(cl["decoded"][0]))
            assert abs(float(zd[0]) - cl["decoded"][1]) <= 4e-6 * max(1.0, abs(cl["decoded"][1]))


def test_model_is_the_second_order_expansion_of_the_helix():
    rng = np.random.default_rng(11)
    n = 40
    part = synth._particles(rng, n, np.exp(rng.uniform(np.log(0.3), np.log(5.0), n)), -0.9, 0.9,
                            phi=np.deg2rad(rng.uniform(-8.0, 8.0, n)))
    alpha = synth.sector_alpha(0)
    h = 0.1   # central differences: truncation error h^2 y''' / 6 below 1e-6 for these tracks
    checked = 0
    for i in range(n):
        X = 120.0
        oks = [synth.helix_state_at_row(part, i, alpha, X + d) for d in (-h, 0.0, h)]
        if not all(o for o, _ in oks):
            continue
        ym, y0, yp = (st[0] for _, st in oks)
        zm, z0, zp = (st[1] for _, st in oks)
        coef = oracle.codec_coef(oks[1][1].astype(np.float32), synth.BZ_TESLA)
        d1y, d2y = (yp - ym) / (2 * h), (yp - 2 * y0 + ym) / h ** 2
        d1z, d2z = (zp - zm) / (2 * h), (zp - 2 * z0 + zm) / h ** 2
        assert abs(coef[1] - d1y) <= 1e-5 * max(1.0, abs(d1y)), (i, coef[1], d1y)
        assert abs(2 * coef[2] - d2y) <= 2e-3 * abs(d2y) + 1e-8, (i, 2 * coef[2], d2y)
        assert abs(coef[4] - d1z) <= 1e-5 * max(1.0, abs(d1z)), (i, coef[4], d1z)
        assert abs(2 * coef[5] - d2z) <= 2e-3 * abs(d2z) + 1e-8, (i, 2 * coef[5], d2z)
        checked += 1
    assert checked >= 30


def _frame_with_tracks(seed, n_tracks=50, n_noise=300, q_noise=0.05):
    """Clusters of straight-ish model tracks plus noise clusters, in one sector (input order = row order)."""
    rng = np.random.default_rng(seed)
    row_x, _ = synth.row_geometry()
    R = len(row_x)
    recs = []   # (row, y, z, track or -1)
    tracks = []
    for t in range(n_tracks):
        r0 = int(rng.integers(0, R - 40))
        rows = np.arange(r0, r0 + int(rng.integers(20, 40)))
        p = np.array([rng.uniform(-20, 20), rng.uniform(-100, 100), rng.uniform(-0.5, 0.5), rng.uniform(-1, 1),
                      rng.uniform(-3, 3)], np.float32)
        xr = np.float32(row_x[r0])
        tracks.append((p, xr))
        coef = oracle.codec_coef(p, synth.BZ_TESLA).astype(np.float64)
        for r in rows:
            u = row_x[r] - float(xr)
            y = coef[0] + u * (coef[1] + u * coef[2]) + rng.normal(0, q_noise)
            z = coef[3] + u * (coef[4] + u * coef[5]) + rng.normal(0, q_noise)
            recs.append((r, y, z, t))
    for _ in range(n_noise):
        recs.append((int(rng.integers(0, R)), rng.uniform(-30, 30), rng.uniform(-200, 200), -1))
    recs.append((5, 1e4, 0.0, 0))     # far off track 0: escaped
    recs.sort(key=lambda a: a[0])
    row = np.array([a[0] for a in recs])
    y = np.array([a[1] for a in recs], np.float32)
    z = np.array([a[2] for a in recs], np.float32)
    trk = np.array([a[3] for a in recs])
    ro = np.searchsorted(row, np.arange(R + 1)).astype(np.uint32)
    first, ids = [0], []
    for t in range(n_tracks):
        own = np.flatnonzero(trk == t)
        own = own[np.argsort(row[own], kind="stable")]
        ids.extend(own.tolist())
        first.append(len(ids))
    x_ref = np.array([xr for _, xr in tracks], np.float32)
    param = np.array([p for p, _ in tracks], np.float32)
    return row_x, ro, y, z, np.array(first, np.uint32), np.array(ids, np.uint32), x_ref, param


@pytest.mark.parametrize("qy,qz", [(0.01, 0.01), (0.05, 0.05), (0.01, 0.04)])
def test_round_trip_within_half_a_quantum(qy, qz):
    row_x, ro, y, z, first, ids, x_ref, param = _frame_with_tracks(5)
    s = oracle.codec_encode(row_x, synth.BZ_TESLA, qy, qz, first, ids, x_ref, param, y, z, ro)
    yd, zd = oracle.codec_decode(row_x, qy, qz, s)
    esc = s["code"][:, 0] == oracle.CODEC_ESCAPE
    assert s["n_escaped"] == int(esc.sum()) >= 1
    ym, zm = y[ids], z[ids]
    assert np.array_equal(yd[esc], ym[esc]) and np.array_equal(zd[esc], zm[esc])
    ok = ~esc
    tol_y = 0.5 * qy * (1 + 1e-5) + 4 * np.spacing(np.abs(ym[ok]).astype(np.float32))
    tol_z = 0.5 * qz * (1 + 1e-5) + 4 * np.spacing(np.abs(zm[ok]).astype(np.float32))
    assert np.all(np.abs(yd[ok].astype(np.float64) - ym[ok]) <= tol_y)
    assert np.all(np.abs(zd[ok].astype(np.float64) - zm[ok]) <= tol_z)
    # rows of the track clusters and the unassigned clusters, in input order
    R = len(row_x)
    row_of = np.searchsorted(ro, np.arange(len(y)), side="right") - 1
    assert np.array_equal(s["row"], row_of[ids] % R)
    un = np.setdiff1d(np.arange(len(y)), ids)
    assert np.array_equal(s["un_row"], row_of[un] % R)
    assert np.array_equal(s["un_yz"][:, 0], y[un]) and np.array_equal(s["un_yz"][:, 1], z[un])
    # residual codes of model tracks are small: |k| <= 5 sigma / q for all but the escaped cluster
    assert np.abs(s["code"][ok][:, 0]).max() <= math.ceil(5 * 0.05 / qy) + 1
    assert np.abs(s["code"][ok][:, 1]).max() <= math.ceil(5 * 0.05 / qz) + 1
