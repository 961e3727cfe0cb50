"""Detector model and synthetic generator: closed-form checks (CPU)."""
import math

import numpy as np
import pytest

from paper_2502_09138_amd import synth


def test_row_geometry_closed_form():
    x, hy = synth.row_geometry()
    assert len(x) == 152
    pitch = np.array([0.75] * 63 + [1.0] * 64 + [1.5] * 25)
    assert pitch.sum() == 148.75
    # lower edge of row r = 85 + sum of earlier pitches; centre = edge + pitch/2
    assert x[0] == 85.375 and x[62] == 131.875 and x[63] == 132.75
    assert x[126] == 195.75 and x[127] == 197.0 and x[151] == 233.0
    assert x[151] + 0.75 == 233.75
    assert np.all(x.astype(np.float32).astype(np.float64) == x)      # exact in float32
    assert np.all((x * 8) == np.round(x * 8))                        # multiples of 1/8 cm
    assert np.allclose(hy, x * math.tan(math.radians(10.0)), rtol=0, atol=1e-12)


def _global_point(sector, X, yl):
    a = synth.sector_alpha(sector)
    return X * math.cos(a) - yl * math.sin(a), X * math.sin(a) + yl * math.cos(a)


def test_noiseless_clusters_lie_on_helix():
    ev = synth.single_sector(seed=5, n_tracks=50, smear=synth.NOISELESS)
    x, _ = synth.row_geometry()
    P = ev.particles
    rows = np.repeat(np.arange(152), np.diff(ev.row_offsets))
    assert np.all(ev.particle >= 0)
    worst_r, worst_z = 0.0, 0.0
    for i in range(ev.n_clusters):
        p = ev.particle[i]
        gx, gy = _global_point(0, x[rows[i]], ev.y_true[i])
        kap = synth.curvature(P["q"][p], P["pt"][p])
        cx = P["vx"][p] - math.sin(P["phi"][p]) / kap
        cy = P["vy"][p] + math.cos(P["phi"][p]) / kap
        # on the circle of radius 1/|kappa| around the centre
        worst_r = max(worst_r, abs(math.hypot(gx - cx, gy - cy) - 1.0 / abs(kap)))
        # z = tan(lambda) * arc length from the vertex; arc from the turning angle
        a0 = math.atan2(P["vy"][p] - cy, P["vx"][p] - cx)
        a1 = math.atan2(gy - cy, gx - cx)
        dphi = math.remainder(a1 - a0, 2 * math.pi)
        s = abs(dphi / kap)
        worst_z = max(worst_z, abs(ev.z_true[i] - P["tanl"][p] * s))
    assert worst_r < 1e-9 and worst_z < 1e-9


def test_generator_deterministic_and_sized():
    a = synth.single_sector(seed=1)
    b = synth.single_sector(seed=1)
    c = synth.single_sector(seed=2)
    assert np.array_equal(a.y, b.y) and np.array_equal(a.row_offsets, b.row_offsets)
    assert not np.array_equal(a.y, c.y[: len(a.y)]) if len(c.y) >= len(a.y) else True
    assert 18_000 < a.n_clusters < 32_000
    assert a.row_offsets[0] == 0 and np.all(np.diff(a.row_offsets.astype(np.int64)) >= 0)
    hy = synth.row_geometry()[1]
    rows = np.repeat(np.arange(152), np.diff(a.row_offsets))
    assert np.all(np.abs(a.y) <= hy[rows].astype(np.float32) + 1e-4)
    noise = (a.particle < 0).mean()
    assert 0.03 < noise < 0.06


def test_time_frame_drift_coordinate_small():
    ev = synth.time_frame(seed=7, n_orbits=1)
    hi = synth.DRIFT_VELOCITY * synth.ORBIT_US + 250.0
    assert np.allclose(ev.sector_z_hi, hi) and np.all(ev.sector_z_lo == 0)
    sig = ev.particle >= 0
    assert np.all(ev.z_true[sig] >= 0) and np.all(ev.z_true[sig] <= hi + 1e-6)


def test_uneven_chunks_targets():
    ev = synth.uneven_chunks(chunks=[0, 1, 2, 3])
    counts = np.diff(ev.row_offsets[::152].astype(np.int64))
    t = ev.particles["target"]
    assert np.all(np.abs(counts - t) <= 0.1 * t + 200)
    assert np.all((t >= 1000) & (t <= 200000))
