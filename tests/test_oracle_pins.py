"""Hand-worked pins of the oracle's discrete rules (CPU).

Each golden under tests/golden/ states a small event, the rule it exercises
and the outcome worked out by hand; a one-token change of the rule in the
oracle (a comparison flipped, a bound dropped, a key reversed) changes the
outcome of at least one case.

* c1_bins.json: the float32 bin rule of C1 -- clamps at both ends, NaN/inf,
  integer u, rounding of a and b in float32.
* c5_stop_rules.json: C5 miss counter outward and below the start row,
  search window min(g*sqrt(C_yy + sigma_y^2), cap) with the cap and the gate
  binding, edge-margin stops outward and inward below the start row.
* c6_selector.json: C6 ownership key order (nHits, then smaller start) and
  the owned-fraction boundary; C7 output order.
* C2 in float32 (as defined) against C2 evaluated in double: on the
  single-sector and central-event workloads every hit whose links differ is
  a near-tie, i.e. the two deciding quantities differ by less than the
  float32 evaluation error bound of the quantities involved.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle
from paper_2502_09138_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------------- C1 bins
def test_bin_rule_golden():
    f = np.float32
    for c in _load("c1_bins.json")["cases"]:
        v, lo, iw, n = float(c["v"]), float(c["lo"]), float(c["inv_w"]), int(c["n"])
        got, _ = oracle.bin_of(v, 0.0, lo, iw, 0.0, 1.0, n, 1)
        assert got == c["bin"], c
        # the same from a float32 evaluation written out in numpy (one rounding per operation)
        with np.errstate(all="ignore"):
            u = f(f(f(v) - f(lo)) * f(f(n) * f(iw)))
        u = f(0) if not (u >= 0) else u
        u = f(n - 1) if u > f(n - 1) else u
        assert int(u) == c["bin"], c


# ---------------------------------------------------------------------- C5 stop and search rules
R40 = 40


def _c5_config(cfg, cuts):
    c = dict(cfg)
    c["row_x"] = 100.0 + np.arange(R40, dtype=np.float64)
    c["row_half_y"] = np.full(R40, 20.0)
    c.update(bz=0.0, min_tracklet_hits=8, min_track_hits=8)
    c.update(cuts or {})
    return c


def _gate_width(rows_fitted, x_pred, slope, sigma_y, c0_sinphi, gate):
    """g*sqrt(C_yy + sigma_y^2) at x_pred after fitting a straight line to hits at
    x = rows_fitted (sigma_y each) with prior variance c0_sinphi on sin(phi): the
    batch least-squares covariance of (y at x_pred, sin phi)."""
    s = slope / math.sqrt(1.0 + slope * slope)
    c3 = (1.0 - s * s) ** 1.5
    J = np.array([[1.0, (x - x_pred) / c3] for x in rows_fitted])
    info = J.T @ J / sigma_y ** 2 + np.diag([0.0, 1.0 / c0_sinphi])
    cyy = np.linalg.inv(info)[0, 0]
    return gate * math.sqrt(cyy + sigma_y ** 2)


def _c5_event(case, cfg):
    ln = case["line"]
    hits = {r: [(ln["y0"] + ln["slope"] * r, ln["z"])] for r in case["rows"]}
    for row, dy, dz in case.get("extra", []):
        hits.setdefault(row, []).append((ln["y0"] + ln["slope"] * row + dy, ln["z"] + dz))
    if "extra_gate" in case:
        eg = case["extra_gate"]
        row = eg["row"]
        fitted = [100.0 + r for r in case["rows"] if 1 <= r < row]   # the chain: rows 1..row-1
        w = _gate_width(fitted, 100.0 + row, ln["slope"], cfg["sigma_y"], cfg["c0_sinphi"], cfg["gate_nsigma"])
        assert w < cfg["win_cap"]
        hits.setdefault(row, []).append((ln["y0"] + ln["slope"] * row + eg["frac"] * w, ln["z"]))
    counts = [len(hits.get(r, [])) for r in range(R40)]
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.uint32)
    y = np.array([h[0] for r in range(R40) for h in hits.get(r, [])], np.float64)
    z = np.array([h[1] for r in range(R40) for h in hits.get(r, [])], np.float64)
    return offs, y, z


@pytest.mark.parametrize("case", _load("c5_stop_rules.json")["cases"], ids=lambda c: c["name"])
def test_c5_stop_rules_golden(cfg, case):
    c = _c5_config(cfg, case.get("cuts"))
    offs, y, z = _c5_event(case, c)
    res = oracle.Run(c, offs, y, z, np.float32([0.0]), np.float32([250.0])).run_all().result()
    e = case["expect"]
    row_of = np.repeat(np.arange(R40), np.diff(offs.astype(np.int64)))
    assert len(res["starts"]) == e["n_starts"]
    assert row_of[res["sorted_id"][res["starts"][0]]] == e["start_row"]
    assert res["tk_nhits"][0] == e["nhits"]
    hit_rows = np.nonzero(res["tk_rowhit"][0] >= 0)[0]
    assert hit_rows.tolist() == e["hit_rows"]
    # one hit per row and it is the hit on the line (the extra hit where it was taken)
    for r in hit_rows:
        assert row_of[res["sorted_id"][res["tk_rowhit"][0][r]]] == r
    assert c["row_x"][res["tk_xref_row"][0]] == e["x_ref"]
    assert len(res["trk_tracklet"]) == e["n_tracks"]
    assert sorted(row_of[res["trk_clusters"]].tolist()) == e["hit_rows"]


# ---------------------------------------------------------------------- C6 selector
def test_c6_selector_golden(cfg):
    g = _load("c6_selector.json")
    R = g["n_rows"]
    c = dict(cfg)
    c["row_x"] = 100.0 + np.arange(R, dtype=np.float64)
    c["row_half_y"] = np.full(R, 20.0)
    c.update(min_tracklet_hits=4, min_track_hits=4, min_owned_frac=0.5)
    T = len(g["tracklets"])
    rowhit = np.full((T, R), -1, np.int32)
    for i, t in enumerate(g["tracklets"]):
        for row, cid in t["hits"]:
            assert cid // 3 == row
            rowhit[i, row] = cid
    nhits = [len(t["hits"]) for t in g["tracklets"]]
    starts = [t["start"] for t in g["tracklets"]]
    res = oracle.Run.from_tracklets(c, g["n_clusters"], nhits, starts, rowhit).select().result()
    exp = g["expect"]["tracks"]
    assert res["trk_tracklet"].tolist() == [e["tracklet"] for e in exp]
    for k, e in enumerate(exp):
        assert res["trk_clusters"][res["trk_first"][k]:res["trk_first"][k + 1]].tolist() == e["ids"], e


# ---------------------------------------------------------------------- C2 float32 vs FP64
EPS32 = 2.0 ** -24


def _c2_quantities(cfg, row_x, r, yh, zh, yd, zd, yu, zu):
    """FP64 deviation of a pair and a bound on its float32 evaluation error."""
    du, dd = row_x[r + 1] - row_x[r], row_x[r] - row_x[r - 1]
    t = dd / (dd + du)
    rho = (cfg["sigma_y"] / cfg["sigma_z"]) ** 2
    ey = yh - (yd + t * (yu - yd))
    ez = zh - (zd + t * (zu - zd))
    dev = ey * ey + rho * ez * ez
    Y = max(abs(yh), abs(yd), abs(yu))
    Z = max(abs(zh), abs(zd), abs(zu))
    # yp, zp: two roundings of magnitude <= Y (Z) plus the rounding of t; ey, ez: one more;
    # dev: squares, product with rho and the sum (relative 4 eps)
    e_ey = 6 * EPS32 * Y
    e_ez = 6 * EPS32 * Z
    err = 2 * abs(ey) * e_ey + e_ey ** 2 + rho * (2 * abs(ez) * e_ez + e_ez ** 2) + 4 * EPS32 * dev
    return dev, err


def _c2_near_tie(cfg, row_x, r, h, pair_a, pair_b, sy, sz):
    """True if the C2 decisions for hit h (coordinates sy/sz, FP64) under pairs
    pair_a (float32 result) and pair_b (FP64 result) differ only within the float32
    evaluation error: deviation vs deviation, deviation vs cut, or a window edge."""
    du, dd = row_x[r + 1] - row_x[r], row_x[r] - row_x[r - 1]
    t = dd / (dd + du)
    dmax = (cfg["link_nsigma"] ** 2 * cfg["sigma_y"] ** 2) * ((1 + t * t) + (1 - t) ** 2)
    yh, zh = sy[h], sz[h]
    devs = []
    for u, d in (pair_a, pair_b):
        if u < 0:
            devs.append(None)
            continue
        devs.append(_c2_quantities(cfg, row_x, r, yh, zh, sy[d], sz[d], sy[u], sz[u]))
    if devs[0] and devs[1] and abs(devs[0][0] - devs[1][0]) <= devs[0][1] + devs[1][1]:
        return "dev-dev"
    for dv in devs:
        if dv and abs(dv[0] - dmax) <= dv[1] + 2 * EPS32 * dmax:
            return "dev-cut"
    for (u, d) in (pair_a, pair_b):
        if u < 0:
            continue
        for q, dist in ((u, du), (d, dd)):
            wy, wz = cfg["win_a_y"] * dist + cfg["win_b_y"], cfg["win_a_z"] * dist + cfg["win_b_z"]
            if abs(abs(sy[q] - yh) - wy) <= 4 * EPS32 * (abs(sy[q]) + abs(yh) + wy) or \
               abs(abs(sz[q] - zh) - wz) <= 4 * EPS32 * (abs(sz[q]) + abs(zh) + wz):
                return "window"
    return None


def _c2_diffs(cfg, offs, y, z, lo, hi, R):
    a = oracle.Run(cfg, offs, y, z, lo, hi).grid().links().result()
    b = oracle.Run(cfg, offs, y, z, lo, hi).grid().links(fp64=True).result()
    sid = a["sorted_id"].astype(np.int64)
    sy, sz = np.asarray(y, np.float64)[sid], np.asarray(z, np.float64)[sid]
    row_of = np.repeat(np.arange(len(offs) - 1) % R, np.diff(offs.astype(np.int64)))
    diff = np.nonzero((a["up0"] != b["up0"]) | (a["down0"] != b["down0"]))[0]
    out = []
    for h in diff:
        kind = _c2_near_tie(cfg, np.asarray(cfg["row_x"]), int(row_of[h]), int(h),
                            (int(a["up0"][h]), int(a["down0"][h])), (int(b["up0"][h]), int(b["down0"][h])), sy, sz)
        out.append((int(h), kind))
    return out


def test_c2_near_tie_classifier_on_a_constructed_tie(cfg):
    """Two up-candidates whose FP64 deviations differ by 1e-26 but coincide after
    rounding to float32: float32 takes the smaller position, FP64 the smaller
    deviation; the classifier calls it a near-tie.  A clear difference is not one."""
    row_x = np.array([100.0, 101.0, 102.0])
    c = dict(cfg, row_x=row_x, row_half_y=np.full(3, 20.0))
    y = np.array([0.0, 0.0, -(1e-4 + 1e-13), 1e-4])     # d, h, u_a (first in its bin), u_b
    z = np.array([10.0, 10.0, 10.0, 10.0])
    offs = np.uint32([0, 1, 2, 4])
    diffs = _c2_diffs(c, offs, y, z, np.float32([0.0]), np.float32([250.0]), 3)
    assert len(diffs) == 1 and diffs[0][1] == "dev-dev", diffs
    sy = y
    sz = z
    assert _c2_near_tie(c, row_x, 1, 1, (2, 0), (3, 0), sy, sz) == "dev-dev"
    sy2 = np.array([0.0, 0.0, -0.3, 0.1])
    assert _c2_near_tie(c, row_x, 1, 1, (2, 0), (3, 0), sy2, sz) is None


@pytest.mark.parametrize("workload", ["single_sector", "central_event"])
def test_c2_float32_and_fp64_differ_only_at_near_ties(cfg, workload):
    ev = synth.single_sector(seed=1) if workload == "single_sector" else synth.central_event(seed=2)
    diffs = _c2_diffs(cfg, ev.row_offsets, ev.y, ev.z, ev.sector_z_lo, ev.sector_z_hi, synth.N_ROWS)
    print(workload, "hits whose links differ between float32 and FP64 C2:", len(diffs), diffs[:10])
    assert all(kind is not None for _, kind in diffs), diffs
    assert len(diffs) <= 1e-4 * ev.n_clusters


def test_c2_cut_is_inclusive(cfg):
    """A pair whose float32 deviation equals Delta_max exactly is kept (dev <= cut).
    Equal pitches give t = 0.5; with d and u at y = 0 the deviation is y_h^2, and
    y_h = 0.48989794f squares to exactly float(0.24) = Delta_max (n = 4,
    sigma_y = 0.1: 16 * 0.01 * (1 + 0.25 + 0.25))."""
    row_x = np.array([100.0, 101.0, 102.0])
    c = dict(cfg, row_x=row_x, row_half_y=np.full(3, 20.0))
    yh = np.float32(0.48989794)
    assert np.float32(yh * yh) == np.float32(0.24)
    y = np.array([0.0, float(yh), 0.0])
    z = np.array([10.0, 10.0, 10.0])
    res = oracle.Run(c, np.uint32([0, 1, 2, 3]), y, z, np.float32([0.0]), np.float32([250.0])).grid().links().result()
    assert res["up0"][1] == 2 and res["down0"][1] == 0
    y2 = np.array([0.0, float(np.nextafter(yh, np.float32(1))), 0.0])
    res = oracle.Run(c, np.uint32([0, 1, 2, 3]), y2, z, np.float32([0.0]), np.float32([250.0])).grid().links().result()
    assert res["up0"][1] == -1
