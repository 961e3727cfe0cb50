"""Pins for the oracle's tracker steps C1-C7 (CPU).

* C1 grid: stable order by (bin, input id) equals numpy's stable argsort;
  bins respect their geometric edges; dims follow hand-worked values.
* C2 neighbours: grid-accelerated search equals all-pairs brute force
  (no grid) on tiny random sectors, including exact ties and window edges.
* C3/C4: mutual-link invariants; starts = chains of >= 3 hits found by an
  independent walk.
* C5: noiseless helices are recovered to 1e-9; pulls are standard normal;
  every covariance is positive definite.
* C6/C7: each cluster in at most one track; a lone track is found whole.
* A hand-worked 5-row event (tests/golden) pins C2-C7 end to end.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle
from paper_2502_09138_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cfg_rows(cfg, row_x, row_half_y, **kw):
    c = dict(cfg)
    c["row_x"] = np.asarray(row_x, np.float64)
    c["row_half_y"] = np.asarray(row_half_y, np.float64)
    c.update(kw)
    return c


# ---------------------------------------------------------------------- C1
def test_grid_dims_golden():
    g = json.load(open(os.path.join(GOLDEN, "grid_dims.json")))
    for c in g["cases"]:
        assert oracle.grid_dims(c["n"], c["K"], c["Ly"], c["Lz"]) == (c["nY"], c["nZ"]), c


def test_grid_dims_identities():
    for n in list(range(0, 300)) + [1000, 5000, 65535]:
        for ly, lz in [(340, 2500), (900, 2500), (565, 75920), (100, 10)]:
            ny, nz = oracle.grid_dims(n, 2, ly, lz)
            B = max(1, n // 2)
            assert 1 <= ny <= B and nz >= 1 and ny * nz <= B
            assert nz == max(1, B // ny)


def test_grid_order_is_stable_sort_and_bins_respect_edges(cfg):
    ev = synth.single_sector(seed=3)
    run = oracle.Run.from_event(cfg, ev).grid()
    res = run.result()
    x, hy = synth.row_geometry()
    offs = ev.row_offsets.astype(np.int64)
    lz = math.ceil(10.0 * (float(ev.sector_z_hi[0]) - float(ev.sector_z_lo[0])))
    for r in range(152):
        a, b = offs[r], offs[r + 1]
        ny, nz = int(res["row_dims"][r] & 0xFFFF), int(res["row_dims"][r] >> 16)
        assert (ny, nz) == oracle.grid_dims(b - a, 2, math.ceil(20 * hy[r]), lz)
        y, z = ev.y[a:b], ev.z[a:b]
        iy = np.array([oracle.bin_of(float(y[j]), float(z[j]), np.float32(-hy[r]), np.float32(1 / (2 * hy[r])),
                                     float(ev.sector_z_lo[0]), np.float32(1 / 250.0), ny, nz) for j in range(b - a)])
        key = iy[:, 1] * ny + iy[:, 0]
        order = np.argsort(key, kind="stable")
        assert np.array_equal(res["sorted_id"][a:b], a + order)
        # geometric edges (float tolerance)
        wy, wz = 2 * hy[r] / ny, 250.0 / nz
        lo_y = -hy[r] + iy[:, 0] * wy
        inner = (iy[:, 0] > 0) & (iy[:, 0] < ny - 1)
        assert np.all(y[inner] >= lo_y[inner] - 1e-4) and np.all(y[inner] <= lo_y[inner] + wy + 1e-4)
        lo_z = iy[:, 1] * wz
        innz = (iy[:, 1] > 0) & (iy[:, 1] < nz - 1)
        assert np.all(z[innz] >= lo_z[innz] - 1e-3) and np.all(z[innz] <= lo_z[innz] + wz + 1e-3)
        # bin starts = cumulative histogram
        base = a + 2 * r
        hist = np.bincount(key, minlength=ny * nz)
        assert np.array_equal(res["bin_start"][base:base + ny * nz + 1], a + np.concatenate([[0], np.cumsum(hist)]))


# ---------------------------------------------------------------------- C2
def _brute_links(cfg, row_x, offs, y, z, sorted_id):
    """All-pairs search without a grid; float32 arithmetic as the definition states."""
    f = np.float32
    R = len(row_x)
    pos_of = np.empty(len(sorted_id), np.int64)
    pos_of[sorted_id] = np.arange(len(sorted_id))
    rho = f((cfg["sigma_y"] / cfg["sigma_z"]) ** 2)
    up0 = -np.ones(len(y), np.int64)
    dn0 = -np.ones(len(y), np.int64)
    for r in range(1, R - 1):
        du, dd = row_x[r + 1] - row_x[r], row_x[r] - row_x[r - 1]
        t = dd / (dd + du)
        tf = f(t)
        wyu, wzu = f(cfg["win_a_y"] * du + cfg["win_b_y"]), f(cfg["win_a_z"] * du + cfg["win_b_z"])
        wyd, wzd = f(cfg["win_a_y"] * dd + cfg["win_b_y"]), f(cfg["win_a_z"] * dd + cfg["win_b_z"])
        n2, s2 = cfg["link_nsigma"] ** 2, cfg["sigma_y"] ** 2
        dmax = f((n2 * s2) * ((1.0 + t * t) + (1.0 - t) * (1.0 - t)))
        for h in range(offs[r], offs[r + 1]):
            yh, zh = f(y[h]), f(z[h])
            U = [u for u in range(offs[r + 1], offs[r + 2]) if abs(f(y[u]) - yh) <= wyu and abs(f(z[u]) - zh) <= wzu]
            D = [d for d in range(offs[r - 1], offs[r]) if abs(f(y[d]) - yh) <= wyd and abs(f(z[d]) - zh) <= wzd]
            best = None
            for d in D:
                for u in U:
                    yp = f(y[d]) + f(tf * f(f(y[u]) - f(y[d])))
                    zp = f(z[d]) + f(tf * f(f(z[u]) - f(z[d])))
                    ey, ez = f(yh - yp), f(zh - zp)
                    dev = f(f(ey * ey) + f(rho * f(ez * ez)))
                    if dev <= dmax:
                        cand = (float(dev), pos_of[u], pos_of[d])
                        best = cand if best is None or cand < best else best
            if best is not None:
                up0[pos_of[h]], dn0[pos_of[h]] = best[1], best[2]
    return up0, dn0


@pytest.mark.parametrize("seed", range(12))
def test_links_equal_brute_force_tiny(cfg, seed):
    rng = np.random.default_rng(100 + seed)
    R = 8
    row_x = synth.row_geometry()[0][60:60 + R]          # spans the 0.75 -> 1.0 cm pitch change
    hy = np.full(R, 6.0)
    counts = rng.integers(0, 40, R)
    counts[rng.integers(0, R)] = 0                        # an empty row
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.uint32)
    N = int(offs[-1])
    y = rng.uniform(-3, 3, N).astype(np.float32)
    z = rng.uniform(0, 6, N).astype(np.float32)
    # exact duplicates (ties) and points exactly on a window edge
    for k in range(min(6, N // 4)):
        i, j = rng.integers(0, N, 2)
        y[j], z[j] = y[i], z[i]
    c = _cfg_rows(cfg, row_x, hy)
    run = oracle.Run(c, offs, y, z, np.float32([0.0]), np.float32([6.0])).grid().links()
    res = run.result()
    up0, dn0 = _brute_links(c, row_x, offs.astype(np.int64), y, z, res["sorted_id"].astype(np.int64))
    assert np.array_equal(res["up0"], up0) and np.array_equal(res["down0"], dn0)


def test_links_window_edge_inclusive(cfg):
    # du = dd = 1: W_y = 2.5 exactly; u sits exactly 2.5 cm away and must be a candidate
    row_x = np.array([100.0, 101.0, 102.0])
    c = _cfg_rows(cfg, row_x, [20.0] * 3, link_nsigma=1e3)
    y = np.float32([-2.5, 0.0, 2.5])
    z = np.float32([10.0, 10.0, 10.0])
    offs = np.uint32([0, 1, 2, 3])
    res = oracle.Run(c, offs, y, z, np.float32([0.0]), np.float32([250.0])).grid().links().result()
    assert res["up0"][1] == 2 and res["down0"][1] == 0
    y2 = np.float32([-2.5, 0.0, np.nextafter(np.float32(2.5), np.float32(9))])
    res = oracle.Run(c, offs, y2, z, np.float32([0.0]), np.float32([250.0])).grid().links().result()
    assert res["up0"][1] == -1


def test_link_deviation_slope_form(cfg):
    # equal pitches: Delta = dx^2/4 * [(y_u-y_h)/dx - (y_h-y_d)/dx]^2 for z on a line
    row_x = np.array([100.0, 101.0, 102.0])
    c = _cfg_rows(cfg, row_x, [20.0] * 3, link_nsigma=1e3)
    for yd, yh, yu in [(0.0, 0.25, 0.0), (1.0, 1.5, 2.5), (-1.0, -0.5, 0.5)]:
        y = np.float32([yd, yh, yu])
        z = np.float32([10.0, 10.5, 11.0])
        res = oracle.Run(c, np.uint32([0, 1, 2, 3]), y, z, np.float32([0.0]), np.float32([250.0])).grid().links().result()
        assert res["up0"][1] == 2  # accepted with an effectively open cut
        slope_diff = (yu - yh) - (yh - yd)
        dev = 0.25 * slope_diff ** 2
        nsig_needed = math.sqrt(dev / (0.01 * 1.5)) if dev else 0.0
        c2 = _cfg_rows(cfg, row_x, [20.0] * 3, link_nsigma=nsig_needed * 0.999)
        res2 = oracle.Run(c2, np.uint32([0, 1, 2, 3]), y, z, np.float32([0.0]), np.float32([250.0])).grid().links().result()
        assert (res2["up0"][1] == -1) == (dev > 0)


# ---------------------------------------------------------------------- C3/C4
def test_clean_and_start_invariants(cfg):
    ev = synth.single_sector(seed=4)
    res = oracle.Run.from_event(cfg, ev).grid().links().starts().result()
    up1, dn1 = res["up1"], res["down1"]
    up0, dn0 = res["up0"], res["down0"]
    N = len(up1)
    for h in range(N):
        if up1[h] >= 0:
            assert dn1[up1[h]] == h and up0[h] == up1[h]
        if dn1[h] >= 0:
            assert up1[dn1[h]] == h and dn0[h] == dn1[h]
        if up0[h] >= 0 and dn0[up0[h]] == h:
            assert up1[h] == up0[h]
    # independent walk: paths in the mutual-link graph with >= 3 nodes
    seen = np.zeros(N, bool)
    bottoms = []
    for h in range(N):
        if dn1[h] == -1 and up1[h] >= 0:
            n, p = 0, h
            while p >= 0:
                assert not seen[p]
                seen[p] = True
                n += 1
                p = up1[p]
            if n >= 3:
                bottoms.append(h)
    assert np.array_equal(res["starts"], np.array(bottoms, np.uint32))


# ---------------------------------------------------------------------- C5
def _match_tracks(ev, res):
    first, cl = res["trk_first"], res["trk_clusters"]
    out = []
    for t in range(len(first) - 1):
        ids = cl[first[t]:first[t + 1]]
        p = ev.particle[ids]
        vals, cnt = np.unique(p, return_counts=True)
        j = cnt.argmax()
        out.append((int(vals[j]), cnt[j] / len(ids), len(ids)))
    return out


def test_noiseless_helices_recovered_to_1e9(cfg):
    ev = synth.single_sector(seed=17, n_tracks=12, smear=synth.NOISELESS, pt_range=(0.25, 5.0))
    run = oracle.Run.from_event(cfg, ev, fp64=(ev.y_true, ev.z_true)).run_all()
    res = run.result()
    x = synth.row_geometry()[0]
    matches = _match_tracks(ev, res)
    good = 0
    for t, (p, purity, n) in enumerate(matches):
        if p < 0 or purity < 1.0 or n != int((ev.particle == p).sum()):
            continue
        i = res["trk_tracklet"][t]
        ok, truth = synth.helix_state_at_row(ev.particles, p, synth.SECTOR_HALF_ANGLE, x[res["tk_xref_row"][i]])
        assert ok
        got = res["tk_param"][i]
        assert np.all(np.abs(got - truth) <= 1e-9 * np.maximum(1.0, np.abs(truth))), (got, truth)
        good += 1
    assert good >= 9, (good, matches)


def test_pulls_and_spd_on_smeared_sector(cfg):
    x = synth.row_geometry()[0]
    pulls, chi2ndf = [], []
    for seed in (1, 2, 3):
        ev = synth.single_sector(seed=seed)
        res = oracle.Run.from_event(cfg, ev).run_all().result()
        for t, (p, purity, n) in enumerate(_match_tracks(ev, res)):
            i = res["trk_tracklet"][t]
            M = oracle.unpack_cov(res["tk_cov"][i])
            np.linalg.cholesky(M)                      # SPD
            # parameters come from the tracklet fit: require every fitted hit from one particle
            fitted = res["tk_rowhit"][i]
            fitted = res["sorted_id"][fitted[fitted >= 0]]
            if p < 0 or n < 60 or np.any(ev.particle[fitted] != p):
                continue
            ok, truth = synth.helix_state_at_row(ev.particles, p, synth.SECTOR_HALF_ANGLE, x[res["tk_xref_row"][i]])
            pulls.append((res["tk_param"][i] - truth) / np.sqrt(np.diag(M)))
            chi2ndf.append(res["tk_chi2"][i] / (2 * res["tk_nhits"][i] - 5))
    pulls = np.array(pulls)
    assert len(pulls) > 400
    mu, sd = pulls.mean(axis=0), pulls.std(axis=0)
    assert np.all(np.abs(mu) < 0.1), mu
    assert np.all((sd > 0.92) & (sd < 1.08)), sd
    assert 0.9 < np.mean(chi2ndf) < 1.1


# ---------------------------------------------------------------------- C6/C7
def test_selector_invariants(cfg):
    ev = synth.single_sector(seed=6)
    res = oracle.Run.from_event(cfg, ev).run_all().result()
    cl = res["trk_clusters"]
    assert len(np.unique(cl)) == len(cl)               # each cluster in at most one track
    first = res["trk_first"]
    tk = res["trk_tracklet"]
    assert np.all(np.diff(tk.astype(np.int64)) > 0)     # canonical order
    assert np.all(res["starts"][tk][1:] > res["starts"][tk][:-1])
    rows = np.repeat(np.arange(152), np.diff(ev.row_offsets))
    for t in range(len(tk)):
        ids = cl[first[t]:first[t + 1]]
        assert len(ids) >= cfg["min_track_hits"]
        assert np.all(np.diff(rows[ids]) > 0)           # ascending rows, one per row
        assert 2 * len(ids) >= res["tk_nhits"][tk[t]]


def test_isolated_track_found_whole(cfg):
    ev = synth.single_sector(seed=23, n_tracks=1, smear=synth.NOISELESS, pt_range=(1.0, 2.0))
    res = oracle.Run.from_event(cfg, ev).run_all().result()
    assert len(res["trk_tracklet"]) == 1
    assert np.array_equal(np.sort(res["trk_clusters"]), np.arange(ev.n_clusters))


def test_golden_straight_line(cfg):
    g = json.load(open(os.path.join(GOLDEN, "straight_line_5rows.json")))
    c = _cfg_rows(cfg, g["row_x"], g["row_half_y"], **g["cuts"])
    hits = [h for row in g["hits_by_row"] for h in row]
    offs = np.concatenate([[0], np.cumsum([len(r) for r in g["hits_by_row"]])]).astype(np.uint32)
    y = np.array([h[0] for h in hits])
    z = np.array([h[1] for h in hits])
    run = oracle.Run(c, offs, y, z, np.float32([g["z_lo"]]), np.float32([g["z_hi"]])).run_all()
    res = run.result()
    sid = res["sorted_id"].astype(np.int64)
    pos_of = np.empty(len(sid), np.int64)
    pos_of[sid] = np.arange(len(sid))
    e = g["expect"]
    up_id = [int(sid[res["up0"][pos_of[i]]]) if res["up0"][pos_of[i]] >= 0 else -1 for i in range(len(hits))]
    dn_id = [int(sid[res["down0"][pos_of[i]]]) if res["down0"][pos_of[i]] >= 0 else -1 for i in range(len(hits))]
    assert up_id == e["up0_by_input_id"] and dn_id == e["down0_by_input_id"]
    assert len(res["starts"]) == e["n_starts"] and sid[res["starts"][0]] == e["start_input_id"]
    assert len(res["trk_tracklet"]) == e["n_tracks"]
    assert sorted(res["trk_clusters"].tolist()) == e["track_input_ids"]
    i = res["trk_tracklet"][0]
    assert g["row_x"][res["tk_xref_row"][i]] == e["x_ref"]
    assert np.allclose(res["tk_param"][i], e["param"], rtol=0, atol=1e-9)


# ---------------------------------------------------------------------- truth gates
def _efficiency(ev, res, per_sector=False):
    R = 152
    sec_of = np.repeat(np.arange(ev.n_sectors), np.diff(ev.row_offsets[::R].astype(np.int64)))
    part = ev.particle
    key_all = part.astype(np.int64) * 64 + sec_of
    u, c = np.unique(key_all[part >= 0], return_counts=True)
    findable = dict(zip(u.tolist(), c.tolist()))
    matched, fakes = set(), 0
    m = _match_tracks(ev, res)
    first, cl = res["trk_first"], res["trk_clusters"]
    for t, (p, purity, n) in enumerate(m):
        if p >= 0 and purity >= 0.9:
            matched.add(p * 64 + int(sec_of[cl[first[t]]]))
        else:
            fakes += 1
    return findable, matched, fakes / max(1, len(m))


def test_truth_gates_single_sector(cfg):
    ev = synth.single_sector(seed=1)
    res = oracle.Run.from_event(cfg, ev).run_all().result()
    findable, matched, fake = _efficiency(ev, res)
    pt = ev.particles["pt"]
    sel = [k for k, n in findable.items() if n >= 30 and pt[k // 64] > 0.3]
    eff = np.mean([k in matched for k in sel])
    assert eff >= 0.95 and fake <= 0.02, (eff, fake)


@pytest.mark.slow
def test_truth_gates_central_event(cfg):
    ev = synth.central_event(seed=2)
    sub = ev.sector_slice([0, 7, 20, 33])
    sub.particles = ev.particles
    res = oracle.Run.from_event(cfg, sub).run_all().result()
    findable, matched, fake = _efficiency(sub, res)
    sel = [k for k, n in findable.items() if n >= 30]
    eff = np.mean([k in matched for k in sel])
    assert eff >= 0.90 and fake <= 0.05, (eff, fake)
