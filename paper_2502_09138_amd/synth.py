"""Seeded synthetic TPC events: geometry, helices, clusters and truth.

This module is the single source of inputs for both the HIP path and the
FP64 oracle.  It simulates the detector (charged particles on helices in a
solenoidal field, crossing the pad-row planes of 20-degree sectors) and holds
none of the tracking method's arithmetic: it never propagates a track state,
fits, links or selects anything.  Crossings are solved in the global frame
from the particle's circle, which keeps the generator independent of the
local-frame propagation the tracker uses, so it can serve as a closed-form
check of that propagation.

Workloads (the shapes of the paper's 50 kHz Pb-Pb and 650 kHz pp data, which
are not available, replaced by synthetic stand-ins; paper section 1 and
Tables 1-3 for the data-taking context):

* ``single_sector``   one 20-degree sector, 200 primaries, pT log-uniform
                      0.2-5 GeV (about 22k clusters);
* ``central_event``   one central heavy-ion-like event in all 36 sectors,
                      8000 primaries + 800 secondaries (about 1.25M);
* ``time_frame``      a 32-orbit continuous-readout time frame at 50 kHz with
                      the drift coordinate as the sector z (about 10M);
* ``uneven_chunks``   independent sector-sized chunks with log-uniform
                      occupancy between 1k and 200k clusters.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# ---------------------------------------------------------------------------
# Geometry and physics constants
# ---------------------------------------------------------------------------
N_ROWS = 152
N_SECTORS_PER_SIDE = 18
N_SECTORS = 36
SECTOR_HALF_ANGLE = math.pi / 18.0          # 10 degrees
C_LIGHT_B = 0.00299792458                   # GeV / (T cm): pT = c_B * B * R
BZ_TESLA = 0.5
SIGMA_Y = 0.1                               # cm
SIGMA_Z = 0.15                              # cm
TPC_HALF_LENGTH = 250.0                     # cm
DRIFT_VELOCITY = 2.58                       # cm / us
ORBIT_US = 88.924                           # LHC orbit, us


def row_geometry():
    """Pad-row centres X_r and sector half-widths Y_r (cm), float64 [152].

    63 rows of 0.75 cm pitch, 64 of 1.0 cm and 25 of 1.5 cm, starting at
    85 cm; the centre of row r is its lower edge plus half its pitch.  All
    centres are multiples of 1/8 cm, so they are exact in float32.
    """
    pitch = np.array([0.75] * 63 + [1.0] * 64 + [1.5] * 25, dtype=np.float64)
    edges = 85.0 + np.concatenate([[0.0], np.cumsum(pitch)])
    row_x = edges[:-1] + 0.5 * pitch
    row_half_y = row_x * math.tan(SECTOR_HALF_ANGLE)
    return row_x, row_half_y


def sector_alpha(sector):
    """Azimuth of the centre line of sector s (radians); A side s < 18."""
    return (np.asarray(sector) % N_SECTORS_PER_SIDE) * (2.0 * SECTOR_HALF_ANGLE) + SECTOR_HALF_ANGLE


# ---------------------------------------------------------------------------
# Event container
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Event:
    """Clusters laid out sector-major, row-major; truth alongside.

    ``row_offsets[s*R + r]`` .. ``row_offsets[s*R + r + 1]`` is the index range
    of the clusters of sector s, row r; the index of a cluster in these arrays
    is its input id.
    """
    n_sectors: int
    row_offsets: np.ndarray      # uint32 [S*R+1]
    y: np.ndarray                # float32 [N], sector-local cm
    z: np.ndarray                # float32 [N], cm (drift coordinate for time frames)
    charge: np.ndarray           # uint16 [N]
    sector_z_lo: np.ndarray      # float32 [S]
    sector_z_hi: np.ndarray      # float32 [S]
    particle: np.ndarray         # int32 [N], -1 for noise
    y_true: np.ndarray           # float64 [N], before smearing
    z_true: np.ndarray           # float64 [N]
    particles: dict              # per-particle arrays (pt, phi, tanl, q, vx, vy, vz, t_us)
    name: str = ""

    @property
    def n_clusters(self) -> int:
        return int(self.row_offsets[-1])

    def sector_slice(self, sectors):
        """Sub-event made of the listed sectors (cluster order preserved)."""
        sectors = list(sectors)
        R = N_ROWS
        offs = [0]
        idx = []
        for s in sectors:
            a, b = int(self.row_offsets[s * R]), int(self.row_offsets[(s + 1) * R])
            idx.append(np.arange(a, b))
            base = offs[-1] - a
            offs.extend((self.row_offsets[s * R + 1:(s + 1) * R + 1].astype(np.int64) + base).tolist())
        idx = np.concatenate(idx) if idx else np.zeros(0, np.int64)
        return Event(
            n_sectors=len(sectors),
            row_offsets=np.asarray(offs, dtype=np.uint32),
            y=self.y[idx].copy(), z=self.z[idx].copy(), charge=self.charge[idx].copy(),
            sector_z_lo=self.sector_z_lo[sectors].copy(), sector_z_hi=self.sector_z_hi[sectors].copy(),
            particle=self.particle[idx].copy(), y_true=self.y_true[idx].copy(), z_true=self.z_true[idx].copy(),
            particles=self.particles, name=f"{self.name}[sectors {sectors[:4]}{'...' if len(sectors) > 4 else ''}]")


# ---------------------------------------------------------------------------
# Landau charge table (charge is carried, never read by the tracker)
# ---------------------------------------------------------------------------
_LANDAU_TABLE = None


def _landau_ppf_table():
    global _LANDAU_TABLE
    if _LANDAU_TABLE is None:
        from scipy.stats import landau
        u = np.linspace(1e-4, 1.0 - 1e-3, 4097)
        _LANDAU_TABLE = (u, landau.ppf(u))
    return _LANDAU_TABLE


def landau_charge(rng, n):
    """uint16 charge = clamp(round(50 + 10 L)), L a standard Landau variate."""
    u_tab, l_tab = _landau_ppf_table()
    lam = np.interp(rng.random(n), u_tab, l_tab)
    return np.clip(np.rint(50.0 + 10.0 * lam), 0, 65535).astype(np.uint16)


# ---------------------------------------------------------------------------
# Helix / row-plane crossings (global circle, solved per sector)
# ---------------------------------------------------------------------------
def curvature(q, pt, bz=BZ_TESLA):
    """Signed curvature d(phi)/ds_T (1/cm); positive = counter-clockwise."""
    return -C_LIGHT_B * bz * np.asarray(q, dtype=np.float64) / np.asarray(pt, dtype=np.float64)


def crossings(vx, vy, vz, phi, tanl, kappa, alpha, X):
    """First outward crossing of the plane x_local = X within the first half-turn.

    All arguments broadcast.  Returns (ok, y_local, z, s_T, sin_phi_local).
    The particle starts at (vx, vy, vz) with transverse direction phi and moves
    on a circle of signed curvature kappa; x_local = x cos(a) + y sin(a).
    """
    ca, sa = np.cos(alpha), np.sin(alpha)
    xl0 = vx * ca + vy * sa
    yl0 = -vx * sa + vy * ca
    psi0 = phi - alpha                       # direction angle in the local frame
    v = np.sin(psi0) + kappa * (X - xl0)     # sin(psi) at the crossing
    ok = np.abs(v) < 1.0
    psi = np.arcsin(np.clip(v, -1.0, 1.0))   # outward crossing: cos(psi) > 0
    d = psi - psi0
    two_pi = 2.0 * math.pi
    pos = kappa > 0
    dpos = np.mod(d, two_pi)
    dneg = -np.mod(-d, two_pi)
    dpsi = np.where(pos, dpos, dneg)
    ok &= np.abs(dpsi) <= math.pi
    with np.errstate(divide="ignore", invalid="ignore"):
        s = dpsi / kappa
        # y_l(s) - y_l(0) = (cos psi0 - cos psi)/kappa = 2 sin(mid) sin(dpsi/2)/kappa
        yl = yl0 + 2.0 * np.sin(0.5 * (psi + psi0)) * (np.sin(0.5 * dpsi) / kappa)
    z = vz + tanl * s
    ok &= s >= 0.0
    return ok, yl, z, s, np.sin(psi)


def _candidate_sectors(vx, vy, phi, kappa, n_side_sector=18, r_min=80.0, r_max=240.0):
    """Sector indices (0..17) that a particle's arc may enter, as (track, sector) pairs."""
    n = len(phi)
    ns = 48
    smax = np.minimum(math.pi / np.abs(kappa), 2.2 * r_max)
    frac = np.linspace(0.0, 1.0, ns)[None, :]
    s = smax[:, None] * frac
    ang = phi[:, None] + kappa[:, None] * s
    with np.errstate(divide="ignore", invalid="ignore"):
        x = vx[:, None] + (np.sin(ang) - np.sin(phi)[:, None]) / kappa[:, None]
        y = vy[:, None] - (np.cos(ang) - np.cos(phi)[:, None]) / kappa[:, None]
    r = np.hypot(x, y)
    inside = (r >= r_min - 10.0) & (r <= r_max + 10.0)
    sec = np.floor(np.mod(np.arctan2(y, x), 2.0 * math.pi) / (2.0 * SECTOR_HALF_ANGLE)).astype(np.int64) % n_side_sector
    mask = np.zeros((n, n_side_sector), dtype=bool)
    ti = np.repeat(np.arange(n), ns)[inside.ravel()]
    si = sec.ravel()[inside.ravel()]
    for d in (-1, 0, 1):
        mask[ti, (si + d) % n_side_sector] = True
    return np.nonzero(mask)


@dataclasses.dataclass
class Smearing:
    sigma_y: float = SIGMA_Y
    sigma_z: float = SIGMA_Z
    efficiency: float = 0.95
    noise_frac: float = 0.05


NOISELESS = Smearing(0.0, 0.0, 1.0, 0.0)


def _signal_clusters(rng, part, sector_ids, row_x, row_half_y, time_frame=None, bz=BZ_TESLA,
                     fixed_alpha=None):
    """Ideal crossings of all particles with the rows of the given sectors.

    Returns dict of arrays: sector (0..S-1 in the event's numbering), row,
    particle, y, z_phys, s.  ``sector_ids`` maps the event's sector index to a
    physical sector 0..35; with ``fixed_alpha`` every event sector uses that
    azimuth (independent chunks) and particles carry their chunk in
    ``part['chunk']``.
    """
    vx, vy, vz = part["vx"], part["vy"], part["vz"]
    phi, tanl, q, pt = part["phi"], part["tanl"], part["q"], part["pt"]
    kap = curvature(q, pt, bz)
    out = {k: [] for k in ("sector", "row", "particle", "y", "z", "s")}
    if fixed_alpha is not None:
        ti = np.arange(len(phi))
        evsec = part["chunk"].astype(np.int64)
        alpha = np.full(len(phi), fixed_alpha)
    else:
        ti, si = _candidate_sectors(vx, vy, phi, kap)
        side = (tanl[ti] < 0).astype(np.int64)   # vz = 0: z sign follows tan(lambda)
        phys = si + 18 * side
        lut = -np.ones(N_SECTORS, dtype=np.int64)
        lut[np.asarray(sector_ids)] = np.arange(len(sector_ids))
        evsec = lut[phys]
        keep = evsec >= 0
        ti, evsec, phys = ti[keep], evsec[keep], phys[keep]
        alpha = sector_alpha(phys)
    X = row_x[None, :]
    ok, yl, z, s, _ = crossings(vx[ti, None], vy[ti, None], vz[ti, None], phi[ti, None], tanl[ti, None],
                                kap[ti, None], alpha[:, None], X)
    ok &= np.abs(yl) <= row_half_y[None, :] + 2.0     # coarse pre-cut; exact acceptance after smearing
    ok &= np.abs(z) < TPC_HALF_LENGTH
    if fixed_alpha is None:
        aside = evsec < 0  # placeholder to keep shapes
        side_ok = np.where((np.asarray(sector_ids)[evsec] < 18)[:, None], z >= 0.0, z < 0.0)
        ok &= side_ok
        del aside
    t_idx, r_idx = np.nonzero(ok)
    out["sector"] = evsec[t_idx]
    out["row"] = r_idx
    out["particle"] = ti[t_idx]
    out["y"] = yl[t_idx, r_idx]
    out["z"] = z[t_idx, r_idx]
    out["s"] = s[t_idx, r_idx]
    return out


def _assemble(rng, n_sectors, sig, smear, row_x, row_half_y, z_lo, z_hi, z_map=None, name=""):
    """Smear, apply efficiency/acceptance, add noise and lay out sector-major."""
    n = len(sig["row"])
    keep = rng.random(n) < smear.efficiency if smear.efficiency < 1.0 else np.ones(n, bool)
    y_true = sig["y"]
    z_true = sig["z"] if z_map is None else z_map(sig)
    y_meas = y_true + (rng.normal(0.0, smear.sigma_y, n) if smear.sigma_y > 0 else 0.0)
    z_meas = z_true + (rng.normal(0.0, smear.sigma_z, n) if smear.sigma_z > 0 else 0.0)
    keep &= np.abs(y_meas) <= row_half_y[sig["row"]]
    sec = sig["sector"][keep]
    row = sig["row"][keep]
    prt = sig["particle"][keep].astype(np.int32)
    y_t, z_t = y_true[keep], z_true[keep]
    y_m, z_m = y_meas[keep], z_meas[keep]
    # noise: round(frac * n_signal) per sector, uniform in row, y, z
    if smear.noise_frac > 0:
        nsig = np.bincount(sec, minlength=n_sectors)
        nnoise = np.rint(smear.noise_frac * nsig).astype(np.int64)
        nsec = np.repeat(np.arange(n_sectors), nnoise)
        nrow = rng.integers(0, N_ROWS, len(nsec))
        hw = row_half_y[nrow]
        ny = rng.uniform(-hw, hw)
        nz = rng.uniform(z_lo[nsec].astype(np.float64), z_hi[nsec].astype(np.float64))
        sec = np.concatenate([sec, nsec])
        row = np.concatenate([row, nrow])
        prt = np.concatenate([prt, -np.ones(len(nsec), np.int32)])
        y_t = np.concatenate([y_t, ny]); z_t = np.concatenate([z_t, nz])
        y_m = np.concatenate([y_m, ny]); z_m = np.concatenate([z_m, nz])
    key = sec.astype(np.int64) * N_ROWS + row
    order = np.lexsort((rng.random(len(key)), key))    # random order inside each (sector, row)
    key = key[order]
    counts = np.bincount(key, minlength=n_sectors * N_ROWS)
    row_offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.uint32)
    N = len(key)
    return Event(
        n_sectors=n_sectors, row_offsets=row_offsets,
        y=y_m[order].astype(np.float32), z=z_m[order].astype(np.float32),
        charge=landau_charge(rng, N),
        sector_z_lo=np.asarray(z_lo, np.float32), sector_z_hi=np.asarray(z_hi, np.float32),
        particle=prt[order], y_true=y_t[order], z_true=z_t[order], particles={}, name=name)


def _particles(rng, n, pt, eta_lo, eta_hi, phi=None, vertex_r=0.0, chunk=None, t_us=None):
    eta = rng.uniform(eta_lo, eta_hi, n)
    p = dict(pt=np.asarray(pt, np.float64), tanl=np.sinh(eta),
             phi=rng.uniform(0.0, 2 * math.pi, n) if phi is None else phi,
             q=np.where(rng.random(n) < 0.5, -1.0, 1.0))
    if vertex_r > 0:
        r = vertex_r * np.sqrt(rng.random(n))
        a = rng.uniform(0.0, 2 * math.pi, n)
        p["vx"], p["vy"] = r * np.cos(a), r * np.sin(a)
    else:
        p["vx"], p["vy"] = np.zeros(n), np.zeros(n)
    p["vz"] = np.zeros(n)
    if chunk is not None:
        p["chunk"] = chunk
    p["t_us"] = np.zeros(n) if t_us is None else t_us
    return p


def _concat(a, b):
    return {k: np.concatenate([a[k], b[k]]) for k in a}


def _physical_z_extent(sector_ids):
    s = np.asarray(sector_ids)
    lo = np.where(s < 18, 0.0, -TPC_HALF_LENGTH).astype(np.float32)
    hi = np.where(s < 18, TPC_HALF_LENGTH, 0.0).astype(np.float32)
    return lo, hi


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------
def single_sector(seed=1, n_tracks=200, smear=Smearing(), pt_range=(0.2, 5.0)):
    """One A-side sector (sector 0), primaries aimed at its centre line +-10 deg at r = 160 cm."""
    rng = np.random.default_rng(seed)
    row_x, row_half_y = row_geometry()
    pt = np.exp(rng.uniform(math.log(pt_range[0]), math.log(pt_range[1]), n_tracks))
    q = np.where(rng.random(n_tracks) < 0.5, -1.0, 1.0)
    kap = curvature(q, pt)
    theta = rng.uniform(0.0, 2.0 * SECTOR_HALF_ANGLE, n_tracks)
    phi = theta - np.arcsin(np.clip(kap * 160.0 / 2.0, -1, 1))
    part = _particles(rng, n_tracks, pt, 0.0, 0.9, phi=phi)
    part["q"] = q
    sig = _signal_clusters(rng, part, [0], row_x, row_half_y)
    lo, hi = _physical_z_extent([0])
    ev = _assemble(rng, 1, sig, smear, row_x, row_half_y, lo, hi, name=f"single_sector(seed={seed})")
    ev.particles = part
    return ev


def central_event(seed=2, n_primaries=8000, secondary_frac=0.1, smear=Smearing(), sectors=None):
    """All 36 sectors of one central event: pT = 0.1 + Exp(0.5) GeV, |eta| < 0.9."""
    rng = np.random.default_rng(seed)
    row_x, row_half_y = row_geometry()
    part = _particles(rng, n_primaries, 0.1 + rng.exponential(0.5, n_primaries), -0.9, 0.9)
    ns = int(round(secondary_frac * n_primaries))
    if ns:
        part = _concat(part, _particles(rng, ns, 0.1 + rng.exponential(0.5, ns), -0.9, 0.9, vertex_r=50.0))
    sector_ids = list(range(N_SECTORS)) if sectors is None else list(sectors)
    sig = _signal_clusters(rng, part, sector_ids, row_x, row_half_y)
    lo, hi = _physical_z_extent(sector_ids)
    ev = _assemble(rng, len(sector_ids), sig, smear, row_x, row_half_y, lo, hi, name=f"central_event(seed={seed})")
    ev.particles = part
    return ev


def time_frame(seed=3, n_orbits=32, rate_khz=50.0, mult_mean=500.0, mult_cap=8000, smear=Smearing(),
               tracks_per_collision=None):
    """Continuous-readout time frame; sector z is the drift coordinate.

    zeta = (250 - |z|) + v_drift * t_collision, so every sector's grid spans
    [0, v_drift * T_frame + 250] cm.  Clusters with |z| >= 250 cm are dropped.
    ``tracks_per_collision`` (callable rng -> int) overrides the exponential
    multiplicity (used for pp-like frames).
    """
    rng = np.random.default_rng(seed)
    row_x, row_half_y = row_geometry()
    t_frame = n_orbits * ORBIT_US
    n_coll = rng.poisson(rate_khz * 1e-3 * t_frame)
    t_c = rng.uniform(0.0, t_frame, n_coll)
    if tracks_per_collision is None:
        mult = np.minimum(mult_cap, np.maximum(1, np.rint(rng.exponential(mult_mean, n_coll)))).astype(np.int64)
    else:
        mult = np.asarray([tracks_per_collision(rng) for _ in range(n_coll)], np.int64)
    n = int(mult.sum())
    part = _particles(rng, n, 0.1 + rng.exponential(0.5, n), -0.9, 0.9, t_us=np.repeat(t_c, mult))
    sector_ids = list(range(N_SECTORS))
    sig = _signal_clusters(rng, part, sector_ids, row_x, row_half_y)
    t_of = part["t_us"]

    def zmap(sg):
        return (TPC_HALF_LENGTH - np.abs(sg["z"])) + DRIFT_VELOCITY * t_of[sg["particle"]]

    hi = np.full(N_SECTORS, DRIFT_VELOCITY * t_frame + TPC_HALF_LENGTH, np.float32)
    lo = np.zeros(N_SECTORS, np.float32)
    ev = _assemble(rng, N_SECTORS, sig, smear, row_x, row_half_y, lo, hi, z_map=zmap,
                   name=f"time_frame(seed={seed}, orbits={n_orbits}, collisions={n_coll})")
    ev.particles = part
    return ev


def uneven_chunks(n_chunks=512, seed0=1000, n_min=1000, n_max=200000, smear=Smearing(), chunks=None):
    """Independent sector-sized chunks (sector-0 frame, A side), log-uniform occupancy.

    Chunk i uses seed ``seed0 + i``; particles (pT = 0.1 + Exp(0.5) GeV,
    eta in (0, 0.9)) aimed into the sector are added until the expected
    cluster count reaches its target.  ``chunks`` selects a subset of chunk
    indices (each chunk's content does not depend on the others).
    """
    row_x, row_half_y = row_geometry()
    idx = list(range(n_chunks)) if chunks is None else list(chunks)
    parts, targets = [], []
    for k, i in enumerate(idx):
        rng = np.random.default_rng(seed0 + i)
        target = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        targets.append(target)
        got, batch = [], max(16, target // 120)
        total = 0
        while total < target / (1.0 + smear.noise_frac):
            pt = 0.1 + rng.exponential(0.5, batch)
            q = np.where(rng.random(batch) < 0.5, -1.0, 1.0)
            kap = curvature(q, pt)
            theta = rng.uniform(0.0, 2.0 * SECTOR_HALF_ANGLE, batch)
            phi = theta - np.arcsin(np.clip(kap * 160.0 / 2.0, -1, 1))
            p = _particles(rng, batch, pt, 0.0, 0.9, phi=phi, chunk=np.full(batch, k))
            p["q"] = q
            sg = _signal_clusters(rng, p, None, row_x, row_half_y, fixed_alpha=SECTOR_HALF_ANGLE)
            cnt = np.bincount(sg["particle"], minlength=batch)
            csum = np.cumsum(cnt) * smear.efficiency
            need = target / (1.0 + smear.noise_frac) - total
            m = int(np.searchsorted(csum, need) + 1)
            m = min(m, batch)
            got.append({kk: vv[:m] for kk, vv in p.items()})
            total += float(csum[m - 1])
        cp = got[0]
        for g in got[1:]:
            cp = _concat(cp, g)
        parts.append(cp)
    part = parts[0]
    for p in parts[1:]:
        part = _concat(part, p)
    rng = np.random.default_rng(seed0 + 10_000_000)
    sig = _signal_clusters(rng, part, None, row_x, row_half_y, fixed_alpha=SECTOR_HALF_ANGLE)
    lo, hi = _physical_z_extent([0] * len(idx))
    ev = _assemble(rng, len(idx), sig, smear, row_x, row_half_y, lo, hi,
                   name=f"uneven_chunks(n={len(idx)}, seed0={seed0})")
    ev.particles = part
    ev.particles["target"] = np.asarray(targets)
    return ev


def pp_time_frame(seed, n_orbits, rate_khz=650.0, mean_tracks=12.0, smear=Smearing()):
    """pp-like frame: 650 kHz pile-up, Poisson(12) tracks per collision."""
    return time_frame(seed=seed, n_orbits=n_orbits, rate_khz=rate_khz, smear=smear,
                      tracks_per_collision=lambda rng: int(rng.poisson(mean_tracks)))


def boundary_crossers(seed=7, n_tracks=60, smear=Smearing(), pt_range=(0.3, 2.0), sectors=(0, 1, 2)):
    """A-side sectors 0..2 with primaries aimed at the 20 degree edge between sectors 0 and 1
    (azimuth at r = 160 cm uniform in 20 +- 4 degrees), so that most leave track segments
    in two neighbouring sectors; the sector merger's workload."""
    rng = np.random.default_rng(seed)
    row_x, row_half_y = row_geometry()
    pt = np.exp(rng.uniform(math.log(pt_range[0]), math.log(pt_range[1]), n_tracks))
    q = np.where(rng.random(n_tracks) < 0.5, -1.0, 1.0)
    kap = curvature(q, pt)
    theta = np.deg2rad(rng.uniform(16.0, 24.0, n_tracks))
    phi = theta - np.arcsin(np.clip(kap * 160.0 / 2.0, -1, 1))
    part = _particles(rng, n_tracks, pt, 0.05, 0.9, phi=phi)
    part["q"] = q
    sig = _signal_clusters(rng, part, list(sectors), row_x, row_half_y)
    lo, hi = _physical_z_extent(list(sectors))
    ev = _assemble(rng, len(sectors), sig, smear, row_x, row_half_y, lo, hi, name=f"boundary_crossers(seed={seed})")
    ev.particles = part
    return ev


def helix_state_at_row(part, i, alpha, X, bz=BZ_TESLA):
    """True local track state (y, z, sin phi, tan lambda, q/pT) where particle i crosses x_local = X."""
    kap = curvature(part["q"][i], part["pt"][i], bz)
    ok, yl, z, s, sphi = crossings(part["vx"][i], part["vy"][i], part["vz"][i], part["phi"][i],
                                   part["tanl"][i], kap, alpha, X)
    return bool(ok), np.array([yl, z, sphi, part["tanl"][i], part["q"][i] / part["pt"][i]], np.float64)


WORKLOADS = {
    "single_sector": single_sector,
    "central_event": central_event,
    "time_frame": time_frame,
    "uneven_chunks": uneven_chunks,
}
