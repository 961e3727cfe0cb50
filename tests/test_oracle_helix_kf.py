"""Pins for the oracle's helix transport, Jacobian, seed and Kalman update (CPU).

Each check compares the oracle with something other than itself: the
generator's global-frame circle, finite differences, Monte Carlo, the scalar
textbook Kalman formula, batch weighted least squares, or a straight line.
"""
import math

import numpy as np
import pytest

from oracle import oracle
from paper_2502_09138_amd import synth

BZ = synth.BZ_TESLA


def _random_particles(rng, n, pt_lo=0.2, pt_hi=5.0):
    pt = np.exp(rng.uniform(math.log(pt_lo), math.log(pt_hi), n))
    q = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    kap = synth.curvature(q, pt)
    theta = rng.uniform(0, 2 * synth.SECTOR_HALF_ANGLE, n)
    phi = theta - np.arcsin(np.clip(kap * 80.0, -1, 1))
    return dict(pt=pt, q=q, phi=phi, tanl=np.sinh(rng.uniform(-0.9, 0.9, n)),
                vx=rng.uniform(-3, 3, n), vy=rng.uniform(-3, 3, n), vz=rng.uniform(-5, 5, n))


def test_propagation_matches_generator_circle():
    rng = np.random.default_rng(11)
    P = _random_particles(rng, 200)
    alpha = synth.SECTOR_HALF_ANGLE
    x = synth.row_geometry()[0]
    worst = np.zeros(5)
    n = 0
    for i in range(200):
        a, b = sorted(rng.choice(152, 2, replace=False))
        ok1, s1 = synth.helix_state_at_row(P, i, alpha, x[a])
        ok2, s2 = synth.helix_state_at_row(P, i, alpha, x[b])
        if not (ok1 and ok2) or abs(s1[2]) > 0.95 or abs(s2[2]) > 0.95:
            continue
        # the generator only reports the first crossing; skip arcs that turn back
        rc, q, _ = oracle.propagate(s1, x[a], x[b], BZ, s_max=0.999)
        assert rc == 0
        worst = np.maximum(worst, np.abs(q - s2))
        # and back down
        rc, q2, _ = oracle.propagate(s2, x[b], x[a], BZ, s_max=0.999)
        worst = np.maximum(worst, np.abs(q2 - s1))
        n += 1
    assert n > 150
    assert np.all(worst < 1e-9), worst


def test_propagation_composition_and_identity():
    rng = np.random.default_rng(3)
    for _ in range(100):
        p = np.array([rng.uniform(-20, 20), rng.uniform(-200, 200), rng.uniform(-0.8, 0.8),
                      rng.uniform(-1, 1), rng.uniform(-5, 5)])
        x1, x2, x3 = np.sort(rng.uniform(85, 234, 3))
        rc1, a, _ = oracle.propagate(p, x1, x2, BZ)
        rc2, b, _ = oracle.propagate(a, x2, x3, BZ)
        rc3, c, _ = oracle.propagate(p, x1, x3, BZ)
        if rc1 or rc2 or rc3:
            continue
        assert np.allclose(b, c, rtol=0, atol=1e-10)
        rc, same, F = oracle.propagate(p, x1, x1, BZ)
        assert rc == 0 and np.array_equal(same, p) and np.allclose(F, np.eye(5))


def test_straight_line_when_field_off():
    p = np.array([3.0, 10.0, 0.3, 0.5, 2.0])
    rc, q, F = oracle.propagate(p, 100.0, 110.0, 0.0)
    c = math.sqrt(1 - 0.3 ** 2)
    assert rc == 0
    assert abs(q[0] - (3.0 + 10.0 * 0.3 / c)) < 1e-12
    assert abs(q[1] - (10.0 + 0.5 * 10.0 / c)) < 1e-12
    assert q[2] == 0.3


def test_jacobian_matches_central_differences():
    rng = np.random.default_rng(5)
    for _ in range(60):
        p = np.array([rng.uniform(-20, 20), rng.uniform(-100, 100), rng.uniform(-0.7, 0.7),
                      rng.uniform(-1, 1), rng.uniform(-8, 8)])
        x1 = rng.uniform(85, 230)
        dx = rng.choice([-1.5, -1.0, -0.75, 0.75, 1.0, 1.5, 10.0, -12.0])
        rc, q, F = oracle.propagate(p, x1, x1 + dx, BZ)
        if rc:
            continue
        num = np.zeros((5, 5))
        for j in range(5):
            h = 1e-6 * max(1.0, abs(p[j]))
            pp, pm = p.copy(), p.copy()
            pp[j] += h
            pm[j] -= h
            _, qp, _ = oracle.propagate(pp, x1, x1 + dx, BZ)
            _, qm, _ = oracle.propagate(pm, x1, x1 + dx, BZ)
            num[:, j] = (qp - qm) / (2 * h)
        scale = np.maximum(1.0, np.abs(num))
        assert np.all(np.abs(F - num) / scale < 1e-6), (F, num)


def test_covariance_transport_matches_monte_carlo():
    rng = np.random.default_rng(9)
    p = np.array([2.0, 30.0, 0.2, 0.4, 1.5])
    A = rng.normal(size=(5, 5)) * np.array([1e-3, 1e-3, 1e-4, 1e-4, 1e-3])
    Cm = A @ A.T + np.diag([1e-6, 1e-6, 1e-8, 1e-8, 1e-6])
    c15 = np.array([Cm[i, j] for i in range(5) for j in range(i + 1)])
    rc, q, c2 = oracle.propagate_cov(p, c15, 120.0, 125.0, BZ)
    assert rc == 0
    L = np.linalg.cholesky(Cm)
    samples = p + rng.normal(size=(40000, 5)) @ L.T
    out = np.array([oracle.propagate(s, 120.0, 125.0, BZ)[1] for s in samples])
    emp = np.cov(out.T)
    got = oracle.unpack_cov(c2)
    sd = np.sqrt(np.diag(got))
    corr_err = np.abs(emp - got) / np.outer(sd, sd)
    assert np.all(corr_err < 0.05), corr_err


def test_seed_recovers_exact_helix(cfg):
    rng = np.random.default_rng(21)
    P = _random_particles(rng, 300, pt_lo=0.25)
    x = synth.row_geometry()[0]
    alpha = synth.SECTOR_HALF_ANGLE
    n = 0
    for i in range(300):
        r0, rm, rl = sorted(rng.choice(np.arange(5, 150), 3, replace=False))
        oks, st = zip(*[synth.helix_state_at_row(P, i, alpha, x[r]) for r in (r0, rm, rl)])
        if not all(oks) or abs(st[0][2]) > 0.9:
            continue
        rc, p = oracle.seed(cfg, x[r0], st[0][0], st[0][1], x[rm], st[1][0], x[rl], st[2][0], st[2][1])
        assert rc == 0
        assert np.all(np.abs(p - st[0]) <= 1e-9 * np.maximum(1.0, np.abs(st[0]))), (p, st[0])
        n += 1
    assert n > 200


def _c15(M):
    return np.array([M[i, j] for i in range(5) for j in range(i + 1)])


def test_kf_update_scalar_closed_form():
    # prior with y correlated to sinphi only; z uncorrelated
    M = np.diag([0.04, 0.09, 0.01, 0.02, 1.0])
    M[0, 2] = M[2, 0] = 0.012
    p = np.array([1.0, 2.0, 0.1, 0.2, 0.5])
    vy, vz = 0.01, 0.0225
    ym, zm = 1.3, 1.8
    q, c, chi2 = oracle.kf_update(p, _c15(M), ym, zm, vy, vz)
    ky = 0.04 / (0.04 + vy)
    assert abs(q[0] - (1.0 + ky * 0.3)) < 1e-14
    assert abs(q[2] - (0.1 + 0.012 / (0.04 + vy) * 0.3)) < 1e-14
    assert abs(q[1] - (2.0 + 0.09 / (0.09 + vz) * (-0.2))) < 1e-14
    assert q[3] == 0.2 and q[4] == 0.5
    C2 = oracle.unpack_cov(c)
    assert abs(C2[0, 0] - 0.04 * vy / (0.04 + vy)) < 1e-15
    assert abs(C2[2, 2] - (0.01 - 0.012 ** 2 / (0.04 + vy))) < 1e-15
    assert abs(chi2 - (0.3 ** 2 / (0.04 + vy) + 0.2 ** 2 / (0.09 + vz))) < 1e-13


def test_kf_zero_residual_fixed_point_and_spd():
    rng = np.random.default_rng(4)
    A = rng.normal(size=(5, 5))
    M = A @ A.T + np.eye(5) * 0.1
    p = rng.normal(size=5)
    q, c, chi2 = oracle.kf_update(p, _c15(M), p[0], p[1], 0.01, 0.02)
    assert np.array_equal(q, p) and chi2 == 0.0
    np.linalg.cholesky(oracle.unpack_cov(c))


def test_kf_sequence_equals_batch_least_squares():
    # with no transport, n updates = information-form posterior (batch weighted LSQ)
    rng = np.random.default_rng(8)
    A = rng.normal(size=(5, 5))
    C0 = A @ A.T + np.eye(5)
    p0 = rng.normal(size=5)
    vy, vz = 0.01, 0.0225
    H = np.zeros((2, 5))
    H[0, 0] = H[1, 1] = 1
    Vi = np.diag([1 / vy, 1 / vz])
    p, c = p0.copy(), _c15(C0)
    info = np.linalg.inv(C0)
    rhs = info @ p0
    for _ in range(7):
        m = rng.normal(size=2)
        p, c, _ = oracle.kf_update(p, c, m[0], m[1], vy, vz)
        info = info + H.T @ Vi @ H
        rhs = rhs + H.T @ Vi @ m
    Cb = np.linalg.inv(info)
    assert np.allclose(p, Cb @ rhs, rtol=1e-9, atol=1e-11)
    assert np.allclose(oracle.unpack_cov(c), Cb, rtol=1e-8, atol=1e-12)
