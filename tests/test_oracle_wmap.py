"""Pins of the oracle's WMAP field (Sec. 3.1) and of its reverse pass."""
import math

import numpy as np
import pytest

from paper_2410_01136_amd import inputs as I
from parity import oracle_geom


def fields(orc, th, r):
    return orc.fields_at(orc.Field(orc.WMAP, th), np.asarray(r, dtype=np.float64))


def test_field_strength_is_b0_in_the_ring(orc):
    th = I.wmap_theta()
    rng = np.random.default_rng(1)
    for _ in range(200):
        rho = rng.uniform(3.0, 20.0)
        ph = rng.uniform(0, 2 * np.pi)
        z = rng.uniform(-4, 4)
        B, ne, n0 = fields(orc, th, (rho * np.cos(ph), rho * np.sin(ph), z))
        assert np.linalg.norm(B) == pytest.approx(th[0], rel=1e-13)


def test_field_vanishes_outside_the_ring(orc):
    th = I.wmap_theta()
    for r in [(1.0, 2.0, 0.3), (0.0, 0.0, 0.0), (21.0, 1.0, -0.5), (-2.9, 0.0, 1.0)]:
        B, _, _ = fields(orc, th, r)
        assert np.all(B == 0.0)


def test_axisymmetry_and_z_parity(orc):
    th = I.wmap_theta()
    r = np.array([6.0, -4.0, 0.7])
    B, _, n0 = fields(orc, th, r)
    a = 1.1
    R = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
    Br, _, n0r = fields(orc, th, R @ r)
    np.testing.assert_allclose(Br, R @ B, rtol=1e-12, atol=1e-14)
    assert n0r == pytest.approx(n0, rel=1e-13)
    Bm, _, n0m = fields(orc, th, r * np.array([1, 1, -1]))
    np.testing.assert_allclose(Bm, B * np.array([1, 1, -1]), rtol=1e-12, atol=1e-14)
    assert n0m == pytest.approx(n0, rel=1e-13)


def test_pitch_and_tilt_at_the_reference_radius(orc):
    # at rho = 8 kpc the log term vanishes: the field makes the angle psi0 with
    # rho^ in the plane (b0 cos psi0 on rho^, b0 sin psi0 on phi^ at z = 0) and
    # tilts by chi0 tanh(1) at z = 1 kpc
    th = I.wmap_theta()
    B, _, _ = fields(orc, th, (0.0, 8.0, 0.0))   # rho^ = +y, phi^ = -x
    assert B[1] == pytest.approx(th[0] * math.cos(th[1]), rel=1e-13)
    assert -B[0] == pytest.approx(th[0] * math.sin(th[1]), rel=1e-13)
    B1, _, _ = fields(orc, th, (0.0, 8.0, 1.0))
    assert B1[2] == pytest.approx(th[0] * math.sin(th[3] * math.tanh(1.0)), rel=1e-13)


def test_cosmic_ray_density_is_normalised_at_earth(orc):
    th = I.wmap_theta(earth=(-8.3, 0.0, 0.006))
    _, _, n0 = fields(orc, th, (-8.3, 0.0, 0.006))
    assert n0 == pytest.approx(4.0e-5, rel=1e-13)
    # sech^2 profile: half-maximum at z = h_z arccosh(sqrt 2)
    _, _, a = fields(orc, th, (0.0, 8.0, 0.0))
    _, _, b = fields(orc, th, (0.0, 8.0, math.acosh(math.sqrt(2.0))))
    assert b / a == pytest.approx(0.5, rel=1e-12)


def test_theta_gradient_against_differences(orc):
    th = I.wmap_theta()
    g = I.geometry("E1", nside=2, n_steps=48, freqs_hz=(2.4e9,), r_obs=(-8.5, 0.0, 0.0))
    og = oracle_geom(orc, g)
    dm = I.cotangents((1, 3, g.npix), seed=11).astype(np.float64)

    def L(t):
        return float((orc.forward(og, orc.Field(orc.WMAP, t)) * dm).sum())

    grad, _, _ = orc.adjoint(og, orc.Field(orc.WMAP, th), dm)
    for k in (0, 1, 2, 3, 9, 10, 11, 13, 14):
        h = 1e-5 * max(abs(th[k]), 1e-2)
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (L(tp) - L(tm)) / (2 * h)
        scale = max(abs(grad[k]) * max(abs(th[k]), 1e-2), 1e-12)
        assert abs(fd - grad[k]) * max(abs(th[k]), 1e-2) <= 1e-5 * scale + 1e-12, (k, fd, grad[k])
