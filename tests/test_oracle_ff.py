"""Pins of the oracle's free-free emission and absorption.

The paper leaves these processes to future work (Sec. 5) and prints no
formulas; the oracle follows the reading stated in its header: the Mezger &
Henderson (1967) opacity, the Rayleigh-Jeans source function T_e, and
attenuation by e^-tau to each segment's midpoint.  Pinned here by:
  * the classical radio free-free opacity with the Gaunt factor (Oster 1961;
    Rybicki & Lightman 1979, Eq. 5.18b in the Rayleigh-Jeans limit), computed
    from CODATA constants: the approximation agrees to a few per cent;
  * an optically thick uniform medium, whose brightness is T_e;
  * the exact geometric series of a uniform medium (with the segment opacity
    taken from an optically thin run, not from the formula), for free-free
    alone and for attenuated synchrotron on the equator, where B_par = 0;
  * the reduction to the plain march when T_e = 0 or n_e = 0;
  * central finite differences of the reverse pass.
"""
import math

import numpy as np
import pytest

from paper_2410_01136_amd import inputs as I

QE, ME, KB, C, PC = 4.80320471e-10, 9.1093837015e-28, 1.380649e-16, 2.99792458e10, 3.0856775814913673e18
EULER_GAMMA = 0.5772156649015329


def kappa_gaunt_per_pc(nu, T):
    """Free-free absorption per pc per (n_e n_i / cm^-6), Rayleigh-Jeans limit."""
    g = math.sqrt(3) / math.pi * (math.log((2 * KB * T) ** 1.5 / (math.pi * QE ** 2 * math.sqrt(ME) * nu))
                                  - 2.5 * EULER_GAMMA)
    return 4 * QE ** 6 / (3 * ME * KB * C) * math.sqrt(2 * math.pi / (3 * KB * ME)) * T ** -1.5 * nu ** -2 * g * PC


def test_opacity_matches_gaunt_factor_formula(orc):
    for T in (4000.0, 6000.0, 8000.0, 1e4, 1.5e4):
        for nu in (0.03e9, 0.1e9, 0.3e9, 1e9, 3e9, 10e9):
            r = orc.kff(nu, T) / kappa_gaunt_per_pc(nu, T)
            assert 0.97 < r < 1.12, (T, nu, r)
            if 0.3e9 <= nu <= 3e9 and T <= 1e4:
                assert abs(r - 1) < 0.025, (T, nu, r)


def _sphere(orc, B=(0.0, 0.0, 0.0), ne=0.0, n0=0.0, te=0.0, R=5.0):
    th = I.sphere_theta(B_uG=B, ne=ne, n0=n0, R0_kpc=R, centre=(-8.5, 0.0, 0.0))
    return orc.Field(orc.SPHERE, th, te_k=te)


def _geom(orc, n_steps, freqs, nside=2, L=4.0):
    # every sightline has length L inside the sphere of radius 5 around the observer
    return orc.make_geom(nside, n_steps, freqs, r_obs=(-8.5, 0.0, 0.0), r_max=L)


def _series(x, n):
    """sum_{k<n} e^{-x (k + 1/2)}"""
    return math.exp(-x / 2) * -math.expm1(-n * x) / -math.expm1(-x)


def test_optically_thick_medium_shines_at_te(orc):
    # tau ~ 40 over the path in 4096 segments of depth x ~ 0.01: the midpoint
    # sum is T_e (1 - e^-tau) x e^{-x/2} / (1 - e^-x) = T_e (1 - O(x^2 / 24))
    te = 7500.0
    g = _geom(orc, 4096, [0.2e9, 0.25e9], nside=1)
    maps = orc.forward(g, _sphere(orc, ne=33.5, te=te))
    tau = [orc.kff(nu, te) * 33.5 ** 2 * 4000.0 for nu in (0.2e9, 0.25e9)]
    assert min(tau) > 25.0 and max(tau) / 4096 < 0.02
    np.testing.assert_allclose(maps[:, 0], te, rtol=2e-5)
    assert np.abs(maps[:, 1:]).max() == 0.0


def _segment_depth(orc, g, te, ne, nu_index):
    """Optical depth of one segment, solved from an optically thin run."""
    n = g.n_steps
    t = orc.forward(g, _sphere(orc, ne=ne, te=te))[nu_index, 0, 0] / te
    x = t / n
    for _ in range(50):  # Newton on x * sum e^{-x (k + 1/2)} = t
        f = x * _series(x, n) - t
        h = 1e-6 * x
        df = ((x + h) * _series(x + h, n) - (x - h) * _series(x - h, n)) / (2 * h)
        x -= f / df
    return x


@pytest.mark.parametrize("n_steps", [1, 7, 64])
def test_uniform_medium_is_a_geometric_series(orc, n_steps):
    te, ne_thin = 9000.0, 0.05
    g = _geom(orc, n_steps, [0.1e9, 0.4e9])
    x_thin = [_segment_depth(orc, g, te, ne_thin, k) for k in range(2)]
    for m in (3.0, 10.0, 40.0):
        maps = orc.forward(g, _sphere(orc, ne=ne_thin * m, te=te))
        for k in range(2):
            x = x_thin[k] * m * m  # the opacity scales as n_e^2
            want = te * x * _series(x, n_steps)
            assert maps[k, 0] == pytest.approx(np.full(maps.shape[-1], want), rel=1e-10)
    # the thin-limit depth follows T_e^-1.35 nu^-2.1 (Mezger & Henderson)
    assert x_thin[0] / x_thin[1] == pytest.approx(4.0 ** 2.1, rel=1e-9)


def test_synchrotron_is_attenuated_on_the_equator(orc):
    # B along z: sightlines in the Galactic plane see B_perp = B_z and B_par = 0,
    # so their synchrotron is uniform along the path with a fixed angle
    te, ne = 8000.0, 3.0
    nside, n_steps = 4, 32
    g = _geom(orc, n_steps, [0.15e9, 0.5e9], nside=nside)
    base = orc.forward(g, _sphere(orc, B=(0, 0, 6.0), ne=ne, n0=4e-5))
    att = orc.forward(g, _sphere(orc, B=(0, 0, 6.0), ne=ne, n0=4e-5, te=te))
    ring = [p for p in range(12 * nside * nside) if abs(orc.pix2zphi(nside, p)[0]) < 1e-15]
    assert len(ring) == 4 * nside
    for k in range(2):
        x = _segment_depth(orc, g, te, ne, k)
        s = _series(x, n_steps) / n_steps
        for p in ring:
            assert att[k, 0, p] == pytest.approx(base[k, 0, p] * s + te * x * n_steps * s, rel=1e-10)
            assert att[k, 1, p] == pytest.approx(base[k, 1, p] * s, rel=1e-10, abs=1e-14)
            assert att[k, 2, p] == pytest.approx(base[k, 2, p] * s, rel=1e-10, abs=1e-14)


def test_no_electrons_or_no_temperature_is_the_plain_march(orc):
    g = orc.make_geom(4, 48, [0.3e9, 1.4e9], r_max=20.0)
    plain = orc.forward(g, orc.Field(orc.MODEL16, I.THETA0))
    np.testing.assert_array_equal(orc.forward(g, orc.Field(orc.MODEL16, I.THETA0, te_k=0.0)), plain)
    th = I.THETA0.copy()
    th[13] = 0.0  # n0 = 0: no Faraday rotation and no free-free
    a = orc.forward(g, orc.Field(orc.MODEL16, th))
    b = orc.forward(g, orc.Field(orc.MODEL16, th, te_k=8000.0))
    np.testing.assert_array_equal(a, b)


# a medium dense enough for tau ~ 0.2 at 150 MHz over 2 kpc, with a weak field
# (Faraday phases of ~200 rad) and a strong CR density so that synchrotron and
# free-free brightness are comparable
THETA_FF = np.array([0.005, -0.25, 0.15, 0.35, 7.0, 1.2, 0.002, 1.4, 9.0,
                     42.0, 7.5, 1.1, 2.85, 3.0, 0.9, 0.02])
FREQS_FF = [0.15e9, 0.3e9]
TE = 8000.0


def _loss(orc, g, f, dm):
    return float((orc.forward(g, f) * dm).sum())


def test_free_free_is_not_negligible_in_the_gradient_case(orc):
    g = orc.make_geom(4, 48, FREQS_FF, r_max=2.0)
    plain = orc.forward(g, orc.Field(orc.MODEL16, THETA_FF))
    ff = orc.forward(g, orc.Field(orc.MODEL16, THETA_FF, te_k=TE))
    ratio = ff[0, 0] / plain[0, 0]
    assert ratio.min() < 0.95 or ratio.max() > 1.05  # absorption or emission shows


def test_theta_gradient_with_free_free_matches_finite_differences(orc):
    g = orc.make_geom(4, 48, FREQS_FF, r_max=2.0)
    dm = I.cotangents((2, 3, 192), seed=31).astype(np.float64)
    dth, _, _ = orc.adjoint(g, orc.Field(orc.MODEL16, THETA_FF, te_k=TE), dm)
    scale = 0.0
    fds = []
    for k in range(16):
        h = 1e-5 * max(abs(THETA_FF[k]), 1e-2 if k not in (9, 13) else abs(THETA_FF[k]))

        def d(hh):
            tp, tm = THETA_FF.copy(), THETA_FF.copy()
            tp[k] += hh
            tm[k] -= hh
            return (_loss(orc, g, orc.Field(orc.MODEL16, tp, te_k=TE), dm) -
                    _loss(orc, g, orc.Field(orc.MODEL16, tm, te_k=TE), dm)) / (2 * hh)

        fds.append((4 * d(h / 2) - d(h)) / 3)
    fd = np.array(fds)
    sk = np.maximum(np.abs(THETA_FF), 1e-2)
    scale = np.abs(fd * sk).max()
    for k in range(16):
        assert abs(dth[k] - fd[k]) * sk[k] <= 2e-7 * scale, (k, dth[k], fd[k])
    # the electron-density parameters carry real weight here
    assert abs(dth[13] * THETA_FF[13]) > 1e-2 * scale


def test_grid_gradient_with_free_free_matches_finite_differences(orc):
    lo, hi = (-12.0, -10.0, -3.0), (12.0, 10.0, 3.0)
    bn, c = orc.sample_model16(THETA_FF, (6, 5, 4), lo, hi)
    rng = np.random.default_rng(5)
    bn = bn + (rng.standard_normal(bn.shape) * 0.002).astype(np.float32)
    bn[..., 3] = np.abs(bn[..., 3]) + 0.5
    f = orc.Field(orc.GRID, THETA_FF, grid_bn=bn, grid_c=c, grid_lo=lo, grid_hi=hi, te_k=TE)
    g = orc.make_geom(4, 40, FREQS_FF, r_max=2.5, box_lo=lo, box_hi=hi)
    dm = I.cotangents((2, 3, 192), seed=32).astype(np.float64)
    _, gbn, gc = orc.adjoint(g, f, dm, want_grid=True)
    nz, ny, nx, _ = bn.shape
    scale = max(np.abs(gbn * f.grid_bn).max(), np.abs(gc * f.grid_c).max())
    checked = 0
    # every n_e voxel (absorption and emission act through it), plus random others
    cases = [(iz, iy, ix, 3) for iz in range(nz) for iy in range(ny) for ix in range(nx)]
    cases += [(rng.integers(nz), rng.integers(ny), rng.integers(nx), rng.integers(5)) for _ in range(30)]
    for iz, iy, ix, ch in cases:
        arr = f.grid_bn if ch < 4 else f.grid_c
        idx = (iz, iy, ix, ch) if ch < 4 else (iz, iy, ix)
        v0 = float(arr[idx])
        ana = gbn[idx] if ch < 4 else gc[idx]

        def d(h):
            arr[idx] = np.float32(v0 + h)
            vp = float(arr[idx])
            lp = _loss(orc, g, f, dm)
            arr[idx] = np.float32(v0 - h)
            vm = float(arr[idx])
            lm = _loss(orc, g, f, dm)
            arr[idx] = np.float32(v0)
            return (lp - lm) / (vp - vm)

        h = 2.0 ** np.floor(np.log2(max(abs(v0), 1e-6) * 2e-5))
        fd = (4 * d(h / 2) - d(h)) / 3
        assert abs(fd - ana) * abs(v0) <= 1e-6 * scale + 1e-9 * abs(ana * v0), (idx, fd, ana)
        checked += abs(ana * v0) > 1e-3 * scale and ch == 3
    assert checked >= 5  # n_e voxels on the sightlines carry weight
