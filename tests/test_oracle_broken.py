"""Pins of the oracle's broken power-law CR spectrum.

The paper evaluates Eqs. ji and jp for one power law and names a fuller CR
spectrum as future work (Sec. 2.1).  The oracle's broken power law (index a1
below the break Lorentz factor gamma_b, a2 above, continuous at the break)
reduces the electron integral to incomplete x-moments of the synchrotron
functions F and G, taken through the upper incomplete gamma function.  Pinned
against what does not share that reduction:
  * Gamma(a, y), F(x), G(x) against SciPy's incomplete gamma and Bessel K;
  * the complete moments (the Gamma-function factors of Eqs. ji and jp) against
    quadrature of x^mu F(x) and x^mu G(x) with SciPy's F and G;
  * the tail shares against the same quadrature over [xb, inf);
  * j_I and j_P against the electron integral (1/4 pi) int N(gamma) P(nu, gamma)
    dgamma taken directly in gamma with SciPy's Bessel functions;
  * the limits: a1 = a2 (any break), gamma_b -> inf (all electrons below the
    break) and gamma_b -> 1 (all above it) give the one-index Eqs. ji and jp;
    the spectral slope of j_I runs from (1 - a1)/2 at low frequency to
    (1 - a2)/2 at high frequency;
  * the emissivity's B_trans slope and the maps' reverse pass against central
    differences of the oracle forward, and N0-linearity of the maps.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

from paper_2410_01136_amd import inputs as I

QE, ME, C = 4.80320471e-10, 9.1093837015e-28, 2.99792458e10


def scipy_F(x):
    # int_x^inf K_5/3: below z = 1 in ln z (the integrand grows as z^-5/3 there)
    k = lambda z: special.kv(5.0 / 3.0, z)
    val = integrate.quad(k, max(x, 1.0), np.inf, epsabs=0, epsrel=1e-13, limit=400)[0]
    if x < 1.0:
        val += integrate.quad(lambda u: k(math.exp(u)) * math.exp(u), math.log(x), 0.0, epsabs=0,
                              epsrel=1e-13, limit=400)[0]
    return x * val


def scipy_G(x):
    return x * special.kv(2.0 / 3.0, x)


@pytest.mark.parametrize("a", [0.7, 1.25, 2.0, 2.85, 3.6])
def test_gamma_upper_matches_scipy(orc, a):
    for y in (1e-9, 1e-3, 0.2, 1.0, a + 0.9, a + 1.1, 4.0, 12.0, 40.0, 75.0):
        ref = special.gammaincc(a, y) * special.gamma(a)
        assert orc.gamma_upper(a, y) == pytest.approx(ref, rel=1e-12, abs=1e-300), (a, y)
    assert orc.gamma_upper(a, 0.0) == pytest.approx(special.gamma(a), rel=1e-14)


def test_synchrotron_functions_match_scipy(orc):
    for x in (1e-9, 1e-5, 1e-2, 0.2858, 1.0, 3.0, 10.0, 30.0):
        assert orc.synch_F(x) == pytest.approx(scipy_F(x), rel=1e-10), x
        assert orc.synch_G(x) == pytest.approx(scipy_G(x), rel=1e-10), x
    # textbook values: F peaks near x = 0.29 at 0.918; F(1) = 0.652 (3 digits)
    assert orc.synch_F(0.2858) == pytest.approx(0.918, abs=1e-3)
    assert orc.synch_F(1.0) == pytest.approx(0.652, abs=1e-3)


@pytest.mark.parametrize("alpha", [0.9, 2.0, 2.85, 4.2])
def test_complete_moments_and_tails(orc, alpha):
    mu = 0.5 * (alpha - 3.0)

    def quadF(lo, hi):
        return integrate.quad(lambda x: x ** mu * scipy_F(x), lo, hi, epsabs=0, epsrel=1e-11,
                              limit=400)[0]

    def quadG(lo, hi):
        return integrate.quad(lambda x: x ** mu * scipy_G(x), lo, hi, epsabs=0, epsrel=1e-11,
                              limit=400)[0]

    # the complete moments behind Eqs. ji and jp
    totF = quadF(0, 1) + quadF(1, 60) + quadF(60, np.inf)
    totG = quadG(0, 1) + quadG(1, 60) + quadG(60, np.inf)
    assert orc.moment_F(mu) == pytest.approx(totF, rel=1e-9)
    assert orc.moment_G(mu) == pytest.approx(totG, rel=1e-9)
    # the tail shares: 1 at xb -> 0, 0 beyond the cut, quadrature in between
    tF, tG = orc.moment_tails(alpha, 0.0)
    assert (tF, tG) == (1.0, 1.0)
    for xb in (1e-6, 0.05, 0.7, 3.0, 9.0):
        tF, tG = orc.moment_tails(alpha, xb)
        refF = (quadF(xb, max(60, 2 * xb)) + quadF(max(60, 2 * xb), np.inf)) / totF
        refG = (quadG(xb, max(60, 2 * xb)) + quadG(max(60, 2 * xb), np.inf)) / totG
        assert tF == pytest.approx(refF, abs=1e-10, rel=1e-9), (alpha, xb)
        assert tG == pytest.approx(refG, abs=1e-10, rel=1e-9), (alpha, xb)
    tF, tG = orc.moment_tails(alpha, 1e-14)
    # the trapezoid over the whole s-range reproduces the closed forms
    assert 1.0 - tF == pytest.approx(0.0, abs=max(1e-12, 10 * (1e-14) ** (alpha / 2 - 1 / 6)))
    assert orc.moment_tails(alpha, 200.0)[0] < 1e-80


def electron_integral(a1, a2, gb, nu, bt, polarised):
    """(1/4 pi) int N(gamma) sqrt(3) q^3 B / (m c^2) F(nu / nu_c) dgamma with
    N0 = 1, straight from the single-electron spectrum, in u = ln gamma."""
    kern = scipy_G if polarised else scipy_F
    x0 = 4 * math.pi * nu * ME * C / (3 * QE * bt)

    def n_of(g):
        return g ** -a1 if g < gb else gb ** (a2 - a1) * g ** -a2

    def integrand(u):
        g = math.exp(u)
        return n_of(g) * kern(x0 / (g * g)) * g

    # the kernel is negligible below x = 1e-14 ** ... and above x = 120
    ulo, uhi = 0.5 * math.log(x0 / 120.0), 0.5 * math.log(x0 / 1e-16)
    ub = math.log(gb)
    pts = sorted(u for u in (ulo, ub, uhi) if ulo <= u <= uhi)
    tot = 0.0
    for lo, hi in zip(pts[:-1], pts[1:]):
        tot += integrate.quad(integrand, lo, hi, epsabs=0, epsrel=1e-11, limit=400)[0]
    return math.sqrt(3) * QE ** 3 * bt / (ME * C * C) * tot / (4 * math.pi)


@pytest.mark.parametrize("a1,a2,gb,nu,bt", [
    (2.2, 3.4, 8.0e3, 1.4e9, 6e-6),
    (2.85, 3.6, 2.5e4, 0.4e9, 3e-6),
    (3.0, 2.4, 5.0e3, 5.0e9, 1e-5),  # a hardening break
])
def test_emissivity_equals_the_electron_integral(orc, a1, a2, gb, nu, bt):
    j = orc.j_broken(a1, a2, gb, nu, bt, 1.0)
    assert j[0] == pytest.approx(electron_integral(a1, a2, gb, nu, bt, False), rel=1e-8)
    assert j[1] == pytest.approx(electron_integral(a1, a2, gb, nu, bt, True), rel=1e-8)


def test_one_index_limits(orc):
    nu, bt, n0 = 1.4e9, 5e-6, 3e-5
    for a in (2.2, 3.0):
        for gb in (30.0, 1e4, 1e7):
            j = orc.j_broken(a, a, gb, nu, bt, n0)
            assert j[0] == pytest.approx(orc.j_I(a, nu, bt, n0), rel=1e-13)
            assert j[1] == pytest.approx(orc.j_P(a, nu, bt, n0), rel=1e-13)
    a1, a2 = 2.4, 3.3
    # (nearly) every emitting electron below the break: xb ~ 5e-11, see
    # test_maps_limits_and_linearity for the size of what is left
    j = orc.j_broken(a1, a2, 1e9, nu, bt, n0)
    assert j[0] == pytest.approx(orc.j_I(a1, nu, bt, n0), rel=1e-8)
    assert j[1] == pytest.approx(orc.j_P(a1, nu, bt, n0), rel=1e-8)
    j = orc.j_broken(a1, a2, 1.0, nu, bt, n0)  # every one above it
    assert j[0] == pytest.approx(orc.j_I(a2, nu, bt, n0), rel=1e-13)
    assert j[1] == pytest.approx(orc.j_P(a2, nu, bt, n0), rel=1e-13)


def test_spectral_slope_runs_between_the_two_indices(orc):
    a1, a2, gb, bt = 2.3, 3.5, 1e4, 5e-6

    def slope(nu):
        lo, hi = orc.j_broken(a1, a2, gb, nu / 1.01, bt, 1.0)[0], orc.j_broken(a1, a2, gb, nu * 1.01, bt, 1.0)[0]
        return math.log(hi / lo) / math.log(1.01 ** 2)

    assert slope(1e3) == pytest.approx((1 - a1) / 2, abs=2e-3)
    assert slope(1e15) == pytest.approx((1 - a2) / 2, abs=2e-3)
    s = [slope(nu) for nu in np.geomspace(1e6, 1e13, 15)]
    # steepening through the break (flat to rounding once every electron
    # that emits sits above it)
    assert all(x >= y - 1e-9 for x, y in zip(s[:-1], s[1:]))
    assert s[0] - s[-1] > 0.55


def test_emissivity_slope_in_b_trans(orc):
    a1, a2, gb, nu = 2.3, 3.4, 9e3, 1.4e9
    for bt in (1e-6, 5e-6, 3e-5):
        j = orc.j_broken(a1, a2, gb, nu, bt, 1.0)
        for k in (0, 1):
            def d(h):
                return (orc.j_broken(a1, a2, gb, nu, bt + h, 1.0)[k] -
                        orc.j_broken(a1, a2, gb, nu, bt - h, 1.0)[k]) / (2 * h)
            h = bt * 1e-4
            assert j[2 + k] == pytest.approx((4 * d(h / 2) - d(h)) / 3, rel=1e-8)


THETA_T = np.array([5.0, -0.25, 0.15, 0.35, 7.0, 1.2, 2.0, 1.4, 9.0,
                    4.2e-5, 7.5, 1.1, 2.3, 0.028, 0.9, 0.02])
FREQS = [0.8e9, 1.4e9]
BROKEN = (3.4, 9.0e3)  # a2, gamma_b: the break sits near x ~ 1 at these frequencies


def _loss(orc, g, f, dm):
    return float((orc.forward(g, f) * dm).sum())


def test_maps_limits_and_linearity(orc):
    g = orc.make_geom(4, 48, FREQS, r_max=20.0)
    pl1 = orc.forward(g, orc.Field(orc.MODEL16, THETA_T))
    th2 = THETA_T.copy()
    th2[12] = BROKEN[0]
    pl2 = orc.forward(g, orc.Field(orc.MODEL16, th2))
    # gamma_b = 1e9 puts the break at xb ~ 1e-10: the electrons above it add
    # ~xb^(a1/2 - 1/6) ~ 1e-10 of the emission (and the FP64 rounding of the
    # share below xb, ~1e-16, enters scaled by the upper law's normalisation,
    # ~xb^((a1 - a2)/2) ~ 1e5)
    hi = orc.forward(g, orc.Field(orc.MODEL16, THETA_T, broken=(BROKEN[0], 1e9)))
    lo = orc.forward(g, orc.Field(orc.MODEL16, THETA_T, broken=(BROKEN[0], 1.0)))
    np.testing.assert_allclose(hi, pl1, rtol=1e-8, atol=1e-8 * np.abs(pl1).max())
    np.testing.assert_allclose(lo, pl2, rtol=1e-12, atol=1e-12 * np.abs(pl2).max())
    br = orc.forward(g, orc.Field(orc.MODEL16, THETA_T, broken=BROKEN))
    # the break removes emission relative to the low-energy law continued upward
    assert np.all(br[:, 0] < pl1[:, 0])
    th3 = THETA_T.copy()
    th3[9] *= 3.0
    br3 = orc.forward(g, orc.Field(orc.MODEL16, th3, broken=BROKEN))
    np.testing.assert_allclose(br3, 3.0 * br, rtol=1e-12, atol=1e-14 * np.abs(br).max())


def test_broken_spectrum_is_validated(orc):
    g = orc.make_geom(2, 8, FREQS, r_max=20.0)
    for bad in ((0.2, 1e4), (3.4, 0.0), (3.4, math.inf), (math.nan, 1e4)):
        with pytest.raises(Exception):
            orc.forward(g, orc.Field(orc.MODEL16, THETA_T, broken=bad))


def test_theta_gradient_matches_finite_differences(orc):
    g = orc.make_geom(4, 48, FREQS, r_max=20.0)
    dm = I.cotangents((2, 3, 192), seed=21).astype(np.float64)
    dth, _, _ = orc.adjoint(g, orc.Field(orc.MODEL16, THETA_T, broken=BROKEN), dm)
    assert dth.shape == (18,)

    def fd(k, rel=1e-5):
        h = rel * max(abs(THETA_T[k]), 1e-2 if k not in (9, 13) else abs(THETA_T[k]))

        def d(hh):
            tp, tm = THETA_T.copy(), THETA_T.copy()
            tp[k] += hh
            tm[k] -= hh
            return (_loss(orc, g, orc.Field(orc.MODEL16, tp, broken=BROKEN), dm) -
                    _loss(orc, g, orc.Field(orc.MODEL16, tm, broken=BROKEN), dm)) / (2 * hh)

        return (4 * d(h / 2) - d(h)) / 3

    ks = list(range(16))
    ref = {k: fd(k) for k in ks}
    scale = max(abs(ref[k]) * max(abs(THETA_T[k]), 1e-2) for k in ks)
    for k in ks:
        sk = max(abs(THETA_T[k]), 1e-2)
        assert abs(dth[k] - ref[k]) * sk <= 1e-7 * scale, (k, dth[k], ref[k])
    L = _loss(orc, g, orc.Field(orc.MODEL16, THETA_T, broken=BROKEN), dm)
    assert THETA_T[9] * dth[9] == pytest.approx(L, rel=1e-12)  # maps linear in N0


def test_grid_gradient_matches_finite_differences(orc):
    lo, hi = (-12.0, -10.0, -3.0), (12.0, 10.0, 3.0)
    g = orc.make_geom(4, 40, FREQS, box_lo=lo, box_hi=hi)
    bn, c = orc.sample_model16(THETA_T, (6, 5, 4), lo, hi)
    rng = np.random.default_rng(5)
    bn = bn + (rng.standard_normal(bn.shape) * 0.5).astype(np.float32)
    bn[..., 3] = np.abs(bn[..., 3]) + 0.005
    f = orc.Field(orc.GRID, THETA_T, grid_bn=bn, grid_c=c, grid_lo=lo, grid_hi=hi, broken=BROKEN)
    dm = I.cotangents((2, 3, 192), seed=22).astype(np.float64)
    dth, gbn, gc = orc.adjoint(g, f, dm, want_grid=True)
    L = _loss(orc, g, f, dm)
    assert (gc * f.grid_c).sum() == pytest.approx(L, rel=1e-12)
    scale = max(np.abs(gbn * f.grid_bn).max(), np.abs(gc * f.grid_c).max())
    checked = 0
    for _ in range(40):
        iz, iy, ix, ch = rng.integers(4), rng.integers(5), rng.integers(6), rng.integers(5)
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
        fdv = (4 * d(h / 2) - d(h)) / 3
        assert abs(fdv - ana) * abs(v0) <= 1e-6 * scale + 1e-9 * abs(ana * v0), (idx, fdv, ana)
        checked += abs(ana * v0) > 1e-3 * scale
    assert checked >= 8


def test_spectral_parameter_gradient_matches_finite_differences(orc):
    """The gradient in (alpha_hi, ln gamma_b) (dtheta[16], [17]) and in the index
    below the break (dtheta[12]) against central differences of the maps, with
    and without free-free."""
    g = orc.make_geom(4, 40, FREQS, r_max=20.0)
    dm = I.cotangents((2, 3, 192), seed=23).astype(np.float64)
    for te in (0.0, 8000.0):
        dth, _, _ = orc.adjoint(g, orc.Field(orc.MODEL16, THETA_T, te_k=te, broken=BROKEN), dm)

        def loss(a1, a2, lng):
            th = THETA_T.copy()
            th[12] = a1
            return _loss(orc, g, orc.Field(orc.MODEL16, th, te_k=te, broken=(a2, math.exp(lng))), dm)

        p0 = np.array([THETA_T[12], BROKEN[0], math.log(BROKEN[1])])
        for k, idx in ((0, 12), (1, 16), (2, 17)):
            def d(h):
                e = np.zeros(3)
                e[k] = h
                return (loss(*(p0 + e)) - loss(*(p0 - e))) / (2 * h)
            h = 1e-3
            fdv = (4 * d(h / 2) - d(h)) / 3
            assert dth[idx] == pytest.approx(fdv, rel=1e-6), (te, k, dth[idx], fdv)


def test_spectral_derivatives_of_the_emissivity(orc):
    # the numerical derivatives against an independent closed form where one
    # exists: with equal indices the gamma_b dependence cancels (d/d ln gb = 0)
    # and d/da of j at a1 = a2 = a sums to d j(a) / d a of Eq. ji
    nu, bt = 1.4e9, 5e-6
    for a in (2.4, 3.0):
        dI, dP = orc.dj_broken(a, a, 1e4, nu, bt, 1.0)
        assert abs(dI[2]) <= 1e-9 * orc.j_I(a, nu, bt, 1.0)
        h = 1e-4
        ref = (orc.j_I(a + h, nu, bt, 1.0) - orc.j_I(a - h, nu, bt, 1.0)) / (2 * h)
        assert dI[0] + dI[1] == pytest.approx(ref, rel=1e-6)
        refp = (orc.j_P(a + h, nu, bt, 1.0) - orc.j_P(a - h, nu, bt, 1.0)) / (2 * h)
        assert dP[0] + dP[1] == pytest.approx(refp, rel=1e-6)
