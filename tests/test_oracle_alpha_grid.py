"""Pins of the oracle's spatially varying CR spectral index (a gridded alpha).

The paper evaluates Eqs. ji and jp with one power-law index alpha and leaves a
fuller CR spectrum to future work (Sec. 2.1); the first step taken here lets
alpha vary in space as one more gridded field, with the emissivities evaluated
at the local index.  Pinned by:
  * a constant alpha grid reproduces the plain march at that alpha;
  * alpha linear in z (which trilinear interpolation reproduces exactly) on a
    field without Faraday rotation: each pixel's I and polarised intensity are
    the sums of Eqs. ji and jp at alpha(z) of every midpoint, computed here
    from the midpoints alone;
  * the gradient with respect to B, n_e and N0 against central differences,
    and no theta[12] gradient once alpha is gridded.
"""
import numpy as np
import pytest

from paper_2410_01136_amd import inputs as I

LO, HI = (-6.0, -6.0, -3.0), (6.0, 6.0, 3.0)
FREQS = [0.4e9, 1.4e9]


def _uniform_grid(n=(5, 5, 7), B=(0.0, 0.0, 5.0), ne=0.0, n0=4e-5):
    nx, ny, nz = n
    bn = np.zeros((nz, ny, nx, 4), dtype=np.float32)
    bn[..., 0:3] = B
    bn[..., 3] = ne
    c = np.full((nz, ny, nx), n0, dtype=np.float32)
    return bn, c


def _geom(orc, nside=2, n_steps=40):
    return orc.make_geom(nside, n_steps, FREQS, r_obs=(0.5, -0.3, 0.2), box_lo=LO, box_hi=HI)


@pytest.mark.parametrize("a", [3.0, 2.625])  # exact in FP32 (the grid holds floats)
def test_constant_alpha_grid_is_the_plain_march(orc, a):
    th = I.THETA0.copy()
    th[12] = a
    bn, c = _uniform_grid(B=(1.0, -2.0, 4.0), ne=0.05)
    nz, ny, nx, _ = bn.shape
    alpha = np.full((nz, ny, nx), a, dtype=np.float32)
    g = _geom(orc)
    th_other = th.copy()
    th_other[12] = 3.3  # ignored once alpha is gridded
    plain = orc.forward(g, orc.Field(orc.GRID, th, grid_bn=bn, grid_c=c, grid_lo=LO, grid_hi=HI))
    va = orc.forward(g, orc.Field(orc.GRID, th_other, grid_bn=bn, grid_c=c, grid_lo=LO, grid_hi=HI,
                                  grid_alpha=alpha))
    np.testing.assert_allclose(va, plain, rtol=1e-12, atol=1e-14 * np.abs(plain).max())


def test_alpha_linear_in_z_sums_the_local_emissivities(orc):
    # alpha(z) = a0 + a1 z: 2.375 .. 3.125 over the box, exact in FP32 at the
    # nodes (z = -3 .. 3 kpc in steps of 1), so the interpolation is exactly linear
    a0, a1 = 2.75, 0.125
    bn, c = _uniform_grid(B=(0.0, 0.0, 5.0), ne=0.0, n0=4e-5)
    nz, ny, nx, _ = bn.shape
    zs = np.linspace(LO[2], HI[2], nz)
    alpha = np.broadcast_to((a0 + a1 * zs)[:, None, None], (nz, ny, nx)).astype(np.float32)
    g = _geom(orc)
    f = orc.Field(orc.GRID, I.THETA0, grid_bn=bn, grid_c=c, grid_lo=LO, grid_hi=HI, grid_alpha=alpha)
    maps = orc.forward(g, f)
    npix = 48
    pix = np.arange(npix)
    mids = orc.midpoints(g, pix)  # [pix][step][3] kpc
    for p in pix:
        nhat = mids[p, 1] - mids[p, 0]
        nhat /= np.linalg.norm(nhat)
        dcm = np.linalg.norm(mids[p, 1] - mids[p, 0]) * 3.0856775814913673e21
        bt = 5e-6 * np.sqrt(1.0 - nhat[2] ** 2)  # |B_z e_z| transverse to the sightline
        for k, nu in enumerate(FREQS):
            aI = [a0 + a1 * z for z in mids[p, :, 2]]
            n0 = float(np.float32(4e-5))  # the grid holds floats
            jI = sum(orc.j_I(a, nu, bt, n0) for a in aI) * dcm
            jP = sum(orc.j_P(a, nu, bt, n0) for a in aI) * dcm
            rj = orc.rayleigh_jeans(nu)
            assert maps[k, 0, p] == pytest.approx(rj * jI, rel=1e-12)
            assert np.hypot(maps[k, 1, p], maps[k, 2, p]) == pytest.approx(rj * jP, rel=1e-12)


def test_gradient_with_gridded_alpha_matches_finite_differences(orc):
    th = I.THETA0.copy()
    reg_bn, reg_c = orc.sample_model16(th, (6, 5, 4), LO, HI)
    rng = np.random.default_rng(9)
    bn = reg_bn + (rng.standard_normal(reg_bn.shape) * 0.5).astype(np.float32)
    bn[..., 3] = np.abs(bn[..., 3]) + 0.005
    alpha = (2.7 + 0.4 * rng.random((4, 5, 6))).astype(np.float32)
    f = orc.Field(orc.GRID, th, grid_bn=bn, grid_c=reg_c, grid_lo=LO, grid_hi=HI, grid_alpha=alpha)
    g = orc.make_geom(4, 40, FREQS, r_obs=(0.5, -0.3, 0.2), box_lo=LO, box_hi=HI)
    dm = I.cotangents((2, 3, 192), seed=17).astype(np.float64)
    dth, gbn, gc = orc.adjoint(g, f, dm, want_grid=True)
    assert dth[12] == 0.0

    def loss():
        return float((orc.forward(g, f) * dm).sum())

    scale = max(np.abs(gbn * f.grid_bn).max(), np.abs(gc * f.grid_c).max())
    checked = 0
    for _ in range(50):
        iz, iy, ix, ch = rng.integers(4), rng.integers(5), rng.integers(6), rng.integers(5)
        arr = f.grid_bn if ch < 4 else f.grid_c
        idx = (iz, iy, ix, ch) if ch < 4 else (iz, iy, ix)
        v0 = float(arr[idx])
        ana = gbn[idx] if ch < 4 else gc[idx]

        def d(h):
            arr[idx] = np.float32(v0 + h)
            vp = float(arr[idx])
            lp = loss()
            arr[idx] = np.float32(v0 - h)
            vm = float(arr[idx])
            lm = loss()
            arr[idx] = np.float32(v0)
            return (lp - lm) / (vp - vm)

        h = 2.0 ** np.floor(np.log2(max(abs(v0), 1e-6) * 2e-5))
        fd = (4 * d(h / 2) - d(h)) / 3
        assert abs(fd - ana) * abs(v0) <= 1e-6 * scale + 1e-9 * abs(ana * v0), (idx, fd, ana)
        checked += abs(ana * v0) > 1e-3 * scale
    assert checked >= 10
