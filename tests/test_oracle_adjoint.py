"""Pins of the oracle's hand-derived reverse pass.

The gradient of L = sum(dmaps * maps) is checked against central finite
differences of the oracle forward (Richardson-extrapolated, FP64) and against
the Euler homogeneity identities of the emission model:
  * maps are linear in N0, so sum_v N0_v dL/dN0_v = L (and C0 dL/dC0 = L);
  * scaling every B by s and every n_e by 1/s leaves the Faraday depth fixed
    while j ~ B_perp^{(alpha+1)/2}, so sum B dL/dB - sum n_e dL/dn_e
    = ((alpha + 1) / 2) L.
"""
import numpy as np
import pytest

from paper_2410_01136_amd import inputs as I

THETA_T = np.array([5.0, -0.25, 0.15, 0.35, 7.0, 1.2, 2.0, 1.4, 9.0,
                    4.2e-5, 7.5, 1.1, 2.85, 0.028, 0.9, 0.02])
FREQS = [0.8e9, 1.4e9]


def _loss(orc, g, f, dm):
    return float((orc.forward(g, f) * dm).sum())


def _fd_theta(orc, g, th, dm, k, rel=1e-5):
    # the Faraday phase reaches hundreds of radians, so steps stay far below 1e-3
    h = rel * max(abs(th[k]), 1e-2 if k not in (9, 13) else abs(th[k]))

    def d(hh):
        tp, tm = th.copy(), th.copy()
        tp[k] += hh
        tm[k] -= hh
        return (_loss(orc, g, orc.Field(orc.MODEL16, tp), dm) -
                _loss(orc, g, orc.Field(orc.MODEL16, tm), dm)) / (2 * hh)

    return (4 * d(h / 2) - d(h)) / 3


def test_theta_gradient_matches_finite_differences(orc):
    g = orc.make_geom(4, 48, FREQS, r_max=20.0)
    dm = I.cotangents((2, 3, 192), seed=11).astype(np.float64)
    dth, _, _ = orc.adjoint(g, orc.Field(orc.MODEL16, THETA_T), dm)
    fd = np.array([_fd_theta(orc, g, THETA_T, dm, k) for k in range(16)])
    scale = np.abs(fd * np.maximum(np.abs(THETA_T), 1e-2)).max()
    for k in range(16):
        # compare the parameter-scaled sensitivities theta_k dL/dtheta_k
        sk = max(abs(THETA_T[k]), 1e-2)
        assert abs(dth[k] - fd[k]) * sk <= 1e-7 * scale, (k, dth[k], fd[k])


def test_theta_gradient_euler_identities(orc):
    g = orc.make_geom(4, 64, FREQS, r_max=20.0)
    dm = I.cotangents((2, 3, 192), seed=12).astype(np.float64)
    f = orc.Field(orc.MODEL16, THETA_T)
    L = _loss(orc, g, f, dm)
    dth, _, _ = orc.adjoint(g, f, dm)
    th = THETA_T
    assert th[9] * dth[9] == pytest.approx(L, rel=1e-12)
    lhs = th[0] * dth[0] + th[6] * dth[6] - th[13] * dth[13]
    assert lhs == pytest.approx((th[12] + 1) / 2 * L, rel=1e-11)


def _small_grid(orc, with_c=True, n=(6, 5, 4), seed=3):
    lo, hi = (-12.0, -10.0, -3.0), (12.0, 10.0, 3.0)
    bn, c = orc.sample_model16(THETA_T, n, lo, hi)
    rng = np.random.default_rng(seed)
    bn = bn + (rng.standard_normal(bn.shape) * 0.5).astype(np.float32)
    bn[..., 3] = np.abs(bn[..., 3]) + 0.005
    f = orc.Field(orc.GRID, THETA_T, grid_bn=bn, grid_c=c if with_c else None,
                  grid_lo=lo, grid_hi=hi)
    return f, lo, hi


def test_grid_gradient_matches_finite_differences(orc):
    g = orc.make_geom(4, 40, FREQS, box_lo=(-12, -10, -3), box_hi=(12, 10, 3))
    f, lo, hi = _small_grid(orc)
    dm = I.cotangents((2, 3, 192), seed=13).astype(np.float64)
    _, gbn, gc = orc.adjoint(g, f, dm, want_grid=True)
    rng = np.random.default_rng(7)
    nz, ny, nx, _ = f.grid_bn.shape
    scale = max(np.abs(gbn * f.grid_bn).max(), np.abs(gc * f.grid_c).max())
    checked = 0
    for _ in range(60):
        iz, iy, ix, ch = rng.integers(nz), rng.integers(ny), rng.integers(nx), rng.integers(5)
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

        # small steps: B_perp and the Faraday phase make L strongly curved in a voxel
        h = 2.0 ** np.floor(np.log2(max(abs(v0), 1e-6) * 2e-5))
        fd = (4 * d(h / 2) - d(h)) / 3
        assert abs(fd - ana) * abs(v0) <= 1e-6 * scale + 1e-9 * abs(ana * v0), (idx, fd, ana)
        checked += abs(ana * v0) > 1e-3 * scale
    assert checked >= 10  # enough voxels on the sightlines carry weight


def test_grid_gradient_euler_identities(orc):
    g = orc.make_geom(4, 40, FREQS, box_lo=(-12, -10, -3), box_hi=(12, 10, 3))
    f, lo, hi = _small_grid(orc)
    dm = I.cotangents((2, 3, 192), seed=14).astype(np.float64)
    L = _loss(orc, g, f, dm)
    dth, gbn, gc = orc.adjoint(g, f, dm, want_grid=True)
    bn = f.grid_bn.astype(np.float64)
    assert (gc * f.grid_c).sum() == pytest.approx(L, rel=1e-12)
    lhs = (gbn[..., :3] * bn[..., :3]).sum() - (gbn[..., 3] * bn[..., 3]).sum()
    assert lhs == pytest.approx((THETA_T[12] + 1) / 2 * L, rel=1e-11)
    # alpha enters through the emissivity alone: its derivative matches FD
    th = THETA_T.copy()

    def loss_alpha(a):
        th2 = th.copy()
        th2[12] = a
        f2 = orc.Field(orc.GRID, th2, grid_bn=f.grid_bn, grid_c=f.grid_c, grid_lo=lo, grid_hi=hi)
        return _loss(orc, g, f2, dm)

    h = 1e-3
    d = lambda hh: (loss_alpha(th[12] + hh) - loss_alpha(th[12] - hh)) / (2 * hh)
    assert dth[12] == pytest.approx((4 * d(h / 2) - d(h)) / 3, rel=1e-7)


def test_grid_with_analytic_cr_gradient(orc):
    # grid B / n_e with analytic N0: the CR parameters get theta gradients
    g = orc.make_geom(4, 40, FREQS, box_lo=(-12, -10, -3), box_hi=(12, 10, 3))
    f, lo, hi = _small_grid(orc, with_c=False)
    dm = I.cotangents((2, 3, 192), seed=15).astype(np.float64)
    L = _loss(orc, g, f, dm)
    dth, gbn, gc = orc.adjoint(g, f, dm, want_grid=True)
    assert gc is None
    assert THETA_T[9] * dth[9] == pytest.approx(L, rel=1e-12)
    for k in (10, 11):
        def loss_k(v):
            th2 = THETA_T.copy()
            th2[k] = v
            f2 = orc.Field(orc.GRID, th2, grid_bn=f.grid_bn, grid_c=None, grid_lo=lo, grid_hi=hi)
            return _loss(orc, g, f2, dm)
        h = 1e-3 * THETA_T[k]
        d = lambda hh: (loss_k(THETA_T[k] + hh) - loss_k(THETA_T[k] - hh)) / (2 * hh)
        assert dth[k] == pytest.approx((4 * d(h / 2) - d(h)) / 3, rel=1e-7)
    # field parameters of the analytic model do not reach a gridded B / n_e
    assert np.all(dth[[0, 1, 2, 3, 4, 5, 6, 7, 8, 13, 14, 15]] == 0.0)
