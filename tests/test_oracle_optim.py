"""Pins of the grid-fitting reference (Adam of Kingma & Ba 2015; chi^2 of Sec. 3.1)."""
import numpy as np
import pytest

from oracle import optim


def test_adam_first_step_closed_form():
    # t = 1 from zero moments: m_hat = g, v_hat = g^2, so the step is lr g / (|g| + eps)
    rng = np.random.default_rng(1)
    g = rng.standard_normal(50) * 10.0 ** rng.uniform(-6, 3, 50)
    p0 = rng.standard_normal(50)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    optim.adam_step(p, g, m, v, 1, lr=0.3, eps=1e-8)
    np.testing.assert_allclose(p, p0 - 0.3 * g / (np.abs(g) + 1e-8), rtol=1e-13, atol=1e-15)


def test_adam_constant_gradient_steps_are_constant():
    # with a constant gradient the bias corrections make m_hat = g and v_hat = g^2 at every t
    g = np.array([2.0, -0.5, 1e-3, -7.0])
    p, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    prev = p.copy()
    for t in range(1, 12):
        optim.adam_step(p, g, m, v, t, lr=0.01, beta1=0.8, beta2=0.95, eps=1e-12)
        np.testing.assert_allclose(p - prev, -0.01 * g / (np.abs(g) + 1e-12), rtol=1e-9)
        prev = p.copy()


def test_adam_minimises_a_quadratic():
    rng = np.random.default_rng(2)
    a = rng.standard_normal(20) * 3.0
    x, m, v = np.zeros(20), np.zeros(20), np.zeros(20)
    for t in range(1, 3001):
        optim.adam_step(x, 2.0 * (x - a), m, v, t, lr=0.02)
    assert np.abs(x - a).max() < 2e-2


def test_adam_mask_selects_channels():
    p = np.arange(12, dtype=np.float64)
    g = np.ones(12)
    m, v = np.zeros(12), np.zeros(12)
    optim.adam_step(p, g, m, v, 1, lr=1.0, period=4, mask=0b0101)
    changed = p != np.arange(12)
    assert changed.tolist() == [True, False, True, False] * 3
    assert np.all(m[~changed] == 0) and np.all(v[~changed] == 0)


def test_chi2_gradient_matches_differences():
    rng = np.random.default_rng(3)
    maps = rng.standard_normal((2, 3, 7))
    tgt = rng.standard_normal((2, 3, 7))
    inv = rng.uniform(0.5, 2.0, (2, 3))
    c, d = optim.chi2(maps, tgt, inv)
    assert optim.chi2(tgt, tgt, inv)[0] == 0.0
    h = 1e-6
    for idx in [(0, 0, 0), (1, 2, 6), (0, 1, 3)]:
        e = np.zeros_like(maps)
        e[idx] = h
        fd = (optim.chi2(maps + e, tgt, inv)[0] - optim.chi2(maps - e, tgt, inv)[0]) / (2 * h)
        assert fd == pytest.approx(d[idx], rel=1e-7)


def test_fit_grid_reduces_chi2(orc):
    # a few oracle iterations on a tiny problem lower chi^2 (descent property)
    from paper_2410_01136_amd import inputs as I
    from parity import oracle_geom
    g = I.geometry("C0", nside=2, n_steps=24, freqs_hz=(2.4e9,))
    lo, hi = (-12.0, -12.0, -3.0), (12.0, 12.0, 3.0)
    og = oracle_geom(orc, g)
    reg, _ = orc.sample_model16(I.THETA0, (7, 7, 5), lo, hi)
    true = I.turbulent_grids(reg, seeds=(71, 72, 73, 74), lo=lo, hi=hi)
    tgt = orc.forward(og, orc.Field(orc.GRID, I.THETA0, grid_bn=true, grid_c=None, grid_lo=lo, grid_hi=hi))
    inv = 1.0 / (0.01 * np.sqrt((tgt ** 2).mean(-1))) ** 2
    hist, fitted = optim.fit_grid(orc, og, I.THETA0, reg, lo, hi, tgt, inv, iters=6, lr=0.05)
    assert np.all(np.diff(hist) < 0) and hist[-1] < 0.9 * hist[0]
    assert np.array_equal(fitted[..., 3], reg[..., 3].astype(np.float64))  # n_e untouched
