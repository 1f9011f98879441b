"""Adam on the GPU (syn_adam_step) against the FP64 reference, and the grid-fitting
loop of Sec. 3.3 (forward, chi^2, grid adjoint, Adam) against the oracle's loop.

Tolerances: Adam runs in FP32, so parameters and moments after each step agree
with the FP64 reference to a few FP32 roundings (1e-5 of the step taken; 1e-6
of the largest gradient, or its square, for the moments).  In the loop the first chi^2 is the map parity; later ones also
carry the FP32-vs-FP64 gradient difference through Adam's normalised steps, so
they are compared to 1e-3 relative.
"""
import numpy as np
import pytest

from oracle import optim
from paper_2410_01136_amd import inputs as I
from parity import oracle_geom

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2410_01136_amd import binding
    return binding


@pytest.mark.parametrize("n,period,mask", [(4096, 4, 0b0111), (1001, 1, 1), (777, 3, 0b101),
                                           (4, 4, 0b1000), (1, 1, 1)])
def test_adam_steps_match_reference(sm, n, period, mask):
    import torch
    rng = np.random.default_rng(n)
    p0 = rng.standard_normal(n).astype(np.float32)
    grads = [(rng.standard_normal(n) * 10.0 ** rng.uniform(-4, 1, n)).astype(np.float32)
             for _ in range(4)]
    p, m, v = (torch.from_numpy(x.copy()).cuda() for x in (p0, np.zeros(n, np.float32),
                                                           np.zeros(n, np.float32)))
    rp, rm, rv = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    for t, g in enumerate(grads, start=1):
        sm.adam_step(p, torch.from_numpy(g).cuda(), m, v, t, lr=0.01, beta1=0.9, beta2=0.99,
                     eps=1e-6, period=period, mask=mask)
        optim.adam_step(rp, g.astype(np.float64), rm, rv, t, lr=0.01, beta1=0.9, beta2=0.99,
                        eps=1e-6, period=period, mask=mask)
    torch.cuda.synchronize()
    gp, gm, gv = (x.cpu().numpy().astype(np.float64) for x in (p, m, v))
    sel = ((mask >> (np.arange(n) % period)) & 1).astype(bool)
    assert np.array_equal(gp[~sel], p0[~sel].astype(np.float64))  # untouched, bit for bit
    assert np.all(gm[~sel] == 0) and np.all(gv[~sel] == 0)
    step = np.abs(rp - p0)
    assert np.all(np.abs(gp - rp) <= 1e-5 * step + 2e-7 * np.abs(p0) + 1e-12)
    # moments are weighted sums of the gradients: compare on the scale of the
    # largest gradient each element saw (cancellation makes relative errors of
    # small moments meaningless)
    gmax = np.max(np.abs(np.stack(grads)), axis=0).astype(np.float64)
    assert np.all(np.abs(gm - rm) <= 1e-6 * gmax)
    assert np.all(np.abs(gv - rv) <= 1e-6 * gmax ** 2)


def test_grid_fit_loop_matches_oracle_loop(sm, orc):
    import torch
    from paper_2410_01136_amd import optimize
    g = I.geometry("C0", nside=4, n_steps=48, freqs_hz=(2.4e9,))
    lo, hi = (-12.0, -12.0, -3.0), (12.0, 12.0, 3.0)
    og = oracle_geom(orc, g)
    reg, _ = orc.sample_model16(I.THETA0, (9, 9, 5), lo, hi)
    true = I.turbulent_grids(reg, seeds=(81, 82, 83, 84), lo=lo, hi=hi)
    tgt = orc.forward(og, orc.Field(orc.GRID, I.THETA0, grid_bn=true, grid_c=None, grid_lo=lo,
                                    grid_hi=hi))
    inv = 1.0 / (0.01 * np.sqrt((tgt ** 2).mean(-1))) ** 2
    ref_hist, ref_grid = optim.fit_grid(orc, og, I.THETA0, reg, lo, hi, tgt, inv, iters=4, lr=0.05)
    res = optimize.fit_grid(sm.geom_from(g), I.THETA0, torch.from_numpy(reg).cuda(), lo, hi,
                            torch.from_numpy(tgt.astype(np.float32)).cuda(), inv, iters=4, lr=0.05)
    hist = res["chi2"]
    print("chi2 gpu", hist, "oracle", ref_hist, flush=True)
    assert hist[0] == pytest.approx(ref_hist[0], rel=1e-4)
    np.testing.assert_allclose(hist, ref_hist, rtol=1e-3)
    fitted = res["grid"].cpu().numpy()
    assert np.array_equal(fitted[..., 3], reg[..., 3])  # n_e never updated
    moved = np.abs(ref_grid[..., :3] - reg[..., :3])
    assert np.median(np.abs(fitted[..., :3] - ref_grid[..., :3])[moved > 0] / moved[moved > 0]) < 1e-2
