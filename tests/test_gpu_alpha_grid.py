"""Gridded CR spectral index on the GPU vs the FP64 oracle, through the C ABI:
maps (forward tolerances of parity.py) on every grid read path, with and
without free-free, and the B / n_e / N0 and CR-parameter gradients
(tolerances of test_gpu_adjoint.py)."""
import numpy as np
import pytest

from paper_2410_01136_amd import inputs as I
from parity import check_grid_gradient, compare_maps, oracle_geom

pytestmark = pytest.mark.gpu

THETA_T = np.array([5.0, -0.25, 0.15, 0.35, 7.0, 1.2, 2.0, 1.4, 9.0,
                    4.2e-5, 7.5, 1.1, 2.85, 0.028, 0.9, 0.02])


@pytest.fixture(scope="module")
def sm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2410_01136_amd import binding
    return binding


@pytest.fixture
def lanes(sm):
    def set_(kind, S, kernel=0):
        sm.set_lanes_per_ray(kernel, kind, S)
    yield set_
    for k in range(3):
        for kind in range(5):
            sm.set_lanes_per_ray(k, kind, 0)


def fields(orc, n=(33, 33, 9), seed0=4201):
    """Turbulent B / n_e on the model, gridded N0, and a spectral index that
    steepens away from the plane (2.4 in the plane to 3.3 at |z| = 4 kpc) with
    a smooth random part."""
    reg_bn, reg_c = orc.sample_model16(THETA_T, n, I.BOX_LO, I.BOX_HI)
    bn = I.turbulent_grids(reg_bn, seeds=(seed0, seed0 + 1, seed0 + 2, seed0 + 3))
    nx, ny, nz = n
    z = np.linspace(I.BOX_LO[2], I.BOX_HI[2], nz)[:, None, None]
    rng = np.random.default_rng(seed0 + 9)
    alpha = 2.4 + 0.225 * np.abs(z) + 0.1 * rng.standard_normal((nz, ny, nx))
    return bn, reg_c, alpha.astype(np.float32)


def gpu_field(sm, bn, c, alpha, te=0.0):
    import torch
    return sm.grid(THETA_T, torch.from_numpy(bn).cuda(), torch.from_numpy(c).cuda(), I.BOX_LO,
                   I.BOX_HI, grid_alpha=torch.from_numpy(alpha).cuda()).with_te(te)


def ofield(orc, bn, c, alpha, te=0.0):
    return orc.Field(orc.GRID, THETA_T, grid_bn=bn, grid_c=c, grid_lo=I.BOX_LO, grid_hi=I.BOX_HI,
                     grid_alpha=alpha, te_k=te)


def check(gpu, ref, label):
    ok, rep = compare_maps(gpu, ref)
    print(label, rep, flush=True)
    assert ok, (label, rep)


@pytest.mark.parametrize("mode", [1, 2, 3])
# (at 0.4 GHz some sightlines through the turbulent n_e are Faraday-thick: Q and
# U cancel below the FP32 phase accuracy of the terms, with or without a
# gridded index; the low-frequency case is the weak-field one below)
@pytest.mark.parametrize("freqs", [(1.0e9, 1.4e9), (1.0e9, 2.3e9, 5.0e9)])
@pytest.mark.parametrize("S", [1, 16])
def test_forward(sm, orc, lanes, mode, freqs, S):
    import torch
    g = I.geometry("C1", nside=16, n_steps=117, freqs_hz=freqs)
    bn, c, alpha = fields(orc)
    lanes(sm.FIELD_GRID, S)
    sm.set_grid_addressing(mode)
    try:
        gpu = sm.forward(sm.geom_from(g), gpu_field(sm, bn, c, alpha))
        torch.cuda.synchronize()
        gpu = gpu.cpu().numpy()
    finally:
        sm.set_grid_addressing(0)
    ref = orc.forward(oracle_geom(orc, g), ofield(orc, bn, c, alpha))
    check(gpu, ref, f"alpha grid mode={mode} nf={len(freqs)} S={S}")


@pytest.mark.parametrize("n", [(33, 33, 9), (9, 9, 129)])
def test_shared_reads_carry_alpha(sm, orc, lanes, n):
    # the shared-read path brings alpha in the cells' LDS records; on the fine
    # z grid most chunks hold more distinct cells than the LDS slots and read
    # their cells per lane: both meet the oracle, and agree with the per-lane
    # path to FP32 rounding (which the general-alpha emission and depolarised
    # Q/U amplify a little more than the alpha = 3 march does)
    import torch
    g = I.geometry("C1", nside=16, n_steps=117, freqs_hz=(1.0e9, 2.3e9, 5.0e9))
    bn, c, alpha = fields(orc, n=n)
    lanes(sm.FIELD_GRID, 16)
    out = []
    try:
        for mode in (3, 2):
            sm.set_grid_addressing(mode)
            out.append(sm.forward(sm.geom_from(g), gpu_field(sm, bn, c, alpha)).cpu().numpy())
    finally:
        sm.set_grid_addressing(0)
    ref = orc.forward(oracle_geom(orc, g), ofield(orc, bn, c, alpha))
    check(out[0], ref, f"alpha grid shared n={n}")
    err = np.abs(out[0] - out[1]).max(axis=-1) / np.abs(out[1]).max(axis=-1)
    print(f"alpha shared vs per-lane n={n}: max rel diff {err.max():.2e}", flush=True)
    assert err.max() <= 1e-5, (n, err)


# dense thermal plasma, weak field, strong CR density (as in test_gpu_ff.py)
THETA_FF = np.array([0.005, -0.25, 0.15, 0.35, 7.0, 1.2, 0.002, 1.4, 9.0,
                     42.0, 7.5, 1.1, 2.85, 3.0, 0.9, 0.02])


@pytest.mark.parametrize("S", [1, 16])
def test_forward_with_free_free_at_low_frequency(sm, orc, lanes, S):
    import torch
    g = I.geometry("C2", nside=8, n_steps=83, freqs_hz=(0.15e9, 0.3e9, 0.6e9), r_max=3.0)
    reg_bn, reg_c = orc.sample_model16(THETA_FF, (33, 33, 9), I.BOX_LO, I.BOX_HI)
    bn = I.turbulent_grids(reg_bn, seeds=(4301, 4302, 4303, 4304))
    bn[..., 3] = np.abs(bn[..., 3])
    _, _, alpha = fields(orc)
    lanes(sm.FIELD_GRID, S)
    field = sm.grid(THETA_FF, torch.from_numpy(bn).cuda(), torch.from_numpy(reg_c).cuda(),
                    I.BOX_LO, I.BOX_HI, grid_alpha=torch.from_numpy(alpha).cuda()).with_te(8000.0)
    gpu = sm.forward(sm.geom_from(g), field)
    torch.cuda.synchronize()
    of = orc.Field(orc.GRID, THETA_FF, grid_bn=bn, grid_c=reg_c, grid_lo=I.BOX_LO,
                   grid_hi=I.BOX_HI, grid_alpha=alpha, te_k=8000.0)
    ref = orc.forward(oracle_geom(orc, g), of)
    check(gpu.cpu().numpy(), ref, f"alpha grid + free-free S={S}")


def test_constant_index_grid_is_the_plain_march(sm, orc):
    import torch
    g = I.geometry("C1", nside=16, n_steps=117, freqs_hz=(0.4e9, 1.4e9))
    bn, c, _ = fields(orc)
    th = THETA_T.copy()
    th[12] = 2.625  # exact in FP32
    alpha = np.full(c.shape, th[12], dtype=np.float32)
    b, cc = torch.from_numpy(bn).cuda(), torch.from_numpy(c).cuda()
    plain = sm.forward(sm.geom_from(g), sm.grid(th, b, cc, I.BOX_LO, I.BOX_HI))
    va = sm.forward(sm.geom_from(g), sm.grid(th, b, cc, I.BOX_LO, I.BOX_HI,
                                             grid_alpha=torch.from_numpy(alpha).cuda()))
    torch.cuda.synchronize()
    check(va.cpu().numpy(), plain.cpu().numpy().astype(np.float64), "constant alpha grid vs plain")


@pytest.mark.parametrize("te", [0.0, 8000.0])
@pytest.mark.parametrize("S", [1, 4, 16])
def test_grid_gradient(sm, orc, lanes, S, te):
    import torch
    g = I.geometry("C2", nside=8, n_steps=83, freqs_hz=(0.6e9, 1.4e9))
    bn, c, alpha = fields(orc, n=(17, 17, 9))
    if te:
        bn[..., 3] = np.abs(bn[..., 3]) * 10.0
    dm = I.cotangents((2, 3, g.npix), seed=51)
    lanes(sm.FIELD_GRID, S, kernel=1)
    field = gpu_field(sm, bn, c, alpha, te)
    geom = sm.geom_from(g)
    ws = sm.alloc_workspace(geom, field)
    sm.forward(geom, field, ws=ws)
    dbn, dc = torch.zeros_like(field.grid_bn), torch.zeros_like(field.grid_c)
    dth = sm.adjoint(geom, field, torch.from_numpy(dm).cuda(), ws, want_theta=True, dgrid_bn=dbn,
                     dgrid_c=dc)
    torch.cuda.synchronize()
    rth, rbn, rc = orc.adjoint(oracle_geom(orc, g), ofield(orc, bn, c, alpha, te),
                               dm.astype(np.float64), want_grid=True)
    assert dth.cpu().numpy()[12] == 0.0 and rth[12] == 0.0
    for a, b, lab in ((dbn.cpu().numpy().astype(np.float64), rbn, "bn"),
                      (dc.cpu().numpy().astype(np.float64), rc, "N0")):
        check_grid_gradient(a, b, f"alpha grid S={S} te={te} {lab}")


def test_theta_gradient_with_analytic_cr(sm, orc):
    # gridded B / n_e / alpha with the analytic N0: theta 9-11 get gradients
    import torch
    g = I.geometry("C2", nside=8, n_steps=96, freqs_hz=(0.6e9, 1.4e9))
    bn, _, alpha = fields(orc, n=(17, 17, 9))
    dm = I.cotangents((2, 3, g.npix), seed=52)
    field = sm.grid(THETA_T, torch.from_numpy(bn).cuda(), None, I.BOX_LO, I.BOX_HI,
                    grid_alpha=torch.from_numpy(alpha).cuda())
    geom = sm.geom_from(g)
    ws = sm.alloc_workspace(geom, field)
    sm.forward(geom, field, ws=ws)
    dth = sm.adjoint(geom, field, torch.from_numpy(dm).cuda(), ws).cpu().numpy()
    of = orc.Field(orc.GRID, THETA_T, grid_bn=bn, grid_c=None, grid_lo=I.BOX_LO, grid_hi=I.BOX_HI,
                   grid_alpha=alpha)
    rth, _, _ = orc.adjoint(oracle_geom(orc, g), of, dm.astype(np.float64))
    idx = [9, 10, 11]
    err = np.abs(dth[idx] - rth[idx]) * THETA_T[idx]
    scale = np.abs(rth[idx] * THETA_T[idx]).max()
    print("alpha grid theta 9-11: max scaled err / scale", err.max() / scale, flush=True)
    assert np.all(err <= 1e-3 * scale)
    assert dth[12] == 0.0


@pytest.mark.parametrize("n_steps,S", [(1, 16), (3, 64), (29, 4)])
def test_tiny_and_ragged_schedules(sm, orc, lanes, n_steps, S):
    import torch
    g = I.geometry("C2", nside=2, n_steps=n_steps, freqs_hz=(1.0e9, 1.4e9))
    bn, c, alpha = fields(orc, n=(17, 17, 9))
    lanes(sm.FIELD_GRID, S)
    lanes(sm.FIELD_GRID, S, kernel=1)
    field = gpu_field(sm, bn, c, alpha)
    geom = sm.geom_from(g)
    ws = sm.alloc_workspace(geom, field)
    maps = sm.forward(geom, field, ws=ws)
    dm = I.cotangents((2, 3, g.npix), seed=53)
    dbn = torch.zeros_like(field.grid_bn)
    sm.adjoint(geom, field, torch.from_numpy(dm).cuda(), ws, want_theta=False, dgrid_bn=dbn)
    torch.cuda.synchronize()
    of = ofield(orc, bn, c, alpha)
    check(maps.cpu().numpy(), orc.forward(oracle_geom(orc, g), of), f"alpha n={n_steps} S={S}")
    _, rbn, _ = orc.adjoint(oracle_geom(orc, g), of, dm.astype(np.float64), want_grid=True)
    check_grid_gradient(dbn.cpu().numpy(), rbn, f"alpha grid n={n_steps} S={S}")
