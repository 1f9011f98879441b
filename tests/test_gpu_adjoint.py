"""GPU reverse pass vs the oracle's gradient (itself pinned by finite differences).

Tolerances (the maps agree to ~1e-6 relative; a gradient is a weighted sum over
residual-sized cotangents, so it amplifies map errors):
  * theta: per component |theta_k (g_gpu - g_ref)_k| <= 1e-3 max_k |theta_k g_ref_k|,
  * grid: relative L2 error <= 1e-3, cosine similarity >= 1 - 1e-6 and every
    voxel within 1e-3 of the largest gradient entry (parity.check_grid_gradient).
"""
import numpy as np
import pytest

from paper_2410_01136_amd import inputs as I
from parity import check_grid_gradient, oracle_geom

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
    def set_(kind, S, kernel=1):
        sm.set_lanes_per_ray(kernel, kind, S)
    yield set_
    for k in range(3):
        for kind in range(5):
            sm.set_lanes_per_ray(k, kind, 0)


def gpu_theta_grad(sm, g, field, dm):
    import torch
    geom = sm.geom_from(g)
    ws = sm.alloc_workspace(geom, field)
    sm.forward(geom, field, ws=ws)
    dth = sm.adjoint(geom, field, torch.from_numpy(dm).cuda(), ws)
    torch.cuda.synchronize()
    return dth.cpu().numpy()


def assert_theta_close(got, ref, theta, label):
    sk = np.maximum(np.abs(theta), 1e-2)
    err = np.abs(got - ref) * sk
    scale = np.abs(ref * sk).max()
    print(label, "max scaled err / scale", err.max() / scale, flush=True)
    assert np.all(err <= 1e-3 * scale), (label, err / scale)


@pytest.mark.parametrize("S", [1, 4, 8, 16, 64])
def test_theta_gradient_model16(sm, orc, lanes, S):
    g = I.geometry("C0", nside=8, n_steps=96, freqs_hz=(0.8e9, 1.4e9))
    dm = I.cotangents((2, 3, g.npix), seed=21)
    lanes(sm.FIELD_MODEL16, S)
    got = gpu_theta_grad(sm, g, sm.model16(THETA_T), dm)
    ref, _, _ = orc.adjoint(oracle_geom(orc, g), orc.Field(orc.MODEL16, THETA_T),
                            dm.astype(np.float64))
    assert_theta_close(got, ref, THETA_T, f"model16 S={S}")


def test_theta_gradient_without_piece_snapshots(sm, orc, lanes):
    # the forward ran with a one-lane reverse pass in force (no pieces, so no
    # piece snapshots); the reverse pass then splits each sightline into 8
    # pieces and finds their starting sums with a pre-pass of its own
    import torch
    g = I.geometry("C0", nside=8, n_steps=96, freqs_hz=(0.8e9, 1.4e9))
    dm = I.cotangents((2, 3, g.npix), seed=25)
    field = sm.model16(THETA_T)
    geom = sm.geom_from(g)
    lanes(sm.FIELD_MODEL16, 1)
    ws = sm.alloc_workspace(geom, field)
    sm.forward(geom, field, ws=ws)
    lanes(sm.FIELD_MODEL16, 8)
    got = sm.adjoint(geom, field, torch.from_numpy(dm).cuda(), ws).cpu().numpy()
    ref, _, _ = orc.adjoint(oracle_geom(orc, g), orc.Field(orc.MODEL16, THETA_T),
                            dm.astype(np.float64))
    assert_theta_close(got, ref, THETA_T, "model16, 8 pieces without snapshots")


def test_theta_gradient_alpha3_theta0(sm, orc):
    g = I.geometry("C2", nside=16, n_steps=128)
    dm = I.cotangents((1, 3, g.npix), seed=22)
    got = gpu_theta_grad(sm, g, sm.model16(I.THETA0), dm)
    ref, _, _ = orc.adjoint(oracle_geom(orc, g), orc.Field(orc.MODEL16, I.THETA0),
                            dm.astype(np.float64))
    assert_theta_close(got, ref, I.THETA0, "alpha=3 theta0")


def _grid(orc, n=(17, 17, 9), with_c=True):
    lo, hi = I.BOX_LO, I.BOX_HI
    reg_bn, reg_c = orc.sample_model16(THETA_T, n, lo, hi)
    bn = I.turbulent_grids(reg_bn, seeds=(2201, 2202, 2203, 2204), lo=lo, hi=hi)
    return bn, (reg_c if with_c else None)


# with a grid gradient, S > 1 splits each sightline into S contiguous pieces:
# 83 steps leave a short last piece at S = 4, 8 and 16, and empty pieces at 16 and 64
@pytest.mark.parametrize("S", [1, 4, 8, 16, 64])
@pytest.mark.parametrize("with_c", [True, False])
def test_grid_gradient(sm, orc, lanes, S, with_c):
    import torch
    g = I.geometry("C2", nside=8, n_steps=83, freqs_hz=(1.0e9, 1.4e9))
    bn, c = _grid(orc, with_c=with_c)
    dm = I.cotangents((2, 3, g.npix), seed=23)
    lanes(sm.FIELD_GRID, S)
    bn_t = torch.from_numpy(bn).cuda()
    c_t = torch.from_numpy(c).cuda() if with_c else None
    field = sm.grid(THETA_T, bn_t, c_t, I.BOX_LO, I.BOX_HI)
    geom = sm.geom_from(g)
    ws = sm.alloc_workspace(geom, field)
    sm.forward(geom, field, ws=ws)
    dbn = torch.zeros_like(bn_t)
    dc = torch.zeros_like(c_t) if with_c else None
    dth = sm.adjoint(geom, field, torch.from_numpy(dm).cuda(), ws, want_theta=True,
                     dgrid_bn=dbn, dgrid_c=dc)
    torch.cuda.synchronize()
    ofield = orc.Field(orc.GRID, THETA_T, grid_bn=bn, grid_c=c, grid_lo=I.BOX_LO, grid_hi=I.BOX_HI)
    rth, rbn, rc = orc.adjoint(oracle_geom(orc, g), ofield, dm.astype(np.float64), want_grid=True)
    got = dbn.cpu().numpy().astype(np.float64)
    pairs = [(got, rbn)]
    if with_c:
        pairs.append((dc.cpu().numpy().astype(np.float64), rc))
    for a, b in pairs:
        check_grid_gradient(a, b, f"grid S={S} with_c={with_c}")
    # alpha (and, with analytic N0, the CR parameters) get theta gradients too
    idx = [12] if with_c else [9, 10, 11, 12]
    th_got = dth.cpu().numpy()
    assert_theta_close(th_got[idx], rth[idx], THETA_T[idx], "grid theta")


def test_autograd_function_matches_adjoint(sm, orc):
    import torch
    g = I.geometry("C0", nside=4, n_steps=64)
    theta = torch.tensor(THETA_T, dtype=torch.float64, requires_grad=True)
    geom = sm.geom_from(g)
    maps = sm.march(theta, geom, sm.model16(THETA_T))
    dm = torch.from_numpy(I.cotangents(tuple(maps.shape), seed=24)).cuda()
    (maps * dm).sum().backward()
    ref, _, _ = orc.adjoint(oracle_geom(orc, g), orc.Field(orc.MODEL16, THETA_T),
                            dm.cpu().numpy().astype(np.float64))
    assert_theta_close(theta.grad.numpy(), ref, THETA_T, "autograd")


def test_theta_gradient_deterministic(sm):
    g = I.geometry("C0", nside=8, n_steps=64)
    dm = I.cotangents((1, 3, g.npix), seed=25)
    a = gpu_theta_grad(sm, g, sm.model16(THETA_T), dm)
    b = gpu_theta_grad(sm, g, sm.model16(THETA_T), dm)
    assert np.array_equal(a, b)


def test_chi2_kernel(sm):
    import torch
    rng = np.random.default_rng(31)
    maps = rng.standard_normal((2, 3, 3001)).astype(np.float32)
    tgt = rng.standard_normal((2, 3, 3001)).astype(np.float32)
    inv = rng.uniform(0.5, 2.0, (2, 3))
    c, dm = sm.chi2(torch.from_numpy(maps).cuda(), torch.from_numpy(tgt).cuda(), inv)
    r = maps.astype(np.float64) - tgt
    ref = (inv[..., None] * r * r).sum()
    assert c.item() == pytest.approx(ref, rel=1e-12)
    np.testing.assert_allclose(dm.cpu().numpy(), (2 * inv[..., None] * r).astype(np.float32),
                               rtol=1e-6)


@pytest.mark.slow
@pytest.mark.parametrize("S", [0, 1])
def test_c2_full_size_theta_gradient(sm, orc, lanes, S):
    """C2 at full size: chi^2 of I/Q/U against a target from perturbed parameters
    plus 1% noise, gradient at theta0 vs the oracle; with the built-in lane
    count and with one lane per sightline, whose FP32 theta sums run over all
    768 steps."""
    import torch
    lanes(sm.FIELD_MODEL16, S)
    g = I.geometry("C2")
    og = oracle_geom(orc, g)
    th_star = I.perturbed_thetas(1, 2001)[0]
    target, inv = I.chi2_noise(orc.forward(og, orc.Field(orc.MODEL16, th_star)), seed=2002)
    geom = sm.geom_from(g)
    field = sm.model16(I.THETA0)
    ws = sm.alloc_workspace(geom, field)
    maps = sm.forward(geom, field, ws=ws)
    chi, dm = sm.chi2(maps, torch.from_numpy(target).cuda(), inv)
    dth = sm.adjoint(geom, field, dm, ws).cpu().numpy()
    ref_maps = orc.forward(og, orc.Field(orc.MODEL16, I.THETA0))
    ref_dm = 2 * inv[..., None] * (ref_maps - target.astype(np.float64))
    ref, _, _ = orc.adjoint(og, orc.Field(orc.MODEL16, I.THETA0), ref_dm)
    assert chi.item() == pytest.approx((inv[..., None] * (ref_maps - target) ** 2).sum(), rel=1e-3)
    assert_theta_close(dth, ref, I.THETA0, "C2 full")


@pytest.mark.parametrize("S", [1, 4, 16])
def test_grid_gradient_sub_box(sm, orc, lanes, S):
    # grid box smaller than the geometry box, fewer nodes than the LDS box on z
    import torch
    lo, hi = (-12.0, -10.0, -3.0), (12.0, 10.0, 3.0)
    reg_bn, reg_c = orc.sample_model16(THETA_T, (21, 19, 7), lo, hi)
    bn = I.turbulent_grids(reg_bn, seeds=(2301, 2302, 2303, 2304), lo=lo, hi=hi)
    g = I.geometry("C2", nside=8, n_steps=64, freqs_hz=(1.4e9,))
    dm = I.cotangents((1, 3, g.npix), seed=26)
    lanes(sm.FIELD_GRID, S)
    bn_t, c_t = torch.from_numpy(bn).cuda(), torch.from_numpy(reg_c).cuda()
    field = sm.grid(THETA_T, bn_t, c_t, lo, hi)
    geom = sm.geom_from(g)
    ws = sm.alloc_workspace(geom, field)
    sm.forward(geom, field, ws=ws)
    dbn, dc = torch.zeros_like(bn_t), torch.zeros_like(c_t)
    sm.adjoint(geom, field, torch.from_numpy(dm).cuda(), ws, want_theta=False, dgrid_bn=dbn,
               dgrid_c=dc)
    torch.cuda.synchronize()
    ofield = orc.Field(orc.GRID, THETA_T, grid_bn=bn, grid_c=reg_c, grid_lo=lo, grid_hi=hi)
    _, rbn, rc = orc.adjoint(oracle_geom(orc, g), ofield, dm.astype(np.float64), want_grid=True)
    for a, b in ((dbn.cpu().numpy().astype(np.float64), rbn), (dc.cpu().numpy().astype(np.float64), rc)):
        check_grid_gradient(a, b, f"sub-box grid S={S}")


@pytest.mark.slow
@pytest.mark.parametrize("S", [0, 1])
def test_c2_full_size_grid_gradient(sm, orc, lanes, S):
    """C2 grid adjoint at full size (N_side 64, 768 steps, B and n_e on 128^3
    nodes sampled from theta0, analytic N0) in the built-in launch shape (S = 0)
    and with one lane per sightline, vs the oracle's gradient."""
    import torch
    g = I.geometry("C2")
    reg_bn, _ = orc.sample_model16(I.THETA0, (128, 128, 128), I.BOX_LO, I.BOX_HI)
    dm = I.cotangents((1, 3, g.npix), seed=27)
    if S:
        lanes(sm.FIELD_GRID, S)
    bn_t = torch.from_numpy(reg_bn).cuda()
    field = sm.grid(I.THETA0, bn_t, None, I.BOX_LO, I.BOX_HI)
    geom = sm.geom_from(g)
    ws = sm.alloc_workspace(geom, field)
    sm.forward(geom, field, ws=ws)
    dbn = torch.zeros_like(bn_t)
    sm.adjoint(geom, field, torch.from_numpy(dm).cuda(), ws, want_theta=False, dgrid_bn=dbn)
    torch.cuda.synchronize()
    ofield = orc.Field(orc.GRID, I.THETA0, grid_bn=reg_bn, grid_c=None, grid_lo=I.BOX_LO,
                       grid_hi=I.BOX_HI)
    _, rbn, _ = orc.adjoint(oracle_geom(orc, g), ofield, dm.astype(np.float64), want_grid=True)
    check_grid_gradient(dbn.cpu().numpy(), rbn,
                        f"C2 full grid S={sm.get_lanes_per_ray(1, sm.FIELD_GRID, g.npix)}")


def test_adjoint_refuses_a_mismatched_workspace(sm):
    """A workspace carries the tag of the forward that wrote it: an adjoint at
    other parameters or another geometry is refused, the matching one runs."""
    import torch
    g = I.geometry("C0", nside=4, n_steps=32)
    geom = sm.geom_from(g)
    f = sm.model16(THETA_T)
    ws = sm.alloc_workspace(geom, f)
    sm.forward(geom, f, ws=ws)
    dm = torch.from_numpy(I.cotangents((1, 3, g.npix), seed=28)).cuda()
    th2 = THETA_T.copy()
    th2[0] *= 1.01
    with pytest.raises(sm.SynError) as e:
        sm.adjoint(geom, sm.model16(th2), dm, ws)
    assert e.value.status == sm.SYN_EWORKSPACE
    geom2 = sm.geom_from(I.geometry("C0", nside=4, n_steps=33))
    with pytest.raises(sm.SynError) as e:
        sm.adjoint(geom2, f, dm, ws)
    assert e.value.status == sm.SYN_EWORKSPACE
    d = sm.adjoint(geom, f, dm, ws)
    torch.cuda.synchronize()
    assert torch.isfinite(d).all()
    # a forward under other parameters re-tags the workspace
    sm.forward(geom, sm.model16(th2), ws=ws)
    with pytest.raises(sm.SynError):
        sm.adjoint(geom, f, dm, ws)
    sm.adjoint(geom, sm.model16(th2), dm, ws)
    torch.cuda.synchronize()


@pytest.mark.parametrize("te", [0.0, 8000.0])
def test_grid_gradient_with_and_without_piece_snapshots(sm, orc, te):
    """A forward that a 4-piece grid-gradient pass will follow stores the sums at
    the piece ends; one run while the reverse pass was set to a single lane per
    sightline stores none, and the 4-piece pass then recomputes its pieces'
    sums itself.  Both agree with the oracle voxel by voxel (83 steps: a short
    last piece), with and without free-free."""
    import torch
    g = I.geometry("C2", nside=8, n_steps=83, freqs_hz=(0.9e9, 1.4e9))
    bn, c = _grid(orc)
    dm = I.cotangents((2, 3, g.npix), seed=29)
    bn_t, c_t = torch.from_numpy(bn).cuda(), torch.from_numpy(c).cuda()
    field = sm.grid(THETA_T, bn_t, c_t, I.BOX_LO, I.BOX_HI).with_te(te)
    geom = sm.geom_from(g)
    ofield = orc.Field(orc.GRID, THETA_T, grid_bn=bn, grid_c=c, grid_lo=I.BOX_LO, grid_hi=I.BOX_HI,
                       te_k=te)
    _, rbn, rc = orc.adjoint(oracle_geom(orc, g), ofield, dm.astype(np.float64), want_grid=True)
    out = []
    try:
        for fwd_lanes in (4, 1):
            sm.set_lanes_per_ray(sm.KERNEL_ADJOINT, sm.FIELD_GRID, fwd_lanes)
            ws = sm.alloc_workspace(geom, field)
            sm.forward(geom, field, ws=ws)
            sm.set_lanes_per_ray(sm.KERNEL_ADJOINT, sm.FIELD_GRID, 4)
            dbn, dc = torch.zeros_like(bn_t), torch.zeros_like(c_t)
            sm.adjoint(geom, field, torch.from_numpy(dm).cuda(), ws, want_theta=False, dgrid_bn=dbn,
                       dgrid_c=dc)
            torch.cuda.synchronize()
            label = "snapshots" if fwd_lanes == 4 else "pre-pass"
            check_grid_gradient(dbn.cpu().numpy(), rbn, f"grid te={te} {label} bn")
            check_grid_gradient(dc.cpu().numpy(), rc, f"grid te={te} {label} N0")
            out.append(dbn.cpu().numpy())
    finally:
        sm.set_lanes_per_ray(sm.KERNEL_ADJOINT, sm.FIELD_GRID, 0)
    a, b = out
    assert np.abs(a - b).max() <= 1e-4 * np.abs(b).max()
