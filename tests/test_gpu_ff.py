"""Free-free emission and absorption on the GPU vs the FP64 oracle, through the
C ABI: maps of every field kind (to the forward tolerances of parity.py) and
the theta and grid gradients (to the tolerances of test_gpu_adjoint.py)."""
import numpy as np
import pytest

from paper_2410_01136_amd import inputs as I
from parity import FP32_TERMS, check_grid_gradient, compare_maps, oracle_geom

pytestmark = pytest.mark.gpu

TE = 8000.0
# dense thermal plasma (tau ~ 0.2-0.7 at 150 MHz over 2-3 kpc), weak field
# (Faraday phases of a few hundred rad), strong CR density
THETA_FF = np.array([0.005, -0.25, 0.15, 0.35, 7.0, 1.2, 0.002, 1.4, 9.0,
                     42.0, 7.5, 1.1, 2.85, 3.0, 0.9, 0.02])
FREQS_FF = (0.15e9, 0.3e9)


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


def gpu_maps(sm, g, field):
    import torch
    maps = sm.forward(sm.geom_from(g), field)
    torch.cuda.synchronize()
    return maps.cpu().numpy()


def check(gpu, ref, label, floor=0.0, max_floor=0):
    ok, rep = compare_maps(gpu, ref, floor=floor, max_floor=max_floor)
    print(label, rep, flush=True)
    assert ok, (label, rep)


@pytest.mark.parametrize("S", [1, 4, 8, 16, 64])
def test_model16_dense_plasma(sm, orc, lanes, S):
    g = I.geometry("C0", nside=8, n_steps=83, freqs_hz=FREQS_FF, r_max=2.0)
    lanes(sm.FIELD_MODEL16, S)
    ref = orc.forward(oracle_geom(orc, g), orc.Field(orc.MODEL16, THETA_FF, te_k=TE))
    plain = orc.forward(oracle_geom(orc, g), orc.Field(orc.MODEL16, THETA_FF))
    assert np.abs(ref[:, 0] / plain[:, 0] - 1).max() > 0.05  # the effect is large here
    check(gpu_maps(sm, g, sm.model16(THETA_FF).with_te(TE)), ref, f"model16 ff S={S}")


# Below ~0.3 GHz the disk model at theta0 is Faraday-thick: Q and U cancel to
# ~1e-3 of the sum of their terms, and the FP32 phase of each term (~6e-8 rad)
# then exceeds 1e-4 PI, with or without free-free; those frequencies are
# covered by the dense-plasma, weak-field cases instead.
@pytest.mark.parametrize("freqs", [(0.4e9, 1.4e9), (0.3e9, 0.408e9, 0.6e9), tuple(np.linspace(0.3e9, 1e9, 6))])
def test_model16_theta0_low_frequencies(sm, orc, freqs):
    # the disk model at its own parameters: thin free-free on top of synchrotron,
    # two and three (four-slot) and six (sixteen-slot) frequencies
    g = I.geometry("C0", freqs_hz=freqs)
    ref = orc.forward(oracle_geom(orc, g), orc.Field(orc.MODEL16, I.THETA0, te_k=TE))
    # (the disk model's most depolarised pixels: the declared FP32 term floor,
    # at most 0.1% of the pixels of each frequency)
    check(gpu_maps(sm, g, sm.model16(I.THETA0).with_te(TE)), ref, f"theta0 ff {len(freqs)} freqs",
          FP32_TERMS, 3 * len(freqs))


def dense_grid(orc, n=(33, 33, 9), lo=I.BOX_LO, hi=I.BOX_HI, seed0=4101):
    reg_bn, reg_c = orc.sample_model16(THETA_FF, n, lo, hi)
    bn = I.turbulent_grids(reg_bn, seeds=(seed0, seed0 + 1, seed0 + 2, seed0 + 3), lo=lo, hi=hi)
    bn[..., 3] = np.abs(bn[..., 3])
    return bn, reg_c


@pytest.mark.parametrize("mode", [1, 2, 3])
@pytest.mark.parametrize("S", [1, 16])
def test_grid_read_paths(sm, orc, lanes, mode, S):
    # 64-bit addresses, per-lane buffer reads and shared reads through LDS
    import torch
    g = I.geometry("C2", nside=8, n_steps=83, freqs_hz=FREQS_FF, r_max=3.0)
    bn, c = dense_grid(orc)
    lanes(sm.FIELD_GRID, S)
    sm.set_grid_addressing(mode)
    try:
        field = sm.grid(THETA_FF, torch.from_numpy(bn).cuda(), torch.from_numpy(c).cuda(),
                        I.BOX_LO, I.BOX_HI).with_te(TE)
        gpu = gpu_maps(sm, g, field)
    finally:
        sm.set_grid_addressing(0)
    ref = orc.forward(oracle_geom(orc, g), orc.Field(orc.GRID, THETA_FF, grid_bn=bn, grid_c=c,
                                                     grid_lo=I.BOX_LO, grid_hi=I.BOX_HI, te_k=TE))
    check(gpu, ref, f"grid ff mode={mode} S={S}")


def test_sphere_and_wmap(sm, orc):
    g = I.geometry("E1", nside=8, n_steps=128, freqs_hz=(0.1e9, 0.3e9))
    th = I.sphere_theta(ne=2.0)
    ref = orc.forward(oracle_geom(orc, g), orc.Field(orc.SPHERE, th, te_k=TE))
    check(gpu_maps(sm, g, sm.sphere(th).with_te(TE)), ref, "sphere ff")
    g = I.geometry("G1", nside=8, n_steps=128, freqs_hz=(0.408e9, 0.6e9))
    th = I.wmap_theta()
    ref = orc.forward(oracle_geom(orc, g), orc.Field(orc.WMAP, th, te_k=TE))
    check(gpu_maps(sm, g, sm.wmap(th).with_te(TE)), ref, "wmap ff")


def test_full_size_c1_geometry_sampled(sm, orc):
    """The headline geometry (N_side 256, 512 steps, three frequencies) at radio
    frequencies where free-free matters, analytic disk model, sampled pixels."""
    g = I.geometry("C1", freqs_hz=(0.408e9, 0.6e9, 1.0e9))
    gpu = gpu_maps(sm, g, sm.model16(I.THETA0).with_te(TE))
    pix = I.sample_pixels(g.npix, 3000, seed=78)
    ref = orc.forward_pixels(oracle_geom(orc, g), orc.Field(orc.MODEL16, I.THETA0, te_k=TE), pix)
    check(gpu[:, :, pix], np.transpose(ref, (1, 2, 0)), "C1 geometry ff sampled")


def _theta_grad(sm, g, field, dm):
    import torch
    geom = sm.geom_from(g)
    ws = sm.alloc_workspace(geom, field)
    sm.forward(geom, field, ws=ws)
    dth = sm.adjoint(geom, field, torch.from_numpy(dm).cuda(), ws)
    torch.cuda.synchronize()
    return dth.cpu().numpy()


def assert_theta_close(got, ref, theta, label, idx=range(16)):
    idx = list(idx)
    sk = np.maximum(np.abs(theta), 1e-2)[idx]
    err = np.abs(got[idx] - ref[idx]) * sk
    scale = np.abs(ref[idx] * sk).max()
    print(label, "max scaled err / scale", err.max() / scale, flush=True)
    assert np.all(err <= 1e-3 * scale), (label, err / scale)


@pytest.mark.parametrize("S", [1, 4, 16])
def test_theta_gradient_model16(sm, orc, lanes, S):
    g = I.geometry("C0", nside=8, n_steps=83, freqs_hz=FREQS_FF, r_max=2.0)
    dm = I.cotangents((2, 3, g.npix), seed=41)
    lanes(sm.FIELD_MODEL16, S, kernel=1)
    got = _theta_grad(sm, g, sm.model16(THETA_FF).with_te(TE), dm)
    ref, _, _ = orc.adjoint(oracle_geom(orc, g), orc.Field(orc.MODEL16, THETA_FF, te_k=TE),
                            dm.astype(np.float64))
    assert_theta_close(got, ref, THETA_FF, f"model16 ff grad S={S}")


def test_theta_gradient_wmap(sm, orc):
    g = I.geometry("G1", nside=8, n_steps=96, freqs_hz=(0.408e9, 0.6e9))
    th = I.wmap_theta()
    th[13] = 0.3  # denser thermal disk: absorption at the per-cent level
    dm = I.cotangents((2, 3, g.npix), seed=42)
    got = _theta_grad(sm, g, sm.wmap(th).with_te(TE), dm)
    ref, _, _ = orc.adjoint(oracle_geom(orc, g), orc.Field(orc.WMAP, th, te_k=TE),
                            dm.astype(np.float64))
    live = [0, 1, 2, 3, 9, 10, 11, 12, 13, 14, 15]
    assert_theta_close(got, ref, th, "wmap ff grad", live)


@pytest.mark.parametrize("S", [1, 4, 16])
def test_grid_gradient(sm, orc, lanes, S):
    # with a grid gradient S > 1 splits sightlines into pieces, which carry the
    # emission-measure sums and their cotangents across pieces
    import torch
    g = I.geometry("C2", nside=8, n_steps=83, freqs_hz=FREQS_FF, r_max=3.0)
    bn, c = dense_grid(orc, n=(17, 17, 9))
    dm = I.cotangents((2, 3, g.npix), seed=43)
    lanes(sm.FIELD_GRID, S, kernel=1)
    bn_t, c_t = torch.from_numpy(bn).cuda(), torch.from_numpy(c).cuda()
    field = sm.grid(THETA_FF, bn_t, c_t, I.BOX_LO, I.BOX_HI).with_te(TE)
    geom = sm.geom_from(g)
    ws = sm.alloc_workspace(geom, field)
    sm.forward(geom, field, ws=ws)
    dbn, dc = torch.zeros_like(bn_t), torch.zeros_like(c_t)
    sm.adjoint(geom, field, torch.from_numpy(dm).cuda(), ws, want_theta=False, dgrid_bn=dbn,
               dgrid_c=dc)
    torch.cuda.synchronize()
    of = orc.Field(orc.GRID, THETA_FF, grid_bn=bn, grid_c=c, grid_lo=I.BOX_LO, grid_hi=I.BOX_HI,
                   te_k=TE)
    _, rbn, rc = orc.adjoint(oracle_geom(orc, g), of, dm.astype(np.float64), want_grid=True)
    got = dbn.cpu().numpy().astype(np.float64)
    for a, b, lab in ((got, rbn, "bn"), (got[..., 3], rbn[..., 3], "n_e"),
                      (dc.cpu().numpy().astype(np.float64), rc, "N0")):
        check_grid_gradient(a, b, f"grid ff S={S} {lab}")


@pytest.mark.parametrize("n_steps,S", [(1, 16), (1, 1), (3, 64), (17, 4)])
def test_tiny_and_ragged_schedules(sm, orc, lanes, n_steps, S):
    # one step (the attenuation of a lone midpoint is e^{-tau/2}), fewer steps
    # than lanes, a ragged last chunk; forward and theta-gradient
    g = I.geometry("C0", nside=1, n_steps=n_steps, freqs_hz=FREQS_FF, r_max=2.0)
    lanes(sm.FIELD_MODEL16, S)
    lanes(sm.FIELD_MODEL16, S, kernel=1)
    ref = orc.forward(oracle_geom(orc, g), orc.Field(orc.MODEL16, THETA_FF, te_k=TE))
    check(gpu_maps(sm, g, sm.model16(THETA_FF).with_te(TE)), ref, f"ff n={n_steps} S={S}")
    dm = I.cotangents((2, 3, g.npix), seed=44)
    got = _theta_grad(sm, g, sm.model16(THETA_FF).with_te(TE), dm)
    rth, _, _ = orc.adjoint(oracle_geom(orc, g), orc.Field(orc.MODEL16, THETA_FF, te_k=TE),
                            dm.astype(np.float64))
    assert_theta_close(got, rth, THETA_FF, f"ff grad n={n_steps} S={S}")


@pytest.mark.parametrize("S", [1, 64])
def test_grid_gradient_few_steps(sm, orc, lanes, S):
    # 5 steps over 64 pieces: most pieces empty, the rest one step long
    import torch
    g = I.geometry("C2", nside=2, n_steps=5, freqs_hz=FREQS_FF, r_max=3.0)
    bn, c = dense_grid(orc, n=(9, 9, 5))
    dm = I.cotangents((2, 3, g.npix), seed=45)
    lanes(sm.FIELD_GRID, S, kernel=1)
    bn_t, c_t = torch.from_numpy(bn).cuda(), torch.from_numpy(c).cuda()
    field = sm.grid(THETA_FF, bn_t, c_t, I.BOX_LO, I.BOX_HI).with_te(TE)
    geom = sm.geom_from(g)
    ws = sm.alloc_workspace(geom, field)
    sm.forward(geom, field, ws=ws)
    dbn, dc = torch.zeros_like(bn_t), torch.zeros_like(c_t)
    sm.adjoint(geom, field, torch.from_numpy(dm).cuda(), ws, want_theta=False, dgrid_bn=dbn,
               dgrid_c=dc)
    torch.cuda.synchronize()
    of = orc.Field(orc.GRID, THETA_FF, grid_bn=bn, grid_c=c, grid_lo=I.BOX_LO, grid_hi=I.BOX_HI,
                   te_k=TE)
    _, rbn, rc = orc.adjoint(oracle_geom(orc, g), of, dm.astype(np.float64), want_grid=True)
    for a, b in ((dbn.cpu().numpy().astype(np.float64), rbn), (dc.cpu().numpy().astype(np.float64), rc)):
        check_grid_gradient(a, b, f"few-step grid ff S={S}")


@pytest.mark.slow
def test_bench_theta_workload(sm, orc):
    """The benchmark's analytic free-free leg as it runs: N_side 64, 768 steps,
    40 x 40 x 8 kpc box, theta0, T_e 8000 K at {0.6, 0.8, 1.0} GHz, forward and
    theta-adjoint of the benchmark's cotangents; maps strict except the disk
    model's most depolarised pixels (declared FP32 term floor, at most 0.1% of
    each frequency's pixels)."""
    import torch
    g = I.geometry("C2", freqs_hz=I.FF_THETA_FREQS)
    nf = len(g.freqs_hz)
    field = sm.model16(I.THETA0).with_te(I.TE_FF)
    geom = sm.geom_from(g)
    ws = sm.alloc_workspace(geom, field)
    maps = sm.forward(geom, field, ws=ws)
    dm = I.cotangents((nf, 3, g.npix), seed=7001)
    dth = sm.adjoint(geom, field, torch.from_numpy(dm).cuda(), ws)
    torch.cuda.synchronize()
    og = oracle_geom(orc, g)
    of = orc.Field(orc.MODEL16, I.THETA0, te_k=I.TE_FF)
    check(maps.cpu().numpy(), orc.forward(og, of), "bench theta ff", FP32_TERMS, nf * g.npix // 1000)
    ref, _, _ = orc.adjoint(og, of, dm.astype(np.float64))
    assert_theta_close(dth.cpu().numpy(), ref, I.THETA0, "bench theta ff gradient")


@pytest.mark.slow
def test_bench_grid_workload(sm, orc, c1_grids):
    """The benchmark's gridded free-free leg as it runs: the 256^3 headline
    grids at N_side 256, 512 steps, {150, 300, 600} MHz, T_e 8000 K, in the
    built-in launch shape; 1500 sampled pixels against the oracle (declared FP32
    term floor for at most 1% of them per frequency)."""
    import torch
    g = I.geometry("C1", freqs_hz=I.FF_GRID_FREQS)
    bn, c = c1_grids
    f = sm.grid(I.THETA0, torch.from_numpy(bn).cuda(), torch.from_numpy(c).cuda(), I.BOX_LO,
                I.BOX_HI).with_te(I.TE_FF)
    gpu = gpu_maps(sm, g, f)
    pix = I.sample_pixels(g.npix, 1500, seed=79)
    ref = orc.forward_pixels(oracle_geom(orc, g), orc.Field(orc.GRID, I.THETA0, grid_bn=bn, grid_c=c,
                                                            grid_lo=I.BOX_LO, grid_hi=I.BOX_HI,
                                                            te_k=I.TE_FF), pix)
    check(gpu[:, :, pix], np.transpose(ref, (1, 2, 0)), "bench grid ff", FP32_TERMS,
          len(g.freqs_hz) * pix.size // 100)
