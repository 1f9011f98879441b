"""The chi^2 entry point that allocates nothing (syn_chi2_cotangent, partial sums
in a static device array) against syn_chi2 with a caller workspace: the same
chi^2 and cotangent, bit for bit, on two calls in a row, the second with a
smaller input (the array keeps the first call's partials, which the second must
not pick up)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2410_01136_amd import binding
    return binding


def _with_workspace(sm, maps, tgt, inv, n_pix, n_maps):
    import torch
    chi = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    dm = torch.full_like(maps, np.nan)
    nws = sm.syn_chi2_workspace_bytes(n_pix, n_maps)
    ws = torch.empty((nws + 7) // 8, dtype=torch.float64, device="cuda")
    sm.check(sm.syn_chi2(n_pix, n_maps, maps.data_ptr(), tgt.data_ptr(), inv.ctypes.data_as(sm._dp),
                         dm.data_ptr(), chi.data_ptr(), ws.data_ptr(), nws, sm._stream()), "syn_chi2")
    return chi, dm


def _no_alloc(sm, maps, tgt, inv, n_pix, n_maps, chi, dm):
    sm.check(sm.syn_chi2_cotangent(n_pix, n_maps, maps.data_ptr(), tgt.data_ptr(),
                                   inv.ctypes.data_as(sm._dp), dm.data_ptr(), chi.data_ptr(),
                                   sm._stream()), "syn_chi2_cotangent")


def test_no_alloc_chi2_matches_workspace_entry_point(sm):
    import torch
    rng = np.random.default_rng(8101)
    # first call: 4 frequencies x 3 Stokes maps of 786,432 pixels (the partial
    # count reaches its 4096 cap); second: 1 x 3 maps of 3,001 pixels (5 partials)
    for n_freq, n_pix in ((4, 786_432), (1, 3_001)):
        n_maps = 3 * n_freq
        print(f"no-alloc chi2: n_maps {n_maps}, n_pix {n_pix}", flush=True)
        maps = torch.from_numpy(rng.standard_normal((n_freq, 3, n_pix)).astype(np.float32)).cuda()
        tgt = torch.from_numpy(rng.standard_normal((n_freq, 3, n_pix)).astype(np.float32)).cuda()
        inv = np.ascontiguousarray(rng.uniform(0.5, 2.0, n_maps))
        ref_chi, ref_dm = _with_workspace(sm, maps, tgt, inv, n_pix, n_maps)
        chi = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
        dm = torch.full_like(maps, np.nan)
        torch.cuda.synchronize()
        _no_alloc(sm, maps, tgt, inv, n_pix, n_maps, chi, dm)
        torch.cuda.synchronize()
        assert chi.item() == ref_chi.item(), (chi.item(), ref_chi.item())
        assert torch.equal(dm, ref_dm)
        r = maps.double() - tgt.double()
        want = (torch.from_numpy(inv).cuda().view(n_freq, 3, 1) * r * r).sum().item()
        assert chi.item() == pytest.approx(want, rel=1e-12)


def test_no_alloc_chi2_rejects_oversized_and_bad_arguments(sm):
    import torch
    x = torch.zeros(8, dtype=torch.float32, device="cuda")
    chi = torch.zeros(1, dtype=torch.float64, device="cuda")
    inv = np.ones(48)
    # n_pix * n_maps beyond SYN_CHI2_MAX_VALUES (nothing is read: the host rejects it)
    st = sm.syn_chi2_cotangent((1 << 36) // 3 + 1, 3, x.data_ptr(), x.data_ptr(),
                               inv.ctypes.data_as(sm._dp), None, chi.data_ptr(), sm._stream())
    assert st == sm.SYN_EINVAL and b"SYN_CHI2_MAX_VALUES" in sm.syn_last_error()
    st = sm.syn_chi2_cotangent(8, 0, x.data_ptr(), x.data_ptr(), inv.ctypes.data_as(sm._dp), None,
                               chi.data_ptr(), sm._stream())
    assert st == sm.SYN_EINVAL
    st = sm.syn_chi2_cotangent(8, 1, x.data_ptr(), None, inv.ctypes.data_as(sm._dp), None,
                               chi.data_ptr(), sm._stream())
    assert st == sm.SYN_EINVAL
    bad = np.array([-1.0])
    st = sm.syn_chi2_cotangent(8, 1, x.data_ptr(), x.data_ptr(), bad.ctypes.data_as(sm._dp), None,
                               chi.data_ptr(), sm._stream())
    assert st == sm.SYN_EINVAL
    # without a cotangent output (chi^2 only), then the binding wrapper
    ones = torch.ones(5, dtype=torch.float32, device="cuda")
    zeros = torch.zeros(5, dtype=torch.float32, device="cuda")
    sm.check(sm.syn_chi2_cotangent(5, 1, ones.data_ptr(), zeros.data_ptr(),
                                   np.array([2.0]).ctypes.data_as(sm._dp), None, chi.data_ptr(),
                                   sm._stream()), "chi2 only")
    torch.cuda.synchronize()
    assert chi.item() == 10.0
    dm = torch.empty_like(ones)
    sm.chi2_cotangent(ones.view(1, 5), zeros.view(1, 5), [0.5], chi, dm.view(1, 5))
    torch.cuda.synchronize()
    assert chi.item() == 2.5 and torch.equal(dm, torch.ones_like(dm))
