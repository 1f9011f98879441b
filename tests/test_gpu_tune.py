"""The autotuner on the GPU: tune a workload, cache it, hand the cache to the
library, and check that the library then launches the tuned shape by itself
(same maps as with that lane count set explicitly)."""
import numpy as np
import pytest

from paper_2410_01136_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2410_01136_amd import binding
    return binding


def test_tuned_shapes_apply_through_the_library(sm, tmp_path, monkeypatch):
    import torch
    from paper_2410_01136_amd import tune
    monkeypatch.setenv("SYNMARCH_TUNE_CACHE", str(tmp_path / "tune.json"))
    g = I.geometry("C0", nside=8, n_steps=96)
    geom = sm.geom_from(g)
    field = sm.model16(I.THETA0)
    try:
        res = tune.tune_forward(geom, field, reps=2)
        assert not res["cached"] and res["lanes"] in tune.CANDIDATES
        sm.set_lanes_per_ray(sm.KERNEL_FORWARD, sm.FIELD_MODEL16, res["lanes"])
        want = sm.forward(geom, field).cpu().numpy()
        sm.set_lanes_per_ray(sm.KERNEL_FORWARD, sm.FIELD_MODEL16, 0)
        assert tune.load() == 1
        lanes, mode = sm._i32(), sm._i32()
        assert sm.syn_autotune_lookup(sm.KERNEL_FORWARD, sm.FIELD_MODEL16, g.npix, g.n_steps, 1,
                                      sm.ctypes.byref(lanes), sm.ctypes.byref(mode)) == 1
        assert lanes.value == res["lanes"] and mode.value == 0
        got = sm.forward(geom, field).cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(got, want)
        # a second tune of the same shape comes from the cache
        assert tune.tune_forward(geom, field, reps=2)["cached"]
    finally:
        sm.syn_autotune_clear()
        sm.set_lanes_per_ray(sm.KERNEL_FORWARD, sm.FIELD_MODEL16, 0)
