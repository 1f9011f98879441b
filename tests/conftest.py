import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle._load()
    return oracle


@pytest.fixture(scope="session")
def c1_grids(orc):
    """The headline's 256^3 node grids over the 40 x 40 x 8 kpc box: the
    spiral-disk model sampled by the oracle plus the seeded k^-11/3 turbulence
    (B: 50% of the local regular field; n_e: lognormal), and the model's N0."""
    from paper_2410_01136_amd import inputs as I
    print("building 256^3 grids", flush=True)
    reg_bn, reg_c = orc.sample_model16(I.THETA0, (256, 256, 256), I.BOX_LO, I.BOX_HI)
    bn = I.turbulent_grids(reg_bn)
    del reg_bn
    return bn, reg_c
