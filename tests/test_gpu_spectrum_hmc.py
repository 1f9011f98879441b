"""Gradient-based inference over a broken power-law CR spectrum (Sec. 2.1 names
inference over fuller spectra with gradient-based sampling as the purpose of
modelling them): HMC over (alpha_lo, alpha_hi, ln gamma_b) from mock I/Q/U maps
at four frequencies across the break, likelihood and gradient from the GPU
forward, chi^2 and adjoint."""
import math

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


def test_hmc_recovers_the_spectrum(sm):
    import torch
    from paper_2410_01136_amd import hmc as H
    g = I.geometry("C0", nside=8, n_steps=128, freqs_hz=(0.4e9, 1.4e9, 5.0e9, 15.0e9))
    truth = np.array([3.0, I.BROKEN[0], math.log(I.BROKEN[1])])
    th = I.THETA0.copy()
    maps = sm.forward(sm.geom_from(g), sm.Field(sm.FIELD_MODEL16, th, broken=I.BROKEN))
    m = maps.cpu().numpy().astype(np.float64)
    rms = np.sqrt((m ** 2).mean(axis=-1))  # [f][3]
    sigma = 0.01 * rms
    rng = np.random.default_rng(8101)
    target = m + rng.standard_normal(m.shape) * sigma[..., None]
    bounds = [(2.0, 4.5), (2.0, 5.0), (math.log(1e3), math.log(1e6))]
    post = H.SpectrumPosterior(g, th, target, (1.0 / sigma ** 2).reshape(-1), bounds)
    # the gradient points back toward the truth from a displaced start
    U0, G0 = post(truth)
    Ud, Gd = post(truth + np.array([0.05, -0.05, 0.1]))
    assert Ud[0] > U0[0]
    inv_mass = H.laplace_inv_mass(post, truth, np.array([1e-3, 1e-3, 1e-3]))
    sd = np.sqrt(np.diag(inv_mass))
    assert np.all(np.isfinite(sd)) and np.all(sd > 0)
    n_chains = 4
    q0 = truth + 0.5 * sd * rng.standard_normal((n_chains, 3))
    out = H.hmc(post, q0, n_iter=60, step=0.4, n_leap=5, inv_mass=inv_mass, rng=rng)
    s = out["samples"][15:].reshape(-1, 3)
    mean, std = s.mean(0), s.std(0)
    acc = out["accept"][15:].mean()
    print(f"spectrum HMC: truth {truth}, posterior mean {mean}, sd {std} (Laplace {sd}), "
          f"acceptance {acc:.2f}, evaluations {post.evals}", flush=True)
    assert acc > 0.5
    assert np.all(np.abs(mean - truth) <= 4.0 * sd), (mean, truth, sd)
    assert np.all(std <= 3.0 * sd) and np.all(std >= sd / 3.0)
