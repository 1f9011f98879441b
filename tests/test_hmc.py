"""The sampler's machinery on a target with a known answer (CPU only): HMC on a
correlated 4-D Gaussian recovers its mean and covariance; the ESS estimator
gives ~n for independent draws and ~n (1 - r) / (1 + r) for an AR(1) chain."""
import numpy as np

from paper_2410_01136_amd import hmc


def gaussian(mu, cov):
    P = np.linalg.inv(cov)

    def pot(q):
        d = q - mu
        return 0.5 * np.einsum("ni,ij,nj->n", d, P, d), d @ P.T
    return pot


def test_hmc_recovers_a_correlated_gaussian():
    rng = np.random.default_rng(7)
    A = rng.standard_normal((4, 4))
    cov = A @ A.T + 0.5 * np.eye(4)
    mu = np.array([1.0, -2.0, 0.5, 3.0])
    out = hmc.hmc(gaussian(mu, cov), mu + rng.standard_normal((32, 4)), n_iter=400, step=0.3,
                  n_leap=6, inv_mass=cov, rng=rng)
    s = out["samples"][100:].reshape(-1, 4)
    assert out["accept"][100:].mean() > 0.9
    sd = np.sqrt(np.diag(cov))
    assert np.all(np.abs(s.mean(0) - mu) < 0.1 * sd)
    np.testing.assert_allclose(np.cov(s.T), cov, rtol=0.15, atol=0.05 * np.abs(cov).max())


def test_hmc_rejects_outside_the_prior():
    def pot(q):
        U = 0.5 * (q ** 2).sum(1)
        return np.where(q[:, 0] > 0.5, np.inf, U), q
    rng = np.random.default_rng(8)
    out = hmc.hmc(pot, np.zeros((16, 2)), n_iter=200, step=0.4, n_leap=5, inv_mass=np.eye(2), rng=rng)
    assert out["samples"][..., 0].max() <= 0.5


def test_ess_estimator():
    rng = np.random.default_rng(9)
    iid = rng.standard_normal((2000, 8))
    assert 0.8 * 16000 < hmc.ess(iid) < 1.25 * 16000
    r = 0.8
    x = np.zeros((4000, 8))
    for t in range(1, 4000):
        x[t] = r * x[t - 1] + np.sqrt(1 - r * r) * rng.standard_normal(8)
    expect = 32000 * (1 - r) / (1 + r)
    assert 0.7 * expect < hmc.ess(x) < 1.4 * expect


def test_laplace_inverse_mass_of_a_quadratic():
    cov = np.array([[2.0, 0.3], [0.3, 0.5]])
    pot = gaussian(np.zeros(2), cov)
    inv = hmc.laplace_inv_mass(pot, np.array([0.2, -0.1]), np.array([1e-3, 1e-3]))
    np.testing.assert_allclose(inv, cov, rtol=1e-8)
