"""HMC over the four WMAP parameters with all chains in one batch plan (Sec. 3.2)."""
import numpy as np
import pytest

from paper_2410_01136_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2410_01136_amd import binding, hmc
    return binding, hmc, torch


def mock(sm, g, th, seed):
    maps = sm.forward(sm.geom_from(g), sm.wmap(th)).cpu().numpy()
    rng = np.random.default_rng(seed)
    return maps + rng.normal(0.0, 1e-3, maps.shape)


def test_batch_potential_matches_single_evaluations(env):
    sm, H, torch = env
    g = I.geometry("G1", nside=4, n_steps=64)
    truth = I.wmap_theta()
    tgt = mock(sm, g, truth, 11)
    inv = np.array([0.0, 1e6, 1e6])
    post = H.BatchPosterior(g, truth, tgt, inv, n_chains=6)
    try:
        rng = np.random.default_rng(12)
        # inside the paper's prior (psi1 = 0.0157 sits near its lower edge)
        q = truth[:4] + rng.normal(0, 0.02, (6, 4)) * np.array([1.0, 1.0, 0.2, 1.0])
        q[:, 2] = np.abs(q[:, 2])
        U, G = post(q)
        for c in range(6):
            th = truth.copy()
            th[:4] = q[c]
            geom = sm.geom_from(g)
            f = sm.wmap(th)
            ws = sm.alloc_workspace(geom, f)
            m = sm.forward(geom, f, ws=ws)
            chi, dm = sm.chi2(m, torch.from_numpy(tgt.astype(np.float32)).cuda(), inv[None])
            d = sm.adjoint(geom, f, dm, ws).cpu().numpy()
            assert U[c] == pytest.approx(0.5 * chi.item(), rel=1e-6)
            np.testing.assert_allclose(G[c], 0.5 * d[:4], rtol=1e-5, atol=1e-6 * np.abs(d[:4]).max())
        q_out = q.copy()
        q_out[0, 0] = -1.0  # outside the prior
        U2, _ = post(q_out)
        assert np.isinf(U2[0]) and np.all(np.isfinite(U2[1:]))
    finally:
        post.close()


def test_hmc_samples_the_wmap_posterior(env):
    sm, H, torch = env
    g = I.geometry("G1", nside=4, n_steps=64)
    truth = I.wmap_theta()
    tgt = mock(sm, g, truth, 13)
    inv = np.array([0.0, 1e6, 1e6])
    post = H.BatchPosterior(g, truth, tgt, inv, n_chains=16)
    try:
        q_star = truth[:4]
        lap = H.BatchPosterior(g, truth, tgt, inv, n_chains=8)
        try:
            inv_mass = H.laplace_inv_mass(lap, q_star, 1e-4 * np.maximum(np.abs(q_star), 1e-2))
        finally:
            lap.close()
        sd = np.sqrt(np.diag(inv_mass))
        rng = np.random.default_rng(14)
        q0 = q_star + 0.5 * sd * rng.standard_normal((16, 4))
        out = H.hmc(post, q0, n_iter=40, step=0.3, n_leap=6, inv_mass=inv_mass, rng=rng)
        acc = out["accept"][10:].mean()
        s = out["samples"][10:].reshape(-1, 4)
        z = (s.mean(0) - q_star) / sd
        print("HMC acceptance", acc, "posterior mean - truth in sigma", z, flush=True)
        assert acc > 0.6
        assert np.all(np.abs(z) < 4.0)
    finally:
        post.close()
