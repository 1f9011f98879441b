"""FP64 reference of the grid-fitting loop (test infrastructure, like the rest of
``oracle``): only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may use it.

Follows Sec. 3.3 of Diao et al. (arXiv:2410.01136): the B field on a voxel grid
is fitted to mock maps by maximising the Gaussian log-likelihood of Sec. 3.1
with the Adam optimiser, the gradient coming from the adjoint march.  Adam is
the published algorithm of Kingma & Ba (2015, arXiv:1412.6980, Algorithm 1),
with its bias-corrected moments written out as defined there.
"""
from __future__ import annotations

import numpy as np


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, period=1, mask=1):
    """One Adam update in place (Kingma & Ba 2015, Algorithm 1), FP64.

    params, grads, m, v: flat arrays of equal length (m, v start at zero);
    t: the step number, 1 for the first update.  Element i takes part iff bit
    (i % period) of `mask` is set; the others keep their parameter and moments.
    """
    idx = np.arange(params.size) % period
    sel = ((mask >> idx) & 1).astype(bool)
    g = grads[sel].astype(np.float64)
    m_new = beta1 * m[sel] + (1.0 - beta1) * g          # biased first moment
    v_new = beta2 * v[sel] + (1.0 - beta2) * g * g      # biased second raw moment
    m_hat = m_new / (1.0 - beta1 ** t)                  # bias corrections
    v_hat = v_new / (1.0 - beta2 ** t)
    params[sel] = params[sel] - lr * m_hat / (np.sqrt(v_hat) + eps)
    m[sel] = m_new
    v[sel] = v_new


def chi2(maps, target, inv_sigma2):
    """Gaussian chi^2 of I/Q/U maps against a target (Sec. 3.1, one sigma per
    Stokes map and frequency) and its gradient with respect to the maps.

    maps, target: [n_freq][3][npix]; inv_sigma2: [n_freq][3].
    """
    r = np.asarray(maps, np.float64) - np.asarray(target, np.float64)
    w = np.asarray(inv_sigma2, np.float64)[..., None]
    return float((w * r * r).sum()), 2.0 * w * r


def fit_grid(orc, geom, theta, grid_bn, lo, hi, target, inv_sigma2, iters, lr, mask=0b0111,
             beta1=0.9, beta2=0.999, eps=1e-8):
    """The grid-fitting loop of Sec. 3.3 on the oracle: forward march, chi^2,
    reverse march into the (B_x, B_y, B_z, n_e) grid, Adam on the channels in
    `mask` (default: the three B components).  Returns (chi^2 before each
    update, fitted grid)."""
    g = np.array(grid_bn, dtype=np.float32, copy=True)
    p = g.reshape(-1).astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    hist = []
    for t in range(1, iters + 1):
        field = orc.Field(orc.GRID, theta, grid_bn=p.reshape(g.shape).astype(np.float32),
                          grid_c=None, grid_lo=lo, grid_hi=hi)
        maps = orc.forward(geom, field)
        c, dm = chi2(maps, target, inv_sigma2)
        hist.append(c)
        _, dbn, _ = orc.adjoint(geom, field, dm, want_grid=True)
        adam_step(p, dbn.reshape(-1), m, v, t, lr, beta1, beta2, eps, period=4, mask=mask)
    return np.array(hist), p.reshape(g.shape)
