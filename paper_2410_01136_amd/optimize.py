"""Fitting a gridded magnetic field to observed maps (Sec. 3.3 of Diao et al.,
arXiv:2410.01136).

The B components on a voxel grid are the parameters; each iteration runs the
forward march, the Gaussian chi^2 of I/Q/U against the target (Sec. 3.1), the
reverse march into the grid and one Adam update (Kingma & Ba 2015) -- all four
in the HIP library (syn_forward, syn_chi2, syn_adjoint, syn_adam_step), with
PyTorch holding the buffers.  n_e (the fourth channel of the grid) and the
analytic cosmic-ray density stay fixed.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import binding as sm

B_CHANNELS = 0b0111  # (B_x, B_y, B_z, n_e): update the B components only


def fit_grid(geom, theta, grid_bn: torch.Tensor, lo, hi, target: torch.Tensor, inv_sigma2,
             iters: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
             mask: int = B_CHANNELS, sync_each: bool = False):
    """Runs `iters` Adam iterations from `grid_bn` ([nz][ny][nx][4], float32, cuda).

    Returns {"chi2": chi^2 before each update (numpy [iters]), "grid": fitted grid,
    "seconds": wall time of the loop, "iter_ms": per-iteration wall time}.
    """
    grid = grid_bn.detach().clone().contiguous()
    field = sm.grid(theta, grid, None, lo, hi)  # reads `grid`, which Adam updates in place
    ws = sm.alloc_workspace(geom, field)
    npix = 12 * geom.nside ** 2
    maps = torch.empty((geom.n_freq, 3, npix), dtype=torch.float32, device=grid.device)
    m = torch.zeros_like(grid)
    v = torch.zeros_like(grid)
    dgrid = torch.empty_like(grid)
    chi = torch.empty(iters, dtype=torch.float64, device=grid.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(1, iters + 1):
        sm.forward(geom, field, maps=maps, ws=ws)
        c, dm = sm.chi2(maps, target, inv_sigma2)
        chi[t - 1:t].copy_(c)
        dgrid.zero_()
        sm.adjoint(geom, field, dm, ws, want_theta=False, dgrid_bn=dgrid)
        sm.adam_step(grid, dgrid, m, v, t, lr, beta1, beta2, eps, period=4, mask=mask)
        if sync_each:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    return {"chi2": chi.cpu().numpy(), "grid": grid, "seconds": secs,
            "iter_ms": 1e3 * secs / max(iters, 1)}
