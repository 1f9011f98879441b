"""Shared helpers of the GPU parity tests (not collected by pytest).

Tolerances of the forward maps, per pixel (the stated target: relative 1e-5 on
I, 1e-4 of the polarised intensity on Q and U), strict by default:
    |I_gpu - I_ref| <= 1e-5 |I_ref|,
    |Q_gpu - Q_ref|, |U_gpu - U_ref| <= 1e-4 PI_ref,  PI_ref = |Q_ref + i U_ref|.

A test may declare the FP32 term floor (``floor=FP32_TERMS``): Q and U of a
pixel may then also deviate by up to 4 FP32 unit roundoffs (2^-22) of the
pixel's own I, which bounds the sum of magnitudes of its polarised terms
(|j_P| <= j_I).  That floor matters only for sightlines whose Q + iU cancels to
below ~2e-3 of their terms (Faraday-thick, depolarised): there the error of an
FP32-per-term sum, a few roundoffs of the terms, exceeds 1e-4 of the small
remainder whatever the order of summation.  A test that declares the floor
also states how many pixels may need it (``max_floor``); the report counts
them (``needed_floor``), names the worst pixel and gives its PI/I.
"""
from __future__ import annotations

import numpy as np

from paper_2410_01136_amd import inputs as I

TOL_I = 1e-5
TOL_P = 1e-4
FP32_TERMS = 2.0 ** -22  # 4 FP32 unit roundoffs, relative to the pixel's I


def oracle_geom(orc, g: I.Geometry):
    return orc.make_geom(g.nside, g.n_steps, g.freqs_hz, g.r_obs, g.r_max, g.box_lo, g.box_hi)


def compare_maps(gpu: np.ndarray, ref: np.ndarray, floor: float = 0.0, max_floor: int = 0):
    """gpu, ref: [n_freq][3][n].  Returns (ok, report).  ok needs every pixel
    within the strict bounds, except at most ``max_floor`` pixels that are
    within the declared floor (``floor`` x |I_ref| added to the Q/U bound)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    aI = np.abs(ref[:, 0])
    dI = np.abs(gpu[:, 0] - ref[:, 0])
    pi = np.hypot(ref[:, 1], ref[:, 2])
    dQU = np.maximum(np.abs(gpu[:, 1] - ref[:, 1]), np.abs(gpu[:, 2] - ref[:, 2]))
    okI = dI <= TOL_I * aI
    strictQU = dQU <= TOL_P * pi
    flooredQU = dQU <= TOL_P * pi + floor * aI
    needed = int((okI & ~strictQU & flooredQU).sum())
    ok = bool(okI.all() and flooredQU.all() and needed <= max_floor)
    with np.errstate(divide="ignore", invalid="ignore"):
        rQU = dQU / pi
        worst = np.unravel_index(int(np.nanargmax(np.where(np.isfinite(rQU), rQU, -1.0))), rQU.shape)
        depol = pi / aI
        rep = {
            "max_rel_I": float(np.nanmax(dI / aI)),
            "max_QU_over_PI": float(rQU[worst]),
            "worst_pixel": [int(v) for v in worst],
            "worst_PI_over_I": float(depol[worst]),
            "min_PI_over_I": float(np.nanmin(depol)),
            "fail_I": int((~okI).sum()),
            "fail_QU": int((~flooredQU).sum()),
            "n": int(aI.size),
            "needed_floor": needed,
            "max_floor": int(max_floor),
        }
    return ok, rep


def failing_pixels(gpu: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Boolean [n]: pixels outside the strict bounds at any frequency."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    pi = np.hypot(ref[:, 1], ref[:, 2])
    badI = np.abs(gpu[:, 0] - ref[:, 0]) > TOL_I * np.abs(ref[:, 0])
    badQU = np.maximum(np.abs(gpu[:, 1] - ref[:, 1]), np.abs(gpu[:, 2] - ref[:, 2])) > TOL_P * pi
    return (badI | badQU).any(axis=0)


# Grid gradients (a gradient is a weighted sum over residual-sized cotangents,
# so it amplifies the maps' ~1e-6 errors): relative L2 error <= 1e-3, cosine
# similarity >= 1 - 1e-6, and on every voxel and channel
# |g_gpu - g_ref| <= 1e-3 max|g_ref| (so a wrong voxel at an LDS-box edge, a
# piece boundary or an atomic path cannot hide in the norm).
GRAD_L2 = 1e-3
GRAD_COS = 1e-6
GRAD_VOXEL = 1e-3


def check_grid_gradient(got, ref, label):
    a = np.asarray(got, dtype=np.float64)
    b = np.asarray(ref, dtype=np.float64)
    assert a.shape == b.shape, (label, a.shape, b.shape)
    nb = np.linalg.norm(b)
    rel = np.linalg.norm(a - b) / nb
    cos = (a * b).sum() / (np.linalg.norm(a) * nb)
    d = np.abs(a - b)
    worst = np.unravel_index(int(np.argmax(d)), d.shape)
    vox = d[worst] / np.abs(b).max()
    print(f"{label}: rel L2 {rel:.2e}, 1-cos {1 - cos:.2e}, worst voxel {tuple(int(v) for v in worst)} "
          f"|dg|/max|g| {vox:.2e}", flush=True)
    assert rel <= GRAD_L2 and cos >= 1 - GRAD_COS and vox <= GRAD_VOXEL, (label, rel, cos, vox, worst)
