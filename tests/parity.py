"""Shared helpers of the GPU parity tests (not collected by pytest).

Tolerances of the forward maps, per pixel (from the stated target: relative
1e-5 on I, 1e-4 of the polarised intensity on Q and U):
    |I_gpu - I_ref| <= 1e-5 |I_ref|,
    |Q_gpu - Q_ref|, |U_gpu - U_ref| <= 1e-4 PI_ref,  PI_ref = |Q_ref + i U_ref|,
plus an absolute floor of 1e-8 of the map's largest I (one FP32 rounding step
of the brightest pixel), which only matters for sightlines that see almost no
emission or are depolarised to below that level; the report counts the pixels
that needed the floor.
"""
from __future__ import annotations

import numpy as np

from paper_2410_01136_amd import inputs as I

TOL_I = 1e-5
TOL_P = 1e-4
FLOOR = 1e-8


def oracle_geom(orc, g: I.Geometry):
    return orc.make_geom(g.nside, g.n_steps, g.freqs_hz, g.r_obs, g.r_max, g.box_lo, g.box_hi)


def compare_maps(gpu: np.ndarray, ref: np.ndarray, pix=None):
    """gpu, ref: [n_freq][3][n]; returns (ok, report dict)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    floor = FLOOR * np.abs(ref[:, 0]).max(axis=-1, keepdims=True)
    dI = np.abs(gpu[:, 0] - ref[:, 0])
    pi = np.hypot(ref[:, 1], ref[:, 2])
    dQ = np.abs(gpu[:, 1] - ref[:, 1])
    dU = np.abs(gpu[:, 2] - ref[:, 2])
    okI = dI <= TOL_I * np.abs(ref[:, 0]) + floor
    okQ = dQ <= TOL_P * pi + floor
    okU = dU <= TOL_P * pi + floor
    strict = (dI <= TOL_I * np.abs(ref[:, 0])) & (dQ <= TOL_P * pi) & (dU <= TOL_P * pi)
    ok = bool(okI.all() and okQ.all() and okU.all())
    with np.errstate(divide="ignore", invalid="ignore"):
        rep = {
            "max_rel_I": float(np.nanmax(dI / np.abs(ref[:, 0]))),
            "max_QU_over_PI": float(np.nanmax(np.maximum(dQ, dU) / pi)),
            "fail_I": int((~okI).sum()),
            "fail_Q": int((~okQ).sum()),
            "fail_U": int((~okU).sum()),
            "n": int(ref[:, 0].size),
            "needed_floor": int((~strict).sum()),
        }
    return ok, rep
