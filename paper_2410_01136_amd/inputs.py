"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds configuration values and random-number recipes only: none
of the ray-march arithmetic (no field model, no emissivity, no sums).  The
regular part of a gridded field is always sampled by the caller -- the oracle
for reference inputs, the HIP library for benchmark inputs -- and handed in.

Workloads (the paper's own workloads are the toy sphere of Sec. 2.4 and the
WMAP-model maps of Sec. 3.1; these synthetic configurations follow the same
shapes and value ranges):

* ``C0`` plain forward, analytic spiral-disk model, N_side 16, 256 steps,
  1 GHz, sightlines capped at 20 kpc.
* ``C1`` gridded forward, N_side 256, 512 steps, {1, 2.3, 5} GHz, five FP32
  channels on 256^3 nodes over a 40x40x8 kpc box: analytic model plus a
  seeded k^-11/3 Gaussian random field (50% rms of the regular B, lognormal
  n_e).
* ``C2`` adjoint, N_side 64, 768 steps, 1.4 GHz, chi^2 against a target at
  perturbed parameters plus 1% noise; 16 parameters and a 128^3 B/n_e grid.
* ``C3`` 256 parameter sets with N_side in {32, 64, 128} mixed 1:2:1, 512
  steps, 1 GHz, forward + adjoint.
* ``C4`` coordinate-MLP field surrogate, N_side 512, 1024 steps, 1 GHz.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

import numpy as np

# Parameter vector of the 16-parameter analytic model (index: name, unit).
PARAM_NAMES = (
    "B0_uG", "psi0_rad", "psi1_rad", "chiB0_rad", "R_B_kpc", "z_B_kpc",
    "BH0_uG", "z_H_kpc", "R_H_kpc", "C0_cm3", "hr_CR_kpc", "hz_CR_kpc",
    "alpha", "n0_cm3", "hz_ne_kpc", "kappa_ne_per_kpc",
)

# Spiral-disk test configuration: B0 = 6 uG, pitch -12 deg, exponential disk
# R = 8 kpc, z = 1 kpc; CR power law alpha = 3 with N0 = 4e-5 cm^-3 at the Sun;
# n_e = 0.03 cm^-3 exponential disk with 1 kpc scale height.
THETA0 = np.array([
    6.0, math.radians(-12.0), 0.0, 0.0, 8.0, 1.0,
    0.0, 1.5, 8.0,
    4.0e-5, 8.0, 1.0, 3.0,
    0.03, 1.0, 0.0,
], dtype=np.float64)

# Perturbation scales: 5% of non-zero entries; fixed scales for zero entries.
THETA_SIGMA = np.where(THETA0 != 0.0, 0.05 * np.abs(THETA0), 0.0)
THETA_SIGMA[2] = 0.05   # psi1 [rad]
THETA_SIGMA[3] = 0.05   # chiB0 [rad]
THETA_SIGMA[6] = 0.5    # BH0 [uG]
THETA_SIGMA[15] = 0.01  # kappa_ne [1/kpc]

R_OBS = (-8.5, 0.0, 0.0)
BOX_LO = (-20.0, -20.0, -4.0)
BOX_HI = (20.0, 20.0, 4.0)
INF3 = (math.inf, math.inf, math.inf)
NINF3 = (-math.inf, -math.inf, -math.inf)


@dataclass
class Geometry:
    nside: int
    n_steps: int
    freqs_hz: Tuple[float, ...]
    r_obs: Tuple[float, float, float] = R_OBS
    r_max: float = math.inf
    box_lo: Tuple[float, float, float] = NINF3
    box_hi: Tuple[float, float, float] = INF3

    @property
    def npix(self) -> int:
        return 12 * self.nside * self.nside

    @property
    def units(self) -> int:
        """Sightline-steps counted as pixels x steps x frequencies."""
        return self.npix * self.n_steps * len(self.freqs_hz)


FIT_BOX_LO = (-20.0, -20.0, -5.0)
FIT_BOX_HI = (20.0, 20.0, 5.0)
FIT_GRID = (128, 128, 32)  # nodes (x, y, z) of the fitted B grid


# Free-free workloads (T_e = 8000 K): the 256^3 gridded headline forward at low
# radio frequencies, and the N_side 64 / 768-step analytic forward + adjoint at
# frequencies where the disk model at theta0 is not yet so Faraday-thick that
# FP32 field values limit its depolarised Q/U (below ~0.5 GHz over the
# 40 x 40 x 8 kpc box).
TE_FF = 8000.0
FF_GRID_FREQS = (0.15e9, 0.3e9, 0.6e9)
FF_THETA_FREQS = (0.6e9, 0.8e9, 1.0e9)

# Broken power-law CR spectrum of the workloads that use one: (index above the
# break, Lorentz factor of the break) with theta[12] below it.  A break at
# gamma ~ 1.2e4 (~6 GeV) puts xb = nu / nu_c(gamma_b) near 0.3 at 1 GHz in a
# 6 uG field, so the {1, 2.3, 5} GHz maps straddle the steepening.
BROKEN = (3.6, 1.2e4)


def geometry(name: str, **over) -> Geometry:
    """The geometry of a named configuration (keyword overrides allowed)."""
    base = {
        "C0": dict(nside=16, n_steps=256, freqs_hz=(1.0e9,), r_max=20.0),
        "C1": dict(nside=256, n_steps=512, freqs_hz=(1.0e9, 2.3e9, 5.0e9),
                   box_lo=BOX_LO, box_hi=BOX_HI),
        "C2": dict(nside=64, n_steps=768, freqs_hz=(1.4e9,), box_lo=BOX_LO, box_hi=BOX_HI),
        "C3": dict(nside=64, n_steps=512, freqs_hz=(1.0e9,), r_max=20.0),
        "C4": dict(nside=512, n_steps=1024, freqs_hz=(1.0e9,), box_lo=BOX_LO, box_hi=BOX_HI),
        # homogeneous-sphere test of the paper (Sec. 2.4): N_side 64, 1024 steps,
        # 2.4 GHz, box (40, 40, 10) kpc
        "E1": dict(nside=64, n_steps=1024, freqs_hz=(2.4e9,), r_obs=(-8.3, 0.0, 0.006),
                   box_lo=(-20.0, -20.0, -5.0), box_hi=(20.0, 20.0, 5.0)),
        # grid fitting of Sec. 3.3: B on 128 x 128 x 32 voxels over a (40, 40, 10)
        # kpc box, N_side 64 with 512 steps at 2.4 GHz (the Sec. 3.1 map setup)
        "G1": dict(nside=64, n_steps=512, freqs_hz=(2.4e9,), box_lo=FIT_BOX_LO,
                   box_hi=FIT_BOX_HI),
    }[name]
    base.update(over)
    return Geometry(**base)


def sphere_theta(B_uG=(6.0, 0.0, 0.0), ne=0.01, n0=4.01e-5, R0_kpc=4.0,
                 centre=(-8.3, 0.0, 0.006), alpha=3.0) -> np.ndarray:
    """Parameter vector of the homogeneous sphere (Sec. 2.4 values by default).

    Layout: 0-2 B [uG], 3 n_e, 4 N0 [cm^-3], 5 radius [kpc] (<= 0: everywhere),
    6-8 centre [kpc], 12 alpha.
    """
    th = np.zeros(16)
    th[0:3] = B_uG
    th[3] = ne
    th[4] = n0
    th[5] = R0_kpc
    th[6:9] = centre
    th[12] = alpha
    return th


def wmap_theta(b0_uG=1.2, psi0=0.4712, psi1=0.0157, chi0=0.4363, n0_earth=4.0e-5,
               earth=(-8.5, 0.0, 0.0), h_r=5.0, h_z=1.0, ring=(3.0, 20.0), alpha=3.0,
               ne=(0.03, 1.0, 0.0)) -> np.ndarray:
    """Parameter vector of the WMAP field of Sec. 3.1 (the paper's true values by
    default; b0 = 1.2e-6 gauss).  C0 is set so that N0 at `earth` is n0_earth.
    n_e = (n0, h_z, kappa) of the exponential disk standing in for YMW16.

    Layout: 0 b0 [uG], 1 psi0, 2 psi1, 3 chi0 [rad], 4-5 ring radii [kpc],
    9 C0 [cm^-3], 10 h_r, 11 h_z [kpc], 12 alpha, 13-15 n_e disk.
    """
    th = np.zeros(16)
    th[0:4] = (b0_uG, psi0, psi1, chi0)
    th[4:6] = ring
    rho_e = float(np.hypot(earth[0], earth[1]))
    th[9] = n0_earth * np.exp(rho_e / h_r) * np.cosh(earth[2] / h_z) ** 2
    th[10], th[11], th[12] = h_r, h_z, alpha
    th[13:16] = ne
    return th


def perturbed_thetas(n: int, seed: int) -> np.ndarray:
    """n parameter vectors drawn from N(THETA0, THETA_SIGMA^2), seeded."""
    rng = np.random.default_rng(seed)
    return THETA0[None, :] + rng.standard_normal((n, 16)) * THETA_SIGMA[None, :]


def c3_nsides(n_sets: int = 256, seed: int = 3002) -> np.ndarray:
    """N_side of each set: 32, 64, 128 mixed 1:2:1 in a seeded order."""
    q = n_sets // 4
    ns = np.array([32] * q + [64] * (n_sets - 2 * q) + [128] * q, dtype=np.int32)
    rng = np.random.default_rng(seed)
    rng.shuffle(ns)
    return ns


def grid_nodes(n: Sequence[int]) -> Tuple[int, int, int]:
    return tuple(int(v) for v in n)  # (nx, ny, nz)


def grf(shape_zyx: Sequence[int], spacing_zyx: Sequence[float], seed: int,
        slope: float = -11.0 / 3.0) -> np.ndarray:
    """Periodic Gaussian random field with power spectrum P(k) ~ k^slope.

    White noise is shaped in Fourier space with physical wavenumbers of the
    node grid, the k = 0 mode is removed and the result is scaled to unit
    variance.  float32 output, C order [z][y][x].
    """
    rng = np.random.default_rng(seed)
    nz, ny, nx = (int(v) for v in shape_zyx)
    white = rng.standard_normal((nz, ny, nx))
    fk = np.fft.rfftn(white)
    del white
    kz = np.fft.fftfreq(nz, d=spacing_zyx[0])[:, None, None]
    ky = np.fft.fftfreq(ny, d=spacing_zyx[1])[None, :, None]
    kx = np.fft.rfftfreq(nx, d=spacing_zyx[2])[None, None, :]
    k2 = kz * kz + ky * ky + kx * kx
    k2[0, 0, 0] = 1.0
    amp = k2 ** (slope / 4.0)  # sqrt(P) = k^(slope/2) = (k^2)^(slope/4)
    amp[0, 0, 0] = 0.0
    fk *= amp
    g = np.fft.irfftn(fk, s=(nz, ny, nx), axes=(0, 1, 2))
    g /= g.std()
    return g.astype(np.float32)


def turbulence_noise(shape_zyx: Sequence[int], seeds=(1001, 1002, 1003, 1004), lo=BOX_LO,
                     hi=BOX_HI) -> np.ndarray:
    """Four unit-variance k^-11/3 fields [4][nz][ny][nx] (B_x, B_y, B_z, n_e)."""
    nz, ny, nx = (int(v) for v in shape_zyx)
    spacing = [(hi[2] - lo[2]) / (nz - 1), (hi[1] - lo[1]) / (ny - 1), (hi[0] - lo[0]) / (nx - 1)]
    return np.stack([grf((nz, ny, nx), spacing, s) for s in seeds])


def apply_turbulence(reg_bn: np.ndarray, noise: np.ndarray, b_frac: float = 0.5,
                     ne_sigma: float = 0.5) -> np.ndarray:
    """Add seeded random fluctuations to a regular B/n_e node grid.

    reg_bn: [nz][ny][nx][4] float32 (Bx, By, Bz [uG], n_e [cm^-3]) sampled from
    the analytic model by the caller.  B gets a local Gaussian fluctuation of
    rms b_frac * |B_reg| (per component |B_reg| b_frac / sqrt(3) times a unit
    k^-11/3 field); n_e is multiplied by exp(s g - s^2 / 2), s = ne_sigma
    (lognormal, mean preserving).  Returns a new float32 array.
    """
    out = np.array(reg_bn, dtype=np.float32, copy=True)
    bmag = np.sqrt((reg_bn[..., :3].astype(np.float64) ** 2).sum(-1))
    for k in range(3):
        out[..., k] += (b_frac / math.sqrt(3.0) * bmag * noise[k]).astype(np.float32)
    out[..., 3] = (reg_bn[..., 3] * np.exp(ne_sigma * noise[3] - 0.5 * ne_sigma ** 2)).astype(np.float32)
    return out


def turbulent_grids(reg_bn: np.ndarray, seeds=(1001, 1002, 1003, 1004),
                    lo=BOX_LO, hi=BOX_HI, b_frac: float = 0.5,
                    ne_sigma: float = 0.5) -> np.ndarray:
    """apply_turbulence with freshly generated noise of the given seeds."""
    noise = turbulence_noise(reg_bn.shape[:3], seeds, lo, hi)
    return apply_turbulence(reg_bn, noise, b_frac, ne_sigma)


def chi2_noise(maps: np.ndarray, seed: int, frac: float = 0.01):
    """Target = maps + Gaussian noise of sigma_X = frac * rms(X) per Stokes map.

    maps: [n_freq][3][npix].  Returns (target float32, inv_sigma2 [n_freq][3]).
    """
    rng = np.random.default_rng(seed)
    rms = np.sqrt((maps.astype(np.float64) ** 2).mean(axis=-1))
    sigma = frac * rms
    target = maps + rng.standard_normal(maps.shape) * sigma[..., None]
    inv_s2 = 1.0 / (sigma * sigma)
    return target.astype(np.float32), inv_s2


def cotangents(shape, seed: int) -> np.ndarray:
    """Seeded random map cotangents for adjoint tests."""
    return np.random.default_rng(seed).standard_normal(shape).astype(np.float32)


def sample_pixels(npix: int, n: int, seed: int) -> np.ndarray:
    """n distinct pixel indices plus both ends of the RING order."""
    rng = np.random.default_rng(seed)
    pix = rng.choice(npix, size=min(n, npix), replace=False)
    return np.unique(np.concatenate([pix, [0, npix - 1]])).astype(np.int64)
