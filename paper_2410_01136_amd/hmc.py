"""Gradient-based sampling of field parameters with many chains per launch.

Sec. 3.2 of Diao et al. (arXiv:2410.01136) samples the four WMAP field
parameters {b0, psi0, psi1, chi0} from the Gaussian likelihood of mock Q/U maps
with a gradient-based sampler.  Here every chain is one parameter set of a batch
plan, so one persistent launch evaluates the likelihood and its gradient for
all chains (syn_batch_set_theta, syn_batch_run); the sampler is plain
Hamiltonian Monte Carlo (Duane et al. 1987; leapfrog integration with a
Metropolis correction, Neal 2011) with a dense mass matrix, vectorised over
chains on the host -- its arithmetic is a few numbers per chain and step.
"""
from __future__ import annotations

import ctypes
import time
from typing import Callable, Sequence

import numpy as np
import torch

from . import binding as sm

PAPER_PRIOR = ((0.0, 10.0), (0.0, np.pi / 2), (0.0, np.pi / 2), (0.0, np.pi / 2))


class BatchPosterior:
    """U(q) = chi^2 / 2 (the negative log-likelihood of Sec. 3.2, flat prior
    inside `bounds`, infinite outside) and dU/dq for n chains in one launch.

    geom: inputs.Geometry of the maps (one frequency); base_theta: the field's
    16 parameters, of which `free` are sampled; target: maps [1][3][npix];
    inv_sigma2: [3] weights of I, Q, U.
    """

    def __init__(self, geom, base_theta, target, inv_sigma2, n_chains: int, free=(0, 1, 2, 3),
                 bounds: Sequence = PAPER_PRIOR, kind: int = sm.FIELD_WMAP, use_graph: bool = True):
        self.n = int(n_chains)
        self.free = np.asarray(free, dtype=np.int64)
        self.bounds = np.asarray(bounds, dtype=np.float64)
        self.base = np.asarray(base_theta, dtype=np.float64)
        self.theta = np.ascontiguousarray(np.tile(self.base, (self.n, 1)))
        self.inv = np.ascontiguousarray(np.asarray(inv_sigma2, dtype=np.float64).reshape(3))
        desc = sm.SynBatchDesc()
        self._ns = np.full(self.n, geom.nside, dtype=np.int32)
        desc.n_sets = self.n
        desc.nside = self._ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        desc.theta = self.theta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        desc.geom = sm.geom_from(geom)
        desc.use_graph = int(use_graph)
        desc.kind = int(kind)
        self.plan = ctypes.c_void_p()
        sm.check(sm.syn_batch_create(ctypes.byref(desc), ctypes.byref(self.plan)), "syn_batch_create")
        total = int(sm.syn_batch_total_pixels(self.plan))
        npix = 12 * geom.nside ** 2
        t = torch.as_tensor(np.asarray(target, dtype=np.float32).reshape(3, npix)).cuda()
        self.target = t.repeat(1, self.n).contiguous()  # every chain fits the same maps
        assert self.target.shape[1] == total
        self.maps = torch.empty((3, total), dtype=torch.float32, device="cuda")
        self.dmaps = torch.empty_like(self.maps)
        self.chi2 = torch.empty(self.n, dtype=torch.float64, device="cuda")
        self.dth = torch.empty((self.n, 16), dtype=torch.float64, device="cuda")
        self.evals = 0

    def inside(self, q):
        return np.all((q >= self.bounds[:, 0]) & (q <= self.bounds[:, 1]), axis=1)

    def __call__(self, q: np.ndarray):
        q = np.asarray(q, dtype=np.float64)
        ok = self.inside(q)
        qc = np.clip(q, self.bounds[:, 0], self.bounds[:, 1])  # chains outside run at the edge
        self.theta[:, self.free] = qc
        stream = sm._stream()
        sm.check(sm.syn_batch_set_theta(self.plan, self.theta.ctypes.data_as(sm._dp), stream),
                 "syn_batch_set_theta")
        sm.check(sm.syn_batch_run(self.plan, self.target.data_ptr(), self.inv.ctypes.data_as(sm._dp),
                                  self.maps.data_ptr(), self.dmaps.data_ptr(), self.chi2.data_ptr(),
                                  self.dth.data_ptr(), stream), "syn_batch_run")
        self.evals += 1
        U = 0.5 * self.chi2.cpu().numpy()
        g = 0.5 * self.dth.cpu().numpy()[:, self.free]
        U = np.where(ok, U, np.inf)
        return U, g

    def close(self):
        if self.plan:
            sm.syn_batch_destroy(self.plan)
            self.plan = ctypes.c_void_p()


class SpectrumPosterior:
    """U(q) = chi^2 / 2 of multi-frequency I/Q/U maps and dU/dq for the broken
    power-law CR spectrum's parameters q = (alpha_lo, alpha_hi, ln gamma_b) --
    the inference over CR spectra with gradient-based sampling that Sec. 2.1
    names as the purpose of a fuller spectrum.  Flat prior inside `bounds`.

    Chains are evaluated one after another (forward, chi^2, adjoint through the
    C ABI); each evaluation rebuilds the spectrum table for its indices into
    one device buffer (syn_spectrum_table: ~0.3 ms on the host after the
    first).  geom: inputs.Geometry; theta: the field's 16 parameters (theta[12]
    is replaced by alpha_lo); target: maps [n_freq][3][npix]; inv_sigma2:
    [n_freq * 3] weights.
    """

    def __init__(self, geom, theta, target, inv_sigma2, bounds, kind: int = sm.FIELD_MODEL16):
        self.g = sm.geom_from(geom)
        self.theta = np.asarray(theta, dtype=np.float64).copy()
        self.kind = int(kind)
        self.bounds = np.asarray(bounds, dtype=np.float64)
        self.target = torch.as_tensor(np.asarray(target, dtype=np.float32)).cuda().contiguous()
        self.inv = np.asarray(inv_sigma2, dtype=np.float64).reshape(-1)
        nb = int(sm.syn_spectrum_table_bytes())
        self.table = torch.empty((nb + 3) // 4, dtype=torch.float32, device="cuda")
        self.nb = nb
        self.maps = torch.empty_like(self.target)
        self.ws = sm.alloc_workspace(self.g, self._field(self.bounds.mean(axis=1)))
        self.evals = 0

    def _field(self, q):
        th = self.theta.copy()
        th[12] = q[0]
        f = sm.Field(self.kind, th)
        f.s.spectrum, f.s.alpha_hi, f.s.gamma_break = sm.SPEC_BROKEN, float(q[1]), float(np.exp(q[2]))
        f.s.spectrum_table = self.table.data_ptr()
        sm.check(sm.syn_spectrum_table(float(q[0]), float(q[1]), self.table.data_ptr(), self.nb,
                                       sm._stream()), "syn_spectrum_table")
        return f

    def one(self, q):
        f = self._field(q)
        sm.forward(self.g, f, maps=self.maps, ws=self.ws)
        chi2, dm = sm.chi2(self.maps, self.target, self.inv)
        dth = sm.adjoint(self.g, f, dm, self.ws)
        self.evals += 1
        d = dth.cpu().numpy()
        return 0.5 * float(chi2.cpu()[0]), 0.5 * d[[12, 16, 17]]

    def __call__(self, Q: np.ndarray):
        Q = np.atleast_2d(np.asarray(Q, dtype=np.float64))
        U = np.full(Q.shape[0], np.inf)
        G = np.zeros_like(Q)
        for i, q in enumerate(Q):
            if np.all((q >= self.bounds[:, 0]) & (q <= self.bounds[:, 1])):
                U[i], G[i] = self.one(q)
        return U, G


def hmc(potential: Callable, q0: np.ndarray, n_iter: int, step: float, n_leap: int,
        inv_mass: np.ndarray, rng: np.random.Generator):
    """Hamiltonian Monte Carlo for all chains at once.

    potential(q [n][k]) -> (U [n], dU/dq [n][k]); inv_mass: [k][k] (the
    kinetic energy is p^T inv_mass p / 2, momenta are drawn from N(0, inv_mass^-1)).
    Returns {"samples": [n_iter][n][k], "accept": [n_iter][n], "dH": [n_iter][n]}.
    """
    q = np.array(q0, dtype=np.float64)
    n, k = q.shape
    Minv = np.asarray(inv_mass, dtype=np.float64)
    L_mass = np.linalg.cholesky(np.linalg.inv(Minv))  # p = L_mass z ~ N(0, M)
    U, g = potential(q)
    samples = np.empty((n_iter, n, k))
    accept = np.zeros((n_iter, n), dtype=bool)
    dH = np.zeros((n_iter, n))
    for it in range(n_iter):
        p0 = rng.standard_normal((n, k)) @ L_mass.T
        qn, p = q.copy(), p0.copy()
        p = p - 0.5 * step * g
        Un, gn = U, g
        for j in range(n_leap):
            qn = qn + step * p @ Minv.T
            Un, gn = potential(qn)
            if j < n_leap - 1:
                p = p - step * gn
        p = p - 0.5 * step * gn
        H0 = U + 0.5 * np.einsum("ni,ij,nj->n", p0, Minv, p0)
        H1 = Un + 0.5 * np.einsum("ni,ij,nj->n", p, Minv, p)
        d = H1 - H0
        acc = np.isfinite(d) & (np.log(rng.uniform(size=n)) < -d)
        q[acc], U[acc], g[acc] = qn[acc], Un[acc], gn[acc]
        samples[it], accept[it], dH[it] = q, acc, np.where(np.isfinite(d), d, np.inf)
    return {"samples": samples, "accept": accept, "dH": dH}


def ess(x: np.ndarray) -> float:
    """Effective sample size of chains x [n_iter][n_chains] (one parameter): the
    chain-averaged autocorrelation summed with Geyer's initial positive
    sequence (Geyer 1992), times the number of draws."""
    x = np.asarray(x, dtype=np.float64)
    T, C = x.shape
    xc = x - x.mean(axis=0)
    var = (xc ** 2).mean()
    if var == 0.0:
        return float(T * C)
    f = np.fft.rfft(xc, n=2 * T, axis=0)
    ac = np.fft.irfft(f * np.conj(f), axis=0)[:T].mean(axis=1) / (T * var)
    tau = -1.0
    for t in range(0, T - 1, 2):
        pair = ac[t] + ac[t + 1]
        if pair <= 0.0:
            break
        tau += 2.0 * pair
    return float(T * C / max(tau, 1.0 / (T * C)))


def laplace_inv_mass(potential_grad: Callable, q_star: np.ndarray, h: np.ndarray) -> np.ndarray:
    """Inverse Hessian of U at q_star from central differences of the exact
    gradient (one batch evaluation of 2k parameter sets), symmetrised."""
    k = q_star.size
    Q = np.tile(q_star, (2 * k, 1))
    for i in range(k):
        Q[2 * i, i] += h[i]
        Q[2 * i + 1, i] -= h[i]
    _, G = potential_grad(Q)
    H = np.empty((k, k))
    for i in range(k):
        H[i] = (G[2 * i] - G[2 * i + 1]) / (2 * h[i])
    H = 0.5 * (H + H.T)
    return np.linalg.inv(H)
